// Fused projection for unfoldings with at most 8 rows onto cores with at
// most 8 columns (the first level of a high-order stream: n_1 = 8 in the
// order-8 reshaped field), in FP64 or FP32 arithmetic.  Per column z_j it
// computes c_j = U^T z_j in the state's arithmetic (the next level's data,
// eq:project_further), ||z_j||^2, and the residual energy of eq:first_resid
// formed explicitly, ||z_j - U c~_j||^2 in FP64 from the rounded
// coefficients c~_j (= ||R||^2 + ||c~_j - c_j||^2 for orthonormal U: never
// below the true energy, so the norm test stays on the safe side in either
// arithmetic).  A column of 8 values is far too short for a matrix-core
// tile: the pass is a plain stream of the input (32 bytes per column) and of
// the FP64 outputs (up to 80 bytes per column).  Each thread owns one group
// of four consecutive columns (one thread per group: measured faster than
// grid-stride loops, which cost occupancy), loads all its rows at once with
// 16-byte nontemporal loads (the batch is read once), and applies U (staged
// per block in LDS, read as a broadcast) with vector FMAs.  Every sum runs
// in a fixed order (rows, then core columns).
#include <hip/hip_ext.h>

#include "proj_common.h"

namespace ttice {
namespace {

using proj::store_vec;
using proj::Vec;

constexpr int kShortThreads = 256;

// four consecutive 16- or 32-byte aligned values, read once (the scalar
// nontemporal loads merge into vector loads)
template <typename T>
__device__ __forceinline__ Vec<T, 4> load_once(const T* p) {
  const T* q = (const T*)__builtin_assume_aligned(p, 4 * sizeof(T));
  return Vec<T, 4>{{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1), __builtin_nontemporal_load(q + 2),
                    __builtin_nontemporal_load(q + 3)}};
}

// RHO: rho2 is written (a kernel without it holds fewer registers)
template <typename TIn, typename TA, bool RHO>
__global__ __launch_bounds__(kShortThreads) void k_proj_short(int32_t rows, int32_t r, int32_t ngroups, View vz,
                                                              const TIn* __restrict__ Z,
                                                              const double* __restrict__ U, int64_t ldu,
                                                              double* __restrict__ C, View vc,
                                                              double* __restrict__ znorm2,
                                                              double* __restrict__ rho2) {
  constexpr int R = kShortRows;
  // U[i][t] at [i R + t] in the arithmetic TA and in FP64, zero outside rows x r
  __shared__ TA us[R * R];
  __shared__ double ud[R * R];
  for (int q = threadIdx.x; q < R * R; q += kShortThreads) {
    const int i = q / R, t = q % R;
    const double u = (i < rows && t < r) ? U[(int64_t)i * ldu + t] : 0.0;
    us[q] = (TA)u;
    ud[q] = u;
  }
  __syncthreads();
  const int32_t g = (int32_t)blockIdx.x * kShortThreads + (int32_t)threadIdx.x;
  if (g >= ngroups) return;
  const int32_t j = 4 * g;
  const int64_t zo = col_off(vz, j);
  Vec<TIn, 4> z[R];
#pragma unroll
  for (int i = 0; i < R; ++i)
    if (i < rows) z[i] = load_once(Z + (int64_t)i * vz.rs + zo);
  double zz[4] = {0.0, 0.0, 0.0, 0.0};
  TA c[R][4];
#pragma unroll
  for (int t = 0; t < R; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) c[t][k] = (TA)0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i >= rows) break;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double zd = (double)z[i].v[k];
      zz[k] = fma(zd, zd, zz[k]);
      const TA za = (TA)zd;
#pragma unroll
      for (int t = 0; t < R; ++t) c[t][k] = fma(us[i * R + t], za, c[t][k]);
    }
  }
  const int64_t co = col_off(vc, j);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    if (t >= r) break;
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (double)c[t][k];
    if (C) store_vec<4>(C + row_off(vc, t) + co, v);
  }
  if (znorm2) store_vec<4>(znorm2 + j, zz);
  if constexpr (RHO) {
    // ||z - U c~||^2, row by row
    double e[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i >= rows) break;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double ri = (double)z[i].v[k];
#pragma unroll
        for (int t = 0; t < R; ++t) {
          if (t >= r) break;
          ri = fma(-ud[i * R + t], (double)c[t][k], ri);
        }
        e[k] = fma(ri, ri, e[k]);
      }
    }
    store_vec<4>(rho2 + j, e);
  }
}

template <typename TIn, typename TA>
hipError_t launch_short(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                        const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                        hipEvent_t ev0, hipEvent_t ev1) {
  const int32_t ngroups = Ncol / 4;
  const dim3 grid((unsigned)((ngroups + kShortThreads - 1) / kShortThreads));
  if (rho2)
    hipExtLaunchKernelGGL((k_proj_short<TIn, TA, true>), grid, dim3(kShortThreads), 0u, st, ev0, ev1, 0u, rows, r,
                          ngroups, vz, Z, U, ldu, C, vc, znorm2, rho2);
  else
    hipExtLaunchKernelGGL((k_proj_short<TIn, TA, false>), grid, dim3(kShortThreads), 0u, st, ev0, ev1, 0u, rows, r,
                          ngroups, vz, Z, U, ldu, C, vc, znorm2, rho2);
  return hipGetLastError();
}

}  // namespace

bool proj_short_fits(int prec, int32_t rows, int32_t r) {
  return (prec == kProjFP64 || prec == kProjFP32) && rows >= 1 && rows <= kShortRows && r >= 0 && r <= kShortRows;
}

template <typename TIn>
hipError_t proj_columns_short(hipStream_t st, int prec, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z,
                              View vz, const double* U, int64_t ldu, double* C, View vc, double* znorm2,
                              double* rho2, hipEvent_t ev0, hipEvent_t ev1) {
  if (!proj_short_fits(prec, rows, r) || (Ncol % 4) != 0 || Ncol <= 0) return hipErrorInvalidValue;
  if (prec == kProjFP32)
    return launch_short<TIn, float>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_short<TIn, double>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
}

template hipError_t proj_columns_short<float>(hipStream_t, int, int32_t, int32_t, int32_t, const float*, View,
                                              const double*, int64_t, double*, View, double*, double*, hipEvent_t,
                                              hipEvent_t);
template hipError_t proj_columns_short<double>(hipStream_t, int, int32_t, int32_t, int32_t, const double*, View,
                                               const double*, int64_t, double*, View, double*, double*, hipEvent_t,
                                               hipEvent_t);

}  // namespace ttice
