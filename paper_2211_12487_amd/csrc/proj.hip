// Fused projection kernel for the levels whose core is narrow (the
// HBM-bound level 1 of every increment and the chain projection of TT-ICE*).
//
// For every column z_j of the level unfolding [Z(0) ... Z(N-1)] (rows x
// N*cols; eq:first_resid, eq:project_further) one pass over the data gives
//   c_j = U^T z_j            (written to the next level / the last core),
//   ||z_j||^2                (Corollary 1's ||Y||, eq:relerror's ||Y(b)||),
//   ||z_j||^2 - ||c_j||^2    = ||(I - U U^T) z_j||^2 for orthonormal U
// (the residual energy of eq:first_resid / eq:ithresidual by Pythagoras; in
// FP64 the cancellation costs ~1e-13 relative at the tolerances used, so the
// residual itself is only formed when a core is actually updated).
//
// Layout: a block owns 64 consecutive columns (one per lane) and splits the
// rows over its 4 waves; U (rows x r, FP64) is staged in LDS and read as
// wave-wide broadcasts; each lane keeps RMAX FP64 accumulators; the 4 row
// partials are combined through LDS in a fixed order.  Loads of Z are
// coalesced along the columns of a frame (a frame boundary inside a wave's
// 64 columns only splits its load into two runs).
#include "kernels.h"

namespace ttice {
namespace {

constexpr int kProjWaves = 4;

template <typename TIn, typename TOut, int RMAX>
__global__ __launch_bounds__(64 * kProjWaves) void k_proj_col(int32_t rows, int32_t r, int32_t Ncol, View vz,
                                                              const TIn* __restrict__ Z, const double* __restrict__ U,
                                                              int64_t ldu, TOut* __restrict__ C, View vc,
                                                              double* __restrict__ znorm2,
                                                              double* __restrict__ rho2) {
  HIP_DYNAMIC_SHARED(double, lds);
  double* Us = lds;                               // rows x RMAX (zero-padded)
  double* part = lds + (int64_t)rows * RMAX;      // kProjWaves x (RMAX + 1) x 64
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t q = threadIdx.x; q < (int64_t)rows * RMAX; q += 64 * kProjWaves) {
    const int32_t i = (int32_t)(q / RMAX), k = (int32_t)(q % RMAX);
    Us[q] = k < r ? U[(int64_t)i * ldu + k] : 0.0;
  }
  __syncthreads();
  const int32_t j = (int32_t)blockIdx.x * 64 + lane;
  const bool valid = j < Ncol;
  const TIn* zc = Z + (valid ? col_off(vz, j) : 0);
  // rows of this wave: [i0, i1)
  const int32_t per = (rows + kProjWaves - 1) / kProjWaves;
  const int32_t i0 = wid * per, i1 = min(rows, i0 + per);
  double acc[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; ++k) acc[k] = 0.0;
  double zz = 0.0;
  if (valid) {
    int32_t i = i0;
    for (; i + 4 <= i1; i += 4) {
      double z[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) z[u] = (double)zc[row_off(vz, i + u)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        zz = fma(z[u], z[u], zz);
        const double* ui = Us + (int64_t)(i + u) * RMAX;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) acc[k] = fma(ui[k], z[u], acc[k]);
      }
    }
    for (; i < i1; ++i) {
      const double z = (double)zc[row_off(vz, i)];
      zz = fma(z, z, zz);
      const double* ui = Us + (int64_t)i * RMAX;
#pragma unroll
      for (int k = 0; k < RMAX; ++k) acc[k] = fma(ui[k], z, acc[k]);
    }
  }
  // combine the row partials of the 4 waves (fixed order)
  double* pw = part + (int64_t)wid * (RMAX + 1) * 64;
#pragma unroll
  for (int k = 0; k < RMAX; ++k) pw[k * 64 + lane] = acc[k];
  pw[RMAX * 64 + lane] = zz;
  __syncthreads();
  if (wid == 0 && valid) {
    double cc = 0.0;
    const int64_t co = col_off(vc, j);
    for (int k = 0; k < r; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kProjWaves; ++w) s += part[(int64_t)w * (RMAX + 1) * 64 + k * 64 + lane];
      if (C) C[row_off(vc, k) + co] = (TOut)s;
      cc = fma(s, s, cc);
    }
    double zs = 0.0;
#pragma unroll
    for (int w = 0; w < kProjWaves; ++w) zs += part[(int64_t)w * (RMAX + 1) * 64 + RMAX * 64 + lane];
    if (znorm2) znorm2[j] = zs;
    if (rho2) rho2[j] = zs - cc;
  }
}

template <typename TIn, typename TOut, int RMAX>
hipError_t launch_proj(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                       const double* U, int64_t ldu, TOut* C, View vc, double* znorm2, double* rho2) {
  const size_t lds = ((size_t)rows * RMAX + (size_t)kProjWaves * (RMAX + 1) * 64) * sizeof(double);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_proj_col<TIn, TOut, RMAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_proj_col<TIn, TOut, RMAX>), dim3((unsigned)((Ncol + 63) / 64)), dim3(64 * kProjWaves), lds,
                     st, rows, r, Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
  return hipGetLastError();
}

}  // namespace

bool proj_fits(int32_t rows, int32_t r) {
  if (r > 64 || rows <= 0) return false;
  const int32_t R = r <= 8 ? 8 : (r <= 16 ? 16 : (r <= 32 ? 32 : 64));
  return ((size_t)rows * R + (size_t)kProjWaves * (R + 1) * 64) * sizeof(double) <= 150 * 1024;
}

template <typename TIn, typename TOut>
hipError_t proj_columns(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                        const double* U, int64_t ldu, TOut* C, View vc, double* znorm2, double* rho2) {
  if (Ncol <= 0) return hipSuccess;
  if (r <= 8) return launch_proj<TIn, TOut, 8>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2);
  if (r <= 16) return launch_proj<TIn, TOut, 16>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2);
  if (r <= 32) return launch_proj<TIn, TOut, 32>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2);
  return launch_proj<TIn, TOut, 64>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2);
}

template hipError_t proj_columns<float, double>(hipStream_t, int32_t, int32_t, int32_t, const float*, View,
                                                const double*, int64_t, double*, View, double*, double*);
template hipError_t proj_columns<double, double>(hipStream_t, int32_t, int32_t, int32_t, const double*, View,
                                                 const double*, int64_t, double*, View, double*, double*);

}  // namespace ttice
