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
// The product runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64: a
// 16 x 4 tile of U^T times a 4 x 16 tile of Z per instruction).  Layout:
//  * a block owns 16*VEC consecutive columns; lane (kq = lane / 16,
//    n = lane % 16) holds VEC consecutive columns 16*VEC*blk + VEC*n + g of
//    row 4*q + kq of every row quad q, loaded as one VEC-wide vector (one
//    load instruction moves 4 rows x 16*VEC columns), and column slot g
//    feeds MFMA group g;
//  * the A operand of quad q is U[4q + kq, 16t + n] (one FP64 per lane per
//    16-wide tile t of U's columns; U is small and cache resident);
//  * the W waves of a block split the row quads, and their FP64 partial
//    tiles are summed by a fixed-order tree through LDS (deterministic);
//  * output element i of a D tile on lane (kq, n) is row 16t + 4i + kq.
// VEC > 1 needs the columns of a frame, the row and frame strides and the
// base pointers of Z and C to be VEC-aligned (checked on the host).
#include <hip/hip_ext.h>

#include "proj_common.h"

namespace ttice {
namespace {

using proj::aligned_cols;
using proj::kChunkQuads;
using proj::store_vec;
using proj::Vec;
typedef double d4 __attribute__((ext_vector_type(4)));

// the kernel body for column block blk
template <typename TIn, int VEC, int RT, int W>
__device__ __forceinline__ void proj_mfma_body(int32_t blk, int32_t rows, int32_t r, int32_t Ncol, View vz,
                                               const TIn* __restrict__ Z, const double* __restrict__ U, int64_t ldu,
                                               double* __restrict__ C, View vc, double* __restrict__ znorm2,
                                               double* __restrict__ rho2) {
  constexpr int NV = RT * VEC * 4 + VEC;  // doubles per lane: D tiles + ||z||^2 partials
  HIP_DYNAMIC_SHARED(double, red);        // (W / 2) x NV x 64
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kq = lane >> 4, n = lane & 15;
  const int32_t j = blk * (16 * VEC) + VEC * n;  // first of this lane's VEC columns
  const bool valid = j < Ncol;
  // lanes past the last column read column 0 and are never stored
  const int64_t coff = valid ? col_off(vz, j) : 0;
  const int64_t rs = vz.rs;
  const int32_t nq = (rows + 3) >> 2;
  const int32_t per = (nq + W - 1) / W;
  const int32_t q0 = wid * per, q1 = min(nq, q0 + per);

  d4 acc[RT][VEC];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int g = 0; g < VEC; ++g) acc[t][g] = d4{0.0, 0.0, 0.0, 0.0};
  double zz[VEC];
#pragma unroll
  for (int g = 0; g < VEC; ++g) zz[g] = 0.0;

  for (int32_t qb = q0; qb < q1; qb += kChunkQuads) {
    // all loads of the chunk first (rows clamped in bounds, masked below)
    Vec<TIn, VEC> zr[kChunkQuads];
    double ur[kChunkQuads][RT];
#pragma unroll
    for (int u = 0; u < kChunkQuads; ++u) {
      const int32_t i = min((qb + u) * 4 + kq, rows - 1);
      zr[u] = Vec<TIn, VEC>::load(Z + (int64_t)i * rs + coff);
#pragma unroll
      for (int t = 0; t < RT; ++t) ur[u][t] = U[(int64_t)i * ldu + 16 * t + n];
    }
#pragma unroll
    for (int u = 0; u < kChunkQuads; ++u) {
      const bool live = qb + u < q1 && (qb + u) * 4 + kq < rows;
#pragma unroll
      for (int g = 0; g < VEC; ++g) {
        const double z = live ? (double)zr[u].v[g] : 0.0;
        zz[g] = fma(z, z, zz[g]);
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(ur[u][t], z, acc[t][g], 0, 0, 0);
      }
    }
  }

  // fixed-order tree over the waves' row partials
#pragma unroll
  for (int h = W / 2; h >= 1; h /= 2) {
    if (wid >= h && wid < 2 * h) {
      double* o = red + (int64_t)(wid - h) * NV * 64 + lane;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int g = 0; g < VEC; ++g)
#pragma unroll
          for (int i = 0; i < 4; ++i) o[((t * VEC + g) * 4 + i) * 64] = acc[t][g][i];
#pragma unroll
      for (int g = 0; g < VEC; ++g) o[(RT * VEC * 4 + g) * 64] = zz[g];
    }
    __syncthreads();
    if (wid < h) {
      const double* o = red + (int64_t)wid * NV * 64 + lane;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int g = 0; g < VEC; ++g)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[t][g][i] += o[((t * VEC + g) * 4 + i) * 64];
#pragma unroll
      for (int g = 0; g < VEC; ++g) zz[g] += o[(RT * VEC * 4 + g) * 64];
    }
    __syncthreads();
  }
  if (wid != 0) return;

  double cc[VEC];
#pragma unroll
  for (int g = 0; g < VEC; ++g) cc[g] = 0.0;
  const int64_t co = valid ? col_off(vc, j) : 0;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * t + 4 * i + kq;
      if (m < r) {
        double v[VEC];
#pragma unroll
        for (int g = 0; g < VEC; ++g) {
          v[g] = acc[t][g][i];
          cc[g] = fma(v[g], v[g], cc[g]);
        }
        if (C && valid) store_vec<VEC>(C + row_off(vc, m) + co, v);
      }
    }
  // sum over the four row phases kq (lanes n, n + 16, n + 32, n + 48)
#pragma unroll
  for (int g = 0; g < VEC; ++g) {
    cc[g] += __shfl_xor(cc[g], 16);
    cc[g] += __shfl_xor(cc[g], 32);
    zz[g] += __shfl_xor(zz[g], 16);
    zz[g] += __shfl_xor(zz[g], 32);
  }
  if (kq == 0 && valid) {
    if (znorm2) store_vec<VEC>(znorm2 + j, zz);
    if (rho2) {
      double e[VEC];
#pragma unroll
      for (int g = 0; g < VEC; ++g) e[g] = zz[g] - cc[g];
      store_vec<VEC>(rho2 + j, e);
    }
  }
}

template <typename TIn, int VEC, int RT, int W>
__global__ __launch_bounds__(64 * W) void k_proj_mfma(int32_t rows, int32_t r, int32_t Ncol, View vz,
                                                      const TIn* __restrict__ Z, const double* __restrict__ U,
                                                      int64_t ldu, double* __restrict__ C, View vc,
                                                      double* __restrict__ znorm2, double* __restrict__ rho2) {
  proj_mfma_body<TIn, VEC, RT, W>((int32_t)blockIdx.x, rows, r, Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
}

// Several projections in one launch (one column per lane): block b belongs
// to the descriptor q with g.start[q] <= b < g.start[q + 1], and computes
// exactly what the single launch's block b - g.start[q] computes.
template <typename TIn, int RT, int W>
__global__ __launch_bounds__(64 * W) void k_proj_mfma_group(ProjGroup g) {
  int q = 0;
  while (q + 1 < g.n && (int32_t)blockIdx.x >= g.start[q + 1]) ++q;
  const ProjDesc& p = g.d[q];
  proj_mfma_body<TIn, 1, RT, W>((int32_t)blockIdx.x - g.start[q], p.rows, p.r, p.Ncol, p.vz, (const TIn*)p.Z, p.U,
                                p.ldu, p.C, p.vc, p.znorm2, p.rho2);
}

template <typename TIn, int VEC, int RT, int W>
hipError_t launch_proj_w(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                         const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                         hipEvent_t ev0, hipEvent_t ev1) {
  constexpr size_t lds = proj::red_bytes(W, RT * VEC * 4 + VEC);
  static_assert(lds <= 80 * 1024, "reduction buffer");
  // once per process (thread-safe static initialisation)
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_proj_mfma<TIn, VEC, RT, W>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const int32_t cols_per_block = 16 * VEC;
  const dim3 grid((unsigned)((Ncol + cols_per_block - 1) / cols_per_block));
  if (ev0 || ev1)
    hipExtLaunchKernelGGL((k_proj_mfma<TIn, VEC, RT, W>), grid, dim3(64 * W), (uint32_t)lds, st, ev0, ev1, 0u, rows,
                          r, Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
  else
    hipLaunchKernelGGL((k_proj_mfma<TIn, VEC, RT, W>), grid, dim3(64 * W), lds, st, rows, r, Ncol, vz, Z, U, ldu, C,
                       vc, znorm2, rho2);
  return hipGetLastError();
}

// Waves per block: enough to give each a chunk of row quads, so short
// columns (a few quads) take one or two waves and no idle ones or LDS sum.
template <typename TIn, int VEC, int RT>
hipError_t launch_proj(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                       const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                       hipEvent_t ev0, hipEvent_t ev1) {
  const int32_t nq = (rows + 3) / 4;
  if (nq <= kChunkQuads)
    return launch_proj_w<TIn, VEC, RT, 1>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (nq <= 2 * kChunkQuads)
    return launch_proj_w<TIn, VEC, RT, 2>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_proj_w<TIn, VEC, RT, RT == 4 ? 4 : 8>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0,
                                                      ev1);
}

template <typename TIn, int VEC>
hipError_t launch_rt(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                     const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                     hipEvent_t ev0, hipEvent_t ev1) {
  if (r <= 16) return launch_proj<TIn, VEC, 1>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (r <= 32) return launch_proj<TIn, VEC, 2>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_proj<TIn, VEC, 4>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
}

}  // namespace

bool proj_fits(int32_t rows, int32_t r) { return r <= 64 && rows > 0; }

template <typename TIn>
hipError_t proj_columns(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                        const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2, int prec,
                        hipEvent_t ev0, hipEvent_t ev1, int vmax, bool* rho_explicit) {
  if (rho_explicit) *rho_explicit = false;
  if (Ncol <= 0) return hipSuccess;
  if (vz.rpf != kUnframed || vc.rpf != kUnframed || r > 64 || rows <= 0) return hipErrorInvalidValue;
  // the widest instantiation reads 16 * 4 doubles of every row of U
  static_assert(kProjTail >= 64, "core allocations must cover the widest row read");
  int vec = 1;
  for (int v : {4, 2}) {
    if (v <= vmax && (Ncol % v) == 0 && aligned_cols(vz, Z, sizeof(TIn), v) && (!C || aligned_cols(vc, C, sizeof(double), v))) {
      vec = v;
      break;
    }
  }
  // short columns (at most 8 rows) stream through the vector-ALU kernel
  if (vec == 4 && proj_short_fits(prec, rows, r)) {
    if (rho_explicit) *rho_explicit = true;
    return proj_columns_short<TIn>(st, prec, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  }
  // FP64 input: two columns per lane already load 16 bytes, and half the
  // accumulators of four leave room for three or four waves per SIMD
  if (sizeof(TIn) == 8 && vec == 4) vec = 2;
  if (prec != kProjFP64)
    return proj_columns_lp<TIn>(st, prec, vec, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (vec == 4) return launch_rt<TIn, 4>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (vec == 2) return launch_rt<TIn, 2>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_rt<TIn, 1>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
}

template hipError_t proj_columns<float>(hipStream_t, int32_t, int32_t, int32_t, const float*, View, const double*,
                                        int64_t, double*, View, double*, double*, int, hipEvent_t, hipEvent_t, int,
                                        bool*);
template hipError_t proj_columns<double>(hipStream_t, int32_t, int32_t, int32_t, const double*, View, const double*,
                                         int64_t, double*, View, double*, double*, int, hipEvent_t, hipEvent_t, int,
                                         bool*);

// ---- grouped launches (one column per lane, the single launch's shape)
int32_t proj_shape(int prec, int32_t rows, int32_t r) {
  const int32_t rt = r <= 16 ? 1 : r <= 32 ? 2 : 4;
  int32_t w;
  if (prec == kProjFP64) {
    const int32_t nq = (rows + 3) / 4;
    w = nq <= kChunkQuads ? 1 : nq <= 2 * kChunkQuads ? 2 : (rt == 4 ? 4 : 8);
  } else {
    const int32_t step = prec == kProjFP32 ? 4 * kChunkQuads : 32;
    const int32_t nb = (rows + step - 1) / step;
    w = nb <= 1 ? 1 : nb <= 2 ? 2 : 4;
  }
  return 8 * w + rt;
}

namespace {
template <typename TIn, int RT, int W>
hipError_t launch_group_w(hipStream_t st, const ProjGroup& g) {
  constexpr size_t lds = proj::red_bytes(W, RT * 4 + 1);
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_proj_mfma_group<TIn, RT, W>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_proj_mfma_group<TIn, RT, W>), dim3((unsigned)g.start[g.n]), dim3(64 * W), lds, st, g);
  return hipGetLastError();
}
template <typename TIn, int RT>
hipError_t launch_group_rt(hipStream_t st, const ProjGroup& g, int32_t w) {
  if (w == 1) return launch_group_w<TIn, RT, 1>(st, g);
  if (w == 2) return launch_group_w<TIn, RT, 2>(st, g);
  if (w == 4) return launch_group_w<TIn, RT, 4>(st, g);
  return launch_group_w<TIn, RT, 8>(st, g);
}
}  // namespace

template <typename TIn>
hipError_t proj_group(hipStream_t st, int prec, const ProjGroup& g) {
  if (g.n < 1 || g.n > kGroupMax || g.start[0] != 0) return hipErrorInvalidValue;
  const int32_t shape = proj_shape(prec, g.d[0].rows, g.d[0].r);
  for (int q = 0; q < g.n; ++q) {
    const ProjDesc& p = g.d[q];
    if (p.rows <= 0 || p.r < 0 || p.r > 64 || p.Ncol <= 0 || p.vz.rpf != kUnframed || p.vc.rpf != kUnframed ||
        proj_shape(prec, p.rows, p.r) != shape || g.start[q + 1] - g.start[q] != (p.Ncol + 15) / 16)
      return hipErrorInvalidValue;
  }
  if (prec != kProjFP64) return proj_group_lp<TIn>(st, prec, g);
  const int32_t w = shape / 8, rt = shape % 8;
  if (rt == 1) return launch_group_rt<TIn, 1>(st, g, w);
  if (rt == 2) return launch_group_rt<TIn, 2>(st, g, w);
  return launch_group_rt<TIn, 4>(st, g, w);
}
template hipError_t proj_group<float>(hipStream_t, int, const ProjGroup&);
template hipError_t proj_group<double>(hipStream_t, int, const ProjGroup&);

}  // namespace ttice
