// Reduced-precision variants of the fused column projection (see proj.hip
// for the FP64 kernel, the layout and the quantities computed):
//
//  * FP32: v_mfma_f32_16x16x4f32 on a 16 x 4 tile of U^T (rounded to FP32)
//    times a 4 x 16 tile of Z, FP32 accumulation;
//  * split BF16 ("BF16x3"): each FP32 operand x is written as hi + lo with
//    hi = bf16(x) and lo = bf16(x - hi) (16 significant bits together), and
//    U^T z is accumulated in FP32 from the three products hi*hi + hi*lo +
//    lo*hi on v_mfma_f32_16x16x32_bf16 (the lo*lo term is below FP32
//    rounding of the sum).
//
// In both, ||z||^2 is accumulated in FP64 from the input values and the
// residual energy ||z||^2 - ||c||^2 is formed in FP64 from the rounded
// coefficients.  The host engine takes the decision of the norm test again
// in FP64 when that energy lands within the rounding band of the tolerance.
//
// Output element i of an FP32-accumulated 16 x 16 tile on lane (kq, n) is
// row 4*kq + i, column n (measured on the device).
#include <hip/hip_ext.h>

#include "proj_common.h"

namespace ttice {
namespace {

using proj::kChunkQuads;
using proj::store_vec;
using proj::Vec;
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f8 __attribute__((ext_vector_type(8)));

// x = hi + lo + O(2^-16 |x|): hi = bf16(x), lo = bf16(x - hi), both rounded
// to nearest even by the hardware's packed FP32 -> BF16 conversion (two
// values per instruction; widening back to FP32 is a shift)
__device__ __forceinline__ void split_bf16(const f8& x, bf16x8& hi, bf16x8& lo) {
  hi = __builtin_convertvector(x, bf16x8);
  lo = __builtin_convertvector(x - __builtin_convertvector(hi, f8), bf16x8);
}

// Sum of the W waves' FP64 partials (NV per lane) into wave 0, in the fixed
// order w = 0, 1, ..., W-1: waves 1.. write theirs to LDS, one barrier, wave
// 0 adds them (one barrier in all, where a pairwise tree needs two per
// level).  red: (W-1) NV 64 doubles.
template <int W, int NV>
__device__ __forceinline__ void waves_to_first(double (&v)[NV], double* red, int wid, int lane) {
  if (W == 1) return;
  if (wid > 0) {
    double* o = red + (int64_t)(wid - 1) * NV * 64 + lane;
#pragma unroll
    for (int q = 0; q < NV; ++q) o[q * 64] = v[q];
  }
  __syncthreads();
  if (wid == 0)
#pragma unroll
    for (int w = 1; w < W; ++w) {
      const double* o = red + (int64_t)(w - 1) * NV * 64 + lane;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] += o[q * 64];
    }
}
constexpr size_t flat_red_bytes(int W, int NV) { return (size_t)(W > 1 ? W - 1 : 1) * NV * 64 * sizeof(double); }
constexpr size_t kRedBudget = 80 * 1024;

// Pairwise fixed-order tree (two barriers per level, half the LDS of the
// flat sum), for partials too wide for the flat buffer.
template <int W, int NV>
__device__ __forceinline__ void wave_tree(double (&v)[NV], double* red, int wid, int lane) {
#pragma unroll
  for (int h = W / 2; h >= 1; h /= 2) {
    if (wid >= h && wid < 2 * h) {
      double* o = red + (int64_t)(wid - h) * NV * 64 + lane;
#pragma unroll
      for (int q = 0; q < NV; ++q) o[q * 64] = v[q];
    }
    __syncthreads();
    if (wid < h) {
      const double* o = red + (int64_t)wid * NV * 64 + lane;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] += o[q * 64];
    }
    __syncthreads();
  }
}

template <int W, int NV>
constexpr bool use_flat() { return flat_red_bytes(W, NV) <= kRedBudget; }
template <int W, int NV>
constexpr size_t red_lds_bytes() { return use_flat<W, NV>() ? flat_red_bytes(W, NV) : proj::red_bytes(W, NV); }
template <int W, int NV>
__device__ __forceinline__ void reduce_waves(double (&v)[NV], double* red, int wid, int lane) {
  if constexpr (use_flat<W, NV>())
    waves_to_first<W, NV>(v, red, wid, lane);
  else
    wave_tree<W, NV>(v, red, wid, lane);
}

// Wave 0's epilogue: v holds the RT x VEC x 4 tile values (element i of tile
// (t, g) is row 16t + 4kq + i) then the VEC column energies.
template <int VEC, int RT, int NV>
__device__ __forceinline__ void proj_store(const double (&v)[NV], int kq, bool valid, int32_t j, int32_t r,
                                           double* __restrict__ C, const View& vc, double* __restrict__ znorm2,
                                           double* __restrict__ rho2) {
  double cc[VEC], zz[VEC];
#pragma unroll
  for (int g = 0; g < VEC; ++g) {
    cc[g] = 0.0;
    zz[g] = v[RT * VEC * 4 + g];
  }
  const int64_t co = valid ? col_off(vc, j) : 0;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * t + 4 * kq + i;
      if (m < r) {
        double c[VEC];
#pragma unroll
        for (int g = 0; g < VEC; ++g) {
          c[g] = v[(t * VEC + g) * 4 + i];
          cc[g] = fma(c[g], c[g], cc[g]);
        }
        if (C && valid) store_vec<VEC>(C + row_off(vc, m) + co, c);
      }
    }
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

// ---- FP32 matrix cores: row quads, as the FP64 kernel
template <typename TIn, int VEC, int RT, int W>
__device__ __forceinline__ void f32_body(int32_t blk, int32_t rows, int32_t r, int32_t Ncol, View vz,
                                         const TIn* __restrict__ Z, const double* __restrict__ U, int64_t ldu,
                                         double* __restrict__ C, View vc, double* __restrict__ znorm2,
                                         double* __restrict__ rho2) {
  constexpr int NV = RT * VEC * 4 + VEC;
  HIP_DYNAMIC_SHARED(double, red);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kq = lane >> 4, n = lane & 15;
  const int32_t j = blk * (16 * VEC) + VEC * n;
  const bool valid = j < Ncol;
  const int64_t coff = valid ? col_off(vz, j) : 0;
  const int64_t rs = vz.rs;
  const int32_t nq = (rows + 3) >> 2;
  const int32_t per = (nq + W - 1) / W;
  const int32_t q0 = wid * per, q1 = min(nq, q0 + per);

  f4 acc[RT][VEC];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int g = 0; g < VEC; ++g) acc[t][g] = f4{0.f, 0.f, 0.f, 0.f};
  double zz[VEC];
#pragma unroll
  for (int g = 0; g < VEC; ++g) zz[g] = 0.0;

  for (int32_t qb = q0; qb < q1; qb += kChunkQuads) {
    Vec<TIn, VEC> zr[kChunkQuads];
    float ur[kChunkQuads][RT];
#pragma unroll
    for (int u = 0; u < kChunkQuads; ++u) {
      const int32_t i = min((qb + u) * 4 + kq, rows - 1);
      zr[u] = Vec<TIn, VEC>::load(Z + (int64_t)i * rs + coff);
#pragma unroll
      for (int t = 0; t < RT; ++t) ur[u][t] = (float)U[(int64_t)i * ldu + 16 * t + n];
    }
#pragma unroll
    for (int u = 0; u < kChunkQuads; ++u) {
      const bool live = qb + u < q1 && (qb + u) * 4 + kq < rows;
#pragma unroll
      for (int g = 0; g < VEC; ++g) {
        const double zd = live ? (double)zr[u].v[g] : 0.0;
        zz[g] = fma(zd, zd, zz[g]);
        const float z = (float)zd;
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[u][t], z, acc[t][g], 0, 0, 0);
      }
    }
  }
  double v[NV];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int g = 0; g < VEC; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[(t * VEC + g) * 4 + i] = (double)acc[t][g][i];
#pragma unroll
  for (int g = 0; g < VEC; ++g) v[RT * VEC * 4 + g] = zz[g];
  reduce_waves<W, NV>(v, red, wid, lane);
  if (wid != 0) return;
  proj_store<VEC, RT, NV>(v, kq, valid, j, r, C, vc, znorm2, rho2);
}

// ---- split BF16 on BF16 matrix cores: row blocks of 32, lane (kq, n) holds
// rows 8kq .. 8kq+7 of the block (the 16x16x32 operand layout)
constexpr int kOcts = 2;  // 32-row blocks whose loads are issued together

template <typename TIn, int VEC, int RT, int W>
__device__ __forceinline__ void bf3_body(int32_t blk, int32_t rows, int32_t r, int32_t Ncol, View vz,
                                         const TIn* __restrict__ Z, const double* __restrict__ U, int64_t ldu,
                                         double* __restrict__ C, View vc, double* __restrict__ znorm2,
                                         double* __restrict__ rho2) {
  constexpr int NV = RT * VEC * 4 + VEC;
  HIP_DYNAMIC_SHARED(double, red);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kq = lane >> 4, n = lane & 15;
  const int32_t j = blk * (16 * VEC) + VEC * n;
  const bool valid = j < Ncol;
  const int64_t coff = valid ? col_off(vz, j) : 0;
  const int64_t rs = vz.rs;
  const int32_t no = (rows + 31) >> 5;
  const int32_t per = (no + W - 1) / W;
  const int32_t o0 = wid * per, o1 = min(no, o0 + per);

  f4 acc[RT][VEC];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int g = 0; g < VEC; ++g) acc[t][g] = f4{0.f, 0.f, 0.f, 0.f};
  double zz[VEC];
#pragma unroll
  for (int g = 0; g < VEC; ++g) zz[g] = 0.0;

  for (int32_t ob = o0; ob < o1; ob += kOcts) {
    Vec<TIn, VEC> zr[kOcts][8];
    double ur[kOcts][8][RT];
#pragma unroll
    for (int o = 0; o < kOcts; ++o)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t i = min((ob + o) * 32 + 8 * kq + q, rows - 1);
        zr[o][q] = Vec<TIn, VEC>::load(Z + (int64_t)i * rs + coff);
#pragma unroll
        for (int t = 0; t < RT; ++t) ur[o][q][t] = U[(int64_t)i * ldu + 16 * t + n];
      }
#pragma unroll
    for (int o = 0; o < kOcts; ++o) {
      if (ob + o >= o1) break;  // uniform over the wave
      bf16x8 ahi[RT], alo[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        f8 a;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool live = (ob + o) * 32 + 8 * kq + q < rows;
          a[q] = live ? (float)ur[o][q][t] : 0.f;
        }
        split_bf16(a, ahi[t], alo[t]);
      }
#pragma unroll
      for (int g = 0; g < VEC; ++g) {
        f8 z;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool live = (ob + o) * 32 + 8 * kq + q < rows;
          const double zd = live ? (double)zr[o][q].v[g] : 0.0;
          zz[g] = fma(zd, zd, zz[g]);
          z[q] = (float)zd;
        }
        bf16x8 bh, bl;
        split_bf16(z, bh, bl);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          acc[t][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[t], bh, acc[t][g], 0, 0, 0);
          acc[t][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[t], bl, acc[t][g], 0, 0, 0);
          acc[t][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[t], bh, acc[t][g], 0, 0, 0);
        }
      }
    }
  }
  double v[NV];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int g = 0; g < VEC; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[(t * VEC + g) * 4 + i] = (double)acc[t][g][i];
#pragma unroll
  for (int g = 0; g < VEC; ++g) v[RT * VEC * 4 + g] = zz[g];
  reduce_waves<W, NV>(v, red, wid, lane);
  if (wid != 0) return;
  proj_store<VEC, RT, NV>(v, kq, valid, j, r, C, vc, znorm2, rho2);
}

template <typename TIn, int VEC, int RT, int W>
__global__ __launch_bounds__(64 * W) void k_proj_f32(int32_t rows, int32_t r, int32_t Ncol, View vz,
                                                     const TIn* __restrict__ Z, const double* __restrict__ U,
                                                     int64_t ldu, double* __restrict__ C, View vc,
                                                     double* __restrict__ znorm2, double* __restrict__ rho2) {
  f32_body<TIn, VEC, RT, W>((int32_t)blockIdx.x, rows, r, Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
}
template <typename TIn, int VEC, int RT, int W>
__global__ __launch_bounds__(64 * W) void k_proj_bf3(int32_t rows, int32_t r, int32_t Ncol, View vz,
                                                     const TIn* __restrict__ Z, const double* __restrict__ U,
                                                     int64_t ldu, double* __restrict__ C, View vc,
                                                     double* __restrict__ znorm2, double* __restrict__ rho2) {
  bf3_body<TIn, VEC, RT, W>((int32_t)blockIdx.x, rows, r, Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
}

// Several projections in one launch (one column per lane; see ProjGroup)
template <int P, typename TIn, int RT, int W>
__global__ __launch_bounds__(64 * W) void k_proj_lp_group(ProjGroup g) {
  int q = 0;
  while (q + 1 < g.n && (int32_t)blockIdx.x >= g.start[q + 1]) ++q;
  const ProjDesc& p = g.d[q];
  const int32_t blk = (int32_t)blockIdx.x - g.start[q];
  if constexpr (P == kProjFP32)
    f32_body<TIn, 1, RT, W>(blk, p.rows, p.r, p.Ncol, p.vz, (const TIn*)p.Z, p.U, p.ldu, p.C, p.vc, p.znorm2, p.rho2);
  else
    bf3_body<TIn, 1, RT, W>(blk, p.rows, p.r, p.Ncol, p.vz, (const TIn*)p.Z, p.U, p.ldu, p.C, p.vc, p.znorm2, p.rho2);
}

template <int P, typename TIn, int VEC, int RT, int W>
hipError_t launch_lp_w(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz, const double* U,
                       int64_t ldu, double* C, View vc, double* znorm2, double* rho2, hipEvent_t ev0,
                       hipEvent_t ev1) {
  constexpr size_t lds = red_lds_bytes<W, RT * VEC * 4 + VEC>();
  static_assert(lds <= kRedBudget, "reduction buffer");
  const void* fn = P == kProjFP32 ? (const void*)k_proj_f32<TIn, VEC, RT, W> : (const void*)k_proj_bf3<TIn, VEC, RT, W>;
  // once per process (thread-safe static initialisation)
  static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((Ncol + 16 * VEC - 1) / (16 * VEC)));
  if constexpr (P == kProjFP32)
    hipExtLaunchKernelGGL((k_proj_f32<TIn, VEC, RT, W>), grid, dim3(64 * W), (uint32_t)lds, st, ev0, ev1, 0u, rows, r,
                          Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
  else
    hipExtLaunchKernelGGL((k_proj_bf3<TIn, VEC, RT, W>), grid, dim3(64 * W), (uint32_t)lds, st, ev0, ev1, 0u, rows, r,
                          Ncol, vz, Z, U, ldu, C, vc, znorm2, rho2);
  return hipGetLastError();
}

// Four waves split the row blocks (measured: beats eight, whose sum costs
// more); columns of at most one or two blocks of the kernel's row step (4
// rows FP32, 32 rows split BF16) per wave take one or two waves.
template <int P, typename TIn, int VEC, int RT>
hipError_t launch_lp(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz, const double* U,
                     int64_t ldu, double* C, View vc, double* znorm2, double* rho2, hipEvent_t ev0,
                     hipEvent_t ev1) {
  const int32_t step = P == kProjFP32 ? 4 * kChunkQuads : 32;
  const int32_t nb = (rows + step - 1) / step;
  if (nb <= 1)
    return launch_lp_w<P, TIn, VEC, RT, 1>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (nb <= 2)
    return launch_lp_w<P, TIn, VEC, RT, 2>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_lp_w<P, TIn, VEC, RT, 4>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
}

template <int P, typename TIn, int VEC>
hipError_t launch_lp_rt(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                        const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                        hipEvent_t ev0, hipEvent_t ev1) {
  if (r <= 16) return launch_lp<P, TIn, VEC, 1>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (r <= 32) return launch_lp<P, TIn, VEC, 2>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_lp<P, TIn, VEC, 4>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
}

template <int P, typename TIn>
hipError_t launch_lp_vec(hipStream_t st, int vec, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                         const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                         hipEvent_t ev0, hipEvent_t ev1) {
  if (vec == 4) return launch_lp_rt<P, TIn, 4>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (vec == 2) return launch_lp_rt<P, TIn, 2>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return launch_lp_rt<P, TIn, 1>(st, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
}

template <int P, typename TIn, int RT, int W>
hipError_t launch_lp_group_w(hipStream_t st, const ProjGroup& g) {
  constexpr size_t lds = red_lds_bytes<W, RT * 4 + 1>();
  static_assert(lds <= kRedBudget, "reduction buffer");
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_proj_lp_group<P, TIn, RT, W>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_proj_lp_group<P, TIn, RT, W>), dim3((unsigned)g.start[g.n]), dim3(64 * W), lds, st, g);
  return hipGetLastError();
}
template <int P, typename TIn, int RT>
hipError_t launch_lp_group_rt(hipStream_t st, const ProjGroup& g, int32_t w) {
  if (w == 1) return launch_lp_group_w<P, TIn, RT, 1>(st, g);
  if (w == 2) return launch_lp_group_w<P, TIn, RT, 2>(st, g);
  return launch_lp_group_w<P, TIn, RT, 4>(st, g);
}
template <int P, typename TIn>
hipError_t launch_lp_group(hipStream_t st, const ProjGroup& g, int32_t shape) {
  const int32_t w = shape / 8, rt = shape % 8;
  if (rt == 1) return launch_lp_group_rt<P, TIn, 1>(st, g, w);
  if (rt == 2) return launch_lp_group_rt<P, TIn, 2>(st, g, w);
  return launch_lp_group_rt<P, TIn, 4>(st, g, w);
}

}  // namespace

template <typename TIn>
hipError_t proj_columns_lp(hipStream_t st, int prec, int vec, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z,
                           View vz, const double* U, int64_t ldu, double* C, View vc, double* znorm2,
                           double* rho2, hipEvent_t ev0, hipEvent_t ev1) {
  if (prec == kProjFP32)
    return launch_lp_vec<kProjFP32, TIn>(st, vec, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  if (prec == kProjBF16x3)
    return launch_lp_vec<kProjBF16x3, TIn>(st, vec, rows, r, Ncol, Z, vz, U, ldu, C, vc, znorm2, rho2, ev0, ev1);
  return hipErrorInvalidValue;
}

template hipError_t proj_columns_lp<float>(hipStream_t, int, int, int32_t, int32_t, int32_t, const float*, View,
                                           const double*, int64_t, double*, View, double*, double*, hipEvent_t,
                                           hipEvent_t);
template hipError_t proj_columns_lp<double>(hipStream_t, int, int, int32_t, int32_t, int32_t, const double*, View,
                                            const double*, int64_t, double*, View, double*, double*, hipEvent_t,
                                            hipEvent_t);

// (descriptors validated by proj_group)
template <typename TIn>
hipError_t proj_group_lp(hipStream_t st, int prec, const ProjGroup& g) {
  const int32_t shape = proj_shape(prec, g.d[0].rows, g.d[0].r);
  if (prec == kProjFP32) return launch_lp_group<kProjFP32, TIn>(st, g, shape);
  if (prec == kProjBF16x3) return launch_lp_group<kProjBF16x3, TIn>(st, g, shape);
  return hipErrorInvalidValue;
}
template hipError_t proj_group_lp<float>(hipStream_t, int, const ProjGroup&);
template hipError_t proj_group_lp<double>(hipStream_t, int, const ProjGroup&);

}  // namespace ttice
