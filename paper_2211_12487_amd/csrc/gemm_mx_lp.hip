// Matrix-core tiled products (gemm_mx.h): the reduced arithmetics, split
// BF16 and FP32.
// Each operand is rounded to FP32 and split into hi = bf16(x) and
// lo = bf16(x - hi) when its K tile is written to LDS (hi and lo planes,
// rows padded to 40 bf16); a lane's eight consecutive k of a row are one
// 16-byte LDS read, the A operand of v_mfma_f32_16x16x32_bf16 (row n16,
// k 8 kq .. 8 kq + 7) or its B operand (column n16, the same k).  The
// small products lo*hi and hi*lo are accumulated before hi*hi.
#include "gemm_mx.h"

namespace ttice {
namespace mx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <>
struct Tile<kMxBF3> {
  static constexpr int PA = BK + 8;  // bf16 per row, hi and lo planes
  static constexpr int PB = BK + 8;
  static constexpr size_t bytes = (size_t)2 * (BM * PA + BN * PB) * sizeof(__bf16);
};

template <>
struct Acc<kMxBF3> {
  f4 v[2][4];
};

__device__ __forceinline__ void split2(double v, __bf16& hi, __bf16& lo) {
  const float x = (float)v;
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <>
struct Ops<kMxBF3> {
  static __device__ __forceinline__ void store_tile(void* buf, bool a_kfast, int32_t M, int32_t m0, int32_t N,
                                                    int32_t n0, int32_t k0, int32_t K, int t, const double (&a)[16],
                                                    const double (&b)[8]) {
    using T = Tile<kMxBF3>;
    const int bn = t & 63;
    const bool bvalid = n0 + bn < N;
    __bf16* Ah = (__bf16*)buf;
    __bf16* Al = Ah + BM * T::PA;
    __bf16* Bh = Al + BM * T::PA;
    __bf16* Bl = Bh + BN * T::PB;
    __bf16 hi, lo;
    if (a_kfast) {
      const int kk = t & 31;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int mm = (t >> 5) + 8 * u;
        split2((m0 + mm < M && k0 + kk < K) ? a[u] : 0.0, hi, lo);
        Ah[mm * T::PA + kk] = hi;
        Al[mm * T::PA + kk] = lo;
      }
    } else {
      const int mm = t & 127;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int kk = (t >> 7) + 2 * u;
        split2((m0 + mm < M && k0 + kk < K) ? a[u] : 0.0, hi, lo);
        Ah[mm * T::PA + kk] = hi;
        Al[mm * T::PA + kk] = lo;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kk = (t >> 6) + 4 * u;
      split2((bvalid && k0 + kk < K) ? b[u] : 0.0, hi, lo);
      Bh[bn * T::PB + kk] = hi;
      Bl[bn * T::PB + kk] = lo;
    }
  }

  static __device__ __forceinline__ void mma_tile(const void* buf, int w, int lane, Acc<kMxBF3>& acc) {
    using T = Tile<kMxBF3>;
    const int n16 = lane & 15, kq = lane >> 4;
    const __bf16* Ah = (const __bf16*)buf;
    const __bf16* Al = Ah + BM * T::PA;
    const __bf16* Bh = Al + BM * T::PA;
    const __bf16* Bl = Bh + BN * T::PB;
    bf16x8 ah[2], al[2], bh[4], bl[4];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      const int o = (32 * w + 16 * ti + n16) * T::PA + 8 * kq;
      __builtin_memcpy(&ah[ti], Ah + o, sizeof(bf16x8));
      __builtin_memcpy(&al[ti], Al + o, sizeof(bf16x8));
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      const int o = (16 * tj + n16) * T::PB + 8 * kq;
      __builtin_memcpy(&bh[tj], Bh + o, sizeof(bf16x8));
      __builtin_memcpy(&bl[tj], Bl + o, sizeof(bf16x8));
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        f4 c = acc.v[ti][tj];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ti], bh[tj], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ti], bl[tj], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ti], bh[tj], c, 0, 0, 0);
        acc.v[ti][tj] = c;
      }
  }
};

// FP32: operands rounded to FP32 in LDS, v_mfma_f32_16x16x4f32 (the A
// operand of lane (kq, n16) is row n16, k = kq of a 4-deep step; B column
// n16, the same k), FP32 accumulation.
constexpr int kMxF32 = kProjFP32;

template <>
struct Tile<kMxF32> {
  static constexpr int PA = kb<kMxF32>() + 1;  // floats per row (m-major, k contiguous)
  static constexpr int PB = kb<kMxF32>() + 1;
  static constexpr size_t bytes = (size_t)(BM * PA + BN * PB) * sizeof(float);
};

template <>
struct Acc<kMxF32> {
  f4 v[2][4];
};

template <>
struct Ops<kMxF32> {
  static __device__ __forceinline__ void store_tile(void* buf, bool a_kfast, int32_t M, int32_t m0, int32_t N,
                                                    int32_t n0, int32_t k0, int32_t K, int t,
                                                    const double (&a)[kb<kMxF32>() / 2],
                                                    const double (&b)[kb<kMxF32>() / 4]) {
    using T = Tile<kMxF32>;
    constexpr int KB = kb<kMxF32>();
    const int bn = t & 63;
    const bool bvalid = n0 + bn < N;
    float* As = (float*)buf;
    float* Bs = As + BM * T::PA;
    if (a_kfast) {
      const int kk = t & (KB - 1);
#pragma unroll
      for (int u = 0; u < KB / 2; ++u) {
        const int mm = t / KB + (kThreads / KB) * u;
        As[mm * T::PA + kk] = (m0 + mm < M && k0 + kk < K) ? (float)a[u] : 0.f;
      }
    } else {
      const int mm = t & 127;
#pragma unroll
      for (int u = 0; u < KB / 2; ++u) {
        const int kk = (t >> 7) + 2 * u;
        As[mm * T::PA + kk] = (m0 + mm < M && k0 + kk < K) ? (float)a[u] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < KB / 4; ++u) {
      const int kk = (t >> 6) + 4 * u;
      Bs[bn * T::PB + kk] = (bvalid && k0 + kk < K) ? (float)b[u] : 0.f;
    }
  }

  static __device__ __forceinline__ void mma_tile(const void* buf, int w, int lane, Acc<kMxF32>& acc) {
    using T = Tile<kMxF32>;
    const int n16 = lane & 15, kq = lane >> 4;
    const float* As = (const float*)buf;
    const float* Bs = As + BM * T::PA;
#pragma unroll
    for (int s = 0; s < kb<kMxF32>() / 4; ++s) {
      const int k = 4 * s + kq;
      float av[2], bv[4];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) av[ti] = As[(32 * w + 16 * ti + n16) * T::PA + k];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) bv[tj] = Bs[(16 * tj + n16) * T::PB + k];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc.v[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc.v[ti][tj], 0, 0, 0);
    }
  }
};

}  // namespace mx

template <typename TB, typename TE, typename TD>
hipError_t gemm_mx_bf3(hipStream_t st, int32_t M, int32_t N, int32_t K, double alpha, const double* A, View va,
                       const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd, double* colpart) {
  constexpr size_t lds = mx::lds_bytes<mx::kMxBF3>();
  static const hipError_t attr = hipFuncSetAttribute((const void*)mx::k_gemm_mx<mx::kMxBF3, TB, TE, TD>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((N + mx::BN - 1) / mx::BN), (unsigned)((M + mx::BM - 1) / mx::BM));
  hipLaunchKernelGGL((mx::k_gemm_mx<mx::kMxBF3, TB, TE, TD>), grid, dim3(mx::kThreads), lds, st, M, N, K, alpha, A,
                     va, B, vb, beta, E, ve, D, vd, colpart);
  return hipGetLastError();
}

template <typename TB, typename TE, typename TD>
hipError_t gemm_mx_f32(hipStream_t st, int32_t M, int32_t N, int32_t K, double alpha, const double* A, View va,
                       const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd, double* colpart) {
  constexpr size_t lds = mx::lds_bytes<mx::kMxF32>();
  static const hipError_t attr = hipFuncSetAttribute((const void*)mx::k_gemm_mx<mx::kMxF32, TB, TE, TD>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((N + mx::BN - 1) / mx::BN), (unsigned)((M + mx::BM - 1) / mx::BM));
  hipLaunchKernelGGL((mx::k_gemm_mx<mx::kMxF32, TB, TE, TD>), grid, dim3(mx::kThreads), lds, st, M, N, K, alpha, A,
                     va, B, vb, beta, E, ve, D, vd, colpart);
  return hipGetLastError();
}

#define TTICE_GEMM_BF3_INST(TB, TE, TD)                                                                          \
  template hipError_t gemm_mx_bf3<TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, double, const double*, View, \
                                              const TB*, View, double, const TE*, View, TD*, View, double*);    \
  template hipError_t gemm_mx_f32<TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, double, const double*, View, \
                                              const TB*, View, double, const TE*, View, TD*, View, double*);
TTICE_GEMM_BF3_INST(double, double, double)
TTICE_GEMM_BF3_INST(float, double, double)
TTICE_GEMM_BF3_INST(double, float, double)
TTICE_GEMM_BF3_INST(float, float, double)
TTICE_GEMM_BF3_INST(double, double, float)
TTICE_GEMM_BF3_INST(float, float, float)
TTICE_GEMM_BF3_INST(double, float, float)
TTICE_GEMM_BF3_INST(float, double, float)

}  // namespace ttice
