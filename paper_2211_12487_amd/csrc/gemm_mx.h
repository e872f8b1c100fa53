// Matrix-core tiled product of the level contractions (C = U^T Z, the next
// level's data, eq:project_further; and Z - U C with its column energies,
// eq:ithresidual), internal to the library.
//
// D = alpha A B + beta E over an M x N output, A FP64 (the cores' master
// copy), B of element type TB, in one of three arithmetics:
//  * P = kMxF64: v_mfma_f64_16x16x4f64, FP64 throughout;
//  * P = kProjFP32: operands rounded to FP32, v_mfma_f32_16x16x4f32 with
//    FP32 accumulation;
//  * P = kMxBF3: split BF16, each operand rounded to FP32 and written as
//    hi + lo bf16 (hi = bf16(x), lo = bf16(x - hi)), the three products
//    hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32
//    accumulation (the lo*lo term is below that sum's rounding).
// Block tile 128 x 64 (four waves of 32 rows x 64 columns, 2 x 4 MFMA tiles
// of 16 x 16 each), K in tiles staged through two LDS buffers (one barrier
// per K tile, the next tile's global loads in flight during the current
// tile's products): 32 deep for split BF16, 16 for FP64 and FP32, whose
// smaller buffers and prefetch registers let three blocks share a CU, so one
// block's barrier and loads overlap the others' products.  Operands are rounded to the arithmetic when
// they are written to LDS.  Views: A unframed (row or column stride 1 picks
// the coalesced load order), B, E and D with unframed rows (columns may be
// framed and renumbered).  The optional column energies colpart[mb N + n] =
// sum of D(m, n)^2 over the 64-row block mb (FP64, fixed order) match the
// other product kernels'.
#pragma once

#include "kernels.h"

namespace ttice {
namespace mx {

constexpr int kMxF64 = kProjFP64, kMxBF3 = kProjBF16x3;
constexpr int BM = 128, BN = 64, BK = 32;
// K tile depth per arithmetic (split BF16 needs 32: its instruction takes 32
// values of k)
template <int P>
constexpr int kb() { return P == kProjBF16x3 ? BK : 16; }
constexpr int kThreads = 256;

typedef double d4 __attribute__((ext_vector_type(4)));

// Per arithmetic: the LDS layout of one buffer (Tile), the accumulators
// (Acc), writing a K tile to LDS (store_tile) and its products (mma_tile).
// The split-BF16 ones are in gemm_mx_lp.hip.
template <int P>
struct Tile;
template <>
struct Tile<kMxF64> {
  static constexpr int PA = kb<kProjFP64>() + 1;  // doubles per A row (m-major, k contiguous)
  static constexpr int PB = kb<kProjFP64>() + 1;
  static constexpr size_t bytes = (size_t)(BM * PA + BN * PB) * sizeof(double);
};

template <int P>
constexpr size_t lds_bytes() { return 2 * Tile<P>::bytes; }

// Global loads of the K tile at k0, KB deep (clamped in-bounds positions,
// masked when written to LDS): KB / 2 values of A and KB / 4 of B per thread
template <int KB, typename TB>
__device__ __forceinline__ void load_tile(const double* __restrict__ A, const View& va, bool a_kfast, int32_t M,
                                          int32_t m0, const TB* __restrict__ B, const View& vb, int64_t bco,
                                          int32_t k0, int32_t K, int t, double (&a)[KB / 2], double (&b)[KB / 4]) {
  static_assert(KB == 16 || KB == 32, "K tile of 16 or 32");
  if (a_kfast) {
    const int kk = t & (KB - 1);
    const int32_t kc = min(k0 + kk, K - 1);
#pragma unroll
    for (int u = 0; u < KB / 2; ++u) {
      const int32_t m = min(m0 + t / KB + (kThreads / KB) * u, M - 1);
      a[u] = A[(int64_t)m * va.rs + (int64_t)kc * va.cs];
    }
  } else {
    const int mm = t & 127;
    const int32_t m = min(m0 + mm, M - 1);
#pragma unroll
    for (int u = 0; u < KB / 2; ++u) {
      const int32_t kc = min(k0 + (t >> 7) + 2 * u, K - 1);
      a[u] = A[(int64_t)m * va.rs + (int64_t)kc * va.cs];
    }
  }
#pragma unroll
  for (int u = 0; u < KB / 4; ++u) {
    const int32_t kc = min(k0 + (t >> 6) + 4 * u, K - 1);
    b[u] = (double)B[(int64_t)kc * vb.rs + bco];
  }
}

template <int P>
struct Acc;
template <>
struct Acc<kMxF64> {
  d4 v[2][4];
};

// Registers -> LDS buffer (zero outside the matrices)
template <int P>
struct Ops;
template <>
struct Ops<kMxF64> {
  static __device__ __forceinline__ void store_tile(void* buf, bool a_kfast, int32_t M, int32_t m0, int32_t N,
                                                    int32_t n0, int32_t k0, int32_t K, int t,
                                                    const double (&a)[kb<kMxF64>() / 2],
                                                    const double (&b)[kb<kMxF64>() / 4]) {
    using T = Tile<kMxF64>;
    constexpr int KB = kb<kMxF64>();
    const int bn = t & 63;
    const bool bvalid = n0 + bn < N;
    double* As = (double*)buf;
    double* Bs = As + BM * T::PA;
    if (a_kfast) {
      const int kk = t & (KB - 1);
#pragma unroll
      for (int u = 0; u < KB / 2; ++u) {
        const int mm = t / KB + (kThreads / KB) * u;
        As[mm * T::PA + kk] = (m0 + mm < M && k0 + kk < K) ? a[u] : 0.0;
      }
    } else {
      const int mm = t & 127;
#pragma unroll
      for (int u = 0; u < KB / 2; ++u) {
        const int kk = (t >> 7) + 2 * u;
        As[mm * T::PA + kk] = (m0 + mm < M && k0 + kk < K) ? a[u] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < KB / 4; ++u) {
      const int kk = (t >> 6) + 4 * u;
      Bs[bn * T::PB + kk] = (bvalid && k0 + kk < K) ? b[u] : 0.0;
    }
  }

  // Products of one LDS buffer into the wave's 2 x 4 tiles (rows 32 w ..)
  static __device__ __forceinline__ void mma_tile(const void* buf, int w, int lane, Acc<kMxF64>& acc) {
    using T = Tile<kMxF64>;
    const int n16 = lane & 15, kq = lane >> 4;
    const double* As = (const double*)buf;
    const double* Bs = As + BM * T::PA;
#pragma unroll
    for (int s = 0; s < kb<kMxF64>() / 4; ++s) {
      const int k = 4 * s + kq;
      double av[2], bv[4];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) av[ti] = As[(32 * w + 16 * ti + n16) * T::PA + k];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) bv[tj] = Bs[(16 * tj + n16) * T::PB + k];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc.v[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc.v[ti][tj], 0, 0, 0);
    }
  }
};

// Row of element i of tile ti on lane (kq, n16): the FP64 instruction's
// layout is row kq + 4 i, the FP32-accumulating ones' 4 kq + i.
template <int P>
__device__ __forceinline__ int tile_row(int kq, int i) {
  return P == kMxF64 ? kq + 4 * i : 4 * kq + i;
}

template <int P, typename TB, typename TE, typename TD>
__device__ __forceinline__ void gemm_mx_body(int32_t M, int32_t N, int32_t kbeg, int32_t K, double alpha,
                                             const double* __restrict__ A, View va, const TB* __restrict__ B,
                                             View vb, double beta, const TE* __restrict__ E, View ve,
                                             TD* __restrict__ D, View vd, double* __restrict__ colpart) {
  HIP_DYNAMIC_SHARED(unsigned char, lds);
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int32_t m0 = (int32_t)blockIdx.y * BM, n0 = (int32_t)blockIdx.x * BN;
  const bool a_kfast = va.cs == 1;
  const int64_t bco = col_off(vb, min(n0 + (t & 63), N - 1));
  Acc<P> acc;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc.v[ti][tj][i] = 0;

  constexpr int KB = kb<P>();
  double a[KB / 2], b[KB / 4];
  if (kbeg < K) load_tile<KB, TB>(A, va, a_kfast, M, m0, B, vb, bco, kbeg, K, t, a, b);
  int buf = 0;
  for (int32_t k0 = kbeg; k0 < K; k0 += KB) {
    void* cur = lds + buf * Tile<P>::bytes;
    Ops<P>::store_tile(cur, a_kfast, M, m0, N, n0, k0, K, t, a, b);
    __syncthreads();
    if (k0 + KB < K) load_tile<KB, TB>(A, va, a_kfast, M, m0, B, vb, bco, k0 + KB, K, t, a, b);
    Ops<P>::mma_tile(cur, w, lane, acc);
    buf ^= 1;
  }

  // epilogue: E read at clamped positions first, then masked
  const int n16 = lane & 15, kq = lane >> 4;
  double csq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
    const int32_t n = n0 + 16 * tj + n16;
    const int64_t eco = E ? col_off(ve, min(n, N - 1)) : 0;
    const int64_t dco = D ? col_off(vd, min(n, N - 1)) : 0;
    double ev[2][4];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t m = min(m0 + 32 * w + 16 * ti + tile_row<P>(kq, i), M - 1);
        ev[ti][i] = E ? (double)E[row_off(ve, m) + eco] : 0.0;
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t m = m0 + 32 * w + 16 * ti + tile_row<P>(kq, i);
        if (m >= M || n >= N) continue;
        double v = alpha * (double)acc.v[ti][tj][i];
        if (E) v = fma(beta, ev[ti][i], v);
        if (D) D[row_off(vd, m) + dco] = (TD)v;
        csq[tj] = fma(v, v, csq[tj]);
      }
  }
  if (colpart == nullptr) return;
  // per column: the four row phases kq, then the two waves of each 64-row
  // block in order
  __syncthreads();  // the LDS buffers are free
  double* red = (double*)lds;  // [4 waves][64 columns]
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
    double s = csq[tj];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (kq == 0) red[w * 64 + 16 * tj + n16] = s;
  }
  __syncthreads();
  if (t < 128) {
    const int h = t >> 6, c = t & 63;
    const int32_t n = n0 + c, mb = m0 / 64 + h;
    if (n < N && mb * 64 < M) colpart[(int64_t)mb * N + n] = red[(2 * h) * 64 + c] + red[(2 * h + 1) * 64 + c];
  }
}

// the reduced arithmetics (gemm_mx_lp.hip)
template <int P, typename TB, typename TE, typename TD>
__global__ __launch_bounds__(kThreads) void k_gemm_mx(int32_t M, int32_t N, int32_t K, double alpha,
                                                      const double* __restrict__ A, View va,
                                                      const TB* __restrict__ B, View vb, double beta,
                                                      const TE* __restrict__ E, View ve, TD* __restrict__ D,
                                                      View vd, double* __restrict__ colpart) {
  gemm_mx_body<P, TB, TE, TD>(M, N, 0, K, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart);
}

// FP64: registers held to three waves per SIMD, so three blocks (3 x 52 KB
// of LDS) share a CU
template <typename TB, typename TE, typename TD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_mx64(
    int32_t M, int32_t N, int32_t K, double alpha, const double* __restrict__ A, View va, const TB* __restrict__ B,
    View vb, double beta, const TE* __restrict__ E, View ve, TD* __restrict__ D, View vd,
    double* __restrict__ colpart) {
  gemm_mx_body<kMxF64, TB, TE, TD>(M, N, 0, K, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart);
}

// FP64, K split over grid z: slice z (K range [z kchunk, (z+1) kchunk))
// writes its partial product A B to part + z M N (M x N, row-major); a
// second kernel adds the slices in order and applies the epilogue
template <typename TB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_mx64_part(
    int32_t M, int32_t N, int32_t K, int32_t kchunk, const double* __restrict__ A, View va,
    const TB* __restrict__ B, View vb, double* __restrict__ part) {
  const int32_t kbeg = (int32_t)blockIdx.z * kchunk;
  const int32_t kend = min(K, kbeg + kchunk);
  View vp;
  vp.rs = N;
  vp.cs = 1;
  gemm_mx_body<kMxF64, TB, double, double>(M, N, kbeg, kend, 1.0, A, va, B, vb, 0.0, (const double*)nullptr,
                                           View(), part + (int64_t)blockIdx.z * M * N, vp, nullptr);
}

}  // namespace mx
}  // namespace ttice
