// gfx950 kernels of the TT-ICE library (generic FP64-accumulating paths).
//
// Every kernel here computes one step of TT-ICE (Algorithm 1 / Algorithm 2 of
// arXiv 2211.12487); the host engine (ttice.hip) sequences them.  Layouts:
// cores are row-major FP64, level data is frame-major [N][rows][cols].
#include "kernels.h"

#include <math.h>

#include <algorithm>

namespace ttice {

namespace {

// Shared epilogue of the tiled products: D(m,n) = alpha*acc + beta*E(m,n),
// and per-column sums of D^2 over the tile's rows into colpart.
template <typename TE, typename TD>
__device__ __forceinline__ void gemm_epilogue(double (&acc)[4][4], int32_t M, int32_t N, int32_t m0, int32_t n0,
                                              double alpha, double beta, const TE* __restrict__ E, const View& ve,
                                              TD* __restrict__ D, const View& vd, double* __restrict__ colpart,
                                              double* red) {
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  double csq[4] = {0.0, 0.0, 0.0, 0.0};
  // E is read from clamped in-bounds positions first (all loads in flight),
  // then masked; M > 0 and E != null are uniform.
  double ev[4][4];
  if (E && M > 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t ero = row_off(ve, min(m0 + ty + 16 * i, M - 1));
#pragma unroll
      for (int j = 0; j < 4; ++j) ev[i][j] = (double)E[ero + col_off(ve, min(n0 + tx + 16 * j, N - 1))];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int32_t m = m0 + ty + 16 * i;
    if (m >= M) continue;
    const int64_t dro = D ? row_off(vd, m) : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t n = n0 + tx + 16 * j;
      if (n >= N) continue;
      double v = alpha * acc[i][j];
      if (E) v = fma(beta, ev[i][j], v);
      if (D) D[dro + col_off(vd, n)] = (TD)v;
      csq[j] = fma(v, v, csq[j]);
    }
  }
  if (colpart != nullptr) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      red[t] = csq[j];
      __syncthreads();
      if (ty == 0) {
        double s = 0.0;
#pragma unroll
        for (int y = 0; y < 16; ++y) s += red[y * 16 + tx];
        const int32_t n = n0 + tx + 16 * j;
        if (n < N) colpart[(int64_t)blockIdx.y * N + n] = s;
      }
      __syncthreads();
    }
  }
}

// One K tile of 16 of the product: thread (lk, ln) loads rows lk, lk+4,
// lk+8, lk+12 of the tile (column ln of A^T and of B) from clamped in-bounds
// positions ...
template <typename TB>
__device__ __forceinline__ void gemm_load(const double* __restrict__ A, const View& va, int64_t aro, bool aload,
                                          const TB* __restrict__ B, const View& vb, int64_t bco, int32_t k0,
                                          int32_t ke, int lk, double (&av)[4], double (&bv)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int32_t kc = min(k0 + lk + 4 * u, ke - 1);
    av[u] = aload ? A[aro + col_off(va, kc)] : 0.0;
    bv[u] = (double)B[row_off(vb, kc) + bco];
  }
}
// ... stores them masked into an LDS buffer (returns their B squares) ...
__device__ __forceinline__ double gemm_store(int32_t k0, int32_t ke, int lk, int ln, bool avalid, bool bvalid,
                                             const double (&av)[4], const double (&bv)[4], double (*As)[65],
                                             double (*Bs)[65]) {
  double bsq = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int kk = lk + 4 * u;
    const bool kin = k0 + kk < ke;
    const double a = (kin && avalid) ? av[u] : 0.0;
    const double b = (kin && bvalid) ? bv[u] : 0.0;
    As[kk][ln] = a;
    Bs[kk][ln] = b;
    bsq = fma(b, b, bsq);
  }
  return bsq;
}
// ... and multiplies a buffered tile into the 4 x 4 micro-tile.
__device__ __forceinline__ void gemm_tile(const double (*As)[65], const double (*Bs)[65], int tx, int ty,
                                          double (&acc)[4][4]) {
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
  }
}

// Fixed-order sum of the S K-split partials of the elements e = e0 + t,
// e0 + t + 256, ... (EP of them) of a tile's Mt x Nt block at (m0, n0), PZ
// partials of each element in flight; the sums go to tile_s[em * 65 + en].
// Each element's partials are added in the order z = 0, 1, ... whatever EP
// and PZ.
template <int EP, int PZ>
__device__ __forceinline__ void split_reduce(const double* __restrict__ part, int32_t S, int64_t MN, int32_t N,
                                             int32_t m0, int32_t n0, int32_t Nt, int32_t Et, double* tile_s,
                                             int32_t e0) {
  const int t = threadIdx.x;
  double acc[EP];
  int64_t off[EP];
  int32_t slot[EP];
#pragma unroll
  for (int i = 0; i < EP; ++i) {
    const int32_t e = e0 + t + 256 * i;
    const int32_t ee = e < Et ? e : 0;  // clamped: every load stays in bounds
    const int32_t em = ee / Nt, en = ee - em * Nt;
    off[i] = (int64_t)(m0 + em) * N + (n0 + en);
    slot[i] = e < Et ? em * 65 + en : -1;
    acc[i] = 0.0;
  }
  int32_t z = 0;
  for (; z + PZ <= S; z += PZ) {
    double q[PZ][EP];
#pragma unroll
    for (int u = 0; u < PZ; ++u)
#pragma unroll
      for (int i = 0; i < EP; ++i) q[u][i] = part[(int64_t)(z + u) * MN + off[i]];
#pragma unroll
    for (int u = 0; u < PZ; ++u)
#pragma unroll
      for (int i = 0; i < EP; ++i) acc[i] += q[u][i];
  }
  for (; z < S; ++z)
#pragma unroll
    for (int i = 0; i < EP; ++i) acc[i] += part[(int64_t)z * MN + off[i]];
#pragma unroll
  for (int i = 0; i < EP; ++i)
    if (slot[i] >= 0) tile_s[slot[i]] = acc[i];
}

// End of a K-split product for one 64 x 64 output tile (256 threads, acc in
// the (ty + 16 i, tx + 16 j) layout): with gridDim.z = S > 1 slices, each
// block stores its partial tile; the last block to arrive at the tile's
// counter adds the S partials in the order z = 0, 1, ... (deterministic:
// the order does not depend on arrival), resets the counter for the next
// product and applies the epilogue.  The sums are spread over the threads
// element by element (one element each when the tile's valid block has at
// most 256), so many partial loads are in flight per thread, and return to
// the acc layout through tile_s (64 x 65 doubles of LDS).
template <typename TE, typename TD>
__device__ void split_finish(double (&acc)[4][4], int32_t M, int32_t N, int32_t m0, int32_t n0, double alpha,
                             double beta, const TE* __restrict__ E, const View& ve, TD* __restrict__ D,
                             const View& vd, double* __restrict__ colpart, double* __restrict__ part,
                             int* __restrict__ cnt, double* tile_s, double* red) {
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int32_t S = (int32_t)gridDim.z;
  if (S > 1) {
    const int64_t MN = (int64_t)M * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int32_t m = m0 + ty + 16 * i, n = n0 + tx + 16 * j;
        if (m < M && n < N) part[(int64_t)blockIdx.z * MN + (int64_t)m * N + n] = acc[i][j];
      }
    // every thread's partials are visible device-wide before the block's
    // arrival is counted
    __threadfence();
    __syncthreads();
    __shared__ int last;
    const int tile = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (t == 0) last = atomicAdd(&cnt[tile], 1) == S - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int32_t Mt = min(64, M - m0), Nt = min(64, N - n0);
    const int32_t Et = Mt * Nt;
    // (16 values in flight per thread: more would set the register count of
    // the whole kernel, and with it the occupancy of its K loop)
    if (Et <= 256)
      split_reduce<1, 16>(part, S, MN, N, m0, n0, Nt, Et, tile_s, 0);
    else
      for (int32_t e0 = 0; e0 < Et; e0 += 1024) split_reduce<4, 4>(part, S, MN, N, m0, n0, Nt, Et, tile_s, e0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int32_t mi = ty + 16 * i, nj = tx + 16 * j;
        acc[i][j] = (mi < Mt && nj < Nt) ? tile_s[mi * 65 + nj] : 0.0;
      }
    if (t == 0) cnt[tile] = 0;
  }
  gemm_epilogue<TE, TD>(acc, M, N, m0, n0, alpha, beta, E, ve, D, vd, colpart, red);
}

// The S K-slice partials of the matrix-core split (part + z M N, row-major)
// added in the order z = 0, 1, ... per element of a 64 x 64 output tile (the
// acc layout of the tiled products), then their epilogue: alpha, beta E, D
// and the column energies.
template <typename TE, typename TD>
__global__ __launch_bounds__(256) void k_mx_split_finish(int32_t M, int32_t N, int32_t S,
                                                         const double* __restrict__ part, double alpha, double beta,
                                                         const TE* __restrict__ E, View ve, TD* __restrict__ D,
                                                         View vd, double* __restrict__ colpart) {
  __shared__ double red[256];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int32_t m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int64_t MN = (int64_t)M * N;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t m = min(m0 + ty + 16 * i, M - 1), n = min(n0 + tx + 16 * j, N - 1);
      const double* p = part + (int64_t)m * N + n;
      double s = 0.0;
      for (int32_t z = 0; z < S; ++z) s += p[z * MN];
      acc[i][j] = s;  // (rows and columns past the output are dropped by the epilogue)
    }
  gemm_epilogue<TE, TD>(acc, M, N, m0, n0, alpha, beta, E, ve, D, vd, colpart, red);
}

// ---------------------------------------------------------------------------
// K-split product on the FP64 matrix cores for small outputs (each tile's
// valid block at most four 16 x 16 sub-blocks: M, N <= 32, or one of them
// <= 16) and a long K whose operands are linear along K
// (A(m, k) = A[row_off(m) + k sa], B(k, n) = B[k sb + col_off(n)]; no
// frames along K).  The block's four waves cover the nsb sub-blocks, and
// when there are fewer sub-blocks than waves the spare waves take further
// parts of the K slice (parts = 4, 2 or 1 for nsb = 1, 2, 3..4): wave w works
// on sub-block w mod nsb over part w / nsb.  v_mfma_f64_16x16x4f64 reads its
// operands straight from memory in the instruction's layout: lane
// (q, i) = (l / 16, l % 16) supplies A(m0 + 16 mb + i, k + q) and
// B(k + q, n0 + 16 nb + i), so no LDS staging and no barrier sit in the K
// loop.  A batch of 32 k-steps (128 values of k) per wave is loaded at once,
// 64 operand doubles per lane all in flight together (data written by
// another kernel is about a microsecond away), then multiplied with two
// accumulator chains; k is clamped into the wave's part and masked, so
// every load is unconditional.  The parts of a sub-block are added through
// LDS in the order part 0, 1, ... into the layout of split_finish.  (Larger
// outputs stay on the LDS-tiled kernel: their single-block reduction of many
// partials costs more than the matrix cores save.)
// ---------------------------------------------------------------------------
typedef double mf4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaBatch = 32;  // k-steps of 4 per load batch

__host__ __device__ constexpr int mfma_parts(int nsb) { return nsb <= 1 ? 4 : nsb == 2 ? 2 : 1; }

template <typename TB, typename TE, typename TD>
__global__ __launch_bounds__(256) void k_gemm_mfma(int32_t M, int32_t N, int32_t K, int32_t kchunk, double alpha,
                                                    const double* __restrict__ A, View va,
                                                    const TB* __restrict__ B, View vb, double beta,
                                                    const TE* __restrict__ E, View ve, TD* __restrict__ D, View vd,
                                                    double* __restrict__ colpart, double* __restrict__ part,
                                                    int* __restrict__ cnt) {
  __shared__ double tile_s[64 * 65];
  __shared__ double part_s[4][256];  // each wave's 16 x 16 accumulator
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int l = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int i16 = l & 15, kq = l >> 4;
  const int32_t m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int32_t kb = (int32_t)blockIdx.z * kchunk;
  const int32_t ke = min(K, kb + kchunk);  // kb < ke: the host sizes the slices
  const int32_t Mt = min(64, M - m0), Nt = min(64, N - n0);
  const int nnb = (Nt + 15) >> 4, nsb = ((Mt + 15) >> 4) * nnb;  // nsb <= 4
  const int parts = mfma_parts(nsb);
  const bool active = w < nsb * parts;  // (nsb = 3: wave 3 idles)
  const int sbk = w % nsb, kp = w / nsb;
  const int mb = sbk / nnb, nb = sbk - (sbk / nnb) * nnb;
  const int32_t m = m0 + 16 * mb + i16, n = n0 + 16 * nb + i16;
  const bool ok = active && m < M;
  const int64_t aro = row_off(va, min(m, M - 1));
  const int64_t bco = col_off(vb, min(n, N - 1));  // columns past N read column N-1; their outputs are dropped
  const int64_t sa = va.cs, sb = vb.rs;
  // this wave's part of the slice: contiguous k-steps of 4
  const int32_t steps = (ke - kb + 3) >> 2, per = (steps + parts - 1) / parts;
  const int32_t kwb = active ? min(ke, kb + 4 * kp * per) : ke;
  const int32_t kwe = active ? min(ke, kb + 4 * (kp + 1) * per) : ke;

  mf4 acc0 = mf4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
  for (int32_t k0 = kwb; k0 < kwe; k0 += 4 * kMfmaBatch) {
    double av[kMfmaBatch], bv[kMfmaBatch];
#pragma unroll
    for (int u = 0; u < kMfmaBatch; ++u) {
      const int32_t k = k0 + 4 * u + kq;
      const int32_t kc = min(k, kwe - 1);
      const double a = A[aro + (int64_t)kc * sa];
      const double b = (double)B[(int64_t)kc * sb + bco];
      av[u] = (k < kwe && ok) ? a : 0.0;
      bv[u] = (k < kwe) ? b : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kMfmaBatch; u += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], bv[u + 1], acc1, 0, 0, 0);
    }
  }
  // element i of lane l of a sub-block: row l / 16 + 4 i, column l % 16
  if (active)
#pragma unroll
    for (int i = 0; i < 4; ++i) part_s[w][(kq + 4 * i) * 16 + i16] = acc0[i] + acc1[i];
  __syncthreads();
  const int tx = t & 15, ty = t >> 4;
  double c[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t mi = ty + 16 * i, nj = tx + 16 * j;
      double v = 0.0;
      if (mi < Mt && nj < Nt) {
        const int sub = (mi >> 4) * nnb + (nj >> 4);
        const int e = (mi & 15) * 16 + (nj & 15);
        for (int q = 0; q < parts; ++q) v += part_s[sub + nsb * q][e];
      }
      c[i][j] = v;
    }
  split_finish<TE, TD>(c, M, N, m0, n0, alpha, beta, E, ve, D, vd, colpart, part, cnt, tile_s, red);
}

// ---------------------------------------------------------------------------
// Generic tiled product  D = alpha A B + beta E  (64 x 64 tiles, 256 threads,
// 4 x 4 register micro-tiles strided by 16 to spread LDS banks, K staged in
// chunks of 16 through LDS, FP64 accumulation).
// ---------------------------------------------------------------------------
template <typename TB, typename TE, typename TD, bool kSplit>
__global__ __launch_bounds__(256) void k_gemm(int32_t M, int32_t N, int32_t K, int32_t kchunk,
                                               double alpha, const double* __restrict__ A, View va,
                                               const TB* __restrict__ B, View vb, double beta,
                                               const TE* __restrict__ E, View ve, TD* __restrict__ D,
                                               View vd, int64_t dz, double* __restrict__ colpart,
                                               double* __restrict__ bnorm, double* __restrict__ part,
                                               int* __restrict__ cnt) {
  // the two K-tile buffers of A and B; a K-split reduction reuses the same
  // 4160 doubles as a 64 x 65 tile
  __shared__ double lds_ab[2 * 2 * 16 * 65];
  double(*As)[16][65] = (double(*)[16][65])lds_ab;
  double(*Bs)[16][65] = (double(*)[16][65])(lds_ab + 2 * 16 * 65);
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int ln = t & 63, lk = t >> 6;
  const int32_t m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int32_t kb = (int32_t)blockIdx.z * kchunk;
  const int32_t ke = min(K, kb + kchunk);

  // Tile loads always read a clamped, in-bounds element and mask it
  // afterwards, so the compiler keeps them in flight together (a guarded load
  // becomes a branch with a wait).  M > 0 is uniform over the block.
  const int32_t bn = n0 + ln;
  const bool bvalid = bn < N;
  const int64_t bco = col_off(vb, min(bn, N - 1));
  const int32_t am = m0 + ln;
  const bool avalid = am < M;
  const bool aload = M > 0;
  const int64_t aro = aload ? row_off(va, min(am, M - 1)) : 0;

  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  double bsq = 0.0;

  // K tiles of 16 go through two LDS buffers; the global loads of the next
  // tile are in flight while the current one is multiplied (one barrier per
  // tile).
  double av[4], bv[4];
  if (kb < ke) gemm_load(A, va, aro, aload, B, vb, bco, kb, ke, lk, av, bv);  // none when K == 0
  int buf = 0;
  for (int32_t k0 = kb; k0 < ke; k0 += 16) {
    bsq += gemm_store(k0, ke, lk, ln, avalid, bvalid, av, bv, As[buf], Bs[buf]);
    __syncthreads();
    if (k0 + 16 < ke) gemm_load(A, va, aro, aload, B, vb, bco, k0 + 16, ke, lk, av, bv);
    gemm_tile(As[buf], Bs[buf], tx, ty, acc);
    buf ^= 1;
  }
  __syncthreads();

  if (bnorm != nullptr && blockIdx.y == 0) {
    red[t] = bsq;
    __syncthreads();
    if (t < 64 && bvalid) bnorm[bn] = (red[t] + red[t + 64]) + (red[t + 128] + red[t + 192]);
    __syncthreads();
  }

  if (kSplit) {
    split_finish<TE, TD>(acc, M, N, m0, n0, alpha, beta, E, ve, D, vd, colpart, part, cnt, lds_ab, red);
    return;
  }
  TD* Dz = D ? D + dz * (int64_t)blockIdx.z : nullptr;
  gemm_epilogue<TE, TD>(acc, M, N, m0, n0, alpha, beta, E, ve, Dz, vd, colpart, red);
}

// Products with at most four output columns and K <= 128 (the Newton-Schulz
// and Gram-Schmidt corrections, U_R = R V, coefficient rows): one wave per
// output row, kSkinnyRows rows per wave, lane l holding k = l and l + 64.
// B's K x N block is loaded once per wave and kept in registers; every load
// of the wave's rows is issued before the first product; each of the row's
// N dot products is a wave sum (fixed order).  D = alpha A B + beta E.
extern "C" __device__ double __ockl_wfred_add_f64(double);
constexpr int kSkinnyRows = 4;
constexpr int kSkinnyMaxK = 128;

template <typename TB, typename TE, typename TD>
__global__ __launch_bounds__(256) void k_gemm_skinny(int32_t M, int32_t N, int32_t K, double alpha,
                                                     const double* __restrict__ A, View va,
                                                     const TB* __restrict__ B, View vb, double beta,
                                                     const TE* __restrict__ E, View ve, TD* __restrict__ D,
                                                     View vd) {
  const int l = threadIdx.x & 63;
  const int32_t row0 = ((int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6)) * kSkinnyRows;
  if (row0 >= M) return;  // uniform over the wave; no barriers below
  double b[2][4], a[kSkinnyRows][2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int32_t k = l + 64 * h;
    const int64_t bro = row_off(vb, min(k, K - 1));
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const double x = (double)B[bro + col_off(vb, min(n, N - 1))];
      b[h][n] = (k < K && n < N) ? x : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < kSkinnyRows; ++q) {
    const int64_t aro = row_off(va, min(row0 + q, M - 1));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t k = l + 64 * h;
      const double x = A[aro + col_off(va, min(k, K - 1))];
      a[q][h] = k < K ? x : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < kSkinnyRows; ++q) {
    const int32_t i = row0 + q;
    if (i >= M) break;  // uniform over the wave
    for (int n = 0; n < N; ++n) {
      const double sn = __ockl_wfred_add_f64(fma(a[q][0], b[0][n], a[q][1] * b[1][n]));
      if (l == 0) {
        double v = alpha * sn;
        if (E) v = fma(beta, (double)E[row_off(ve, i) + col_off(ve, n)], v);
        D[row_off(vd, i) + col_off(vd, n)] = (TD)v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------
extern "C" __device__ double __ockl_wfred_add_f64(double);
__device__ double block_sum_256(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Block (s, f) sums the column slice s (of S) of frame f over the MB row
// blocks: out[f * S + s] (with S = 1, the frame's total).  Loops run over
// the row blocks, then columns: no index division.
__global__ __launch_bounds__(256) void k_frame_sums(const double* __restrict__ part, int32_t MB,
                                                     int64_t ld, int32_t cpf, int32_t cslice,
                                                     double* __restrict__ out) {
  __shared__ double red[256];
  const int32_t s = blockIdx.x, S = gridDim.x, f = blockIdx.y;
  const int32_t c0 = s * cslice, c1 = min(cpf, c0 + cslice);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t mb = 0; mb < MB; ++mb) {
    const double* p = part + (int64_t)mb * ld + (int64_t)f * cpf;
    int32_t c = c0 + threadIdx.x;
    for (; c + 768 < c1; c += 1024) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += p[c + 256 * u];
    }
    for (; c < c1; c += 256) acc[0] += p[c];
  }
  const double v = block_sum_256((acc[0] + acc[1]) + (acc[2] + acc[3]), red);
  if (threadIdx.x == 0) out[(int64_t)f * S + s] = v;
}

// out[f] = sum of the S slice sums of frame f, in slice order
__global__ void k_slice_sums(const double* __restrict__ sl, int32_t S, int32_t F, double* __restrict__ out) {
  const int32_t f = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (f >= F) return;
  double v = 0.0;
  for (int32_t s = 0; s < S; ++s) v += sl[(int64_t)f * S + s];
  out[f] = v;
}

__global__ __launch_bounds__(256) void k_total_sum(const double* __restrict__ x, int64_t n,
                                                    double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  int bad = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = x[i];
    s += v;
    bad |= !isfinite(v);
  }
  const double tot = block_sum_256(s, red);
  const double nb = block_sum_256((double)bad, red);
  if (threadIdx.x == 0) {
    out[0] = tot;
    out[1] = nb > 0 ? 1.0 : 0.0;
  }
}

// out[0] = max_{i,j} |S(i, j) - [i == j]| over the n x n matrix S (row
// stride ld), out[1] = 1 when an entry is not finite; one block
__global__ __launch_bounds__(256) void k_max_off_identity(int32_t n, const double* __restrict__ S, int32_t ld,
                                                          double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  int bad = 0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += 256) {
    const int32_t i = (int32_t)(e / n), j = (int32_t)(e - (int64_t)i * n);
    const double v = S[(int64_t)i * ld + j] - (i == j ? 1.0 : 0.0);
    if (!isfinite(v)) bad = 1;
    m = fmax(m, fabs(v));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double mx = red[0];
  __syncthreads();  // every thread has read red[0] before the next sum reuses red
  const double nb = block_sum_256((double)bad, red);
  if (threadIdx.x == 0) {
    out[0] = mx;
    out[1] = nb > 0 ? 1.0 : 0.0;
  }
}

// out[j] = sum_k X[j ld + k]^2 over the ncol entries of row j, one block per
// row, fixed-order sums
__global__ __launch_bounds__(256) void k_row_sumsq(int32_t ncol, int64_t ld, const double* __restrict__ X,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const double* x = X + (int64_t)blockIdx.x * ld;
  double s = 0.0;
  for (int32_t k = threadIdx.x; k < ncol; k += 256) s = fma(x[k], x[k], s);
  s = block_sum_256(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// The rank from tails t(r) = perp + sum_{j >= r} e[j] (non-increasing in r):
// res[0] = the smallest r in [1, n] with t(r) <= tol2 (n when t(n) is
// above it), res[1] = t(res[0]), res[2] = min(|t(r) - tol2|, |t(r-1) -
// tol2|) / tol2, res[3] = 1 when a value is not finite.  One thread.
__global__ void k_tail_rank(int32_t n, const double* __restrict__ e, const double* __restrict__ perp, double tol2,
                            double* __restrict__ res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = perp[0];  // t(n)
  bool bad = !isfinite(t) || perp[1] != 0.0;
  int32_t best = n;
  double tb = t;
  for (int32_t q = n; q >= 1; --q) {
    if (!(t <= tol2)) break;
    best = q;
    tb = t;
    t += e[q - 1];  // t(q - 1)
  }
  for (int32_t j = 0; j < n; ++j) bad = bad || !isfinite(e[j]);
  const double tp = tb + e[best - 1];  // t(best - 1)
  const double t2 = tol2 > 0.0 ? tol2 : 1e-300;
  res[0] = (double)best;
  res[1] = tb;
  res[2] = fmin(fabs(tb - tol2), fabs(tp - tol2)) / t2;
  res[3] = bad ? 1.0 : 0.0;
}

// err2[b] = max(0, y2[b] - sum_j c[b ld + j]^2), one wave per frame
__global__ __launch_bounds__(256) void k_telescope(int32_t N, int32_t r, const double* __restrict__ c, int64_t ld,
                                                   const double* __restrict__ y2, double* __restrict__ err2) {
  const int32_t b = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
  if (b >= N) return;  // uniform over the wave
  const int l = threadIdx.x & 63;
  double s = 0.0;
  for (int32_t j = l; j < r; j += 64) {
    const double v = c[(int64_t)b * ld + j];
    s = fma(v, v, s);
  }
  s = __ockl_wfred_add_f64(s);
  if (l == 0) err2[b] = fmax(0.0, y2[b] - s);
}

__global__ void k_accumulate(double* __restrict__ acc, const double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] += x[i];
}

__global__ void k_gram_reduce(const double* __restrict__ part, int32_t S, int32_t m,
                              double* __restrict__ G) {
  const int64_t mm = (int64_t)m * m;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mm) return;
  const int32_t p = (int32_t)(idx / m), q = (int32_t)(idx - (int64_t)p * m);
  const int32_t a = min(p, q), b = max(p, q);
  const int64_t src = (int64_t)a * m + b;
  // slices in the order z = 0, 1, ..., eight loads in flight
  double s = 0.0;
  int32_t z = 0;
  for (; z + 8 <= S; z += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * mm + src];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; z < S; ++z) s += part[(int64_t)z * mm + src];
  G[idx] = s;
}

__global__ void k_gather_columns(int32_t rows, int32_t r, const double* __restrict__ V, int32_t ldv,
                                 const int32_t* __restrict__ order, const double* __restrict__ lam,
                                 int32_t scale, double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * r) return;
  const int32_t i = (int32_t)(e / r), tcol = (int32_t)(e % r);
  double v = V[(int64_t)i * ldv + (order ? order[tcol] : tcol)];
  if (scale) v /= sqrt(lam[tcol]);
  W[e] = v;
}

// Blocks 0 .. r-1: column t of W (rows x r, ld = r) times the sign that
// makes its largest-|.| entry (lowest row on ties) positive, written to
// column t of dst (ld ldd).  Blocks from r: zero the zrows x zcols region at
// zdst (ld zld), grid-stride.
__global__ __launch_bounds__(256) void k_sign_place(int32_t rows, int32_t r, const double* __restrict__ W,
                                                    double* __restrict__ dst, int64_t ldd,
                                                    double* __restrict__ zdst, int64_t zrows, int64_t zcols,
                                                    int64_t zld) {
  if ((int32_t)blockIdx.x >= r) {
    const int64_t nz = zrows * zcols;
    const int64_t stride = (int64_t)(gridDim.x - r) * blockDim.x;
    for (int64_t e = (int64_t)(blockIdx.x - r) * blockDim.x + threadIdx.x; e < nz; e += stride) {
      const int64_t i = e / zcols, j = e - i * zcols;
      zdst[i * zld + j] = 0.0;
    }
    return;
  }
  __shared__ double bv[256];
  __shared__ int32_t bi[256];
  const int32_t col = blockIdx.x;
  double best = -1.0;
  int32_t bidx = 0x7fffffff;
  for (int32_t i = threadIdx.x; i < rows; i += 256) {
    const double a = fabs(W[(int64_t)i * r + col]);
    if (a > best || (a == best && i < bidx)) {
      best = a;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double a = bv[threadIdx.x + s];
      const int32_t ia = bi[threadIdx.x + s];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ia < bi[threadIdx.x])) {
        bv[threadIdx.x] = a;
        bi[threadIdx.x] = ia;
      }
    }
    __syncthreads();
  }
  const int32_t k = bi[0];
  const bool flip = (k < rows) && (W[(int64_t)k * r + col] < 0.0);
  for (int32_t i = threadIdx.x; i < rows; i += 256) {
    const double v = W[(int64_t)i * r + col];
    dst[(int64_t)i * ldd + col] = flip ? -v : v;
  }
}

__global__ void k_zero2d(int64_t rows, int64_t cols, double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  dst[i * ldd + j] = 0.0;
}

// ---------------------------------------------------------------------------
// Algorithm 2 decision: eq:relerror, eq:subselectheuristic,
// eq:epsilonmodification inputs, eq:batchrelativeerror
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_star_decide(int32_t N, const double* __restrict__ e2,
                                                     const double* __restrict__ y2, double eps,
                                                     int32_t* __restrict__ dlist,
                                                     double* __restrict__ res) {
  __shared__ double red[256];
  double srel = 0.0, se = 0.0, sy = 0.0, sdc = 0.0, sd = 0.0, cnt = 0.0, near = 1e300;
  for (int32_t b = threadIdx.x; b < N; b += 256) {
    const double e = e2[b] > 0.0 ? e2[b] : 0.0;
    const double y = y2[b];
    const double rel = y > 0.0 ? sqrt(e / y) : 0.0;
    if (y > 0.0) near = fmin(near, fabs(rel / eps - 1.0));
    srel += rel;
    se += e;
    sy += y;
    if (rel > eps) {
      sd += y;
      cnt += 1.0;
    } else {
      sdc += e;
    }
  }
  srel = block_sum_256(srel, red);
  se = block_sum_256(se, red);
  sy = block_sum_256(sy, red);
  sdc = block_sum_256(sdc, red);
  sd = block_sum_256(sd, red);
  cnt = block_sum_256(cnt, red);
  // the closest per-frame relative error to eps (relative distance)
  red[threadIdx.x] = near;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  near = red[0];
  if (threadIdx.x == 0) {
    res[0] = N > 0 ? srel / N : 0.0;
    res[1] = sy > 0.0 ? sqrt(se / sy) : 0.0;
    res[6] = fmin(near, fmin(fabs(res[0] / eps - 1.0), fabs(res[1] / eps - 1.0)));
    res[2] = sdc;
    res[3] = sd;
    res[4] = cnt;
    res[5] = sy;
    int32_t k = 0;
    for (int32_t b = 0; b < N; ++b) {
      const double e = e2[b] > 0.0 ? e2[b] : 0.0;
      const double y = y2[b];
      const double rel = y > 0.0 ? sqrt(e / y) : 0.0;
      if (rel > eps) dlist[k++] = b;
    }
  }
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

constexpr int64_t kMfmaMaxSplit = 32;

}  // namespace

template <typename TB, typename TE, typename TD>
hipError_t gemm(hipStream_t st, int32_t M, int32_t N, int32_t K, int32_t kchunk, double alpha,
                const double* A, View va, const TB* B, View vb, double beta, const TE* E, View ve,
                TD* D, View vd, int64_t dz, double* colpart, double* bnorm, GemmWs ws, int prec) {
  if (N <= 0) return hipSuccess;
  if ((kchunk <= 0 || kchunk >= K) && !bnorm && ws.p) {
    // too few output tiles for the unsplit matrix-core product and a long K:
    // FP64 partials of K slices, then their fixed-order sum and epilogue
    const int32_t S = gemm_mx_split_slices(M, N, K, va, vb, ws.len);
    if (S >= 2) {
      int32_t chunk = (K + S - 1) / S;
      chunk = (chunk + 15) / 16 * 16;
      const int32_t Sx = (K + chunk - 1) / chunk;
      hipError_t e = gemm_mx64_part<TB>(st, M, N, K, Sx, chunk, A, va, B, vb, ws.p);
      if (e != hipSuccess) return e;
      const dim3 grid((unsigned)((N + 63) / 64), (unsigned)gemm_row_blocks(M));
      hipLaunchKernelGGL((k_mx_split_finish<TE, TD>), grid, dim3(256), 0, st, M, N, Sx, (const double*)ws.p, alpha,
                         beta, E, ve, D, vd, colpart);
      return hipGetLastError();
    }
  }
  if ((kchunk <= 0 || kchunk >= K) && gemm_mx_fits(M, N, K, va, vb, ve, vd, E != nullptr, D != nullptr, bnorm))
    return gemm_mx<TB, TE, TD>(st, prec, M, N, K, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart);
  const int32_t gx = (N + 63) / 64, gy = gemm_row_blocks(M);
  const int64_t tiles = (int64_t)gx * gy;
  const bool whole_k = kchunk <= 0 || kchunk >= K;
  // (a short K is not split when there are tens of tiles: the partials'
  // traffic and reduction cost more than the shorter K loop saves; a single
  // tile or a few split from K = 128)
  const bool can_split = whole_k && ws.p && ws.cnt && !bnorm && M > 0 && (K >= 256 || (K >= 128 && tiles <= 4)) &&
                         tiles <= ws.ncnt && tiles < 96;
  // sub-blocks of 16 x 16 per tile: the largest count, that of the first
  const int64_t nsb = ((std::min<int64_t>(M, 64) + 15) / 16) * ((std::min<int64_t>(N, 64) + 15) / 16);
  const int64_t MN = (int64_t)M * N;
  if (whole_k && !bnorm && !colpart && D && M > 0 && K > 0 && N <= 4 && K <= kSkinnyMaxK) {
    const int64_t waves = (M + kSkinnyRows - 1) / kSkinnyRows;
    hipLaunchKernelGGL((k_gemm_skinny<TB, TE, TD>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, M, N, K,
                       alpha, A, va, B, vb, beta, E, ve, D, vd);
    return hipGetLastError();
  }
  if (whole_k && !bnorm && M > 0 && nsb <= 4 && va.cpf == kUnframed && vb.rpf == kUnframed &&
      (can_split || K >= 4 * kMfmaBatch)) {
    // small output tiles, operands linear along K, and either a K split or
    // at least one full load batch (a short K wastes most of the batch; the
    // LDS-tiled kernel is faster there): matrix-core kernel.  With few tiles
    // and a long K the K range is split, one load batch (128 values of k)
    // per slice unless that needs more than kMfmaMaxSplit slices; the last
    // block of each tile adds the partials in order.
    int64_t S = 1;
    if (can_split) {
      const int64_t batch = 4 * kMfmaBatch * mfma_parts((int)nsb);  // k per slice: one batch per wave
      S = std::min<int64_t>({(K + batch - 1) / batch, std::max<int64_t>(1, 1024 / tiles), (int64_t)kMfmaMaxSplit});
      S = std::max<int64_t>(1, std::min<int64_t>(S, ws.len / std::max<int64_t>(MN, 1)));
    }
    int64_t chunk = (K + S - 1) / S;
    chunk = ((chunk + 15) / 16) * 16;
    S = (K + chunk - 1) / chunk;
    hipLaunchKernelGGL((k_gemm_mfma<TB, TE, TD>), dim3(gx, gy, (unsigned)S), dim3(256), 0, st, M, N, K,
                       (int32_t)chunk, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart, ws.p, ws.cnt);
    return hipGetLastError();
  }
  if (can_split) {
    // few output tiles and a long K on the LDS-tiled kernel: K split over
    // grid z (at least two K tiles of 16 per split, at most 16 splits, about
    // 192 blocks in all); the last block of each tile adds the partials in
    // order
    int64_t S = std::min<int64_t>({(K + 31) / 32, std::max<int64_t>(2, 192 / tiles), (int64_t)16});
    S = std::min<int64_t>(S, ws.len / std::max<int64_t>(MN, 1));
    if (S >= 2) {
      int64_t chunk = (K + S - 1) / S;
      chunk = ((chunk + 15) / 16) * 16;
      S = (K + chunk - 1) / chunk;
      hipLaunchKernelGGL((k_gemm<TB, TE, TD, true>), dim3(gx, gy, (unsigned)S), dim3(256), 0, st, M, N, K, (int32_t)chunk,
                         alpha, A, va, B, vb, beta, E, ve, D, vd, (int64_t)0, colpart, (double*)nullptr, ws.p,
                         ws.cnt);
      return hipGetLastError();
    }
  }
  if (kchunk <= 0) kchunk = K > 0 ? K : 1;
  const int32_t S = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)S);
  hipLaunchKernelGGL((k_gemm<TB, TE, TD, false>), grid, dim3(256), 0, st, M, N, K, kchunk, alpha, A, va, B,
                     vb, beta, E, ve, D, vd, dz, colpart, bnorm, (double*)nullptr, (int*)nullptr);
  return hipGetLastError();
}

#define TTICE_GEMM_INST(TB, TE, TD)                                                                  \
  template hipError_t gemm<TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, int32_t, double,      \
                                       const double*, View, const TB*, View, double, const TE*, View, \
                                       TD*, View, int64_t, double*, double*, GemmWs, int);
TTICE_GEMM_INST(double, double, double)
TTICE_GEMM_INST(float, double, double)
TTICE_GEMM_INST(double, float, double)
TTICE_GEMM_INST(float, float, double)
TTICE_GEMM_INST(double, double, float)
TTICE_GEMM_INST(float, float, float)
TTICE_GEMM_INST(double, float, float)
TTICE_GEMM_INST(float, double, float)

int32_t frame_sum_slices(int32_t cpf, int32_t F) {
  // a few hundred blocks in all, slices of at least 8192 columns
  const int64_t by_len = ((int64_t)cpf + 8191) / 8192;
  const int64_t by_grid = std::max<int64_t>(1, 512 / std::max(F, 1));
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>({by_len, by_grid, (int64_t)kFrameSlicesMax}));
}

hipError_t frame_sums(hipStream_t st, const double* part, int32_t MB, int64_t ld, int32_t cpf,
                      int32_t F, double* out, double* scratch) {
  if (F <= 0) return hipSuccess;
  const int32_t S = scratch ? frame_sum_slices(cpf, F) : 1;
  const int32_t cslice = (cpf + S - 1) / S;
  hipLaunchKernelGGL(k_frame_sums, dim3(S, F), dim3(256), 0, st, part, MB, ld, cpf, cslice, S > 1 ? scratch : out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  hipLaunchKernelGGL(k_slice_sums, dim3(nblocks(F, 256)), dim3(256), 0, st, scratch, S, F, out);
  return hipGetLastError();
}

hipError_t total_sum(hipStream_t st, const double* x, int64_t n, double* out) {
  hipLaunchKernelGGL(k_total_sum, dim3(1), dim3(256), 0, st, x, n, out);
  return hipGetLastError();
}

hipError_t max_off_identity(hipStream_t st, int32_t n, const double* S, int32_t ld, double* out) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_max_off_identity, dim3(1), dim3(256), 0, st, n, S, ld, out);
  return hipGetLastError();
}

hipError_t row_sumsq(hipStream_t st, int32_t n, int32_t ncol, int64_t ld, const double* X, double* out) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_sumsq, dim3((unsigned)n), dim3(256), 0, st, ncol, ld, X, out);
  return hipGetLastError();
}

hipError_t tail_rank(hipStream_t st, int32_t n, const double* e, const double* perp, double tol2, double* res) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tail_rank, dim3(1), dim3(64), 0, st, n, e, perp, tol2, res);
  return hipGetLastError();
}

hipError_t telescope(hipStream_t st, int32_t N, int32_t r, const double* c, int64_t ld, const double* y2,
                     double* err2) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_telescope, dim3(nblocks(N, 4)), dim3(256), 0, st, N, r, c, ld, y2, err2);
  return hipGetLastError();
}

hipError_t accumulate(hipStream_t st, double* acc, const double* x, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate, dim3(nblocks(n, 256)), dim3(256), 0, st, acc, x, n);
  return hipGetLastError();
}

hipError_t gram_reduce(hipStream_t st, const double* part, int32_t S, int32_t m, double* G) {
  const int64_t mm = (int64_t)m * m;
  if (mm == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_reduce, dim3(nblocks(mm, 256)), dim3(256), 0, st, part, S, m, G);
  return hipGetLastError();
}

hipError_t gather_columns(hipStream_t st, int32_t rows, int32_t r, const double* V, int32_t ldv,
                          const int32_t* order, const double* lam, bool scale, double* W) {
  const int64_t n = (int64_t)rows * r;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_columns, dim3(nblocks(n, 256)), dim3(256), 0, st, rows, r, V, ldv, order,
                     lam, scale ? 1 : 0, W);
  return hipGetLastError();
}

hipError_t sign_place(hipStream_t st, int32_t rows, int32_t r, const double* W, double* dst, int64_t ldd,
                      double* zdst, int64_t zrows, int64_t zcols, int64_t zld) {
  const int64_t nz = (zdst != nullptr && zrows > 0 && zcols > 0) ? zrows * zcols : 0;
  const int64_t zb = std::min<int64_t>(nblocks(nz, 256), 256);
  if (r <= 0 && zb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_place, dim3((unsigned)(std::max(r, 0) + zb)), dim3(256), 0, st, rows, std::max(r, 0),
                     W, dst, ldd, zdst, nz > 0 ? zrows : 0, nz > 0 ? zcols : 0, zld);
  return hipGetLastError();
}

hipError_t zero2d(hipStream_t st, int64_t rows, int64_t cols, double* dst, int64_t ldd) {
  const int64_t n = rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero2d, dim3(nblocks(n, 256)), dim3(256), 0, st, rows, cols, dst, ldd);
  return hipGetLastError();
}

hipError_t star_decide(hipStream_t st, int32_t N, const double* e2, const double* y2, double eps,
                       int32_t* dlist, double* res) {
  hipLaunchKernelGGL(k_star_decide, dim3(1), dim3(256), 0, st, N, e2, y2, eps, dlist, res);
  return hipGetLastError();
}

}  // namespace ttice
