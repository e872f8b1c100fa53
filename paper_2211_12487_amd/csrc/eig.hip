// Symmetric eigensolver for the truncated SVD of the residual (eq:svdfirst):
// the Gram matrix G = R R^T (or R^T R) is reduced to tridiagonal form by
// Householder reflections (one workgroup), all eigenvalues are found by
// Sturm-sequence multisection (one wave per eigenvalue, returned in
// decreasing order), and only the eigenvectors that TT-ICE keeps are formed
// on the tridiagonal matrix (twisted factorization for isolated
// eigenvalues, inverse iteration with Gram-Schmidt inside clusters)
// followed by the back-transformation with the stored reflectors.
//
// Everything here is latency-bound (one workgroup, long dependent chains),
// so the working sets stay on chip: the trailing block of the reduction
// once it is at most 128 wide in the registers of one workgroup's waves
// (the first reflections of a larger matrix run on many workgroups), the
// tridiagonal matrix in the Sturm counts in LDS, the per-vector LU factors
// of inverse iteration and chunks of reflectors in the back-transformation
// in LDS.
#include "kernels.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace ttice {
namespace {

constexpr int kTriThreads = 512;
constexpr int kWaves = kTriThreads / 64;
constexpr int kTriLdsMax = 124;      // trailing blocks up to this size are reduced in LDS
constexpr int kEigMax = 4096;        // largest Gram matrix the solver accepts
constexpr int kLdsDoubles = 19200;   // 150 KB of dynamic LDS per workgroup

// Wave-wide sum (DPP reduction of the device library; every lane gets it).
extern "C" __device__ double __ockl_wfred_add_f64(double);
__device__ __forceinline__ double wave_sum(double v) { return __ockl_wfred_add_f64(v); }

// Sum over the block; every thread gets the result.  red: >= kWaves doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kWaves; ++i) s += red[i];
  __syncthreads();
  return s;
}

// sum_{i = i0, i0+G, ... < L} col[i*ld] * v[i], with eight independent
// loads in flight (the loop is latency-bound, not bandwidth-bound).
template <int G>
__device__ __forceinline__ double col_dot(const double* col, int64_t ld, const double* v, int32_t i0, int32_t L) {
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int32_t i = i0;
  for (; i + 7 * G < L; i += 8 * G) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = col[(int64_t)(i + u * G) * ld];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = fma(a[u], v[i + u * G], acc[u]);
  }
  for (; i < L; i += G) acc[0] = fma(col[(int64_t)i * ld], v[i], acc[0]);
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// col[i*ld] -= v_i w_j + w_i v_j for i = i0, i0+G, ... < L, where
// w_i = p_i - gam v_i; eight rows per batch.
template <int G>
__device__ __forceinline__ void col_update(double* col, int64_t ld, const double* v, const double* p, double gam,
                                           double vj, double wj, int32_t i0, int32_t L) {
  int32_t i = i0;
  for (; i + 7 * G < L; i += 8 * G) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = col[(int64_t)(i + u * G) * ld];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double vi = v[i + u * G];
      a[u] = a[u] - vi * wj - (p[i + u * G] - gam * vi) * vj;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) col[(int64_t)(i + u * G) * ld] = a[u];
  }
  for (; i < L; i += G) {
    const double vi = v[i];
    col[(int64_t)i * ld] = col[(int64_t)i * ld] - vi * wj - (p[i] - gam * vi) * vj;
  }
}

// Householder reflections k = 0 .. kend-1 (dsytd2 order) of the symmetric
// n x n block A (row-major, row stride ld, full storage): d[k], e[k] of the
// tridiagonal matrix, tau[k], and v_k stored in row k, columns k+1..n-1
// (v_k[0] = 1).  H_k = I - tau_k v_k v_k^T acts on indices k+1..n-1.
//
// Threads form G groups of NC = 512/G: in the matrix-vector product
// p = tau A v, thread (g, c) sums rows i = g (mod G) of columns c, c+NC, ...
// (no shuffles; G partial sums per column in LDS); the rank-2 update
// A -= v w^T + w v^T with w = p - (tau/2)(p.v) v uses the same layout, and
// group 0 (which updates row 0 of the trailing block) also stores the next
// reflection's x and ||x[1:]||^2.  Four barriers per reflection.
// vbuf: 4n doubles (+ G*n when G > 1), in LDS.  red2: kWaves doubles.
template <int G, bool kLds>
__device__ void tri_steps(int32_t n, double* A, int64_t ld, int32_t kend, double* vbuf, double* red,
                          double* red2, double* d, double* e, double* tau) {
  constexpr int NC = kTriThreads / G;
  constexpr int W0 = NC / 64;  // waves in group 0
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const int g = t / NC, c0 = t % NC;
  double* va = vbuf;          // x of the current reflection (read only during the step)
  double* vb = vbuf + n;      // x of the next reflection
  double* vn = vbuf + 2 * n;  // v = [1, x[1:] / (x[0] - beta)]
  double* p = vbuf + 3 * n;
  double* part = vbuf + 4 * n;  // G x n partial sums (G > 1)
  if (kend <= 0) return;
  {
    double s = 0.0;
    for (int32_t i = t; i < n - 1; i += kTriThreads) {
      const double x = A[1 + i];
      va[i] = x;
      if (i > 0) s = fma(x, x, s);
    }
    s = block_sum(s, red);
    if (t < kWaves) red2[t] = (t == 0) ? s : 0.0;
    __syncthreads();
  }
  for (int32_t k = 0; k < kend; ++k) {
    const int32_t L = n - k - 1;
    double* row = A + (int64_t)k * ld + (k + 1);
    double sigma = 0.0;
    for (int w = 0; w < W0; ++w) sigma += red2[w];
    const double alpha = va[0];
    double beta, tk, scale;
    if (sigma == 0.0) {
      tk = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tk = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (t == 0) {
      d[k] = A[(int64_t)k * ld + k];
      e[k] = beta;
      tau[k] = tk;
    }
    for (int32_t i = t; i < L; i += kTriThreads) {
      const double vi = (i == 0) ? 1.0 : va[i] * scale;
      vn[i] = vi;
      row[i] = vi;  // v_k kept for the back-transformation
    }
    __syncthreads();  // (1) v complete; every thread has read red2 and va[0]
    double* sub = A + (int64_t)(k + 1) * ld + (k + 1);
    double sn = 0.0;
    if (tk != 0.0) {
      double pvw = 0.0;
      if (G == 1) {
        for (int32_t j = c0; j < L; j += NC) {
          const double pj = tk * col_dot<1>(sub + j, ld, vn, 0, L);
          p[j] = pj;
          pvw = fma(pj, vn[j], pvw);
        }
        __syncthreads();  // (2)
      } else {
        for (int32_t j = c0; j < L; j += NC) part[g * n + j] = col_dot<G>(sub + j, ld, vn, g, L);
        __syncthreads();  // (2) partial sums complete
        if (g == 0)
          for (int32_t j = c0; j < L; j += NC) {
            double acc = 0.0;
            for (int gg = 0; gg < G; ++gg) acc += part[gg * n + j];
            const double pj = tk * acc;
            p[j] = pj;
            pvw = fma(pj, vn[j], pvw);
          }
      }
      if (g == 0) {
        pvw = wave_sum(pvw);
        if (lane == 0) red[wid] = pvw;
      }
      __syncthreads();  // (3) p and the partial p.v complete
      double pv = 0.0;
      for (int w = 0; w < W0; ++w) pv += red[w];
      const double gam = 0.5 * tk * pv;
      for (int32_t j = c0; j < L; j += NC) {
        const double vj = vn[j], wj = p[j] - gam * vj;
        if (g == 0 && j >= 1) {  // row 0 of the block: also the next reflection's x
          const double nv = sub[j] - vn[0] * wj - (p[0] - gam * vn[0]) * vj;
          sub[j] = nv;
          vb[j - 1] = nv;
          if (j >= 2) sn = fma(nv, nv, sn);
        }
        col_update<G>(sub + j, ld, vn, p, gam, vj, wj, (g == 0 && j >= 1) ? G : g, L);
      }
    } else {
      __syncthreads();  // keep the barrier count uniform
      __syncthreads();
      if (g == 0)
        for (int32_t j = c0; j < L; j += NC)
          if (j >= 1) {
            const double a = sub[j];
            vb[j - 1] = a;
            if (j >= 2) sn = fma(a, a, sn);
          }
    }
    if (g == 0) {
      sn = wave_sum(sn);
      if (lane == 0) red2[wid] = sn;
    }
    if (!kLds) __threadfence_block();
    __syncthreads();  // (4) update, next x and its norm complete
    double* tmp = va;
    va = vb;
    vb = tmp;
  }
}

// The last 2x2 block of the tridiagonal matrix once all reflections are done.
__device__ void tri_tail(int32_t n, const double* A, int64_t ld, double* d, double* e, double* tau) {
  if (threadIdx.x == 0) {
    if (n >= 2) {
      d[n - 2] = A[(int64_t)(n - 2) * ld + (n - 2)];
      e[n - 2] = A[(int64_t)(n - 2) * ld + (n - 1)];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = A[(int64_t)(n - 1) * ld + (n - 1)];
    tau[n - 1] = 0.0;
  }
}

// Tridiagonalise A (m x m, row-major, ld = m) in place.  Reflections whose
// trailing block is wider than kTriLdsMax run on A in global memory (one
// thread per column); the remaining block is then copied to LDS and reduced
// there.  The reflectors end up in A's rows either way.  (Used when no
// workspace is given for the many-workgroup reflections.)
__global__ __launch_bounds__(kTriThreads) void k_tridiag(int32_t m, double* __restrict__ A,
                                                         double* __restrict__ d, double* __restrict__ e,
                                                         double* __restrict__ tau) {
  HIP_DYNAMIC_SHARED(double, lds);
  __shared__ double red[kWaves];
  __shared__ double red2[kWaves];
  int32_t ksw = 0;
  if (m > kTriLdsMax) {
    ksw = m - kTriLdsMax;
    tri_steps<1, false>(m, A, m, ksw, lds, red, red2, d, e, tau);
  }
  const int32_t n = m - ksw;
  double* Ab = A + (int64_t)ksw * m + ksw;
  const int64_t ld = n + 1;
  double* As = lds;
  for (int32_t i = threadIdx.x >> 6; i < n; i += kWaves)
    for (int32_t j = threadIdx.x & 63; j < n; j += 64) As[i * ld + j] = Ab[(int64_t)i * m + j];
  __syncthreads();
  tri_steps<4, true>(n, As, ld, n - 2, lds + (int64_t)n * ld, red, red2, d + ksw, e + ksw, tau + ksw);
  tri_tail(n, As, ld, d + ksw, e + ksw, tau + ksw);
  __syncthreads();
  for (int32_t i = threadIdx.x >> 6; i < n; i += kWaves)
    for (int32_t j = threadIdx.x & 63; j < n; j += 64) Ab[(int64_t)i * m + j] = As[i * ld + j];
}

// 1/q to full double accuracy from the hardware reciprocal estimate and
// one Newton step (the Sturm recurrence only needs q's sign and magnitude).
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// ---- Register-distributed variant for blocks up to kRwMax wide: the
// n x n trailing block at (ksw, ksw) of A (ld = lda) lives in registers,
// wave w holding the RPW consecutive rows from w * RPW and lane l the
// columns l, l + 64 (CPL of them).  One barrier per reflection: the rank-2
// update of reflection k-1 is applied at the start of step k, and column k
// of the updated block is formed directly as x = c - w - w_k v from column
// k as it stood before that update (c, written to LDS by the lanes that hold
// it at the end of step k-1; the first entry of v_{k-1} is 1).  Step k:
//  * the per-wave partial column sums of A v_{k-1} are added in the order
//    w = 0, 1, ..., giving p = tau A v, p.v (wave sum) and
//    w = p - (tau/2)(p.v) v on the lane's columns; the wave's own rows of w
//    come back from a wave-private LDS copy;
//  * x as above, ||x[k+2:]||^2 (wave sum), beta, tau_k and v_k on the lane's
//    columns, and through a second private copy on the wave's rows;
//  * the registers take A -= v w^T + w v^T of reflection k-1;
//  * p = A v_k as column sums of the wave's rows (one partial row per wave
//    to LDS), the lanes holding column k+1 write it; one barrier.
// A wave whose RPW rows are all finished (<= k) writes zero partials and
// skips the rest, so the block's work shrinks with k.  Rows and columns use
// the same v, built from column k.  Same outputs as k_tridiag (dsytd2
// order; v_k in row ksw+k, columns ksw+k+1 ..; d, e, tau from ksw).
constexpr int kRwWaves = 8;
constexpr int kRwMax = 128;

// value of x in lane `lane` (uniform over the wave) of the wave
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// fixed-order pairwise sum of the per-wave partials
template <int NW>
__device__ __forceinline__ double wave_parts_sum(const double (&p)[NW]) {
  static_assert(NW == 4 || NW == 8, "four or eight waves");
  if constexpr (NW == 4)
    return (p[0] + p[1]) + (p[2] + p[3]);
  else
    return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}

template <int CPL, int RPW, int NW = kRwWaves>
__global__ __launch_bounds__(NW * 64) void k_tridiag_rw(int32_t n, int32_t ksw, int32_t lda,
                                                             double* __restrict__ A, double* __restrict__ d,
                                                             double* __restrict__ e, double* __restrict__ tau) {
  static_assert(CPL == 1 || CPL == 2, "one or two columns per lane");
  static_assert(RPW % 2 == 0 && RPW * NW <= 64 * CPL, "rows per wave: even, within the columns");
  typedef double dbl2 __attribute__((ext_vector_type(2)));
  constexpr int NC = 64 * CPL;  // largest n
  __shared__ __attribute__((aligned(16))) double xcol[2][NC];      // column k before the last update
  __shared__ __attribute__((aligned(16))) double part[2][NW][NC];  // per-wave partial column sums of A v
  __shared__ __attribute__((aligned(16))) double wv[NW][NC];       // wave-private w
  __shared__ __attribute__((aligned(16))) double vv[NW][NC];       // wave-private v
  const int l = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int32_t r0 = w * RPW;
  const int wlast = (n - 1) / RPW;  // holds row n - 1: active in every step
  double* Ab = A + (int64_t)ksw * lda + ksw;

  double a[RPW][CPL];
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int32_t i = r0 + q, j = l + 64 * c;
      a[q][c] = (i < n && j < n) ? Ab[(int64_t)i * lda + j] : 0.0;
    }
  // the previous reflection: v on the lane's columns and the wave's rows, tau
  double vc[CPL], vq[RPW];
#pragma unroll
  for (int c = 0; c < CPL; ++c) vc[c] = 0.0;
#pragma unroll
  for (int q = 0; q < RPW; ++q) vq[q] = 0.0;
  double tkp = 0.0;

  // w = p - (tau/2)(p.v) v of the previous reflection (its partial sums in
  // part[pb]) on the lane's columns (wc) and the wave's rows (wq), for the
  // indices >= k; zero when there is none
  auto finish = [&](int32_t k, int pb, double (&wc)[CPL], double (&wq)[RPW]) {
    if (tkp != 0.0) {  // uniform over the block
      double pc[CPL];
      double pv = 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int32_t j = l + 64 * c;
        double pp[NW];
#pragma unroll
        for (int u = 0; u < NW; ++u) pp[u] = part[pb][u][j];
        const double sp = wave_parts_sum<NW>(pp);
        pc[c] = (j >= k && j < n) ? tkp * sp : 0.0;
        pv = fma(pc[c], vc[c], pv);
      }
      pv = wave_sum(pv);
      const double gam = 0.5 * tkp * pv;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        wc[c] = pc[c] - gam * vc[c];
        wv[w][l + 64 * c] = wc[c];
      }
      // LDS operations of one wave complete in order
      __builtin_amdgcn_wave_barrier();
      const dbl2* src = (const dbl2*)&wv[w][r0];
#pragma unroll
      for (int u = 0; u < RPW / 2; ++u) {
        const dbl2 t = src[u];
        wq[2 * u] = t[0];
        wq[2 * u + 1] = t[1];
      }
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) wc[c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPW; ++q) wq[q] = 0.0;
    }
  };
  // A -= v w^T + w v^T with the previous reflection
  auto update = [&](const double (&wc)[CPL], const double (&wq)[RPW]) {
    if (tkp != 0.0) {
#pragma unroll
      for (int q = 0; q < RPW; ++q)
#pragma unroll
        for (int c = 0; c < CPL; ++c) a[q][c] = fma(-wq[q], vc[c], fma(-vq[q], wc[c], a[q][c]));
    }
  };

  // column 0; the slots of both column buffers past the rows the waves
  // hold start at zero (never left to what an earlier kernel put there)
  for (int i = (int)threadIdx.x; i < 2 * NC; i += NW * 64) xcol[i / NC][i % NC] = 0.0;
  __syncthreads();
  if (l == 0 && r0 < n) {
    dbl2* dst = (dbl2*)&xcol[0][r0];
#pragma unroll
    for (int u = 0; u < RPW / 2; ++u) dst[u] = dbl2{a[2 * u][0], a[2 * u + 1][0]};
  }
  __syncthreads();

  // step k; SK and SK1 are the column slots of k and k + 1 (k >> 6 and
  // (k + 1) >> 6), fixed per range of k so that no step selects between slots
  auto step = [&](int32_t k, auto skt, auto sk1t) __attribute__((always_inline)) {
    constexpr int SK = decltype(skt)::value, SK1 = decltype(sk1t)::value;
    const int buf = k & 1;
    if (r0 + RPW - 1 > k && r0 < n) {  // the wave holds rows > k
      const int kl = k & 63, kl1 = (k + 1) & 63;
      double wc[CPL], wq[RPW];
      finish(k, buf ^ 1, wc, wq);
      // column k after the previous reflection
      const double wk = readlane_f64(wc[SK], kl);
      double x[CPL];
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int32_t j = l + 64 * c;
        x[c] = fma(-wk, vc[c], xcol[buf][j] - wc[c]);
        if (j >= k + 2 && j < n) s = fma(x[c], x[c], s);
      }
      const double sigma = wave_sum(s);
      const double alpha = readlane_f64(x[SK1], kl1);
      const double dk = readlane_f64(x[SK], kl);
      update(wc, wq);
      double beta, tk, scale;
      if (sigma == 0.0) {
        tk = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        tk = (beta - alpha) * recip(beta);
        scale = recip(alpha - beta);
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int32_t j = l + 64 * c;
        vc[c] = (j == k + 1) ? 1.0 : ((j > k + 1 && j < n) ? x[c] * scale : 0.0);
        if (w == wlast && j > k && j < n) Ab[(int64_t)k * lda + j] = vc[c];  // v_k for the back-transformation
      }
      if (w == wlast && l == 0) {
        d[ksw + k] = dk;
        e[ksw + k] = beta;
        tau[ksw + k] = tk;
      }
      tkp = tk;
      if (tk != 0.0) {  // uniform over the block
#pragma unroll
        for (int c = 0; c < CPL; ++c) vv[w][l + 64 * c] = vc[c];
        __builtin_amdgcn_wave_barrier();
        const dbl2* src = (const dbl2*)&vv[w][r0];
#pragma unroll
        for (int u = 0; u < RPW / 2; ++u) {
          const dbl2 t = src[u];
          vq[2 * u] = t[0];
          vq[2 * u + 1] = t[1];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < RPW; ++q) p4[q & 3] = fma(a[q][c], vq[q], p4[q & 3]);
          part[buf][w][l + 64 * c] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        }
      }
      // column k + 1 as it stands now (the lane holding it, the wave's rows)
      if (k + 3 < n && l == kl1) {
        double* dst = &xcol[buf ^ 1][r0];
#pragma unroll
        for (int q = 0; q < RPW; ++q) dst[q] = a[q][SK1];
      }
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) part[buf][w][l + 64 * c] = 0.0;
    }
    __syncthreads();
  };
  typedef std::integral_constant<int, 0> S0;
  typedef std::integral_constant<int, CPL - 1> S1;
  const int32_t kend = n - 2;  // steps k = 0 .. n - 3
  int32_t k = 0;
  for (; k < kend && k < 63; ++k) step(k, S0{}, S0{});
  for (; k < kend && k < 64; ++k) step(k, S0{}, S1{});  // k = 63 (CPL = 2)
  for (; k < kend; ++k) step(k, S1{}, S1{});
  // the last reflection's update, then the last 2 x 2 block (or the single
  // entry when n = 1)
  if (n >= 3 && r0 + RPW - 1 >= n - 2 && r0 < n) {
    double wc[CPL], wq[RPW];
    finish(n - 2, (n - 3) & 1, wc, wq);
    update(wc, wq);
  }
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int32_t i = r0 + q, j = l + 64 * c;
      if (i == n - 2 && j == n - 2) d[ksw + n - 2] = a[q][c];
      if (i == n - 2 && j == n - 1) e[ksw + n - 2] = a[q][c];
      if (i == n - 1 && j == n - 1) d[ksw + n - 1] = a[q][c];
    }
  if (threadIdx.x == 0) {
    if (n >= 2) tau[ksw + n - 2] = 0.0;
    tau[ksw + n - 1] = 0.0;
  }
}

// ---- Reflections of a large Gram matrix spread over many workgroups, one
// launch per reflection (k_tri_step), the rank-2 update of reflection k-1
// folded into the launch of reflection k:
//  * every workgroup forms w = p - gamma v of reflection k-1 (p, v and the
//    per-workgroup shares of p.v from the previous launch; gamma =
//    tau p.v / 2 from the shares in a fixed order), row k after that update
//    (x = a_k - w - w_0 v, as the first entry of v is 1; kept in LDS, never
//    stored) and from x reflection k's beta, tau and v_k (the same
//    fixed-order sum for ||x[2:]||^2 in each workgroup, so all agree bit for
//    bit); workgroup 0 stores v_{k-1} in row k-1 for the back-transformation;
//  * each workgroup then takes a contiguous range of the trailing rows
//    k+1 .. m-1, applies A -= v w^T + w v^T of reflection k-1 to them and,
//    from the updated values still in registers, forms p_i = tau_k (A v_k)_i
//    and its share of p.v.
// The launch with k == kend applies the last update only, to the whole
// trailing block from row kend.  Workspace (sym_eig_ws): vbuf[2][m],
// pbuf[2][m], part[2][kMaxMvBlocks], alternating with the parity of k.
constexpr int kMvThreads = 256;
constexpr int kMaxMvBlocks = 256;

__device__ double block_sum_mv(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  const double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// dynamic LDS: 3 (m - k) + (m - k - 1) doubles
__global__ __launch_bounds__(kMvThreads) void k_tri_step(int32_t m, int32_t k, int32_t kend, double* __restrict__ A,
                                                         double* __restrict__ d, double* __restrict__ e,
                                                         double* __restrict__ tau, double* __restrict__ vbuf,
                                                         double* __restrict__ pbuf, double* __restrict__ part,
                                                         int32_t nprev) {
  HIP_DYNAMIC_SHARED(double, sh);
  __shared__ double red[4];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int32_t Lp = m - k;     // reflection k-1 acts on the indices k .. m-1
  const int32_t L = m - k - 1;  // reflection k on k+1 .. m-1
  double* vp = sh;
  double* wp = sh + Lp;
  double* x = sh + 2 * (int64_t)Lp;
  double* v = sh + 3 * (int64_t)Lp;
  const int pb = (k + 1) & 1, cb = k & 1;
  const bool upd = k > 0;
  const double tkp = upd ? tau[k - 1] : 0.0;
  const bool doup = upd && tkp != 0.0;
  if (upd) {
    double pvp = 0.0;
    for (int32_t g = 0; g < nprev; ++g) pvp += part[pb * kMaxMvBlocks + g];
    const double gam = 0.5 * tkp * pvp;
    for (int32_t j = t; j < Lp; j += kMvThreads) {
      const double vj = vbuf[(int64_t)pb * m + j];
      vp[j] = vj;
      wp[j] = doup ? pbuf[(int64_t)pb * m + j] - gam * vj : 0.0;
      if (blockIdx.x == 0) A[(int64_t)(k - 1) * m + k + j] = vj;  // v_{k-1} kept for the back-transformation
    }
    __syncthreads();
  }
  const int32_t G = (int32_t)gridDim.x;
  if (k == kend) {
    // the last update, rows and columns k .. m-1
    if (!doup) return;
    const int32_t per = (Lp + G - 1) / G;
    const int32_t r0 = (int32_t)blockIdx.x * per, r1 = min(Lp, r0 + per);
    for (int32_t i = r0 + wid; i < r1; i += kMvThreads / 64) {
      double* row = A + (int64_t)(k + i) * m + k;
      const double vi = vp[i], wi = wp[i];
      for (int32_t j = lane; j < Lp; j += 64) row[j] = fma(-wi, vp[j], fma(-vi, wp[j], row[j]));
    }
    return;
  }
  // row k after reflection k-1 (columns k .. m-1)
  const double* rowk = A + (int64_t)k * m + k;
  const double w0 = doup ? wp[0] : 0.0;
  for (int32_t q = t; q < Lp; q += kMvThreads) {
    const double a = rowk[q];
    x[q] = doup ? fma(-w0, vp[q], fma(-1.0, wp[q], a)) : a;
  }
  __syncthreads();
  double s = 0.0;
  for (int32_t j = 1 + t; j < L; j += kMvThreads) s = fma(x[j + 1], x[j + 1], s);
  const double sigma = block_sum_mv(s, red);
  const double alpha = x[1];
  double beta, tk, scale;
  if (sigma == 0.0) {
    tk = 0.0;
    beta = alpha;
    scale = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
    tk = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int32_t j = t; j < L; j += kMvThreads) {
    const double vj = (j == 0) ? 1.0 : x[j + 1] * scale;
    v[j] = vj;
    if (blockIdx.x == 0) vbuf[(int64_t)cb * m + j] = vj;
  }
  if (blockIdx.x == 0 && t == 0) {
    d[k] = x[0];
    e[k] = beta;
    tau[k] = tk;
  }
  __syncthreads();
  const int32_t per = (L + G - 1) / G;
  const int32_t r0 = (int32_t)blockIdx.x * per, r1 = min(L, r0 + per);
  double pv = 0.0;
  for (int32_t i = r0 + wid; i < r1; i += kMvThreads / 64) {
    double* row = A + (int64_t)(k + 1 + i) * m + (k + 1);  // columns k+1 .. m-1
    const double vi = doup ? vp[i + 1] : 0.0, wi = doup ? wp[i + 1] : 0.0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int32_t j = lane;
    for (; j + 192 < L; j += 256) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t jj = j + 64 * u;
        double a = row[jj];
        if (doup) {
          a = fma(-wi, vp[jj + 1], fma(-vi, wp[jj + 1], a));
          row[jj] = a;
        }
        acc[u] = fma(a, v[jj], acc[u]);
      }
    }
    for (; j < L; j += 64) {
      double a = row[j];
      if (doup) {
        a = fma(-wi, vp[j + 1], fma(-vi, wp[j + 1], a));
        row[j] = a;
      }
      acc[0] = fma(a, v[j], acc[0]);
    }
    const double pi = tk * wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
    if (lane == 0) {
      pbuf[(int64_t)cb * m + i] = pi;
      pv = fma(pi, v[i], pv);
    }
  }
  pv = block_sum_mv(pv, red);
  if (t == 0) part[cb * kMaxMvBlocks + blockIdx.x] = pv;
}

int32_t mv_blocks(int32_t L) { return std::max(1, std::min(kMaxMvBlocks, (L + 15) / 16)); }

size_t tridiag_lds_bytes(int32_t m) {
  const int32_t n = m < kTriLdsMax ? m : kTriLdsMax;
  const size_t a = (size_t)n * (n + 1) + 8 * (size_t)n;  // block + vectors + 4 partial rows
  const size_t b = m > kTriLdsMax ? 4 * (size_t)m : 0;   // global phase vectors
  return (a > b ? a : b) * sizeof(double);
}


// w[j] = j-th largest eigenvalue of T, j < m, by multisection on the Sturm
// count (LDL^T pivots of T - x I, tiny pivots replaced by -pivmin): one
// workgroup per eigenvalue, its 256 threads each count the eigenvalues below
// one of 256 interior points of the current interval, so it shrinks
// 257-fold per round; 7 rounds (257^7 > 7e16) take the Gershgorin interval
// below rounding level.
constexpr int kSect = 256;
constexpr int kBisectRounds = 7;

// The truncation rank from all m eigenvalues w (RankSelect), by one
// workgroup: w staged in LDS (sw, m doubles), each eigenvalue's rank in
// decreasing order counted against all others (ties by index), then the
// suffix sums of the clamped values from the end (sl, m + 1 doubles) and the
// first rank whose tail is within tol2.
__device__ void select_rank_block(int32_t m, const double* w, const RankSelect& sel, double* sw, double* sl) {
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int32_t i = t; i < m; i += blockDim.x) {
    const double wi = w[i];
    sw[i] = wi;
    if (!isfinite(wi)) bad = 1;
  }
  __syncthreads();
  for (int32_t i = t; i < m; i += blockDim.x) {
    const double wi = sw[i];
    int32_t r = 0;
    for (int32_t j = 0; j < m; ++j) {
      const double wj = sw[j];
      r += (wj > wi) || (wj == wi && j < i);
    }
    const double li = wi > 0.0 ? wi : 0.0;
    sel.order[r] = i;
    sel.lam[r] = li;
    sl[r] = li;
  }
  __syncthreads();
  if (t == 0) {
    double acc = 0.0;
    for (int32_t r = m - 1; r >= 0; --r) {
      acc = acc + sl[r];
      sl[r] = acc;
    }
    sl[m] = 0.0;
    // eigenvalues of a projection of the Gram matrix (Ritz values): the
    // energy they do not account for, trace - sum, belongs to every tail
    double rem = 0.0;
    if (sel.trace != nullptr) {
      const double tr = *sel.trace;
      if (!isfinite(tr)) bad = 1;
      rem = fmax(0.0, tr - sl[0]);
    }
    for (int32_t r = 0; r <= m; ++r) {
      sl[r] += rem;
      sel.tail[r] = sl[r];
    }
    int32_t rr = m;
    for (int32_t r = 0; r <= m; ++r)
      if (sl[r] <= sel.tol2) {
        rr = r;
        break;
      }
    if ((int64_t)rr > sel.cap) rr = (int32_t)sel.cap;
    const double t2 = sel.tol2 > 0.0 ? sel.tol2 : 1e-300;
    double margin = fabs(sl[rr] - sel.tol2) / t2;
    if (rr >= 1) margin = fmin(margin, fabs(sl[rr - 1] - sel.tol2) / t2);
    sel.res[0] = (double)rr;
    sel.res[1] = sl[rr];
    sel.res[2] = margin;
    sel.res[3] = bad ? 1.0 : 0.0;
  }
}

// Eigenvalue blockIdx.x (decreasing order) by Sturm multisection; with a
// RankSelect, the last workgroup to finish (arrival counter sel.cnt) then
// selects the truncation rank from all of them and clears the counter.
// Dynamic LDS: 2m + 1 doubles.
__global__ __launch_bounds__(256) void k_bisect(int32_t m, const double* __restrict__ d,
                                                const double* __restrict__ e, double* __restrict__ w,
                                                RankSelect sel) {
  HIP_DYNAMIC_SHARED(double, lds);
  __shared__ double rlo[4], rhi[4], remax[4];
  __shared__ int rbad[4];
  double* dS = lds;
  double* e2S = lds + m;  // e2S[i] = e[i-1]^2, e2S[0] = 0
  const int t = threadIdx.x;
  double lo = 1e300, hi = -1e300, emax = 0.0;
  bool nonfin = false;
  for (int32_t i = t; i < m; i += 256) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    dS[i] = d[i];
    e2S[i] = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i + 1 < m) emax = fmax(emax, e[i] * e[i]);
    if (!isfinite(d[i] + r)) nonfin = true;
  }
  // (fmin and fmax drop NaN: a non-finite entry is recorded on its own)
  const bool wbad = __ballot(nonfin) != 0;
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
    emax = fmax(emax, __shfl_down(emax, off, 64));
  }
  if ((t & 63) == 0) {
    rlo[t >> 6] = lo;
    rhi[t >> 6] = hi;
    remax[t >> 6] = emax;
    rbad[t >> 6] = wbad ? 1 : 0;
  }
  __syncthreads();
  const bool bad = (rbad[0] | rbad[1] | rbad[2] | rbad[3]) != 0;
  lo = fmin(fmin(rlo[0], rlo[1]), fmin(rlo[2], rlo[3]));
  hi = fmax(fmax(rhi[0], rhi[1]), fmax(rhi[2], rhi[3]));
  emax = fmax(fmax(remax[0], remax[1]), fmax(remax[2], remax[3]));
  const double u = 2.220446049250313e-16;
  const double nrm = fmax(fabs(lo), fabs(hi));
  lo -= 2.0 * u * nrm + 1e-300;
  hi += 2.0 * u * nrm + 1e-300;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);

  __shared__ int kw[2][4];
  const int32_t j = (int32_t)blockIdx.x;  // eigenvalue index (descending)
  const int32_t target = m - 1 - j;      // the target-th smallest (0-based)
  for (int round = 0; round < kBisectRounds; ++round) {
    const double h = (hi - lo) / (double)(kSect + 1);
    const double x = lo + h * (double)(t + 1);
    int32_t c = 0;
    double q = 1.0;
    for (int32_t i = 0; i < m; ++i) {
      q = (dS[i] - x) - e2S[i] * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
    // the threads whose point has at most `target` eigenvalues below it are
    // the first k threads (the count is monotone in x); each wave counts
    // its share
    const int kc = __popcll(__ballot(c <= target));
    if ((t & 63) == 0) kw[round & 1][t >> 6] = kc;
    __syncthreads();
    const int k = (kw[round & 1][0] + kw[round & 1][1]) + (kw[round & 1][2] + kw[round & 1][3]);
    const double nlo = (k == 0) ? lo : lo + h * (double)k;
    const double nhi = (k == kSect) ? hi : lo + h * (double)(k + 1);
    lo = nlo;
    hi = nhi;
  }
  // a non-finite tridiagonal matrix gives NaN eigenvalues, which the rank
  // selection reports
  if (t == 0) w[j] = bad ? __builtin_nan("") : 0.5 * (lo + hi);
  if (sel.cnt == nullptr) return;
  __shared__ int last;
  if (t == 0) {
    __threadfence();  // w[j] is visible before the arrival is counted
    last = atomicAdd(sel.cnt, 1) == m - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  select_rank_block(m, w, sel, lds, lds + m);
  if (t == 0) *sel.cnt = 0;
}

// LU with partial pivoting of T - lc I (tridiagonal, LAPACK gttrf order)
// into DL/DD/DU/DU2/piv; zero or tiny pivots become +-pert; DD holds the
// reciprocal pivots.  Serial; the recurrence runs in registers (the
// current pivot and the current superdiagonal entry), so each step's chain
// is a reciprocal and one FMA and the stores never wait.
__device__ void tri_factor(int32_t m, const double* __restrict__ d, const double* __restrict__ e, double lc,
                           double pert, double* __restrict__ DL, double* __restrict__ DD, double* __restrict__ DU,
                           double* __restrict__ DU2, int32_t* __restrict__ piv) {
  auto store_pivot = [&](int32_t i, double x) {
    if (fabs(x) < pert) x = x < 0.0 ? -pert : pert;
    DD[i] = 1.0 / x;
  };
  double dd = d[0] - lc;              // DD[i] as updated by step i-1
  double du = m > 1 ? e[0] : 0.0;     // DU[i] as updated by step i-1
  // branch-free (both cases formed, one selected), so the loads of the
  // next steps can be issued ahead
#pragma unroll 4
  for (int32_t i = 0; i + 1 < m; ++i) {
    const double dl = e[i];                      // DL[i], untouched so far
    const double dn = d[i + 1] - lc;             // DD[i+1], untouched so far
    const double un = i + 2 < m ? e[i + 1] : 0.0;  // DU[i+1], untouched so far
    const bool keep = fabs(dd) >= fabs(dl);      // else rows i and i+1 are exchanged
    const double p = keep ? (dd == 0.0 ? pert : dd) : dl;  // pivot
    const double q = keep ? dl : dd;
    const double f = q * recip(p);
    DL[i] = f;
    DU[i] = keep ? du : dn;
    DU2[i] = keep ? 0.0 : un;
    piv[i] = keep ? i : i + 1;
    store_pivot(i, p);
    const double ndd = keep ? dn - f * du : du - f * dn;
    du = keep ? un : -f * un;
    dd = ndd;
  }
  store_pivot(m - 1, dd);
}

// y <- (T - lc I)^{-1} y from the factors (DD holds reciprocal pivots),
// rescaled by its largest entry.  Both sweeps carry their recurrence in
// registers: one dependent FMA per step (the backward step's y[i+2] term
// and the pivot scaling are formed off the chain).
__device__ void tri_solve(int32_t m, const double* __restrict__ DL, const double* __restrict__ DD,
                          const double* __restrict__ DU, const double* __restrict__ DU2,
                          const int32_t* __restrict__ piv, double* __restrict__ y) {
  double cur = y[0];  // y[i] after the exchanges of steps < i
#pragma unroll 4
  for (int32_t i = 0; i + 1 < m; ++i) {
    const double nx = y[i + 1];
    const double l = DL[i];
    const bool keep = piv[i] == i;
    y[i] = keep ? cur : nx;
    cur = keep ? nx - l * cur : cur - l * nx;
  }
  double y1 = cur * DD[m - 1];  // y[i+1]
  double y2 = 0.0;              // y[i+2]
  y[m - 1] = y1;
  double mx = fabs(y1);
#pragma unroll 4
  for (int32_t i = m - 2; i >= 0; --i) {
    const double di = DD[i];
    const double t = (y[i] - DU2[i] * y2) * di;  // DU2[m-2] = 0
    const double yi = t - (DU[i] * di) * y1;
    y[i] = yi;
    mx = fmax(mx, fabs(yi));
    y2 = y1;
    y1 = yi;
  }
  const double s = mx > 0.0 ? 1.0 / mx : 1.0;
  for (int32_t i = 0; i < m; ++i) y[i] *= s;
}

// Eigenvector of T for an eigenvalue lc isolated from the rest of the
// spectrum, by the twisted factorization of T - lc I: top-down pivots
// D+_i = (a_i - lc) - e_{i-1}^2 / D+_{i-1}, bottom-up pivots
// D-_i = (a_i - lc) - e_i^2 / D-_{i+1} (tiny pivots become +-pert), the
// twist k minimising |gamma_k| with gamma_k = D+_k + D-_k - (a_k - lc), and
// then z_k = 1, z_i = -(e_i / D+_i) z_{i+1} above k and
// z_i = -(e_{i-1} / D-_i) z_{i-1} below it.  A pair of adjacent lanes
// (role 0 and role 1) shares the work in one instruction stream on mirrored
// indices: first the forward (dp, role 0) and backward (dm, role 1) pivots
// ...
__device__ void twisted_sweep(int32_t m, const double* __restrict__ d, const double* __restrict__ e, double lc,
                              double pert, double* dp, double* dm, int role) {
  auto guard = [pert](double x) { return fabs(x) < pert ? (x < 0.0 ? -pert : pert) : x; };
  double* out = role ? dm : dp;
  const int32_t i0 = role ? m - 1 : 0;
  double p = guard(d[i0] - lc);
  out[i0] = p;
  for (int32_t s = 0; s + 1 < m; ++s) {
    const int32_t i = role ? m - 2 - s : s + 1;
    const double ei = e[role ? i : i - 1];
    p = guard(fma(-ei * ei, recip(p), d[i] - lc));
    out[i] = p;
  }
}

// ... then (both pivot sequences complete) the twist index k (first
// minimum of |dp + dm - (d - lc)|, the same in both lanes) and the lane's
// half of z: role 0 z[k] = 1 and z[k-1 .. 0], role 1 z[k+1 .. m-1].
// Returns the half's sum of squares, and k.
__device__ double twisted_half(int32_t m, const double* __restrict__ d, const double* __restrict__ e, double lc,
                               const double* __restrict__ dp, const double* __restrict__ dm,
                               double* __restrict__ z, int role, int32_t& k) {
  k = 0;
  double best = fabs(dp[0] + dm[0] - (d[0] - lc));
  for (int32_t i = 1; i < m; ++i) {
    const double g = fabs(dp[i] + dm[i] - (d[i] - lc));
    if (g < best) {
      best = g;
      k = i;
    }
  }
  double nn = 0.0, zz = 1.0;
  if (role == 0) {
    z[k] = 1.0;
    nn = 1.0;
  }
  const int32_t len = role ? m - 1 - k : k;
  for (int32_t s = 0; s < len; ++s) {
    const int32_t i = role ? k + 1 + s : k - 1 - s;
    const double ei = e[role ? i - 1 : i];
    zz = -(ei * recip(role ? dm[i] : dp[i])) * zz;
    z[i] = zz;
    nn = fma(zz, zz, nn);
  }
  return nn;
}

__device__ __forceinline__ int64_t refl_offset(int32_t m, int32_t klo, int32_t k) {
  // sum_{j=klo}^{k-1} (m - j - 1)
  const int64_t q = k - klo;
  return q * (m - 1 - klo) - (q * (q - 1)) / 2;
}

// Reflectors klo..khi (staged in refl, refl_offset layout) applied to the
// columns of Y (one wave per column) for m <= 64 YR: the column lives in
// registers, lane l holding y[l + 64 j]; the reflector entries are read
// unconditionally at clamped positions and masked, and tau = 0 needs no
// branch (the update then adds zero).  Per reflector the dependent chain is
// the dot product's wave reduction and one FMA.
template <int YR>
__device__ void back_transform_chunk(int32_t m, int32_t r, int32_t klo, int32_t khi, const double* refl,
                                     const double* __restrict__ tau, double* Y) {
  const int t = threadIdx.x, l = t & 63;
  for (int32_t c = t >> 6; c < r; c += kWaves) {
    double* yc = Y + (int64_t)c * m;
    double y[YR];
#pragma unroll
    for (int j = 0; j < YR; ++j) y[j] = (l + 64 * j < m) ? yc[l + 64 * j] : 0.0;
    for (int32_t k = khi; k >= klo; --k) {
      const double tk = tau[k];
      const int64_t off = refl_offset(m, klo, k) - (k + 1);  // refl[off + a] = v_k[a], a > k
      double v[YR];
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < YR; ++j) {
        const int32_t a = l + 64 * j;
        const bool in = a > k && a < m;
        const double x = refl[off + (in ? a : k + 1)];
        v[j] = in ? x : 0.0;
        acc = fma(v[j], y[j], acc);
      }
      const double f = tk * wave_sum(acc);
#pragma unroll
      for (int j = 0; j < YR; ++j) y[j] = fma(-f, v[j], y[j]);
    }
#pragma unroll
    for (int j = 0; j < YR; ++j)
      if (l + 64 * j < m) yc[l + 64 * j] = y[j];
  }
}

// x from the lane CTRL names (DPP) in each of the two halves of a double
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over each aligned group of G = 8 or 16 lanes: lane pairs (l, l^1),
// (l, l^2), then the half-row and row mirrors; every lane of a group ends
// with the same bits (each step adds the same two values in both lanes).
template <int G>
__device__ __forceinline__ double group_sum(double x) {
  static_assert(G == 8 || G == 16, "groups of 8 or 16 lanes");
  x = x + dpp_f64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x = x + dpp_f64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x = x + dpp_f64<0x141>(x);  // row_half_mirror
  if constexpr (G == 16) x = x + dpp_f64<0x140>(x);  // row_mirror
  return x;
}

// The same reflectors applied to 64 / G columns per wave: a group of G lanes
// holds one column (lane p of the group: y[p + G j], YR of them), so each
// reflector's dot product is a G-lane sum and all of a wave's columns move
// together (for r well above the wave count).  Waves without a column skip.
template <int G, int YR>
__device__ void back_transform_group(int32_t m, int32_t r, int32_t klo, int32_t khi, const double* refl,
                                     const double* __restrict__ tau, double* Y) {
  constexpr int CPW = 64 / G;
  const int t = threadIdx.x, l = t & 63, p = l % G, g = l / G;
  const int w = t >> 6;
  for (int32_t c0 = 0; c0 < r; c0 += kWaves * CPW) {
    if (c0 + w * CPW >= r) continue;  // uniform over the wave
    const int32_t c = c0 + w * CPW + g;
    const bool live = c < r;
    double* yc = Y + (int64_t)(live ? c : 0) * m;
    double y[YR];
#pragma unroll
    for (int j = 0; j < YR; ++j) {
      const int32_t a = p + G * j;
      y[j] = (live && a < m) ? yc[a] : 0.0;
    }
    for (int32_t k = khi; k >= klo; --k) {
      const double tk = tau[k];
      const int64_t off = refl_offset(m, klo, k) - (k + 1);  // refl[off + a] = v_k[a], a > k
      double v[YR];
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < YR; ++j) {
        const int32_t a = p + G * j;
        const bool in = a > k && a < m;
        const double x = refl[off + (in ? a : k + 1)];
        v[j] = in ? x : 0.0;
        acc[j & 3] = fma(v[j], y[j], acc[j & 3]);
      }
      const double f = tk * group_sum<G>((acc[0] + acc[1]) + (acc[2] + acc[3]));
#pragma unroll
      for (int j = 0; j < YR; ++j) y[j] = fma(-f, v[j], y[j]);
    }
#pragma unroll
    for (int j = 0; j < YR; ++j) {
      const int32_t a = p + G * j;
      if (live && a < m) yc[a] = y[j];
    }
  }
}

// Eigenvectors of T for the r largest eigenvalues lam[0..r) (decreasing) by
// inverse iteration, back-transformed x = Q y with the reflectors kept in A's
// rows.  Every vector starts on its own thread (LU + three solves from a
// fixed start vector); vectors whose eigenvalue lies within 1e-3 ||T|| of the
// previous one (a cluster) are then recomputed in order with classical
// Gram-Schmidt (two passes) against the earlier members of their cluster at
// every iteration.  The back-transformation applies the reflectors in chunks
// staged through LDS, one wave per column.  Output X (m x r, row-major).
// kLdsWork: the per-vector factors and Y live in LDS (else in ws, 7*m*r
// doubles).  back = 0: stop before the back-transformation (ws holds Y).
template <bool kLdsWork>
__global__ __launch_bounds__(kTriThreads) void k_tri_eigvecs(int32_t m, int32_t r, const double* __restrict__ d,
                                                             const double* __restrict__ e,
                                                             const double* __restrict__ lam,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ tau,
                                                             double* __restrict__ ws, double* __restrict__ X,
                                                             int32_t back) {
  HIP_DYNAMIC_SHARED(double, lds);
  __shared__ double red[kWaves];
  const int t = threadIdx.x;
  double* dS = lds;
  double* eS = lds + m;
  double *Y, *scr, *refl;
  int64_t refl_cap;
  if (kLdsWork) {
    Y = lds + 2 * m;
    scr = Y + (int64_t)m * r;
    refl = scr + (int64_t)(6 * m + 1) * r;
    refl_cap = kLdsDoubles - (2 * (int64_t)m + (int64_t)(7 * m + 1) * r);
  } else {
    Y = ws;
    scr = ws + (int64_t)m * r;
    refl = lds + 2 * m;
    refl_cap = kLdsDoubles - 2 * (int64_t)m;
  }
  double tn = 0.0;
  for (int32_t i = t; i < m; i += kTriThreads) {
    dS[i] = d[i];
    eS[i] = (i + 1 < m) ? e[i] : 0.0;
    tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0));
  }
  for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_down(tn, off, 64));
  if ((t & 63) == 0) red[t >> 6] = tn;
  __syncthreads();
  tn = 0.0;
  for (int i = 0; i < kWaves; ++i) tn = fmax(tn, red[i]);
  __syncthreads();
  const double u = 2.220446049250313e-16;
  const double pert = fmax(u * tn, 1e-300);
  const double ortol = 1e-3 * tn;

  // phase 1: every vector on a pair of adjacent lanes; an eigenvalue
  // isolated from both neighbours in the whole spectrum (lam holds all m,
  // decreasing) takes the twisted factorization (the two lanes run the two
  // sweeps, then the two halves of the vector), the others inverse
  // iteration on the pair's first lane
  for (int32_t b0 = 0; b0 < 2 * r; b0 += kTriThreads) {  // uniform over the block
    const int32_t c2 = b0 + t;
    const bool act = c2 < 2 * r;
    const int32_t c = act ? (c2 >> 1) : 0;
    const int role = c2 & 1;
    double* base = scr + (int64_t)(6 * m + 1) * c;  // odd stride: vectors on different LDS banks
    double* zc = Y + (int64_t)c * m;
    const double lc = lam[c];
    const bool iso = act && (c == 0 || lam[c - 1] - lc > ortol) && (c + 1 >= m || lc - lam[c + 1] > ortol);
    if (iso) twisted_sweep(m, dS, eS, lc, pert, base, base + m, role);
    // the partner lane's pivots are read below (LDS operations of one wave
    // complete in order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int32_t k = 0;
    const double half = iso ? twisted_half(m, dS, eS, lc, base, base + m, zc, role, k) : 0.0;
    const double other = __shfl_xor(half, 1);
    const double nn = role ? other + half : half + other;  // the same bits in both lanes
    const bool ok = iso && nn > 0.0 && nn < 1e300;
    if (ok) {
      const double inv = 1.0 / sqrt(nn);
      const int32_t i0 = role ? k + 1 : 0, i1 = role ? m : k + 1;
      for (int32_t i = i0; i < i1; ++i) zc[i] *= inv;
    }
    if (act && role == 0 && !ok) {
      double *DL = base, *DD = base + m, *DU = base + 2 * m, *DU2 = base + 3 * m;
      int32_t* piv = (int32_t*)(base + 4 * m);
      double* y = base + 5 * m;
      tri_factor(m, dS, eS, lc, pert, DL, DD, DU, DU2, piv);
      // fixed, non-degenerate start vector (golden-ratio sequence in [0.5, 1.5))
      for (int32_t i = 0; i < m; ++i) {
        const double zq = 0.6180339887498949 * (i + 1) + 0.7548776662466927 * (c + 1);
        y[i] = 0.5 + (zq - floor(zq));
      }
      for (int it = 0; it < 3; ++it) tri_solve(m, DL, DD, DU, DU2, piv, y);
      double ny = 0.0;
      for (int32_t i = 0; i < m; ++i) ny = fma(y[i], y[i], ny);
      const double inv = ny > 0.0 ? 1.0 / sqrt(ny) : 0.0;
      for (int32_t i = 0; i < m; ++i) zc[i] = y[i] * inv;
    }
  }
  __syncthreads();
  // phase 2: clustered vectors, in order; at every iteration two passes of
  // classical Gram-Schmidt against the earlier members b0 .. c-1 of the
  // cluster: all their dot products at once (one wave per member, into
  // dots, which uses the reflector staging area: free until the
  // back-transformation), then one update of y
  // Without LDS work space the member's LU factors and vector sit in
  // global memory; when they fit, they are staged in LDS (after dots) for
  // the single-thread solves, whose every step would otherwise wait on a
  // global load.
  double* dots = refl;
  const int wv = t >> 6, ln = t & 63;
  const bool stage = !kLdsWork && 7 * (int64_t)m <= refl_cap;
  for (int32_t c = 1; c < r; ++c) {
    if (!(fabs(lam[c - 1] - lam[c]) <= ortol)) continue;
    int32_t b0 = c - 1;
    while (b0 > 0 && fabs(lam[b0 - 1] - lam[c]) <= ortol) --b0;
    const int32_t np = c - b0;
    double* base = scr + (int64_t)(6 * m + 1) * c;  // odd stride: vectors on different LDS banks
    double* yg = Y + (int64_t)c * m;
    if (stage) {
      double* sb = dots + m;
      for (int32_t i = t; i < 5 * m; i += kTriThreads) sb[i] = base[i];  // DL, DD, DU, DU2, piv
      for (int32_t i = t; i < m; i += kTriThreads) sb[5 * m + i] = yg[i];
      __syncthreads();
      base = sb;
    }
    double *DL = base, *DD = base + m, *DU = base + 2 * m, *DU2 = base + 3 * m;
    int32_t* piv = (int32_t*)(base + 4 * m);
    double* y = stage ? base + 5 * m : yg;
    for (int it = 0; it < 3; ++it) {
      if (t == 0) tri_solve(m, DL, DD, DU, DU2, piv, y);
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int32_t j = wv; j < np; j += kWaves) {
          const double* yb = Y + (int64_t)(b0 + j) * m;
          double dp = 0.0;
          for (int32_t i = ln; i < m; i += 64) dp = fma(yb[i], y[i], dp);
          dp = wave_sum(dp);
          if (ln == 0) dots[j] = dp;
        }
        __syncthreads();
        for (int32_t i = t; i < m; i += kTriThreads) {
          double s = 0.0;
          for (int32_t j = 0; j < np; ++j) s = fma(dots[j], Y[(int64_t)(b0 + j) * m + i], s);
          y[i] -= s;
        }
        __syncthreads();
      }
      double nn = 0.0;
      for (int32_t i = t; i < m; i += kTriThreads) nn = fma(y[i], y[i], nn);
      nn = block_sum(nn, red);
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int32_t i = t; i < m; i += kTriThreads) y[i] *= inv;
      __syncthreads();
    }
    if (stage) {
      // back to Y before the next member reads it
      for (int32_t i = t; i < m; i += kTriThreads) yg[i] = y[i];
      __syncthreads();
    }
  }
  // (back == 0: the tridiagonal matrix's vectors stay in ws, column c at
  // ws + c m, for the blocked back-transformation)
  if (!back) return;
  // back-transformation x = H_0 H_1 ... H_{m-3} y, reflectors klo..khi
  // staged in LDS per chunk; tau goes to LDS too (dS is free from here on)
  for (int32_t i = t; i < m; i += kTriThreads) dS[i] = tau[i];
  const double* tauS = dS;
  int32_t khi = m - 3;
  while (khi >= 0) {
    int32_t klo = khi;
    int64_t used = m - khi - 1;
    while (klo > 0 && used + (m - klo) <= refl_cap) {
      --klo;
      used += m - klo - 1;
    }
    if (m <= 256) {
      // wave w stages rows klo + w, klo + w + 8, ... four at a time, lane l
      // the entries l, l + 64, ..: all sixteen loads are issued before the
      // first store
      const int l = t & 63;
      for (int32_t k0 = klo + (t >> 6); k0 <= khi; k0 += 4 * kWaves) {
        double v[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t k = k0 + u * kWaves;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int32_t i = l + 64 * j;
            v[u][j] = (k <= khi && i < m - k - 1) ? A[(int64_t)k * m + k + 1 + i] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t k = k0 + u * kWaves;
          if (k > khi) continue;
          const int64_t off = refl_offset(m, klo, k);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int32_t i = l + 64 * j;
            if (i < m - k - 1) refl[off + i] = v[u][j];
          }
        }
      }
    } else {
      for (int32_t k = klo; k <= khi; ++k) {
        const int64_t off = refl_offset(m, klo, k);
        const int32_t L = m - k - 1;
        for (int32_t i = t; i < L; i += kTriThreads) refl[off + i] = A[(int64_t)k * m + k + 1 + i];
      }
    }
    __syncthreads();
    // one wave per column, all reflectors of the chunk without a barrier:
    // lane l always handles the indices a = l (mod 64), so no value passes
    // between lanes through memory
    if (m <= 128 && r <= kWaves)
      back_transform_chunk<2>(m, r, klo, khi, refl, tauS, Y);
    else if (m <= 128 && r <= 4 * kWaves)
      back_transform_group<16, 8>(m, r, klo, khi, refl, tauS, Y);
    else if (m <= 128)
      back_transform_group<8, 16>(m, r, klo, khi, refl, tauS, Y);
    else if (m <= 256 && r <= kWaves)
      back_transform_chunk<4>(m, r, klo, khi, refl, tauS, Y);
    else if (m <= 256)
      back_transform_group<16, 16>(m, r, klo, khi, refl, tauS, Y);
    else
      for (int32_t c = t >> 6; c < r; c += kWaves) {
        double* yc = Y + (int64_t)c * m;
        for (int32_t k = khi; k >= klo; --k) {
          const double tk = tauS[k];
          if (tk == 0.0) continue;
          const int64_t off = refl_offset(m, klo, k) - (k + 1);  // refl[off + a] = v_k[a], a > k
          double acc = 0.0;
          for (int32_t a = t & 63; a < m; a += 64)
            if (a > k) acc = fma(refl[off + a], yc[a], acc);
          const double f = tk * wave_sum(acc);
          for (int32_t a = t & 63; a < m; a += 64)
            if (a > k) yc[a] -= f * refl[off + a];
        }
      }
    __syncthreads();
    khi = klo - 1;
  }
  for (int32_t i = t >> 6; i < m; i += kWaves)
    for (int32_t c = t & 63; c < r; c += 64) X[(int64_t)i * r + c] = Y[(int64_t)c * m + i];
}

// ---- Blocked back-transformation for wide matrices: x = H_0 H_1 ...
// H_{m-3} y applied block by block in the compact WY form, H_{k0} ...
// H_{k0+nb-1} = I - V T V^T (V: the nb reflectors as columns, T upper
// triangular), so each block is three products on the tiled kernels:
// W = V^T Y, W = T W, Y -= V W (last block first).
constexpr int32_t kWyNb = 64;
constexpr int32_t kWyMin = 256;  // wider matrices take this path

// A(k, a) = 0 for a <= k: row k keeps only its reflector's entries (a > k),
// so a block of rows reads as V^T with its zeros in place
__global__ void k_zero_lower(int32_t m, double* __restrict__ A) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int32_t k = (int32_t)(e / m), a = (int32_t)(e - (int64_t)k * m);
  if (a <= k) A[e] = 0.0;
}

// T of block blockIdx.x (reflectors k0 .. k0 + nbc - 1, k0 = block * kWyNb,
// nbc = min(kWyNb, nref - k0)): S = V^T V from row tiles staged in LDS
// (thread t: row i = t / 4 of S, columns 16 (t % 4) ... + 15), then column
// by column T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) S(0:j, j).
// Output Tb + block * kWyNb^2 (kWyNb x kWyNb, zero outside nbc x nbc).
// Dynamic LDS: kWyLds doubles (the row tile, S and T).
constexpr int32_t kWyLds = kWyNb * 33 + 2 * kWyNb * (kWyNb + 1);
__global__ __launch_bounds__(256) void k_wy_t(int32_t m, int32_t nref, const double* __restrict__ A,
                                              const double* __restrict__ tau, double* __restrict__ Tb) {
  HIP_DYNAMIC_SHARED(double, sh);
  double(*Vt)[33] = reinterpret_cast<double(*)[33]>(sh);
  double(*Ss)[kWyNb + 1] = reinterpret_cast<double(*)[kWyNb + 1]>(sh + kWyNb * 33);
  double(*Ts)[kWyNb + 1] = reinterpret_cast<double(*)[kWyNb + 1]>(sh + kWyNb * 33 + kWyNb * (kWyNb + 1));
  const int t = threadIdx.x;
  const int32_t k0 = blockIdx.x * kWyNb;
  const int32_t nbc = min(kWyNb, nref - k0);
  const int i = t >> 2, j0 = (t & 3) * 16;
  double acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0;
  for (int32_t a0 = k0 + 1; a0 < m; a0 += 32) {
    for (int q = t; q < kWyNb * 32; q += 256) {
      const int r = q >> 5, c = q & 31;
      const int32_t a = a0 + c;
      Vt[r][c] = (r < nbc && a < m) ? A[(int64_t)(k0 + r) * m + a] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < 32; ++c) {
      const double vi = Vt[i][c];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = fma(vi, Vt[j0 + u][c], acc[u]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) Ss[i][j0 + u] = acc[u];
  for (int q = t; q < kWyNb * kWyNb; q += 256) Ts[q / kWyNb][q % kWyNb] = 0.0;
  __syncthreads();
  for (int32_t j = 0; j < nbc; ++j) {
    const double tj = tau[k0 + j];
    if (t < j) {
      double s = 0.0;
      for (int32_t l = t; l < j; ++l) s = fma(Ts[t][l], Ss[l][j], s);
      Ts[t][j] = -tj * s;
    } else if (t == j) {
      Ts[j][j] = tj;
    }
    __syncthreads();
  }
  double* out = Tb + (int64_t)blockIdx.x * kWyNb * kWyNb;
  for (int q = t; q < kWyNb * kWyNb; q += 256) out[q] = Ts[q / kWyNb][q % kWyNb];
}

// X (m x r, row-major) = Y (column c at Y + c m)
__global__ void k_cols_to_rows(int32_t m, int32_t r, const double* __restrict__ Y, double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * r) return;
  const int32_t i = (int32_t)(e / r), c = (int32_t)(e - (int64_t)i * r);
  X[e] = Y[(int64_t)c * m + i];
}

hipError_t set_lds_attr(const void* f) {
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsDoubles * sizeof(double)));
}

}  // namespace

int32_t sym_eig_max() { return kEigMax; }

hipError_t sym_eigvals(hipStream_t st, int32_t m, double* A, double* d, double* e, double* tau, double* w,
                       double* ws, const RankSelect* sel) {
  if (sel != nullptr && (m <= 0 || sel->cnt == nullptr)) return hipErrorInvalidValue;
  if (m <= 0) return hipSuccess;
  if (m > kEigMax) return hipErrorInvalidValue;
  // once per process (thread-safe static initialisation)
  static const hipError_t attr = [] {
    hipError_t er = set_lds_attr((const void*)k_tridiag);
    if (er == hipSuccess) er = set_lds_attr((const void*)k_bisect);
    if (er == hipSuccess) er = set_lds_attr((const void*)k_tri_eigvecs<true>);
    if (er == hipSuccess) er = set_lds_attr((const void*)k_tri_eigvecs<false>);
    if (er == hipSuccess) er = set_lds_attr((const void*)k_tri_step);
    return er;
  }();
  if (attr != hipSuccess) return attr;
  if (m <= kRwMax) {
    if (m <= 32)
      hipLaunchKernelGGL((k_tridiag_rw<1, 4>), dim3(1), dim3(kRwWaves * 64), 0, st, m, 0, m, A, d, e, tau);
    else if (m <= 64)
      hipLaunchKernelGGL((k_tridiag_rw<1, 8>), dim3(1), dim3(kRwWaves * 64), 0, st, m, 0, m, A, d, e, tau);
    else if (m <= 96)
      hipLaunchKernelGGL((k_tridiag_rw<2, 12>), dim3(1), dim3(kRwWaves * 64), 0, st, m, 0, m, A, d, e, tau);
    else
      hipLaunchKernelGGL((k_tridiag_rw<2, 16>), dim3(1), dim3(kRwWaves * 64), 0, st, m, 0, m, A, d, e, tau);
  } else if (ws != nullptr) {
    // reflections whose trailing block is wider than kRwMax on many
    // workgroups, the rest in registers
    double* vbuf = ws;
    double* pbuf = ws + 2 * (int64_t)m;
    double* part = ws + 4 * (int64_t)m;
    const int32_t ksw = m - kRwMax;
    for (int32_t k = 0; k <= ksw; ++k) {  // k == ksw: the last update only
      const int32_t L = m - k - 1;
      const int32_t G = mv_blocks(k < ksw ? L : L + 1);
      const int32_t nprev = k > 0 ? mv_blocks(m - k) : 0;
      hipLaunchKernelGGL(k_tri_step, dim3(G), dim3(kMvThreads), (size_t)(3 * (m - k) + L) * sizeof(double), st, m, k,
                         ksw, A, d, e, tau, vbuf, pbuf, part, nprev);
    }
    hipLaunchKernelGGL((k_tridiag_rw<2, 16>), dim3(1), dim3(kRwWaves * 64), 0, st, kRwMax, ksw, m, A, d, e, tau);
  } else {
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kTriThreads), tridiag_lds_bytes(m), st, m, A, d, e, tau);
  }
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return er;
  hipLaunchKernelGGL(k_bisect, dim3(m), dim3(kSect), (size_t)(2 * m + 1) * sizeof(double), st, m, d, e, w,
                     sel != nullptr ? *sel : RankSelect());
  return hipGetLastError();
}

hipError_t sym_eigvecs(hipStream_t st, int32_t m, int32_t r, const double* d, const double* e,
                       const double* lam, double* A, const double* tau, double* ws, double* X, GemmWs gws) {
  if (m <= 0 || r <= 0) return hipSuccess;
  const int64_t base_lds = 2 * (int64_t)m + (7 * (int64_t)m + 1) * r;
  // all work in LDS when that leaves room for at least one reflector
  if (base_lds + m <= kLdsDoubles) {
    hipLaunchKernelGGL(k_tri_eigvecs<true>, dim3(1), dim3(kTriThreads), (size_t)kLdsDoubles * sizeof(double),
                       st, m, r, d, e, lam, A, tau, ws, X, 1);
    return hipGetLastError();
  }
  if (m <= kWyMin) {
    hipLaunchKernelGGL(k_tri_eigvecs<false>, dim3(1), dim3(kTriThreads), (size_t)kLdsDoubles * sizeof(double),
                       st, m, r, d, e, lam, A, tau, ws, X, 1);
    return hipGetLastError();
  }
  // vectors of the tridiagonal matrix into ws (Y, column-major), then the
  // blocked back-transformation on the tiled products
  hipLaunchKernelGGL(k_tri_eigvecs<false>, dim3(1), dim3(kTriThreads), (size_t)kLdsDoubles * sizeof(double), st,
                     m, r, d, e, lam, A, tau, ws, X, 0);
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return er;
  const int32_t nref = m - 2;
  const int32_t nblk = (nref + kWyNb - 1) / kWyNb;
  double* Y = ws;
  double* Tb = ws + (int64_t)m * r;
  double* W = Tb + (int64_t)nblk * kWyNb * kWyNb;
  double* W2 = W + (int64_t)kWyNb * r;
  hipLaunchKernelGGL(k_zero_lower, dim3((unsigned)(((int64_t)m * m + 255) / 256)), dim3(256), 0, st, m, A);
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_wy_t, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(kWyLds * sizeof(double)));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_wy_t, dim3(nblk), dim3(256), (size_t)kWyLds * sizeof(double), st, m, nref, A, tau, Tb);
  er = hipGetLastError();
  if (er != hipSuccess) return er;
  View vy;  // Y rows a, columns c: Y[c m + a]
  vy.rs = 1;
  vy.cs = m;
  View vcol = vy;  // V (rows a, columns j) read from A's rows
  const View vr = row_major(r);
  for (int32_t c = nblk - 1; c >= 0; --c) {
    const int32_t k0 = c * kWyNb, nbc = std::min(kWyNb, nref - k0);
    const int32_t a0 = k0 + 1, K = m - a0;
    const double* Vb = A + (int64_t)k0 * m + a0;
    er = gemm<double, double, double>(st, nbc, r, K, K, 1.0, Vb, row_major(m), Y + a0, vy, 0.0,
                                      (const double*)nullptr, View(), W, vr, 0, nullptr, nullptr, gws);
    if (er != hipSuccess) return er;
    er = gemm<double, double, double>(st, nbc, r, nbc, nbc, 1.0, Tb + (int64_t)c * kWyNb * kWyNb, row_major(kWyNb),
                                      W, vr, 0.0, (const double*)nullptr, View(), W2, vr, 0, nullptr, nullptr, gws);
    if (er != hipSuccess) return er;
    er = gemm<double, double, double>(st, K, r, nbc, nbc, -1.0, Vb, vcol, W2, vr, 1.0, Y + a0, vy, Y + a0, vy, 0,
                                      nullptr, nullptr, gws);
    if (er != hipSuccess) return er;
  }
  hipLaunchKernelGGL(k_cols_to_rows, dim3((unsigned)(((int64_t)m * r + 255) / 256)), dim3(256), 0, st, m, r, Y, X);
  return hipGetLastError();
}

int64_t sym_eigvecs_ws(int32_t m, int32_t r) {
  int64_t w = (7 * (int64_t)m + 1) * r;
  if (m > kWyMin) {
    const int64_t nblk = (m - 2 + kWyNb - 1) / kWyNb;
    w = std::max<int64_t>(w, (int64_t)m * r + nblk * kWyNb * kWyNb + 2 * (int64_t)kWyNb * r);
  }
  return w;
}

}  // namespace ttice
