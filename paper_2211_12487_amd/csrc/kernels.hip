// gfx950 kernels of the TT-ICE library (generic FP64-accumulating paths).
//
// Every kernel here computes one step of TT-ICE (Algorithm 1 / Algorithm 2 of
// arXiv 2211.12487); the host engine (ttice.hip) sequences them.  Layouts:
// cores are row-major FP64, level data is frame-major [N][rows][cols].
#include "kernels.h"

#include <math.h>

namespace ttice {

namespace {

__device__ __forceinline__ int64_t row_off(const View& v, int32_t i) {
  if (v.rpf == kUnframed) return (int64_t)i * v.rs;
  const uint32_t f = (uint32_t)i / (uint32_t)v.rpf;
  const uint32_t w = (uint32_t)i - f * (uint32_t)v.rpf;
  return (int64_t)f * v.rfs + (int64_t)w * v.rs;
}

__device__ __forceinline__ int64_t col_off(const View& v, int32_t j) {
  if (v.cpf == kUnframed) return (int64_t)j * v.cs;
  const uint32_t f = (uint32_t)j / (uint32_t)v.cpf;
  const uint32_t w = (uint32_t)j - f * (uint32_t)v.cpf;
  const int64_t ff = v.cfidx ? (int64_t)v.cfidx[f] : (int64_t)f;
  return ff * v.cfs + (int64_t)w * v.cs;
}

// ---------------------------------------------------------------------------
// Generic tiled product  D = alpha A B + beta E  (64 x 64 tiles, 256 threads,
// 4 x 4 register micro-tiles strided by 16 to spread LDS banks, K staged in
// chunks of 16 through LDS, FP64 accumulation).
// ---------------------------------------------------------------------------
template <typename TB, typename TE, typename TD>
__global__ __launch_bounds__(256) void k_gemm(int32_t M, int32_t N, int32_t K, int32_t kchunk,
                                               double alpha, const double* __restrict__ A, View va,
                                               const TB* __restrict__ B, View vb, double beta,
                                               const TE* __restrict__ E, View ve, TD* __restrict__ D,
                                               View vd, int64_t dz, double* __restrict__ colpart,
                                               double* __restrict__ bnorm) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int ln = t & 63, lk = t >> 6;
  const int32_t m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int32_t kb = (int32_t)blockIdx.z * kchunk;
  const int32_t ke = min(K, kb + kchunk);

  const int32_t bn = n0 + ln;
  const bool bvalid = bn < N;
  const int64_t bco = bvalid ? col_off(vb, bn) : 0;
  const int32_t am = m0 + ln;
  const bool avalid = am < M;
  const int64_t aro = avalid ? row_off(va, am) : 0;

  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  double bsq = 0.0;

  for (int32_t k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = lk + 4 * u;
      const int32_t k = k0 + kk;
      double av = 0.0, bv = 0.0;
      if (k < ke) {
        if (avalid) av = A[aro + col_off(va, k)];
        if (bvalid) bv = (double)B[row_off(vb, k) + bco];
      }
      As[kk][ln] = av;
      Bs[kk][ln] = bv;
      bsq = fma(bv, bv, bsq);
    }
    __syncthreads();
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
    __syncthreads();
  }

  if (bnorm != nullptr && blockIdx.y == 0) {
    red[t] = bsq;
    __syncthreads();
    if (t < 64 && bvalid) bnorm[bn] = (red[t] + red[t + 64]) + (red[t + 128] + red[t + 192]);
    __syncthreads();
  }

  double csq[4] = {0.0, 0.0, 0.0, 0.0};
  TD* Dz = D ? D + dz * (int64_t)blockIdx.z : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int32_t m = m0 + ty + 16 * i;
    if (m >= M) continue;
    const int64_t ero = E ? row_off(ve, m) : 0;
    const int64_t dro = Dz ? row_off(vd, m) : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t n = n0 + tx + 16 * j;
      if (n >= N) continue;
      double v = alpha * acc[i][j];
      if (E) v = fma(beta, (double)E[ero + col_off(ve, n)], v);
      if (Dz) Dz[dro + col_off(vd, n)] = (TD)v;
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

// ---------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------
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

__global__ __launch_bounds__(256) void k_frame_sums(const double* __restrict__ part, int32_t MB,
                                                     int64_t ld, int32_t cpf, double* __restrict__ out) {
  __shared__ double red[256];
  const int32_t f = blockIdx.x;
  double s = 0.0;
  const int64_t per = (int64_t)MB * cpf;
  for (int64_t q = threadIdx.x; q < per; q += 256) {
    const int64_t mb = q / cpf, c = q - mb * cpf;
    s += part[mb * ld + (int64_t)f * cpf + c];
  }
  s = block_sum_256(s, red);
  if (threadIdx.x == 0) out[f] = s;
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
  double s = 0.0;
  for (int32_t z = 0; z < S; ++z) s += part[z * mm + src];
  G[idx] = s;
}

// ---------------------------------------------------------------------------
// Cyclic two-sided Jacobi (Golub & Van Loan, symmetric Schur 2x2 rotations)
// with the round-robin ("circle") parallel ordering: at step t the pairs are
// (t mod (n-1), n-1) and ((t+k) mod (n-1), (t-k) mod (n-1)), k = 1..n/2-1,
// so every index pair is visited once per sweep and the n/2 rotations of a
// step act on disjoint index pairs.  For disjoint pairs the two-sided update
// G <- J^T G J factorises over 2x2 blocks (pair a rows, pair b cols):
// block_ab <- J_a^T block_ab J_b, so each block is updated independently.
// The matrix lives either in LDS (Gs/Vs with row stride ldl) or in global
// memory; the same device routine serves both.
// ---------------------------------------------------------------------------
constexpr int kJacobiThreads = 1024;
constexpr int kJacobiLdsMax = 96;
constexpr int kMaxSweeps = 40;

constexpr int kJacobiGlobalHalf = 2048;  // pairs per step of the global-memory path (m <= 4096)

template <int HALF>
struct JacobiShared {
  int32_t p[HALF];
  int32_t q[HALF];
  double c[HALF];
  double s[HALF];
  double tn[HALF];
  int32_t rot[HALF];
  int32_t any;
  double red[kJacobiThreads / 64];
};

__device__ double block_sum_1024(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kJacobiThreads / 64; ++i) s += red[i];
  __syncthreads();
  if (threadIdx.x == 0) red[0] = s;
  __syncthreads();
  s = red[0];
  __syncthreads();
  return s;
}

__device__ __forceinline__ void pair_of(int32_t t, int32_t k, int32_t n, int32_t& p, int32_t& q) {
  const int32_t n1 = n - 1;
  if (k == 0) {
    p = t % n1;
    q = n1;
  } else {
    p = (t + k) % n1;
    q = (t - k + n1) % n1;
  }
  if (p > q) {
    const int32_t x = p;
    p = q;
    q = x;
  }
}

// G, V: n x n (n even) with row stride ld; indices >= m are padding.
template <bool kLds, int HALF>
__device__ void jacobi_run(int32_t m, int32_t n, double* G, double* V, int64_t ld,
                           JacobiShared<HALF>& sh, int32_t* dsweeps) {
  const int t = threadIdx.x;
  const int32_t half = n / 2;
  // Frobenius norm for the absolute threshold
  double fs = 0.0;
  for (int64_t e = t; e < (int64_t)m * m; e += kJacobiThreads) {
    const int32_t i = (int32_t)(e / m), j = (int32_t)(e % m);
    const double g = G[(int64_t)i * ld + j];
    fs = fma(g, g, fs);
  }
  const double normF = sqrt(block_sum_1024(fs, sh.red));
  const double u = 2.220446049250313e-16;
  const double tol_abs = u * normF / (double)(n > 1 ? n : 1);
  __syncthreads();

  int32_t sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (t == 0) sh.any = 0;
    __syncthreads();
    for (int32_t step = 0; step < n - 1; ++step) {
      for (int32_t k = t; k < half; k += kJacobiThreads) {
        int32_t p, q;
        pair_of(step, k, n, p, q);
        sh.p[k] = p;
        sh.q[k] = q;
        int32_t rot = 0;
        double cs = 1.0, sn = 0.0, tn = 0.0;
        if (q < m) {
          const double a = G[(int64_t)p * ld + p];
          const double b = G[(int64_t)q * ld + q];
          const double c = G[(int64_t)p * ld + q];
          const double thr = fmax(u * sqrt(fabs(a) * fabs(b)), tol_abs);
          if (fabs(c) > thr) {
            const double tau = (b - a) / (2.0 * c);
            const double tt = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                           : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            cs = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * cs;
            tn = tt;
            rot = 1;
          }
        }
        sh.c[k] = cs;
        sh.s[k] = sn;
        sh.tn[k] = tn;
        sh.rot[k] = rot;
        if (rot) sh.any = 1;
      }
      __syncthreads();
      // 2x2 block updates for ka <= kb (mirror kb < ka)
      const int32_t nblk = half * half;
      for (int32_t task = t; task < nblk; task += kJacobiThreads) {
        const int32_t ka = task / half, kb = task - ka * half;
        if (kb < ka) continue;
        const int32_t ra = sh.rot[ka], rb = sh.rot[kb];
        if (!ra && !rb) continue;
        const int32_t pa = sh.p[ka], qa = sh.q[ka], pb = sh.p[kb], qb = sh.q[kb];
        if (ka == kb) {
          const double c = G[(int64_t)pa * ld + qa];
          const double tt = sh.tn[ka];
          G[(int64_t)pa * ld + pa] -= tt * c;
          G[(int64_t)qa * ld + qa] += tt * c;
          G[(int64_t)pa * ld + qa] = 0.0;
          G[(int64_t)qa * ld + pa] = 0.0;
          continue;
        }
        const double ca = sh.c[ka], sa = sh.s[ka], cb = sh.c[kb], sb = sh.s[kb];
        const double g11 = G[(int64_t)pa * ld + pb], g12 = G[(int64_t)pa * ld + qb];
        const double g21 = G[(int64_t)qa * ld + pb], g22 = G[(int64_t)qa * ld + qb];
        const double h11 = ca * g11 - sa * g21, h12 = ca * g12 - sa * g22;
        const double h21 = sa * g11 + ca * g21, h22 = sa * g12 + ca * g22;
        const double n11 = cb * h11 - sb * h12, n12 = sb * h11 + cb * h12;
        const double n21 = cb * h21 - sb * h22, n22 = sb * h21 + cb * h22;
        G[(int64_t)pa * ld + pb] = n11;
        G[(int64_t)pa * ld + qb] = n12;
        G[(int64_t)qa * ld + pb] = n21;
        G[(int64_t)qa * ld + qb] = n22;
        G[(int64_t)pb * ld + pa] = n11;
        G[(int64_t)qb * ld + pa] = n12;
        G[(int64_t)pb * ld + qa] = n21;
        G[(int64_t)qb * ld + qa] = n22;
      }
      // V <- V J
      const int32_t nv = m * half;
      for (int32_t task = t; task < nv; task += kJacobiThreads) {
        const int32_t i = task / half, k = task - i * half;
        if (!sh.rot[k]) continue;
        const int32_t p = sh.p[k], q = sh.q[k];
        const double cs = sh.c[k], sn = sh.s[k];
        const double v1 = V[(int64_t)i * ld + p], v2 = V[(int64_t)i * ld + q];
        V[(int64_t)i * ld + p] = cs * v1 - sn * v2;
        V[(int64_t)i * ld + q] = sn * v1 + cs * v2;
      }
      if (!kLds) __threadfence_block();
      __syncthreads();
    }
    const int32_t any = sh.any;
    __syncthreads();
    if (!any) break;
  }
  if (t == 0 && dsweeps) *dsweeps = sweep;
}

__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_lds(int32_t m, double* __restrict__ G,
                                                               double* __restrict__ V,
                                                               double* __restrict__ w,
                                                               int32_t* dsweeps) {
  HIP_DYNAMIC_SHARED(double, lds);
  __shared__ JacobiShared<kJacobiLdsMax / 2> sh;
  const int32_t n = m + (m & 1);
  const int64_t ld = n + 1;
  double* Gs = lds;
  double* Vs = lds + (int64_t)n * ld;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kJacobiThreads) {
    const int32_t i = (int32_t)(e / n), j = (int32_t)(e % n);
    Gs[i * ld + j] = (i < m && j < m) ? G[(int64_t)i * m + j] : 0.0;
    Vs[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_run<true, kJacobiLdsMax / 2>(m, n, Gs, Vs, ld, sh, dsweeps);
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += kJacobiThreads) {
    const int32_t i = (int32_t)(e / m), j = (int32_t)(e % m);
    V[e] = Vs[i * ld + j];
  }
  for (int32_t i = threadIdx.x; i < m; i += kJacobiThreads) w[i] = Gs[i * ld + i];
}

// Global-memory variant: G and V are n x n buffers (n = m rounded up to
// even), ld = n; the caller provides them padded.
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_global(int32_t m, double* __restrict__ G,
                                                                  double* __restrict__ V,
                                                                  double* __restrict__ w,
                                                                  int32_t* dsweeps) {
  __shared__ JacobiShared<kJacobiGlobalHalf> sh;
  const int32_t n = m + (m & 1);
  jacobi_run<false, kJacobiGlobalHalf>(m, n, G, V, n, sh, dsweeps);
  __syncthreads();
  for (int32_t i = threadIdx.x; i < m; i += kJacobiThreads) w[i] = G[(int64_t)i * n + i];
}

// repack G (m x m, ld m) into an n x n padded buffer with V = I (in place is
// not possible; src and dst differ)
__global__ void k_pad_square(int32_t m, int32_t n, const double* __restrict__ src,
                             double* __restrict__ G, double* __restrict__ V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int32_t i = (int32_t)(e / n), j = (int32_t)(e % n);
  G[e] = (i < m && j < m) ? src[(int64_t)i * m + j] : 0.0;
  V[e] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_unpad_square(int32_t m, int32_t n, const double* __restrict__ V,
                               double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int32_t i = (int32_t)(e / m), j = (int32_t)(e % m);
  dst[e] = V[(int64_t)i * n + j];
}

// ---------------------------------------------------------------------------
// Truncation rank from the Gram eigenvalues (eq:deltasvd / eq:svdfirst)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_select_rank(int32_t m, const double* __restrict__ w,
                                                      double tol2, int64_t cap,
                                                      int32_t* __restrict__ order,
                                                      double* __restrict__ lam,
                                                      double* __restrict__ tail,
                                                      double* __restrict__ res) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int32_t i = threadIdx.x; i < m; i += blockDim.x) {
    const double wi = w[i];
    if (!isfinite(wi)) bad = 1;
    int32_t r = 0;
    for (int32_t j = 0; j < m; ++j) {
      const double wj = w[j];
      r += (wj > wi) || (wj == wi && j < i);
    }
    order[r] = i;
    lam[r] = wi > 0.0 ? wi : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    tail[m] = 0.0;
    for (int32_t r = m - 1; r >= 0; --r) tail[r] = tail[r + 1] + lam[r];
    int32_t rr = m;
    for (int32_t r = 0; r <= m; ++r)
      if (tail[r] <= tol2) {
        rr = r;
        break;
      }
    if ((int64_t)rr > cap) rr = (int32_t)cap;
    const double t2 = tol2 > 0.0 ? tol2 : 1e-300;
    double margin = fabs(tail[rr] - tol2) / t2;
    if (rr >= 1) margin = fmin(margin, fabs(tail[rr - 1] - tol2) / t2);
    res[0] = (double)rr;
    res[1] = tail[rr];
    res[2] = margin;
    res[3] = bad ? 1.0 : 0.0;
  }
}

__global__ void k_gather_columns(int32_t rows, int32_t r, const double* __restrict__ V, int32_t ldv,
                                 const int32_t* __restrict__ order, const double* __restrict__ lam,
                                 int32_t scale, double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * r) return;
  const int32_t i = (int32_t)(e / r), tcol = (int32_t)(e % r);
  double v = V[(int64_t)i * ldv + order[tcol]];
  if (scale) v /= sqrt(lam[tcol]);
  W[e] = v;
}

__global__ __launch_bounds__(256) void k_sign_fix(int32_t rows, double* __restrict__ W, int64_t ld) {
  __shared__ double bv[256];
  __shared__ int32_t bi[256];
  const int32_t col = blockIdx.x;
  double best = -1.0;
  int32_t bidx = 0x7fffffff;
  for (int32_t i = threadIdx.x; i < rows; i += 256) {
    const double a = fabs(W[(int64_t)i * ld + col]);
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
  const bool flip = (k < rows) && (W[(int64_t)k * ld + col] < 0.0);
  __syncthreads();
  if (flip)
    for (int32_t i = threadIdx.x; i < rows; i += 256) W[(int64_t)i * ld + col] = -W[(int64_t)i * ld + col];
}

__global__ void k_copy2d(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                         double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  dst[i * ldd + j] = src[i * lds + j];
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
  double srel = 0.0, se = 0.0, sy = 0.0, sdc = 0.0, sd = 0.0, cnt = 0.0;
  for (int32_t b = threadIdx.x; b < N; b += 256) {
    const double e = e2[b] > 0.0 ? e2[b] : 0.0;
    const double y = y2[b];
    const double rel = y > 0.0 ? sqrt(e / y) : 0.0;
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
  if (threadIdx.x == 0) {
    res[0] = N > 0 ? srel / N : 0.0;
    res[1] = sy > 0.0 ? sqrt(se / sy) : 0.0;
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

}  // namespace

template <typename TB, typename TE, typename TD>
hipError_t gemm(hipStream_t st, int32_t M, int32_t N, int32_t K, int32_t kchunk, double alpha,
                const double* A, View va, const TB* B, View vb, double beta, const TE* E, View ve,
                TD* D, View vd, int64_t dz, double* colpart, double* bnorm) {
  if (N <= 0) return hipSuccess;
  if (kchunk <= 0) kchunk = K > 0 ? K : 1;
  const int32_t S = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)gemm_row_blocks(M), (unsigned)S);
  hipLaunchKernelGGL((k_gemm<TB, TE, TD>), grid, dim3(256), 0, st, M, N, K, kchunk, alpha, A, va, B,
                     vb, beta, E, ve, D, vd, dz, colpart, bnorm);
  return hipGetLastError();
}

#define TTICE_GEMM_INST(TB, TE, TD)                                                                  \
  template hipError_t gemm<TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, int32_t, double,      \
                                       const double*, View, const TB*, View, double, const TE*, View, \
                                       TD*, View, int64_t, double*, double*);
TTICE_GEMM_INST(double, double, double)
TTICE_GEMM_INST(float, double, double)
TTICE_GEMM_INST(double, float, double)
TTICE_GEMM_INST(float, float, double)
TTICE_GEMM_INST(double, double, float)
TTICE_GEMM_INST(float, float, float)
TTICE_GEMM_INST(double, float, float)
TTICE_GEMM_INST(float, double, float)

hipError_t frame_sums(hipStream_t st, const double* part, int32_t MB, int64_t ld, int32_t cpf,
                      int32_t F, double* out) {
  if (F <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_frame_sums, dim3(F), dim3(256), 0, st, part, MB, ld, cpf, out);
  return hipGetLastError();
}

hipError_t total_sum(hipStream_t st, const double* x, int64_t n, double* out) {
  hipLaunchKernelGGL(k_total_sum, dim3(1), dim3(256), 0, st, x, n, out);
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

int32_t sym_eig_lds_max() { return kJacobiLdsMax; }

// Work buffers for the global-memory path live right after G and V: the
// caller allocates G and V with room for n*n doubles each (n = m + (m & 1))
// plus an extra n*n each for the padded copies.
hipError_t sym_eig(hipStream_t st, int32_t m, double* G, double* V, double* w, int32_t* dsweeps) {
  if (m <= 0) return hipSuccess;
  if (m <= kJacobiLdsMax) {
    const int32_t n = m + (m & 1);
    const size_t lds = (size_t)2 * n * (n + 1) * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_lds,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)((size_t)2 * 96 * 97 * sizeof(double)));
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    hipLaunchKernelGGL(k_jacobi_lds, dim3(1), dim3(kJacobiThreads), lds, st, m, G, V, w, dsweeps);
    return hipGetLastError();
  }
  const int32_t n = m + (m & 1);
  double* Gp = G + (int64_t)n * n;  // padded copies (caller-provided room)
  double* Vp = V + (int64_t)n * n;
  hipLaunchKernelGGL(k_pad_square, dim3(nblocks((int64_t)n * n, 256)), dim3(256), 0, st, m, n, G, Gp,
                     Vp);
  hipLaunchKernelGGL(k_jacobi_global, dim3(1), dim3(kJacobiThreads), 0, st, m, Gp, Vp, w, dsweeps);
  hipLaunchKernelGGL(k_unpad_square, dim3(nblocks((int64_t)m * m, 256)), dim3(256), 0, st, m, n, Vp, V);
  return hipGetLastError();
}

hipError_t select_rank(hipStream_t st, int32_t m, const double* w, double tol2, int64_t cap,
                       int32_t* order, double* lam, double* tail, double* res) {
  hipLaunchKernelGGL(k_select_rank, dim3(1), dim3(1024), 0, st, m, w, tol2, cap, order, lam, tail, res);
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

hipError_t sign_fix(hipStream_t st, int32_t rows, int32_t r, double* W, int64_t ld) {
  if (r <= 0 || rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_fix, dim3(r), dim3(256), 0, st, rows, W, ld);
  return hipGetLastError();
}

hipError_t copy2d(hipStream_t st, int64_t rows, int64_t cols, const double* src, int64_t lds,
                  double* dst, int64_t ldd) {
  const int64_t n = rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy2d, dim3(nblocks(n, 256)), dim3(256), 0, st, rows, cols, src, lds, dst, ldd);
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
