// Symmetric eigensolver for the truncated SVD of the residual (eq:svdfirst):
// the Gram matrix G = R R^T (or R^T R) is reduced to tridiagonal form by
// Householder reflections (one workgroup), all eigenvalues are found by
// Sturm-sequence bisection (one thread per eigenvalue, returned in
// decreasing order), and only the eigenvectors that TT-ICE keeps are formed
// by inverse iteration on the tridiagonal matrix followed by the
// back-transformation with the stored reflectors.
#include "kernels.h"

#include <math.h>

namespace ttice {
namespace {

constexpr int kTriThreads = 512;
constexpr int kTriLdsMax = 124;  // (m x (m+1)) FP64 + vectors fit in 160 KB of LDS
constexpr int kWaves = kTriThreads / 64;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;  // valid in lane 0
}

// Sum over the block; every thread gets the result.  red: >= kWaves doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kWaves; ++i) s += red[i];
  return s;
}

// Householder tridiagonalisation (dsytd2 order) of the symmetric m x m
// matrix A (row-major, row stride ld, full storage).  On exit d[0..m),
// e[0..m-1) hold the tridiagonal matrix T = Q^T A Q, Q = H_0 ... H_{m-3},
// H_k = I - tau[k] v_k v_k^T acting on indices k+1..m-1, and row k of A
// holds v_k in columns k+1..m-1 (v_k[0] = 1).
//
// Three barriers per reflection: every thread derives (beta, tau) from the
// shared x[0] and ||x[1:]||^2; wave w forms p_i = tau (A v)_i for rows
// i = w, w + waves, ... (lanes across the row) and a partial p.v; the
// rank-2 update A -= v w^T + w v^T (w = p - (tau/2)(p.v) v) is applied row
// by row, and the wave that updates the first row of the trailing block also
// stores the next reflection's x and ||x[1:]||^2.  vbuf: 4m doubles (two
// alternating x vectors, the normalised v, and p), in LDS.
template <bool kLds>
__device__ void tridiag_run(int32_t m, double* A, int64_t ld, double* vbuf, double* red, double* sc,
                            double* d, double* e, double* tau) {
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  double* va = vbuf;          // x of the current reflection (read only in the step)
  double* vb = vbuf + m;      // x of the next reflection
  double* vn = vbuf + 2 * m;  // v = [1, x[1:] / (x[0] - beta)]
  double* p = vbuf + 3 * m;
  // sc[k & 1] holds ||x[1:]||^2 of reflection k (written during step k-1)
  if (m >= 3) {
    // x of the first reflection: row 0, columns 1..m-1
    double s = 0.0;
    for (int32_t i = t; i < m - 1; i += kTriThreads) {
      const double x = A[1 + i];
      va[i] = x;
      if (i > 0) s = fma(x, x, s);
    }
    s = block_sum(s, red);
    if (t == 0) sc[0] = s;
    __syncthreads();
  }
  for (int32_t k = 0; k + 2 < m; ++k) {
    const int32_t L = m - k - 1;
    double* row = A + (int64_t)k * ld + (k + 1);
    const double sigma = sc[k & 1];
    double* snext = sc + ((k + 1) & 1);
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
    __syncthreads();  // (1) v complete
    double* sub = A + (int64_t)(k + 1) * ld + (k + 1);
    if (tk != 0.0) {
      double pvw = 0.0;
      for (int32_t i = wid; i < L; i += kWaves) {
        const double* ri = sub + (int64_t)i * ld;
        double acc = 0.0;
        for (int32_t j = lane; j < L; j += 64) acc = fma(ri[j], vn[j], acc);
        acc = wave_sum(acc);
        if (lane == 0) {
          p[i] = tk * acc;
          pvw = fma(tk * acc, vn[i], pvw);
        }
      }
      if (lane == 0) red[wid] = pvw;
      __syncthreads();  // (2) p and the partial p.v complete
      double pv = 0.0;
      for (int i = 0; i < kWaves; ++i) pv += red[i];
      const double gam = 0.5 * tk * pv;
      for (int32_t i = wid; i < L; i += kWaves) {
        double* ri = sub + (int64_t)i * ld;
        const double vi = vn[i], wi = p[i] - gam * vi;
        double sn = 0.0;
        for (int32_t j = lane; j < L; j += 64) {
          const double a = ri[j] - vi * (p[j] - gam * vn[j]) - wi * vn[j];
          ri[j] = a;
          if (i == 0 && j >= 1) {
            vb[j - 1] = a;
            if (j >= 2) sn = fma(a, a, sn);
          }
        }
        if (i == 0) {
          sn = wave_sum(sn);
          if (lane == 0) *snext = sn;
        }
      }
    } else {
      // no reflection: the next x is row k+1 as it stands
      if (wid == 0) {
        double sn = 0.0;
        for (int32_t j = lane; j < L; j += 64)
          if (j >= 1) {
            const double a = sub[j];
            vb[j - 1] = a;
            if (j >= 2) sn = fma(a, a, sn);
          }
        sn = wave_sum(sn);
        if (lane == 0) *snext = sn;
      }
    }
    if (!kLds) __threadfence_block();
    __syncthreads();  // (3) update, next x and its norm complete
    double* tmp = va;
    va = vb;
    vb = tmp;
  }
  if (t == 0) {
    if (m >= 2) {
      d[m - 2] = A[(int64_t)(m - 2) * ld + (m - 2)];
      e[m - 2] = A[(int64_t)(m - 2) * ld + (m - 1)];
      tau[m - 2] = 0.0;
    }
    d[m - 1] = A[(int64_t)(m - 1) * ld + (m - 1)];
    tau[m - 1] = 0.0;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kTriThreads) void k_tridiag_lds(int32_t m, double* __restrict__ A,
                                                             double* __restrict__ d, double* __restrict__ e,
                                                             double* __restrict__ tau) {
  HIP_DYNAMIC_SHARED(double, lds);
  __shared__ double red[kWaves];
  __shared__ double sc[4];
  const int64_t ld = m + 1;
  double* As = lds;
  for (int32_t i = threadIdx.x >> 6; i < m; i += kWaves)
    for (int32_t j = threadIdx.x & 63; j < m; j += 64) As[i * ld + j] = A[(int64_t)i * m + j];
  __syncthreads();
  tridiag_run<true>(m, As, ld, lds + (int64_t)m * ld, red, sc, d, e, tau);
  // write the reflectors back (upper part of each row)
  for (int32_t i = threadIdx.x >> 6; i < m; i += kWaves)
    for (int32_t j = threadIdx.x & 63; j < m; j += 64) A[(int64_t)i * m + j] = As[i * ld + j];
}

__global__ __launch_bounds__(kTriThreads) void k_tridiag_global(int32_t m, double* __restrict__ A,
                                                                double* __restrict__ d, double* __restrict__ e,
                                                                double* __restrict__ tau) {
  HIP_DYNAMIC_SHARED(double, lds);
  __shared__ double red[kWaves];
  __shared__ double sc[4];
  tridiag_run<false>(m, A, m, lds, red, sc, d, e, tau);
}

// w[j] = j-th largest eigenvalue of T, j < m, by multisection on the Sturm
// count: 16 lanes per eigenvalue each count the eigenvalues below one of 16
// interior points of the current interval, and the interval shrinks 17-fold
// per round (14 rounds take the Gershgorin interval below rounding level).
constexpr int kSect = 16;
constexpr int kBisectRounds = 14;

__global__ __launch_bounds__(256) void k_bisect(int32_t m, const double* __restrict__ d,
                                                const double* __restrict__ e, double* __restrict__ w) {
  __shared__ double rlo[4], rhi[4], remax[4];
  const int t = threadIdx.x;
  // Gershgorin interval of T (block reduction)
  double lo = 1e300, hi = -1e300, emax = 0.0;
  for (int32_t i = t; i < m; i += 256) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i + 1 < m) emax = fmax(emax, e[i] * e[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
    emax = fmax(emax, __shfl_down(emax, off, 64));
  }
  if ((t & 63) == 0) {
    rlo[t >> 6] = lo;
    rhi[t >> 6] = hi;
    remax[t >> 6] = emax;
  }
  __syncthreads();
  lo = fmin(fmin(rlo[0], rlo[1]), fmin(rlo[2], rlo[3]));
  hi = fmax(fmax(rhi[0], rhi[1]), fmax(rhi[2], rhi[3]));
  emax = fmax(fmax(remax[0], remax[1]), fmax(remax[2], remax[3]));
  const double u = 2.220446049250313e-16;
  const double nrm = fmax(fabs(lo), fabs(hi));
  lo -= 2.0 * u * nrm + 1e-300;
  hi += 2.0 * u * nrm + 1e-300;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);

  const int32_t j = (int32_t)blockIdx.x * (256 / kSect) + t / kSect;  // eigenvalue index (descending)
  const int32_t l = t % kSect;                                        // lane within the group
  const bool valid = j < m;
  const int32_t target = m - 1 - j;  // the target-th smallest (0-based)
  const int gshift = (t & 63) / kSect * kSect;
  for (int round = 0; round < kBisectRounds; ++round) {
    const double h = (hi - lo) / (double)(kSect + 1);
    const double x = lo + h * (double)(l + 1);
    int32_t c = 0;
    if (valid) {
      double q = d[0] - x;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
      for (int32_t i = 1; i < m; ++i) {
        const double ei = e[i - 1];
        q = (d[i] - x) - (ei * ei) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
      }
    }
    // lanes whose point has at most `target` eigenvalues below it; the count
    // is monotone in x, so they are the group's first k lanes
    const unsigned long long bal = __ballot(valid && c <= target);
    const int k = __popcll((bal >> gshift) & ((1ull << kSect) - 1ull));
    const double nlo = (k == 0) ? lo : lo + h * (double)k;
    const double nhi = (k == kSect) ? hi : lo + h * (double)(k + 1);
    lo = nlo;
    hi = nhi;
  }
  if (valid && l == 0) w[j] = 0.5 * (lo + hi);
}

// Inverse iteration for eigenvalue lc of T (d, e) in per-vector scratch:
// LU with partial pivoting of T - lc I (LAPACK gttrf order) into
// DL/DD/DU/DU2/piv, then `iters` solves from the start vector in y, each
// rescaled by its largest entry.  Serial (one thread).
__device__ void tri_factor(int32_t m, const double* __restrict__ d, const double* __restrict__ e, double lc,
                           double pert, double* DL, double* DD, double* DU, double* DU2, int32_t* piv) {
  for (int32_t i = 0; i < m; ++i) {
    DD[i] = d[i] - lc;
    if (i + 1 < m) {
      DL[i] = e[i];
      DU[i] = e[i];
    }
    if (i + 2 < m) DU2[i] = 0.0;
  }
  for (int32_t i = 0; i + 1 < m; ++i) {
    if (fabs(DD[i]) >= fabs(DL[i])) {
      if (DD[i] == 0.0) DD[i] = pert;
      const double f = DL[i] / DD[i];
      DL[i] = f;
      DD[i + 1] -= f * DU[i];
      if (i + 2 < m) DU2[i] = 0.0;
      piv[i] = i;
    } else {
      const double f = DD[i] / DL[i];
      DD[i] = DL[i];
      DL[i] = f;
      const double tmp = DU[i];
      DU[i] = DD[i + 1];
      DD[i + 1] = tmp - f * DD[i + 1];
      if (i + 2 < m) {
        DU2[i] = DU[i + 1];
        DU[i + 1] = -f * DU[i + 1];
      }
      piv[i] = i + 1;
    }
  }
  for (int32_t i = 0; i < m; ++i)
    if (fabs(DD[i]) < pert) DD[i] = DD[i] < 0.0 ? -pert : pert;
}

__device__ void tri_solve(int32_t m, const double* DL, const double* DD, const double* DU, const double* DU2,
                          const int32_t* piv, double* y) {
  for (int32_t i = 0; i + 1 < m; ++i) {
    if (piv[i] == i) {
      y[i + 1] -= DL[i] * y[i];
    } else {
      const double tmp = y[i] - DL[i] * y[i + 1];
      y[i] = y[i + 1];
      y[i + 1] = tmp;
    }
  }
  y[m - 1] /= DD[m - 1];
  if (m >= 2) y[m - 2] = (y[m - 2] - DU[m - 2] * y[m - 1]) / DD[m - 2];
  for (int32_t i = m - 3; i >= 0; --i) y[i] = (y[i] - DU[i] * y[i + 1] - DU2[i] * y[i + 2]) / DD[i];
  double mx = 0.0;
  for (int32_t i = 0; i < m; ++i) mx = fmax(mx, fabs(y[i]));
  const double s = mx > 0.0 ? 1.0 / mx : 1.0;
  for (int32_t i = 0; i < m; ++i) y[i] *= s;
}

// Eigenvectors of T for the r largest eigenvalues lam[0..r) (decreasing) by
// inverse iteration, then back-transformed x = Q y with the reflectors kept
// in A's rows.  Vectors are computed concurrently, one thread each; vectors
// whose eigenvalue lies within 1e-3 ||T|| of the previous one (a cluster) are
// then recomputed in order with modified Gram-Schmidt against the earlier
// members of their cluster at every iteration.  Output X (m x r, row-major).
// One workgroup; ws: 6*m*r + m*r doubles.
__global__ __launch_bounds__(kTriThreads) void k_tri_eigvecs(int32_t m, int32_t r, const double* __restrict__ d,
                                                             const double* __restrict__ e,
                                                             const double* __restrict__ lam,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ tau,
                                                             double* __restrict__ ws, double* __restrict__ X) {
  __shared__ double red[kWaves];
  const int t = threadIdx.x;
  double* Y = ws + (int64_t)6 * m * r;  // column c at Y + c*m
  double tn = 0.0;
  for (int32_t i = t; i < m; i += kTriThreads)
    tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0));
  for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_down(tn, off, 64));
  if ((t & 63) == 0) red[t >> 6] = tn;
  __syncthreads();
  tn = 0.0;
  for (int i = 0; i < kWaves; ++i) tn = fmax(tn, red[i]);
  __syncthreads();
  const double u = 2.220446049250313e-16;
  const double pert = fmax(u * tn, 1e-300);
  const double ortol = 1e-3 * tn;

  // phase 1: every vector on its own thread
  for (int32_t c = t; c < r; c += kTriThreads) {
    double* base = ws + (int64_t)6 * m * c;
    double *DL = base, *DD = base + m, *DU = base + 2 * m, *DU2 = base + 3 * m;
    int32_t* piv = (int32_t*)(base + 4 * m);
    double* y = base + 5 * m;
    tri_factor(m, d, e, lam[c], pert, DL, DD, DU, DU2, piv);
    for (int32_t i = 0; i < m; ++i) y[i] = 1.0 + 0.5 * sin(0.7 * i + 1.3 * c + 0.1);
    for (int it = 0; it < 3; ++it) tri_solve(m, DL, DD, DU, DU2, piv, y);
    double nn = 0.0;
    for (int32_t i = 0; i < m; ++i) nn = fma(y[i], y[i], nn);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int32_t i = 0; i < m; ++i) Y[(int64_t)c * m + i] = y[i] * inv;
  }
  __syncthreads();
  // phase 2: clustered vectors, in order, orthogonalised against their
  // predecessors in the cluster
  for (int32_t c = 1; c < r; ++c) {
    if (!(fabs(lam[c - 1] - lam[c]) <= ortol)) continue;
    double* base = ws + (int64_t)6 * m * c;
    double *DL = base, *DD = base + m, *DU = base + 2 * m, *DU2 = base + 3 * m;
    int32_t* piv = (int32_t*)(base + 4 * m);
    double* y = Y + (int64_t)c * m;
    for (int it = 0; it < 3; ++it) {
      if (t == 0) tri_solve(m, DL, DD, DU, DU2, piv, y);
      __syncthreads();
      for (int32_t b = c - 1; b >= 0 && fabs(lam[b] - lam[c]) <= ortol; --b) {
        const double* yb = Y + (int64_t)b * m;
        double dp = 0.0;
        for (int32_t i = t; i < m; i += kTriThreads) dp = fma(yb[i], y[i], dp);
        dp = block_sum(dp, red);
        for (int32_t i = t; i < m; i += kTriThreads) y[i] -= dp * yb[i];
        __syncthreads();
      }
      double nn = 0.0;
      for (int32_t i = t; i < m; i += kTriThreads) nn = fma(y[i], y[i], nn);
      nn = block_sum(nn, red);
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int32_t i = t; i < m; i += kTriThreads) y[i] *= inv;
      __syncthreads();
    }
  }
  // back-transformation x = H_0 H_1 ... H_{m-3} y, one wave per column
  for (int32_t k = m - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const double* vk = A + (int64_t)k * m + (k + 1);  // v_k, length m-k-1, vk[0] = 1
    const int32_t L = m - k - 1;
    for (int32_t c = t >> 6; c < r; c += kWaves) {
      double* yc = Y + (int64_t)c * m + (k + 1);
      double acc = 0.0;
      for (int32_t i = t & 63; i < L; i += 64) acc = fma(vk[i], yc[i], acc);
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      const double f = tk * acc;
      for (int32_t i = t & 63; i < L; i += 64) yc[i] -= f * vk[i];
    }
    __syncthreads();
  }
  for (int32_t i = t >> 6; i < m; i += kWaves)
    for (int32_t c = t & 63; c < r; c += 64) X[(int64_t)i * r + c] = Y[(int64_t)c * m + i];
}

}  // namespace

int32_t sym_tri_lds_max() { return kTriLdsMax; }

hipError_t sym_eigvals(hipStream_t st, int32_t m, double* A, double* d, double* e, double* tau, double* vp,
                       double* w) {
  if (m <= 0) return hipSuccess;
  if (m <= kTriLdsMax) {
    const size_t lds = ((size_t)m * (m + 1) + 4 * (size_t)m) * sizeof(double);
    static bool attr = false;
    if (!attr) {
      hipError_t er = hipFuncSetAttribute((const void*)k_tridiag_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)(((size_t)kTriLdsMax * (kTriLdsMax + 1) + 4 * kTriLdsMax) *
                                                sizeof(double)));
      if (er != hipSuccess) return er;
      attr = true;
    }
    hipLaunchKernelGGL(k_tridiag_lds, dim3(1), dim3(kTriThreads), lds, st, m, A, d, e, tau);
  } else {
    hipLaunchKernelGGL(k_tridiag_global, dim3(1), dim3(kTriThreads), (size_t)4 * m * sizeof(double), st, m, A,
                       d, e, tau);
  }
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return er;
  hipLaunchKernelGGL(k_bisect, dim3((m + (256 / kSect) - 1) / (256 / kSect)), dim3(256), 0, st, m, d, e, w);
  return hipGetLastError();
}

hipError_t sym_eigvecs(hipStream_t st, int32_t m, int32_t r, const double* d, const double* e,
                       const double* lam, const double* A, const double* tau, double* ws, double* X) {
  if (m <= 0 || r <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_eigvecs, dim3(1), dim3(kTriThreads), 0, st, m, r, d, e, lam, A, tau, ws, X);
  return hipGetLastError();
}

}  // namespace ttice
