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
template <bool kLds>
__device__ void tridiag_run(int32_t m, double* A, int64_t ld, double* v, double* p, double* red,
                            double* sc, double* d, double* e, double* tau) {
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  for (int32_t k = 0; k + 2 < m; ++k) {
    const int32_t L = m - k - 1;
    double* row = A + (int64_t)k * ld + (k + 1);
    // x = A[k, k+1:], sigma = ||x[1:]||^2
    double s = 0.0;
    for (int32_t i = t; i < L; i += kTriThreads) {
      const double x = row[i];
      v[i] = x;
      if (i > 0) s = fma(x, x, s);
    }
    s = block_sum(s, red);
    if (t == 0) {
      const double alpha = v[0];
      double beta, tk, scale;
      if (s == 0.0) {
        tk = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      sc[0] = tk;
      sc[1] = beta;
      sc[2] = scale;
      d[k] = A[(int64_t)k * ld + k];
      e[k] = beta;
      tau[k] = tk;
    }
    __syncthreads();
    const double tk = sc[0], scale = sc[2];
    for (int32_t i = t; i < L; i += kTriThreads) {
      const double vi = (i == 0) ? 1.0 : v[i] * scale;
      v[i] = vi;
      row[i] = vi;  // keep v_k for the back-transformation
    }
    __syncthreads();
    if (tk == 0.0) continue;  // uniform: H_k = I, nothing to update
    // p = tau * A_sub v  (one wave per row, lanes across the row)
    double* sub = A + (int64_t)(k + 1) * ld + (k + 1);
    for (int32_t i = wid; i < L; i += kWaves) {
      const double* ri = sub + (int64_t)i * ld;
      double acc = 0.0;
      for (int32_t j = lane; j < L; j += 64) acc = fma(ri[j], v[j], acc);
      acc = wave_sum(acc);
      if (lane == 0) p[i] = tk * acc;
    }
    __syncthreads();
    // w = p - (tau/2) (p.v) v
    double pv = 0.0;
    for (int32_t i = t; i < L; i += kTriThreads) pv = fma(p[i], v[i], pv);
    pv = block_sum(pv, red);
    const double gam = 0.5 * tk * pv;
    for (int32_t i = t; i < L; i += kTriThreads) p[i] = p[i] - gam * v[i];
    __syncthreads();
    // A_sub -= v w^T + w v^T
    const int64_t LL = (int64_t)L * L;
    for (int64_t q = t; q < LL; q += kTriThreads) {
      const int32_t i = (int32_t)(q / L), j = (int32_t)(q - (int64_t)i * L);
      double* a = sub + (int64_t)i * ld + j;
      *a = *a - v[i] * p[j] - p[i] * v[j];
    }
    if (!kLds) __threadfence_block();
    __syncthreads();
  }
  if (t == 0) {
    if (m >= 2) {
      d[m - 2] = A[(int64_t)(m - 2) * ld + (m - 2)];
      e[m - 2] = A[(int64_t)(m - 2) * ld + (m - 1)];
      tau[m - 2] = 0.0;
    }
    d[m - 1] = A[(int64_t)(m - 1) * ld + (m - 1)];
    if (m >= 1) tau[m - 1] = 0.0;
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
  double* v = lds + (int64_t)m * ld;
  double* p = v + m;
  for (int64_t q = threadIdx.x; q < (int64_t)m * m; q += kTriThreads) {
    const int32_t i = (int32_t)(q / m), j = (int32_t)(q % m);
    As[i * ld + j] = A[q];
  }
  __syncthreads();
  tridiag_run<true>(m, As, ld, v, p, red, sc, d, e, tau);
  // write the reflectors back (upper part of each row)
  for (int64_t q = threadIdx.x; q < (int64_t)m * m; q += kTriThreads) {
    const int32_t i = (int32_t)(q / m), j = (int32_t)(q % m);
    A[q] = As[i * ld + j];
  }
}

__global__ __launch_bounds__(kTriThreads) void k_tridiag_global(int32_t m, double* __restrict__ A,
                                                                double* __restrict__ vp,
                                                                double* __restrict__ d, double* __restrict__ e,
                                                                double* __restrict__ tau) {
  __shared__ double red[kWaves];
  __shared__ double sc[4];
  tridiag_run<false>(m, A, m, vp, vp + m, red, sc, d, e, tau);
}

// w[j] = j-th largest eigenvalue of T, j < m (Gershgorin interval, then
// bisection on the Sturm count until the interval is at rounding level).
__global__ __launch_bounds__(256) void k_bisect(int32_t m, const double* __restrict__ d,
                                                const double* __restrict__ e, double* __restrict__ w) {
  __shared__ double s_lo, s_hi, s_pivmin;
  if (threadIdx.x == 0) {
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int32_t i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      if (i + 1 < m) emax = fmax(emax, e[i] * e[i]);
    }
    const double nrm = fmax(fabs(lo), fabs(hi));
    const double u = 2.220446049250313e-16;
    lo -= 2.0 * u * nrm + 1e-300;
    hi += 2.0 * u * nrm + 1e-300;
    s_lo = lo;
    s_hi = hi;
    s_pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
  }
  __syncthreads();
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int32_t target = m - 1 - j;  // we want the (target)-th smallest (0-based)
  double lo = s_lo, hi = s_hi;
  const double pivmin = s_pivmin;
  const double u = 2.220446049250313e-16;
  const double atol = u * fmax(fabs(lo), fabs(hi));
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= 2.0 * u * fmax(fabs(lo), fabs(hi)) + atol || mid <= lo || mid >= hi) break;
    // count eigenvalues < mid
    int32_t c = 0;
    double q = d[0] - mid;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int32_t i = 1; i < m; ++i) {
      const double ei = e[i - 1];
      q = (d[i] - mid) - (ei * ei) / q;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
    if (c > target) hi = mid;
    else lo = mid;
  }
  w[j] = 0.5 * (lo + hi);
}

// Eigenvectors of T for the r largest eigenvalues lam[0..r) (decreasing),
// by inverse iteration (LU with partial pivoting of T - lam I, three
// iterations, re-orthogonalised against earlier vectors of the same cluster),
// then back-transformed x = Q y with the reflectors stored in A's rows.
// Output X (m x r, row-major, ld = r).  One workgroup; scratch in global:
// ws >= 8*m + m*r doubles.
__global__ __launch_bounds__(kTriThreads) void k_tri_eigvecs(int32_t m, int32_t r, const double* __restrict__ d,
                                                             const double* __restrict__ e,
                                                             const double* __restrict__ lam,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ tau,
                                                             double* __restrict__ ws, double* __restrict__ X) {
  __shared__ double red[kWaves];
  __shared__ double sc[4];
  const int t = threadIdx.x;
  double* DL = ws;
  double* DD = ws + m;
  double* DU = ws + 2 * m;
  double* DU2 = ws + 3 * m;
  int32_t* piv = (int32_t*)(ws + 4 * m);
  double* y = ws + 5 * m;          // current vector
  double* Y = ws + 8 * m;          // m x r, column t contiguous: Y[t*m + i]
  // norm of T for perturbations / cluster tolerance
  double tn = 0.0;
  for (int32_t i = t; i < m; i += kTriThreads) {
    const double a = fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    tn = fmax(tn, a);
  }
  // block max via sum of per-wave maxima is not a max; do a simple LDS max
  {
    for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_down(tn, off, 64));
    __syncthreads();
    if ((t & 63) == 0) red[t >> 6] = tn;
    __syncthreads();
    double mx = 0.0;
    for (int i = 0; i < kWaves; ++i) mx = fmax(mx, red[i]);
    tn = mx;
  }
  const double u = 2.220446049250313e-16;
  const double pert = fmax(u * tn, 1e-300);
  const double ortol = 1e-3 * tn;

  for (int32_t c = 0; c < r; ++c) {
    const double lc = lam[c];
    if (t == 0) {
      // LU of T - lc I with partial pivoting (tridiagonal, LAPACK gttrf order)
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
      // deterministic start vector
      for (int32_t i = 0; i < m; ++i) y[i] = 1.0 + 0.5 * sin(0.7 * i + 1.3 * c + 0.1);
    }
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (t == 0) {
        // solve (T - lc I) y_new = y
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
        sc[0] = mx > 0.0 ? 1.0 / mx : 1.0;
      }
      __syncthreads();
      const double sca = sc[0];
      for (int32_t i = t; i < m; i += kTriThreads) y[i] *= sca;
      __syncthreads();
      // re-orthogonalise against earlier vectors of the same cluster (MGS)
      for (int32_t b = c - 1; b >= 0 && fabs(lam[b] - lc) <= ortol; --b) {
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
    for (int32_t i = t; i < m; i += kTriThreads) Y[(int64_t)c * m + i] = y[i];
    __syncthreads();
  }
  // back-transformation x = H_0 H_1 ... H_{m-3} y for every column
  for (int32_t k = m - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const double* vk = A + (int64_t)k * m + (k + 1);  // v_k, length m-k-1, vk[0] = 1
    const int32_t L = m - k - 1;
    // one wave per column
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
  for (int64_t q = t; q < (int64_t)m * r; q += kTriThreads) {
    const int32_t i = (int32_t)(q / r), c = (int32_t)(q % r);
    X[q] = Y[(int64_t)c * m + i];
  }
}

}  // namespace

int32_t sym_tri_lds_max() { return kTriLdsMax; }

hipError_t sym_eigvals(hipStream_t st, int32_t m, double* A, double* d, double* e, double* tau, double* vp,
                       double* w) {
  if (m <= 0) return hipSuccess;
  if (m <= kTriLdsMax) {
    const size_t lds = ((size_t)m * (m + 1) + 2 * (size_t)m) * sizeof(double);
    static bool attr = false;
    if (!attr) {
      hipError_t er = hipFuncSetAttribute((const void*)k_tridiag_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)(((size_t)kTriLdsMax * (kTriLdsMax + 1) + 2 * kTriLdsMax) *
                                                sizeof(double)));
      if (er != hipSuccess) return er;
      attr = true;
    }
    hipLaunchKernelGGL(k_tridiag_lds, dim3(1), dim3(kTriThreads), lds, st, m, A, d, e, tau);
  } else {
    hipLaunchKernelGGL(k_tridiag_global, dim3(1), dim3(kTriThreads), 0, st, m, A, vp, d, e, tau);
  }
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return er;
  hipLaunchKernelGGL(k_bisect, dim3((m + 255) / 256), dim3(256), 0, st, m, d, e, w);
  return hipGetLastError();
}

hipError_t sym_eigvecs(hipStream_t st, int32_t m, int32_t r, const double* d, const double* e,
                       const double* lam, const double* A, const double* tau, double* ws, double* X) {
  if (m <= 0 || r <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_eigvecs, dim3(1), dim3(kTriThreads), 0, st, m, r, d, e, lam, A, tau, ws, X);
  return hipGetLastError();
}

}  // namespace ttice
