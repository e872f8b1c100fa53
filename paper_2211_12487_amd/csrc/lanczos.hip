// Helpers of the truncated SVD of large residuals (eq:svdfirst) by block
// Lanczos: TT-ICE keeps only the leading r_R directions of a residual whose
// Gram matrix can be thousands wide, and the truncation rank needs only the
// leading eigenvalues (the discarded energy is the trace minus their sum).
// The engine builds an orthonormal block Krylov basis Q of the Gram matrix
// G (applied as R^T (R X) or R (R^T X), never formed) with the tiled
// products, and these kernels supply its small pieces: the deterministic
// start block, the Cholesky QR of each new block, the symmetrised projected
// matrix Q^T G Q, the trace of G, and the residual norms of the Ritz pairs
// that decide whether the result is accepted.
#include "kernels.h"

#include <math.h>

#include <algorithm>

namespace ttice {
namespace {

// A counter-based uniform value in [-1, 1) for entry (i, j) (splitmix64 of
// the entry's index and a seed): the start block is the same in every run.
__device__ __forceinline__ double hash_uniform(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_rand_fill(int64_t m, int32_t b, double* __restrict__ Q, int64_t ld, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * b) return;
  const int64_t i = e / b, j = e - i * b;
  Q[i * ld + j] = hash_uniform(seed * 0x100000001B3ull + (uint64_t)e);
}

// Cholesky S = L L^T of a b x b Gram block (b <= kLzMaxB) in LDS, then
// Li = L^{-T}, so that V Li has orthonormal columns when S = V^T V.  A
// column is dropped (its column of Li is zero, so the product's column is
// zero and the block loses that direction) when it depends on the earlier
// columns of the block to working precision (pivot at most kDepTol^2 times
// its diagonal entry), or, with Spre given (the Gram block of the columns
// before they were orthogonalised against earlier blocks), when
// orthogonalisation left less than kPreTol of its length: normalising such
// a remainder would magnify its rounding error into components along the
// earlier blocks.
// LDS (dynamic): A (b x (b+1)): S, then L in the lower triangle and L^{-1}
// transposed in the strict upper one; diag0, dinv (b each), dead (b ints).
constexpr int kLzMaxB = 128;
constexpr double kDepTol = 1e-13;
constexpr double kPreTol = 1e-7;

size_t chol_lds_bytes(int32_t b) { return ((size_t)b * (b + 1) + 3 * (size_t)b) * sizeof(double); }

__global__ __launch_bounds__(256) void k_chol_inv(int32_t b, const double* __restrict__ S, int32_t lds,
                                                  const double* __restrict__ Spre, int32_t ldpre,
                                                  double* __restrict__ Li, int32_t ldl) {
  HIP_DYNAMIC_SHARED(double, sh);
  const int32_t la = b + 1;
  double* A = sh;
  double* diag0 = sh + (int64_t)b * la;
  double* dinv = diag0 + b;
  int* dead = (int*)(dinv + b);
  const int t = threadIdx.x;
  for (int e = t; e < b * b; e += 256) {
    const int i = e / b, j = e - i * b;
    A[i * la + j] = S[(int64_t)i * lds + j];
  }
  __syncthreads();
  for (int i = t; i < b; i += 256) {
    diag0[i] = A[i * la + i];
    dead[i] = (Spre != nullptr && !(A[i * la + i] > kPreTol * kPreTol * Spre[(int64_t)i * ldpre + i])) ? 1 : 0;
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    if (t == 0) {
      const double dj = A[j * la + j];
      const bool dep = dead[j] || !(dj > kDepTol * kDepTol * diag0[j]) || !(dj > 0.0);
      dead[j] = dep ? 1 : 0;
      A[j * la + j] = dep ? 0.0 : sqrt(dj);
    }
    __syncthreads();
    const double piv = A[j * la + j];
    const bool dj = dead[j] != 0;
    for (int i = j + 1 + t; i < b; i += 256) A[i * la + j] = dj ? 0.0 : A[i * la + j] / piv;
    __syncthreads();
    const int n = b - j - 1;
    for (int e = t; e < n * n; e += 256) {
      const int i = j + 1 + e / n, k = j + 1 + e % n;
      if (k <= i) A[i * la + k] = fma(-A[i * la + j], A[k * la + j], A[i * la + k]);
    }
    __syncthreads();
  }
  // L^{-1} by forward substitution, one column c per thread: its diagonal
  // entry in dinv[c], the entries below in row c of A's upper triangle
  // (L itself stays in the lower triangle); dead indices give zeros
  for (int c = t; c < b; c += 256) {
    dinv[c] = dead[c] ? 0.0 : 1.0 / A[c * la + c];
    for (int i = c + 1; i < b; ++i) {
      double s = 0.0;
      if (!dead[i]) {
        // four partial sums (added in a fixed order) break the FMA chain
        double s0 = -A[i * la + c] * dinv[c], s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int k = c + 1;
        for (; k + 3 < i; k += 4) {
          s0 = fma(-A[i * la + k], A[c * la + k], s0);
          s1 = fma(-A[i * la + k + 1], A[c * la + k + 1], s1);
          s2 = fma(-A[i * la + k + 2], A[c * la + k + 2], s2);
          s3 = fma(-A[i * la + k + 3], A[c * la + k + 3], s3);
        }
        for (; k < i; ++k) s0 = fma(-A[i * la + k], A[c * la + k], s0);
        s = ((s0 + s1) + (s2 + s3)) / A[i * la + i];
      }
      A[c * la + i] = s;
    }
  }
  __syncthreads();
  // Li(k, c) = L^{-1}(c, k): zero below the diagonal
  for (int e = t; e < b * b; e += 256) {
    const int k = e / b, c = e - k * b;
    Li[(int64_t)k * ldl + c] = c > k ? A[k * la + c] : (c == k ? dinv[k] : 0.0);
  }
}

// T = (T + T^T) / 2 in place (n x n, ld)
__global__ void k_symmetrize(int32_t n, double* __restrict__ T, int32_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int32_t i = (int32_t)(e / n), j = (int32_t)(e - (int64_t)i * n);
  if (j <= i) return;
  const double a = T[(int64_t)i * ld + j], c = T[(int64_t)j * ld + i];
  const double s = 0.5 * (a + c);
  T[(int64_t)i * ld + j] = s;
  T[(int64_t)j * ld + i] = s;
}

__device__ double block_sum256(double v, double* red) {
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

// Deterministic sum of squares of x[0 .. n): block g sums the fixed chunk g
// into part[g] ...
__global__ __launch_bounds__(256) void k_sumsq_part(const double* __restrict__ x, int64_t n, int64_t chunk,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s = fma(x[i], x[i], s);
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ... and one block adds the G partials in order
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int32_t G,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int32_t g = threadIdx.x; g < G; g += 256) s += part[g];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) *out = s;
}

// eta2[j] = || GX(:, j) - theta_j X(:, j) ||^2 and theta_out[j] = theta_j,
// one block per column (m x k row-major operands, ld)
__global__ __launch_bounds__(256) void k_ritz_resid(int32_t m, int32_t ld, const double* __restrict__ X,
                                                    const double* __restrict__ GX, const double* __restrict__ theta,
                                                    double* __restrict__ eta2, double* __restrict__ theta_out) {
  __shared__ double red[256];
  const int32_t j = blockIdx.x;
  const double th = theta[j];
  double s = 0.0;
  for (int32_t i = threadIdx.x; i < m; i += 256) {
    const double r = fma(-th, X[(int64_t)i * ld + j], GX[(int64_t)i * ld + j]);
    s = fma(r, r, s);
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) {
    eta2[j] = s;
    theta_out[j] = th;
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int32_t lz_max_block() { return kLzMaxB; }

hipError_t rand_fill(hipStream_t st, int64_t m, int32_t b, double* Q, int64_t ld, uint64_t seed) {
  if (m * b <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rand_fill, dim3(nblk(m * b, 256)), dim3(256), 0, st, m, b, Q, ld, seed);
  return hipGetLastError();
}

hipError_t chol_inv(hipStream_t st, int32_t b, const double* S, int32_t lds, const double* Spre, int32_t ldpre,
                    double* Li, int32_t ldl) {
  if (b <= 0) return hipSuccess;
  if (b > kLzMaxB) return hipErrorInvalidValue;
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_chol_inv,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)chol_lds_bytes(kLzMaxB));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), chol_lds_bytes(b), st, b, S, lds, Spre, ldpre, Li, ldl);
  return hipGetLastError();
}

hipError_t symmetrize(hipStream_t st, int32_t n, double* T, int32_t ld) {
  if (n <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_symmetrize, dim3(nblk((int64_t)n * n, 256)), dim3(256), 0, st, n, T, ld);
  return hipGetLastError();
}

int64_t sumsq_parts(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(1024, (n + 8191) / 8192)); }

hipError_t sumsq(hipStream_t st, const double* x, int64_t n, double* part, double* out) {
  const int64_t G = sumsq_parts(n);
  const int64_t chunk = (n + G - 1) / G;
  hipLaunchKernelGGL(k_sumsq_part, dim3((unsigned)G), dim3(256), 0, st, x, n, std::max<int64_t>(chunk, 1), part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, part, (int32_t)G, out);
  return hipGetLastError();
}

hipError_t ritz_residuals(hipStream_t st, int32_t m, int32_t k, int32_t ld, const double* X, const double* GX,
                          const double* theta, double* eta2, double* theta_out) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ritz_resid, dim3(k), dim3(256), 0, st, m, ld, X, GX, theta, eta2, theta_out);
  return hipGetLastError();
}

}  // namespace ttice
