// Test-only entry point of the emulation build: the matrix-core tiled
// product (FP64 arithmetic) on host matrices, against NumPy in the tests.
#include <hip/hip_runtime.h>

#include "../../paper_2211_12487_amd/csrc/kernels.h"

// D = alpha A B + beta E with A (M x K) row-major (a_trans: A given as its
// transpose K x M row-major), B (K x N) seen as nf frames of N / nf columns
// (frame stride fs), E and D row-major M x N, colpart (M / 64 blocks) x N.
extern "C" int hipemu_gemm_mx(int M, int N, int K, double alpha, const double* A, int a_trans, const double* B,
                              int nf, long fs, double beta, const double* E, double* D, double* colpart) {
  ttice::View va = a_trans ? ttice::transposed(ttice::row_major(M)) : ttice::row_major(K);
  const int cpf = N / nf;
  ttice::View vb = ttice::unfolding(cpf, fs);
  ttice::View vd = ttice::row_major(N);
  return ttice::gemm_mx<double, double, double>(nullptr, 0, M, N, K, alpha, A, va, B, vb, beta, E, vd, D, vd,
                                                colpart) == hipSuccess
             ? 0
             : -1;
}

// The same through gemm() with a K-split workspace of ws_len doubles (the
// matrix-core split for products with few output tiles and a long K):
// A (M x K) row-major, B (K x N) row-major, E, D row-major M x N.
extern "C" int hipemu_gemm_ws(int M, int N, int K, double alpha, const double* A, const double* B, double beta,
                              const double* E, double* D, double* colpart, double* ws, long ws_len, int* cnt) {
  ttice::GemmWs g;
  g.p = ws;
  g.len = ws_len;
  g.cnt = cnt;
  g.ncnt = 256;
  const ttice::View va = ttice::row_major(K), vb = ttice::row_major(N), vd = ttice::row_major(N);
  return ttice::gemm<double, double, double>(nullptr, M, N, K, K, alpha, A, va, B, vb, beta, E, vd, D, vd, 0,
                                             colpart, nullptr, g) == hipSuccess
             ? 0
             : -1;
}

// the number of K slices gemm() gives such a product (0: unsplit)
extern "C" int hipemu_gemm_split_slices(int M, int N, int K, long ws_len) {
  return ttice::gemm_mx_split_slices(M, N, K, ttice::row_major(K), ttice::row_major(N), ws_len);
}
