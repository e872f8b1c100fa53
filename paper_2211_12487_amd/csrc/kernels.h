// Internal interface between the TT-ICE host engine and its gfx950 kernels.
// Not part of the public ABI (include/ttice.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttice {

constexpr int32_t kUnframed = 0x7fffffff;

// A strided view of a matrix whose row and/or column index may be split into
// "frames": element (i, j) lives at
//   base + row_off(i) + col_off(j),
//   row_off(i) = (i / rpf) * rfs + (i % rpf) * rs,
//   col_off(j) = (cfidx ? cfidx[j / cpf] : j / cpf) * cfs + (j % cpf) * cs.
// A batch of N frame-major matrices Z[b] (rows x cols, row-major, frame
// stride fs) seen as the unfolding [Z[0] Z[1] ... Z[N-1]] (rows x N*cols) is
// {rpf=unframed, rs=cols, cpf=cols, cfs=fs, cs=1}.  cfidx optionally
// renumbers column frames (a gathered subset of the batch, read in place).
struct View {
  int32_t rpf = kUnframed;
  int32_t cpf = kUnframed;
  int64_t rfs = 0, rs = 0;
  int64_t cfs = 0, cs = 0;
  const int32_t* cfidx = nullptr;
};

inline View row_major(int64_t ld) {
  View v;
  v.rs = ld;
  v.cs = 1;
  return v;
}
inline View transposed(View v) {
  View t;
  t.rpf = v.cpf;
  t.rfs = v.cfs;
  t.rs = v.cs;
  t.cpf = v.rpf;
  t.cfs = v.rfs;
  t.cs = v.rs;
  t.cfidx = v.cfidx;
  return t;
}
// [Z[0] ... Z[N-1]] for frame-major data, rows x (N*cols)
inline View unfolding(int64_t cols, int64_t fs, const int32_t* fidx = nullptr) {
  View v;
  v.rs = cols;
  v.cpf = (int32_t)cols;
  v.cfs = fs;
  v.cs = 1;
  v.cfidx = fidx;
  return v;
}

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

// Fused one-pass projection of narrow cores (r <= 64, FP64 matrix cores):
// for every column j of Z (rows x Ncol view, rows unframed), C(:, j) =
// U^T z_j (view vc, rows unframed), znorm2[j] = ||z_j||^2 and rho2[j] =
// ||z_j||^2 - ||C(:, j)||^2 (FP64).  Any output may be null.  U is read
// kProjTail doubles wide from the start of each of its rows, so its
// allocation must extend at least kProjTail doubles past row (rows - 1)'s
// start (the values there are never used).
constexpr int kProjTail = 64;
bool proj_fits(int32_t rows, int32_t r);
// prec selects the product's arithmetic (kProj*): FP64 matrix cores; FP32
// matrix cores with FP32 accumulation; or split-BF16, each FP32 operand as a
// hi + lo pair of bf16 and the three products hi*hi + hi*lo + lo*hi on BF16
// matrix cores with FP32 accumulation.  ||z||^2 and the residual energy are
// FP64 in every mode.  With ev_start/ev_stop given, the launch carries them
// as its own start and end timestamps (the dispatch packet's, so they time
// the kernel alone).
constexpr int kProjFP64 = 0, kProjFP32 = 1, kProjBF16x3 = 2;
// vmax caps the columns per lane (1, 2 or 4; the widest the alignment allows
// up to vmax is taken).  *rho_explicit (if given) tells whether rho2 was
// formed explicitly, ||z - U c~||^2 in FP64 from the rounded coefficients
// (the short-column kernel), rather than by Pythagoras.
template <typename TIn>
hipError_t proj_columns(hipStream_t st, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z, View vz,
                        const double* U, int64_t ldu, double* C, View vc, double* znorm2, double* rho2,
                        int prec = kProjFP64, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                        int vmax = 4, bool* rho_explicit = nullptr);

// The short-column form behind proj_columns (at most kShortRows rows and
// core columns, FP64 or FP32 arithmetic, four aligned columns per thread):
// a vector-ALU stream of the input and outputs, for unfoldings too short
// for a matrix-core tile.
constexpr int kShortRows = 8;
bool proj_short_fits(int prec, int32_t rows, int32_t r);
template <typename TIn>
hipError_t proj_columns_short(hipStream_t st, int prec, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z,
                              View vz, const double* U, int64_t ldu, double* C, View vc, double* znorm2,
                              double* rho2, hipEvent_t ev_start, hipEvent_t ev_stop);

// Several independent projections (one per stream of a server) in one
// launch: descriptor q is proj_columns' arguments for one column per lane,
// and its column blocks are blocks start[q] .. start[q + 1] - 1 of the grid.
// Every descriptor of a group shares the input type, the arithmetic and the
// launch shape (proj_shape), so each block computes bit for bit what the
// same block of that projection's own launch (vmax = 1) computes.
struct ProjDesc {
  int32_t rows = 0, r = 0, Ncol = 0;
  View vz, vc;
  const void* Z = nullptr;
  const double* U = nullptr;
  int64_t ldu = 0;
  double* C = nullptr;
  double* znorm2 = nullptr;
  double* rho2 = nullptr;
};
constexpr int kGroupMax = 16;  // descriptors per launch (kernel arguments stay under 4 KB)
struct ProjGroup {
  int32_t n = 0;
  int32_t start[kGroupMax + 1] = {};
  ProjDesc d[kGroupMax];
};
// Launch shape of a projection with one column per lane, 8 * (waves per
// block) + (16-wide column tiles of U): equal for two projections exactly
// when they can share a grouped launch (given the same input type and prec).
int32_t proj_shape(int prec, int32_t rows, int32_t r);
template <typename TIn>
hipError_t proj_group(hipStream_t st, int prec, const ProjGroup& g);
template <typename TIn>
hipError_t proj_group_lp(hipStream_t st, int prec, const ProjGroup& g);
// The reduced-precision launches behind proj_columns (vec = columns per lane,
// already checked for alignment).
template <typename TIn>
hipError_t proj_columns_lp(hipStream_t st, int prec, int vec, int32_t rows, int32_t r, int32_t Ncol, const TIn* Z,
                           View vz, const double* U, int64_t ldu, double* C, View vc, double* znorm2,
                           double* rho2, hipEvent_t ev_start, hipEvent_t ev_stop);

// Scratch the product may use to split a long K-sum across workgroups.
// Workspace of K-split products: partial products (len doubles) and one
// arrival counter per output tile (ncnt of them, zero between products).
struct GemmWs {
  double* p = nullptr;
  int64_t len = 0;  // doubles
  int* cnt = nullptr;
  int32_t ncnt = 0;
};

// D = alpha * A * B + beta * E over an M x N output, K-sum split into
// ceil(K / kchunk) slices along grid z (slice z writes D + z*dz).  A is FP64.
// Optional outputs: colpart[mb*N + n] = sum over the rows of output tile mb of
// D(m, n)^2 (FP64), bnorm[n] = sum_k B(k, n)^2 (only with one K slice).
// Any of E / D / colpart / bnorm may be null.  When one K slice is asked
// for (kchunk >= K), the output has few tiles and K is long, the product is
// split over K into partial sums in ws (if given and large enough) and
// finished by a second kernel that applies alpha, beta*E and colpart; the
// result does not depend on the split (fixed summation order per split).
// prec (kProj*): the arithmetic of large products that fit gemm_mx; every
// other product is FP64.
template <typename TB, typename TE, typename TD>
hipError_t gemm(hipStream_t st, int32_t M, int32_t N, int32_t K, int32_t kchunk, double alpha,
                const double* A, View va, const TB* B, View vb, double beta, const TE* E, View ve,
                TD* D, View vd, int64_t dz, double* colpart, double* bnorm, GemmWs ws = GemmWs(),
                int prec = 0);

inline int32_t gemm_row_blocks(int32_t M) { return M > 0 ? (M + 63) / 64 : 1; }

// The matrix-core tiled product (gemm_mx.h) that gemm() takes for large
// level contractions: FP64 (prec kProjFP64), FP32 (kProjFP32) or split
// BF16 (kProjBF16x3).
// gemm_mx_fits: the shape and views it supports without a K split.
bool gemm_mx_fits(int32_t M, int32_t N, int32_t K, const View& va, const View& vb, const View& ve, const View& vd,
                  bool has_e, bool has_d, bool bnorm);
// Products with too few output tiles to fill the device unsplit and a long
// K: the number of K slices gemm() gives the FP64 matrix-core kernel (0:
// none), at most what ws_len doubles of partials hold; and the launch that
// writes slice z's partial product to part + z M N (row-major).
int32_t gemm_mx_split_slices(int32_t M, int32_t N, int32_t K, const View& va, const View& vb, int64_t ws_len);
template <typename TB>
hipError_t gemm_mx64_part(hipStream_t st, int32_t M, int32_t N, int32_t K, int32_t S, int32_t kchunk,
                          const double* A, View va, const TB* B, View vb, double* part);
template <typename TB, typename TE, typename TD>
hipError_t gemm_mx(hipStream_t st, int prec, int32_t M, int32_t N, int32_t K, double alpha, const double* A,
                   View va, const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd,
                   double* colpart);
template <typename TB, typename TE, typename TD>
hipError_t gemm_mx_bf3(hipStream_t st, int32_t M, int32_t N, int32_t K, double alpha, const double* A, View va,
                       const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd, double* colpart);
template <typename TB, typename TE, typename TD>
hipError_t gemm_mx_f32(hipStream_t st, int32_t M, int32_t N, int32_t K, double alpha, const double* A, View va,
                       const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd, double* colpart);

// out[f] = sum_{mb<MB} sum_{c<cpf} part[mb*ld + f*cpf + c], f < F, in a
// fixed order.  scratch (F * kFrameSlicesMax doubles, or null: one block per
// frame) holds the sums of column slices of each frame.
constexpr int32_t kFrameSlicesMax = 64;
int32_t frame_sum_slices(int32_t cpf, int32_t F);
hipError_t frame_sums(hipStream_t st, const double* part, int32_t MB, int64_t ld, int32_t cpf,
                      int32_t F, double* out, double* scratch);
// out[0] = sum_{i<n} x[i] (deterministic order); out[1] = 1 if any x is not finite.
hipError_t total_sum(hipStream_t st, const double* x, int64_t n, double* out);
// out[0] = max |S(i, j) - [i == j]| over an n x n matrix (row stride ld),
// out[1] = 1 when an entry is not finite.  out may be a pinned host buffer.
hipError_t max_off_identity(hipStream_t st, int32_t n, const double* S, int32_t ld, double* out);
// out[j] = sum_k X[j ld + k]^2 over the ncol entries of each of the n rows
// (fixed order).
hipError_t row_sumsq(hipStream_t st, int32_t n, int32_t ncol, int64_t ld, const double* X, double* out);
// The rank (at least 1, at most n) from the tails t(r) = perp[0] +
// sum_{j>=r} e[j] of n directions: res[0] = the smallest r with t(r) <=
// tol2 (n when none), res[1] = t(res[0]), res[2] = the decision's margin
// (relative distance of t(r) and t(r-1) from tol2), res[3] = 1 when a value
// is not finite (perp[1], total_sum's flag, counts too).  res may be a pinned
// host buffer.
hipError_t tail_rank(hipStream_t st, int32_t n, const double* e, const double* perp, double tol2, double* res);
// err2[b] = max(0, y2[b] - ||c(b, 0:r)||^2) for N frames (c row b at ld):
// the chain's residual energy by the telescoping identity (FP64 path)
hipError_t telescope(hipStream_t st, int32_t N, int32_t r, const double* c, int64_t ld, const double* y2,
                     double* err2);
// acc[i] += x[i]
hipError_t accumulate(hipStream_t st, double* acc, const double* x, int64_t n);

// G (m x m, ld = m) = sum over S slices of the upper triangle of part
// (slice stride m*m), mirrored to be exactly symmetric.
hipError_t gram_reduce(hipStream_t st, const double* part, int32_t S, int32_t m, double* G);

// Rank selection for SVD(R, eps) from the eigenvalues w (m) of the residual's
// Gram matrix (eq:deltasvd / eq:svdfirst): order[t] = index of the t-th
// largest eigenvalue, lam[t] its value clamped to >= 0; tail[r] =
// sum_{t>=r} lam[t] (+ the remainder below, m + 1 entries); r_R = smallest r with tail[r] <= tol2,
// clipped to cap.  res[0] = r_R, res[1] = tail[r_R], res[2] = margin,
// res[3] = 1 if any eigenvalue was not finite.  cnt: one int of device
// memory that is zero on entry and is left zero (the arrival counter of the
// eigenvalue workgroups).
struct RankSelect {
  int* cnt = nullptr;
  double tol2 = 0.0;
  int64_t cap = 0;
  int32_t* order = nullptr;
  double* lam = nullptr;
  double* tail = nullptr;
  double* res = nullptr;
  // optional: the trace of the Gram matrix when the m eigenvalues are those
  // of a projection of it (Ritz values); every tail then includes trace -
  // sum of the m values (clamped at 0)
  const double* trace = nullptr;
};

// Eigenvalues of the symmetric m x m matrix A (row-major, ld = m, m <=
// sym_eig_max()): A is reduced in place to tridiagonal form T = Q^T A Q (d, e;
// reflectors kept in A's rows and tau; d, e, tau: m doubles each) and w
// receives all eigenvalues in decreasing order.
// ws: sym_eig_ws(m) doubles of device workspace, or null (then every
// reflection runs in one workgroup).  sel (optional, m >= 1): the rank
// selection above, run by the last eigenvalue workgroup to finish.
hipError_t sym_eigvals(hipStream_t st, int32_t m, double* A, double* d, double* e, double* tau, double* w,
                       double* ws, const RankSelect* sel = nullptr);
inline int64_t sym_eig_ws(int32_t m) { return 4 * (int64_t)m + 512; }
int64_t sym_eigvecs_ws(int32_t m, int32_t r);
// Eigenvectors of A for its r largest eigenvalues lam[0..r) (from
// sym_eigvals, decreasing): X (m x r, row-major).  ws: sym_eigvecs_ws(m, r)
// doubles.  For m > 256 the reflectors are applied in blocks on the tiled
// products (K split through gws when given), and A's diagonal and the
// entries left of it in each row (not needed by then) are zeroed.
hipError_t sym_eigvecs(hipStream_t st, int32_t m, int32_t r, const double* d, const double* e,
                       const double* lam, double* A, const double* tau, double* ws, double* X,
                       GemmWs gws = GemmWs());
int32_t sym_eig_max();

// (order null: the identity)
// W (rows x r, ld = r) = V[:, order[t]] (left case)  or
// Vs (M x r, ld = r) = V[:, order[t]] / sqrt(lam[t]) (right case, scale = true)
hipError_t gather_columns(hipStream_t st, int32_t rows, int32_t r, const double* V, int32_t ldv,
                          const int32_t* order, const double* lam, bool scale, double* W);
// dst(:, t) = s_t W(:, t) for the r columns of W (rows x r, ld = r), s_t = +-1
// making the column's largest-|.| entry (lowest row index on ties)
// positive; in the same launch, zero the zrows x zcols region at zdst (ld
// zld; none when zdst is null).
hipError_t sign_place(hipStream_t st, int32_t rows, int32_t r, const double* W, double* dst, int64_t ldd,
                      double* zdst, int64_t zrows, int64_t zcols, int64_t zld);
// dst(i, j) = 0 for i < rows, j < cols
hipError_t zero2d(hipStream_t st, int64_t rows, int64_t cols, double* dst, int64_t ldd);

// Algorithm 2 decision from per-frame squared errors e2[b] (old cores) and
// norms y2[b]: res[0] = mean relative error, res[1] = batch relative error,
// res[2] = sum e2 over D_C (frames with rel <= eps), res[3] = ||D||^2,
// res[4] = |D|, res[5] = ||Y||^2, res[6] = the smallest relative distance
// |x / eps - 1| of the mean, the batch and every frame's relative error x;
// dlist = indices of D in increasing order.
hipError_t star_decide(hipStream_t st, int32_t N, const double* e2, const double* y2, double eps,
                       int32_t* dlist, double* res);

// ---- pieces of the block-Lanczos truncated SVD (lanczos.hip)
// Q(i, j) = a fixed pseudo-random value in [-1, 1) for i < m, j < b (ld).
hipError_t rand_fill(hipStream_t st, int64_t m, int32_t b, double* Q, int64_t ld, uint64_t seed);
// Li = L^{-T} (b x b, ld ldl) for the Cholesky factor L of S = V^T V (b x b,
// ld lds, b <= lz_max_block()), so V Li has orthonormal columns; a column
// that depends on the earlier ones to working precision, or (Spre given: the
// Gram block before orthogonalisation against earlier blocks, ld ldpre)
// kept too little of its length, gets a zero column.
int32_t lz_max_block();
hipError_t chol_inv(hipStream_t st, int32_t b, const double* S, int32_t lds, const double* Spre, int32_t ldpre,
                    double* Li, int32_t ldl);
// T = (T + T^T) / 2 (n x n, ld)
hipError_t symmetrize(hipStream_t st, int32_t n, double* T, int32_t ld);
// *out = sum_{i<n} x[i]^2 in a fixed order; part: sumsq_parts(n) doubles
int64_t sumsq_parts(int64_t n);
hipError_t sumsq(hipStream_t st, const double* x, int64_t n, double* part, double* out);
// eta2[j] = ||GX(:, j) - theta_j X(:, j)||^2 and theta_out[j] = theta_j for
// j < k (X, GX: m x k, ld); the outputs may be pinned host memory
hipError_t ritz_residuals(hipStream_t st, int32_t m, int32_t k, int32_t ld, const double* X, const double* GX,
                          const double* theta, double* eta2, double* theta_out);

}  // namespace ttice
