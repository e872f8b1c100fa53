// TT-ICE host engine and C ABI (include/ttice.h).
//
// The engine sequences the gfx950 kernels of kernels.hip through Algorithm 1
// (TT-ICE) and Algorithm 2 (TT-ICE*) of arXiv 2211.12487.  Decisions that
// shape later launches (is a core updated, how many directions are appended)
// come back to the host as a few FP64 scalars per core.
//
// Device layout
//   core U_i (i = 0..d-1): row-major FP64, (r_{i-1} n_i) rows x r_i columns,
//     leading dimension ld >= r_i, row capacity >= rows; rows beyond the
//     committed ones are scratch.  Zero padding (eq:ukpad) appends rows.
//   last core: stored transposed, row j = latent vector of stored tensor j
//     (N_total x r_d, ld >= r_d).  Padding the last core's rows with zeros
//     (eq:lastcore) zero-fills new entries of the old rows.
//   level data Z_i: frame-major [N][rows_i][cols_i], frame stride prod(dims);
//     the C-order reshape of eq:project_further is free in this layout.
#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <vector>

#include "../../include/ttice.h"
#include "kernels.h"
#include "serve.h"

using namespace ttice;

namespace {

// internal results of a capturing update (never returned by the C ABI)
constexpr int kL1Captured = 1000, kL1Plain = 1001;

// Projections that may share a grouped launch have equal keys: the launch
// shape, the arithmetic and the input type.
int32_t serve_key(int prec, int32_t rows, int32_t r, bool f32) {
  return (proj_shape(prec, rows, r) * 3 + prec) * 2 + (f32 ? 1 : 0);
}

bool same_view(const View& a, const View& b) {
  return a.rpf == b.rpf && a.cpf == b.cpf && a.rfs == b.rfs && a.rs == b.rs && a.cfs == b.cfs && a.cs == b.cs &&
         a.cfidx == b.cfidx;
}
bool same_desc(const ProjDesc& a, const ProjDesc& b) {
  return a.rows == b.rows && a.r == b.r && a.Ncol == b.Ncol && same_view(a.vz, b.vz) && same_view(a.vc, b.vc) &&
         a.Z == b.Z && a.U == b.U && a.ldu == b.ldu && a.C == b.C && a.znorm2 == b.znorm2 && a.rho2 == b.rho2;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// A core is allocated kProjTail doubles longer than cap_rows x ld, the
// over-read the fused projection kernel does past its last row.
struct Core {
  double* p = nullptr;
  int64_t cap_rows = 0;
  int64_t ld = 0;
  // capacity growth stops at these (the core's rank bounds, when known)
  int64_t max_rows = std::numeric_limits<int64_t>::max();
  int64_t max_cols = std::numeric_limits<int64_t>::max();
};

int status_of(hipError_t e) {
  if (e == hipSuccess) return TTICE_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return TTICE_ENOMEM;
  return TTICE_EDEVICE;
}

#define CK(expr)                                  \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return status_of(e_);   \
  } while (0)

#define CKS(expr)                      \
  do {                                 \
    int s_ = (expr);                   \
    if (s_ != TTICE_OK) return s_;     \
  } while (0)

// grow-only scratch (contents not preserved); the old buffer is freed once
// the work queued on st (the only stream that uses it) has finished
int ensure_on(DevBuf& b, size_t bytes, hipStream_t st) {
  if (bytes <= b.bytes && b.p) return TTICE_OK;
  size_t nb = std::max(bytes, b.bytes + b.bytes / 2);
  nb = std::max<size_t>(nb, 256);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return TTICE_ENOMEM;
  }
  if (b.p) {
    (void)hipStreamSynchronize(st);  // the old buffer may still be read by queued work
    (void)hipFree(b.p);
  }
  b.p = p;
  b.bytes = nb;
  return TTICE_OK;
}

template <typename T>
T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}

// arrival counters of K-split products (one per output tile; such products
// have fewer than 96 tiles)
constexpr int32_t kTileCounters = 128;

}  // namespace

struct ttice_state {
  int32_t d = 0;
  int64_t dims[TTICE_MAX_D] = {};
  int64_t P = 1;  // prod(dims)
  double eps = 0.0;
  int32_t prec = TTICE_PREC_FP64;
  int32_t algo = TTICE_ALG_PLAIN;
  int32_t skip_rule = TTICE_SKIP_MEAN;
  double tau = 1.0;
  hipStream_t stream = nullptr;
  int device = 0;

  Core U[TTICE_MAX_D];
  Core Gt;  // last core, transposed (frames x r_d)
  int64_t rk[TTICE_MAX_D + 1] = {};  // rk[0] = 1, rk[i] = r_i (committed)
  int64_t n_total = 0;

  // workspace
  DevBuf z[2], rbuf, colpart, bnorm, fres, fy2, e2acc, scal, gpart, gram, tri, order, lam, tail, W, W2, T,
      S, dlist, eigws, splitk, tilecnt;
  double* hs = nullptr;  // pinned host scalars (64 doubles), written by the decision kernels

  // kernel profiling (TTICE_OPT_PROFILE): event pairs recorded during one
  // update and resolved when it has completed
  bool profile = false;
  bool in_update = false;  // an update is running (its chain projections are profiled too)
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  std::vector<double> ev_bytes;
  struct ttice_kernel_stats kstats[1] = {};
  int prof_begin(hipEvent_t* a, hipEvent_t* b);
  int prof_resolve();

  ~ttice_state();

  int64_t cols(int i) const {  // columns per tensor at level i
    int64_t c = 1;
    for (int j = i + 1; j < d; ++j) c *= dims[j];
    return c;
  }
  int grow_core(Core& c, int64_t need_rows, int64_t need_cols, int64_t keep_rows, int64_t keep_cols);
  int ensure(DevBuf& b, size_t bytes) { return ensure_on(b, bytes, stream); }
  // scratch for K-split products (allocated once per state)
  // K-split products' workspace: partials, and arrival counters that start
  // at zero and are left at zero by every product
  int gemm_ws() {
    CKS(ensure(splitk, (size_t)kSplitKDoubles * sizeof(double)));
    if (!tilecnt.p) {
      CKS(ensure(tilecnt, kTileCounters * sizeof(int)));
      CK(hipMemsetAsync(tilecnt.p, 0, kTileCounters * sizeof(int), stream));
    }
    return TTICE_OK;
  }
  GemmWs gws() {
    return GemmWs{as<double>(splitk), (int64_t)(splitk.bytes / sizeof(double)), as<int>(tilecnt), kTileCounters};
  }
  int sync_scalars(int n);
  // truncated SVD of the residual R (rows x Ncol, view vR, in rbuf): r_R,
  // its discarded energy and decision margin, and for r_R > 0 the U_R
  // candidates in W (rows x r_R, ld r_R) before re-orthogonalisation
  int dense_svd(int64_t rows, int64_t Ncol, const View& vR, bool left, double tol2, int64_t cap, int64_t* rR,
                double* tail2, double* margin);
  int lanczos_svd(int level, int32_t b, int64_t rows, int64_t Ncol, const View& vR, bool left, double tol2, int64_t cap,
                  int64_t* rR, double* tail2, double* margin, bool* ok);
  int32_t lz_mode = 1;                       // 1: block Lanczos for wide Gram matrices, 0: dense only
  int64_t last_rR[TTICE_MAX_D] = {};          // last r_R decided per core (solver choice)
  int64_t lz_tries = 0, lz_accepted = 0;      // block-Lanczos SVDs attempted / certified
  double* hl = nullptr;                       // pinned host copy of Ritz values and residuals
  DevBuf lzw;
  // slice sums of frame_sums (null when it cannot be allocated: one block
  // per frame then)
  DevBuf fsl;
  double* fscratch(int64_t N) {
    return ensure(fsl, (size_t)N * kFrameSlicesMax * sizeof(double)) == TTICE_OK ? as<double>(fsl) : nullptr;
  }
  // Serving (server.hip): a served state's level 1 (Algorithm 1) always
  // takes the fused projection with one column per lane, the form a grouped
  // launch over several streams computes bit for bit.  l1_mode 1 stops an
  // update just before that launch and records its arguments in l1_desc
  // (kL1Captured), or stops before any level-1 work when the launch does not
  // apply (kL1Plain); l1_mode 2 runs an update whose level-1 launch has
  // already been made from l1_desc.
  bool served = false;
  int l1_mode = 0;
  ProjDesc l1_desc;
  int32_t l1_key = -1;
  template <typename TIn>
  int core_loop(const TIn* zin0, int64_t N, const int32_t* fidx, double tol_in, int64_t* rk_pend,
                ttice_update_info* info, bool use_occ, double* last_out, int64_t last_ld);
  // Buffers of chain_project given by the caller instead of the state's
  // grow-on-demand workspace (the allocation-free projection)
  struct ChainWs {
    double* z[2];      // level data, N * P doubles each
    double* bnorm;     // N * cols(0)
    double* colpart;   // max over levels of row blocks x columns
    double* fres;      // N
    double* fsl;       // N * kFrameSlicesMax
    double* y2;        // N
    GemmWs g;
  };
  // pp (kProj*): arithmetic of the level products
  template <typename TIn>
  int chain_project(const TIn* zin0, int64_t N, const int64_t* rks, double* coef_out, int64_t coef_ld,
                    double* err2_out, double* y2_out, int* nonfinite, const ChainWs* cw, int pp);
  int proj_prec() const {
    return prec == TTICE_PREC_FP32 ? kProjFP32 : prec == TTICE_PREC_BF16X3 ? kProjBF16x3 : kProjFP64;
  }
  template <typename TIn>
  int update_impl(const TIn* batch, int64_t N, ttice_update_info* info);
  template <typename TD>
  int reconstruct_impl(int64_t first, int64_t count, TD* out);
};

int ttice_state::prof_begin(hipEvent_t* a, hipEvent_t* b) {
  while ((int)ev_pool.size() < ev_used + 2) {
    hipEvent_t e;
    CK(hipEventCreate(&e));
    ev_pool.push_back(e);
  }
  *a = ev_pool[ev_used];
  *b = ev_pool[ev_used + 1];
  ev_used += 2;
  return TTICE_OK;
}

int ttice_state::prof_resolve() {
  for (int k = 0; k + 1 < ev_used; k += 2) {
    float ms = 0.0f;
    CK(hipEventSynchronize(ev_pool[k + 1]));
    CK(hipEventElapsedTime(&ms, ev_pool[k], ev_pool[k + 1]));
    kstats[0].launches += 1;
    kstats[0].total_ms += ms;
    kstats[0].bytes += ev_bytes[k / 2];
  }
  ev_used = 0;
  ev_bytes.clear();
  return TTICE_OK;
}

ttice_state::~ttice_state() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < TTICE_MAX_D; ++i)
    if (U[i].p) (void)hipFree(U[i].p);
  if (Gt.p) (void)hipFree(Gt.p);
  DevBuf* bufs[] = {&z[0], &z[1], &rbuf, &colpart, &bnorm, &fres, &fy2, &e2acc, &scal, &gpart, &gram,
                    &tri, &order, &lam, &tail, &W, &W2, &T, &S, &dlist, &eigws, &splitk, &tilecnt, &lzw, &fsl};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (hs) (void)hipHostFree(hs);
  if (hl) (void)hipHostFree(hl);
}

// Reallocate core storage to at least need_rows x need_cols, preserving the
// keep_rows x keep_cols leading block.
int ttice_state::grow_core(Core& c, int64_t need_rows, int64_t need_cols, int64_t keep_rows,
                           int64_t keep_cols) {
  if (need_rows <= c.cap_rows && need_cols <= c.ld && c.p) return TTICE_OK;
  int64_t nr = std::max<int64_t>(need_rows, c.cap_rows);
  if (need_rows > c.cap_rows) nr = std::max<int64_t>(need_rows, 2 * c.cap_rows);
  int64_t nl = std::max<int64_t>(need_cols, c.ld);
  if (need_cols > c.ld) nl = std::max<int64_t>(need_cols, 2 * c.ld);
  nr = std::min<int64_t>(nr, std::max<int64_t>(need_rows, c.max_rows));
  nl = std::min<int64_t>(nl, std::max<int64_t>(need_cols, c.max_cols));
  nr = std::max<int64_t>(nr, 1);
  nl = std::max<int64_t>(nl, 1);
  double* p = nullptr;
  hipError_t e = hipMalloc(&p, ((size_t)nr * nl + kProjTail) * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return TTICE_ENOMEM;
  }
  if (c.p && keep_rows > 0 && keep_cols > 0) {
    e = hipMemcpy2DAsync(p, nl * sizeof(double), c.p, c.ld * sizeof(double), keep_cols * sizeof(double),
                         keep_rows, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return status_of(e);
    }
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return status_of(e);
    }
  }
  if (c.p) (void)hipFree(c.p);
  c.p = p;
  c.cap_rows = nr;
  c.ld = nl;
  return TTICE_OK;
}

// The decision scalars are written by the kernels straight into the pinned
// host buffer hs (device-visible), so waiting for them needs no copy kernel.
int ttice_state::sync_scalars(int /*n*/) {
  CK(hipStreamSynchronize(stream));
  return TTICE_OK;
}

namespace {

// The fused projection gives each column one lane: below this many columns
// it cannot fill the device and the tiled products are used instead.
constexpr int64_t kFusedMinCols = 8192;

// Split the K-sum of a Gram product so the launch has a few hundred blocks.
int32_t gram_kchunk(int32_t m, int64_t K) {
  const int64_t tiles = (int64_t)((m + 63) / 64) * ((m + 63) / 64);
  int64_t S = std::max<int64_t>(1, 512 / std::max<int64_t>(tiles, 1));
  S = std::min<int64_t>(S, std::max<int64_t>(1, K / 64));
  int64_t chunk = (K + S - 1) / S;
  chunk = ((chunk + 15) / 16) * 16;
  return (int32_t)std::max<int64_t>(chunk, 16);
}

}  // namespace

// Levels i = 0..d-1 of Algorithm 1 (and the update loop of Algorithm 2) on
// N frames read from zin0 (frame stride P, optional frame map fidx).
// tol_in < 0: the per-core tolerance is eps ||Y||_F / sqrt(d) (Corollary 1)
// with ||Y|| computed here; otherwise tol_in is the tolerance.
// rk_pend holds the ranks being built (starts as the committed ones).
// The last level's coefficients go to last_out (row j = frame j, stride
// last_ld); last_out == nullptr means "into the last core after n_total".
namespace {
// Block-Lanczos truncated SVD: kLzSteps blocks of b vectors, a Krylov basis
// of kLzSteps b vectors; used for Gram matrices wider than kLzMinM and at
// least twice the basis.  The block is wider than the core's last r_R + 1 by
// half (a multiple of 32 in [32, 128], doubled while the result is not
// certified): block Krylov methods converge on the leading eigenpairs at a
// rate set by the ratio of the wanted eigenvalues to the (b+1)-st, so a
// block that holds every wanted pair with room to spare converges in a few
// steps even where the spectrum decays slowly.  A basis of at most 128
// vectors keeps the Rayleigh-Ritz eigenproblem on the single-launch
// register tridiagonalisation.
constexpr int32_t kLzBlockMin = 32, kLzBlockMax = 128;
constexpr int32_t kLzBlockForced = 32;  // smallest block when the solver is forced (small test matrices)
constexpr int32_t kLzSteps = 4;
constexpr int32_t kLzBasisMax = kLzBlockMax * kLzSteps;
constexpr int64_t kLzMinM = 256;
// The explicit-residual rank check runs when tol2 < kResolveSafety m^2 u ||R||^2.
constexpr double kResolveSafety = 4.0;
constexpr int kResolveRounds = 8;  // passes of one level at most
// orthonormality reached by the Newton-Schulz steps on appended directions
constexpr double kOrthTol = 1e-13;
constexpr int kNsMaxSteps = 8;
int32_t lz_block(int64_t last_rR, int32_t bmin) {
  const int64_t want = (3 * (last_rR + 1) / 2 + 31) / 32 * 32;
  return (int32_t)std::min<int64_t>(kLzBlockMax, std::max<int64_t>(bmin, want));
}
// Certificate: the rank decision must hold with the kept eigenvalues' error
// bound (sum eta^2 / gap) within kLzTailTol of its distance to the tolerance,
// and the kept subspace's angle bound ||E||_F / gap must be within
// kLzAngleTol, or ||E||_F itself at working accuracy (kLzResUlps units of
// roundoff of the largest eigenvalue: what the dense solver's own rounding
// leaves; E: the residuals G x - theta x).
constexpr double kLzTailTol = 1e-6;
constexpr double kLzAngleTol = 1e-12;
constexpr double kLzResUlps = 64.0;
constexpr int kLzHost = 2 * kLzBasisMax + 16;  // doubles of the pinned host buffer hl
}  // namespace

int ttice_state::dense_svd(int64_t rows, int64_t Ncol, const View& vR, bool left, double tol2, int64_t cap,
                           int64_t* rR_out, double* tail2_out, double* margin_out) {
  hipStream_t st = stream;
  const int64_t m = left ? rows : Ncol;
  const int64_t K = left ? Ncol : rows;
  const View vRt = transposed(vR);  // Ncol x rows
  // (m <= 32 with K linear in memory: one slice, which the matrix-core
  // product kernel splits itself; a frame-major K takes the slices here)
  const bool k_linear = (left ? vR.cpf : vR.rpf) == kUnframed;
  const int32_t kchunk = (m <= 32 && k_linear) ? (int32_t)K : gram_kchunk((int32_t)m, K);
  const int64_t Sg = (K + kchunk - 1) / kchunk;
  CKS(ensure(gpart, (size_t)Sg * m * m * sizeof(double)));
  CKS(ensure(gram, (size_t)m * m * sizeof(double)));
  CKS(ensure(tri, (size_t)(4 * m + sym_eig_ws((int32_t)m)) * sizeof(double)));  // d, e, tau, w, workspace
  CKS(ensure(order, (size_t)m * sizeof(int32_t)));
  CKS(ensure(lam, (size_t)m * sizeof(double)));
  CKS(ensure(tail, (size_t)(m + 1) * sizeof(double)));
  double* dd = as<double>(tri);
  double* ee = dd + m;
  double* tauv = dd + 2 * m;
  double* wv = dd + 3 * m;
  CK((gemm<double, double, double>(st, (int32_t)m, (int32_t)m, (int32_t)K, kchunk, 1.0, as<double>(rbuf),
                                   left ? vR : vRt, as<double>(rbuf), left ? vRt : vR, 0.0, (const double*)nullptr,
                                   View(), as<double>(gpart), row_major(m), m * m, nullptr, nullptr, gws())));
  CK(gram_reduce(st, as<double>(gpart), (int32_t)Sg, (int32_t)m, as<double>(gram)));
  // eigenvalues, then the truncation rank (eq:deltasvd) from them
  RankSelect sel;
  sel.cnt = as<int>(tilecnt);  // zero between kernels (the product kernels clear theirs)
  sel.tol2 = tol2;
  sel.cap = cap;
  sel.order = as<int32_t>(order);
  sel.lam = as<double>(lam);
  sel.tail = as<double>(tail);
  sel.res = hs;
  CK(sym_eigvals(st, (int32_t)m, as<double>(gram), dd, ee, tauv, wv, dd + 4 * m, &sel));
  CKS(sync_scalars(4));
  if (hs[3] != 0.0) return TTICE_EDEVICE;
  const int64_t rR = (int64_t)hs[0];
  *rR_out = rR;
  *tail2_out = hs[1];
  *margin_out = hs[2];
  if (rR == 0) return TTICE_OK;
  CKS(ensure(W, (size_t)rows * rR * sizeof(double)));
  CKS(ensure(W2, (size_t)rows * rR * sizeof(double)));
  CKS(ensure(eigws, (size_t)sym_eigvecs_ws((int32_t)m, (int32_t)rR) * sizeof(double)));
  double* Wp = as<double>(W);
  const View vW = row_major(rR);
  if (left) {
    // eigenvectors of R R^T for the r_R largest eigenvalues
    CK(sym_eigvecs(st, (int32_t)m, (int32_t)rR, dd, ee, wv, as<double>(gram), tauv, as<double>(eigws), Wp, gws()));
  } else {
    // U_R = R V_r Sigma_r^{-1} with V_r the eigenvectors of R^T R
    CKS(ensure(T, (size_t)Ncol * rR * sizeof(double)));
    CK(sym_eigvecs(st, (int32_t)m, (int32_t)rR, dd, ee, wv, as<double>(gram), tauv, as<double>(eigws),
                   as<double>(W2), gws()));
    CK(gather_columns(st, (int32_t)Ncol, (int32_t)rR, as<double>(W2), (int32_t)rR, as<int32_t>(order),
                      as<double>(lam), true, as<double>(T)));
    CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)rR, (int32_t)Ncol, (int32_t)Ncol, 1.0,
                                     as<double>(rbuf), vR, as<double>(T), vW, 0.0, (const double*)nullptr, View(),
                                     Wp, vW, 0, nullptr, nullptr, gws())));
  }
  return TTICE_OK;
}

// The leading eigenpairs of the residual's Gram matrix G (R R^T when left,
// else R^T R; m wide, applied as two products with R, never formed) by
// block Lanczos with full re-orthogonalisation: a pseudo-random start block,
// Krylov blocks G Q_j orthogonalised against all earlier ones (two
// classical Gram-Schmidt passes) and orthonormalised by two Cholesky QR
// passes; then Rayleigh-Ritz on Q^T G Q.  The Ritz values are lower bounds
// of the leading eigenvalues, and the energy they miss (trace - their sum,
// the trace being ||R||_F^2) is added to every tail, so the selected r_R is
// never below the exact one.  The result is accepted (*ok) only when the
// residuals of the kept Ritz pairs and of the first discarded one certify
// it (kLz*Tol); otherwise the caller runs the dense solver.
#ifdef TTICE_EMU_DEBUG
#define LZ_REJECT                                                          \
  do {                                                                     \
    fprintf(stderr, "lanczos m=%ld rejected at line %d\n", (long)m, __LINE__); \
    return TTICE_OK;                                                       \
  } while (0)
#else
#define LZ_REJECT return TTICE_OK
#endif
int ttice_state::lanczos_svd(int level, int32_t b, int64_t rows, int64_t Ncol, const View& vR, bool left, double tol2,
                             int64_t cap, int64_t* rR_out, double* tail2_out, double* margin_out, bool* ok) {
  hipStream_t st = stream;
  *ok = false;
  ++lz_tries;
  const int64_t m = left ? rows : Ncol;
  const int64_t mo = left ? Ncol : rows;  // the other side of R
  const int32_t sb = kLzSteps * b;
  const double* R = as<double>(rbuf);
  const View vRt = transposed(vR);
  if (!hl) {
    if (hipHostMalloc((void**)&hl, kLzHost * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      hl = nullptr;
      return TTICE_ENOMEM;
    }
  }
  // workspace: basis Q and G Q (m x sb each), two candidate blocks (m x b),
  // the other-side products (mo x sb), small matrices, Ritz vectors X and
  // G X (m x sb each), the trace and its partials
  const int64_t nparts = sumsq_parts(rows * Ncol);
  const int64_t need = 2 * m * sb + 2 * m * b + mo * sb + (int64_t)sb * b + 3 * (int64_t)sb * sb +
                       2 * (int64_t)sb * sb + 2 * m * sb + sb + nparts + 8;
  CKS(ensure(lzw, (size_t)need * sizeof(double)));
  CKS(ensure(tri, (size_t)(4 * sb + sym_eig_ws(sb)) * sizeof(double)));
  CKS(ensure(order, (size_t)sb * sizeof(int32_t)));
  CKS(ensure(lam, (size_t)sb * sizeof(double)));
  CKS(ensure(tail, (size_t)(sb + 1) * sizeof(double)));
  double* Q = as<double>(lzw);       // m x sb
  double* GQ = Q + m * sb;           // m x sb
  double* V0 = GQ + m * sb;          // m x b
  double* V1 = V0 + m * b;           // m x b
  double* T1 = V1 + m * b;           // mo x sb
  double* P = T1 + mo * sb;          // sb x b
  double* Sb = P + (int64_t)sb * b;     // b x b (polish: r_R x r_R)
  double* Li = Sb + (int64_t)sb * sb;   // as Sb
  double* Spre = Li + (int64_t)sb * sb;  // b x b
  double* Tm = Spre + (int64_t)sb * sb;  // sb x sb
  double* Sv = Tm + (int64_t)sb * sb;  // sb x sb (eigenvectors of Tm)
  double* X = Sv + (int64_t)sb * sb;   // m x sb
  double* GX = X + m * sb;             // m x sb
  double* eta2 = GX + m * sb;          // sb
  double* parts = eta2 + sb;           // nparts
  double* trace = parts + nparts;      // 1
  const View q = row_major(sb), vb = row_major(b);
  auto G = [&](const double* Xin, View vx, int32_t n, double* out, View vo) -> hipError_t {
    // out = G Xin (m x n): the inner product with R first (mo x n into T1)
    hipError_t e;
    if (left) {
      e = gemm<double, double, double>(st, (int32_t)Ncol, n, (int32_t)rows, (int32_t)rows, 1.0, R, vRt, Xin, vx,
                                       0.0, (const double*)nullptr, View(), T1, row_major(n), 0, nullptr, nullptr,
                                       gws());
      if (e != hipSuccess) return e;
      return gemm<double, double, double>(st, (int32_t)rows, n, (int32_t)Ncol, (int32_t)Ncol, 1.0, R, vR, T1,
                                          row_major(n), 0.0, (const double*)nullptr, View(), out, vo, 0, nullptr,
                                          nullptr, gws());
    }
    e = gemm<double, double, double>(st, (int32_t)rows, n, (int32_t)Ncol, (int32_t)Ncol, 1.0, R, vR, Xin, vx, 0.0,
                                     (const double*)nullptr, View(), T1, row_major(n), 0, nullptr, nullptr, gws());
    if (e != hipSuccess) return e;
    return gemm<double, double, double>(st, (int32_t)Ncol, n, (int32_t)rows, (int32_t)rows, 1.0, R, vRt, T1,
                                        row_major(n), 0.0, (const double*)nullptr, View(), out, vo, 0, nullptr,
                                        nullptr, gws());
  };
  // block j of Q from the candidate block (in, view vin): orthogonalised
  // against Q's first j blocks, then orthonormalised
  auto orth_block = [&](int32_t j, const double* in, View vin) -> hipError_t {
    const int32_t nq = j * b;
    const double* cur = in;
    View vcur = vin;
    hipError_t e = hipSuccess;
    if (nq > 0) {  // the candidates' Gram block before the projection
      e = gemm<double, double, double>(st, b, b, (int32_t)m, (int32_t)m, 1.0, in, transposed(vin), in, vin, 0.0,
                                       (const double*)nullptr, View(), Spre, vb, 0, nullptr, nullptr, gws());
      if (e != hipSuccess) return e;
    }
    for (int pass = 0; pass < 2 && nq > 0; ++pass) {
      e = gemm<double, double, double>(st, nq, b, (int32_t)m, (int32_t)m, 1.0, Q, transposed(q), cur, vcur, 0.0,
                                       (const double*)nullptr, View(), P, vb, 0, nullptr, nullptr, gws());
      if (e != hipSuccess) return e;
      e = gemm<double, double, double>(st, (int32_t)m, b, nq, nq, -1.0, Q, q, P, vb, 1.0, cur, vcur, V0, vb, 0,
                                       nullptr, nullptr, gws());
      if (e != hipSuccess) return e;
      cur = V0;
      vcur = vb;
    }
    // two Cholesky QR passes: cur -> V1 -> block j of Q
    for (int pass = 0; pass < 2; ++pass) {
      e = gemm<double, double, double>(st, b, b, (int32_t)m, (int32_t)m, 1.0, cur, transposed(vcur), cur, vcur, 0.0,
                                       (const double*)nullptr, View(), Sb, vb, 0, nullptr, nullptr, gws());
      if (e != hipSuccess) return e;
      e = chol_inv(st, b, Sb, b, pass == 0 && nq > 0 ? Spre : nullptr, b, Li, b);
      if (e != hipSuccess) return e;
      double* dst = pass == 0 ? V1 : Q + (int64_t)j * b;
      const View vdst = pass == 0 ? vb : q;
      e = gemm<double, double, double>(st, (int32_t)m, b, b, b, 1.0, cur, vcur, Li, vb, 0.0, (const double*)nullptr,
                                       View(), dst, vdst, 0, nullptr, nullptr, gws());
      if (e != hipSuccess) return e;
      cur = V1;
      vcur = vb;
    }
    return hipSuccess;
  };
  CK(sumsq(st, R, rows * Ncol, parts, trace));
  double* dd = as<double>(tri);
  double* ee = dd + sb;
  double* tauv = dd + 2 * sb;
  double* wv = dd + 3 * sb;
  RankSelect sel;
  sel.cnt = as<int>(tilecnt);
  sel.tol2 = tol2;
  sel.cap = cap;
  sel.order = as<int32_t>(order);
  sel.lam = as<double>(lam);
  sel.tail = as<double>(tail);
  sel.res = hs;
  sel.trace = trace;
  CK(rand_fill(st, m, b, V0, b, 0x9E3779B9ull + (uint64_t)level));
  CK(orth_block(0, V0, vb));
  for (int32_t j = 0; j < kLzSteps; ++j) {
    CK(G(Q + (int64_t)j * b, q, b, GQ + (int64_t)j * b, q));
    if (j + 1 < kLzSteps) CK(orth_block(j + 1, GQ + (int64_t)j * b, q));
  }
  // Rayleigh-Ritz: Tm = Q^T G Q (symmetrised), its eigenvalues and the rank
  CK((gemm<double, double, double>(st, sb, sb, (int32_t)m, (int32_t)m, 1.0, Q, transposed(q), GQ, q, 0.0,
                                   (const double*)nullptr, View(), Tm, q, 0, nullptr, nullptr, gws())));
  CK(symmetrize(st, sb, Tm, sb));
  CK(sym_eigvals(st, sb, Tm, dd, ee, tauv, wv, dd + 4 * sb, &sel));
  CKS(sync_scalars(4));
  if (hs[3] != 0.0) LZ_REJECT;  // not finite: left to the dense solver
  const int64_t rR = (int64_t)hs[0];
  double tail2 = hs[1], margin = hs[2];
  if (rR >= sb) LZ_REJECT;  // the basis does not hold enough energy
  if (rR > lz_max_block()) LZ_REJECT;  // more kept pairs than the polishing step's factorisation takes
  if (rR > 0) {
    // Ritz vectors X = Q S of the kept pairs and of the first discarded
    // one.  The kept ones carry the rounding of the Krylov blocks (those of
    // a wide spectrum are ill-conditioned), so one step of subspace
    // iteration polishes them: Y = G X, orthonormalised (a well-conditioned
    // block: its columns scale with the kept eigenvalues), and Rayleigh-Ritz
    // on span(Y).  The first discarded pair (theta, eta) bounds the
    // discarded eigenvalues by theta + eta.
    const int32_t kp = (int32_t)rR, kc = kp + 1;
    const View vc = row_major(kc), vk = row_major(kp);
    CKS(ensure(eigws, (size_t)sym_eigvecs_ws(sb, kc) * sizeof(double)));
    CK(sym_eigvecs(st, sb, kc, dd, ee, wv, Tm, tauv, as<double>(eigws), Sv));
    CK((gemm<double, double, double>(st, (int32_t)m, kc, sb, sb, 1.0, Q, q, Sv, vc, 0.0, (const double*)nullptr,
                                     View(), X, vc, 0, nullptr, nullptr, gws())));
    CK(G(X, vc, kc, GX, vc));  // Y
    // hl: [0, kLzBasisMax) eta_j^2 and [kLzBasisMax, 2 kLzBasisMax) theta_j of
    // the polished pairs; then eta^2, theta of the first discarded pair; trace
    double* hd = hl + 2 * kLzBasisMax;
    CK(ritz_residuals(st, (int32_t)m, 1, kc, X + kp, GX + kp, wv + kp, hd, hd + 1));
    CK(hipMemcpyAsync(hd + 2, trace, sizeof(double), hipMemcpyDeviceToHost, st));
    // two Cholesky QR passes: Y's first r_R columns -> Q (scratch) -> X
    const double* cur = GX;
    View vcur = vc;
    for (int pass = 0; pass < 2; ++pass) {
      double* dst = pass == 0 ? Q : X;
      CK((gemm<double, double, double>(st, kp, kp, (int32_t)m, (int32_t)m, 1.0, cur, transposed(vcur), cur, vcur,
                                       0.0, (const double*)nullptr, View(), Sb, vk, 0, nullptr, nullptr, gws())));
      CK(chol_inv(st, kp, Sb, kp, nullptr, 0, Li, kp));
      CK((gemm<double, double, double>(st, (int32_t)m, kp, kp, kp, 1.0, cur, vcur, Li, vk, 0.0,
                                       (const double*)nullptr, View(), dst, vk, 0, nullptr, nullptr, gws())));
      cur = dst;
      vcur = vk;
    }
    CK(G(X, vk, kp, GX, vk));  // G Y~
    CK((gemm<double, double, double>(st, kp, kp, (int32_t)m, (int32_t)m, 1.0, X, transposed(vk), GX, vk, 0.0,
                                     (const double*)nullptr, View(), Tm, vk, 0, nullptr, nullptr, gws())));
    CK(symmetrize(st, kp, Tm, kp));
    CK(sym_eigvals(st, kp, Tm, dd, ee, tauv, wv, dd + 4 * sb, nullptr));
    CKS(ensure(eigws, (size_t)sym_eigvecs_ws(kp, kp) * sizeof(double)));
    CK(sym_eigvecs(st, kp, kp, dd, ee, wv, Tm, tauv, as<double>(eigws), Sv));
    // the polished pairs (X S, G X S) into the free basis buffers
    CK((gemm<double, double, double>(st, (int32_t)m, kp, kp, kp, 1.0, X, vk, Sv, vk, 0.0, (const double*)nullptr,
                                     View(), Q, vk, 0, nullptr, nullptr, gws())));
    CK((gemm<double, double, double>(st, (int32_t)m, kp, kp, kp, 1.0, GX, vk, Sv, vk, 0.0, (const double*)nullptr,
                                     View(), GQ, vk, 0, nullptr, nullptr, gws())));
    CK(ritz_residuals(st, (int32_t)m, kp, kp, Q, GQ, wv, hl, hl + kLzBasisMax));
    CKS(sync_scalars(0));
    // the decision again from the polished Ritz values (lower bounds of
    // the leading eigenvalues, so trace minus their sum bounds every tail
    // from above): it must agree, and the error bounds of the kept
    // eigenvalues (sum eta^2 / gap) and of the kept subspace's angle
    // (||E||_F / gap) must not be able to move it or the result
    const double* th = hl + kLzBasisMax;
    const double trv = hd[2];
    double esum = 0.0, s_prev = 0.0;
    for (int32_t j = 0; j < kp; ++j) {
      const double e2 = hl[j];
      if (!isfinite(e2) || !isfinite(th[j])) LZ_REJECT;
      esum += std::max(e2, 0.0);
      if (j + 1 < kp) s_prev += std::max(th[j], 0.0);
    }
    const double t_r = std::max(0.0, trv - (s_prev + std::max(th[kp - 1], 0.0)));
    const double t_rm1 = std::max(0.0, trv - s_prev);
    const bool capped = rR == cap;
    if (!capped && !(t_r <= tol2 && t_rm1 > tol2)) LZ_REJECT;
    const double t2 = tol2 > 0.0 ? tol2 : 1e-300;
    margin = std::min(fabs(t_r - tol2), fabs(t_rm1 - tol2)) / t2;
    tail2 = t_r;
    const double up = hd[1] + sqrt(std::max(hd[0], 0.0));
    const double gap = th[kp - 1] - up;
#ifdef TTICE_EMU_DEBUG
    fprintf(stderr, "lanczos m=%ld rR=%ld th0=%g esum=%g gap=%g up=%g margin=%g tol2=%g angle=%g\n", (long)m,
            (long)rR, th[0], esum, gap, up, margin, tol2, sqrt(esum) / gap);
#endif
    if (!(th[0] > 0.0) || !(gap > 0.0)) LZ_REJECT;
    if (!capped && esum / gap > kLzTailTol * margin * tol2) LZ_REJECT;
    if (sqrt(esum) / gap > kLzAngleTol && sqrt(esum) > kLzResUlps * DBL_EPSILON * th[0]) LZ_REJECT;
  }
  // (r_R = 0 is decided by the trace alone, which is exact)
  ++lz_accepted;
  *ok = true;
  *rR_out = rR;
  *tail2_out = tail2;
  *margin_out = margin;
  if (rR == 0) return TTICE_OK;
  CKS(ensure(W, (size_t)rows * rR * sizeof(double)));
  CKS(ensure(W2, (size_t)rows * rR * sizeof(double)));
  // the polished vectors sit in Q (m x r_R), theta_j (decreasing) in wv
  if (left) {
    CK(gather_columns(st, (int32_t)rows, (int32_t)rR, Q, (int32_t)rR, nullptr, wv, false, as<double>(W)));
  } else {
    // U_R = R V_r Sigma_r^{-1}
    CKS(ensure(T, (size_t)Ncol * rR * sizeof(double)));
    CK(gather_columns(st, (int32_t)Ncol, (int32_t)rR, Q, (int32_t)rR, nullptr, wv, true, as<double>(T)));
    CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)rR, (int32_t)Ncol, (int32_t)Ncol, 1.0, R, vR,
                                     as<double>(T), row_major(rR), 0.0, (const double*)nullptr, View(),
                                     as<double>(W), row_major(rR), 0, nullptr, nullptr, gws())));
  }
  return TTICE_OK;
}

template <typename TIn>
int ttice_state::core_loop(const TIn* zin0, int64_t N, const int32_t* fidx, double tol_in,
                           int64_t* rk_pend, ttice_update_info* info, bool use_occ, double* last_out,
                           int64_t last_ld) {
  hipStream_t st = stream;
  double tol2 = tol_in >= 0 ? tol_in * tol_in : -1.0;
  const void* zin = zin0;
  bool zin_is_input = true;
  int64_t r_new_acc = 0;  // directions appended at the current level over its passes
  int rounds = 0;
  for (int i = 0; i < d; ++i) {
    const int64_t rows = rk_pend[i] * dims[i];
    const int64_t cols = this->cols(i);
    const int64_t r = rk_pend[i + 1];
    const int64_t Ncol = N * cols;
    Core& Ui = U[i];
    const bool last = (i == d - 1);
    const int32_t* fmap = zin_is_input ? fidx : nullptr;
    const View vz = unfolding(cols, P, fmap);

    double* out;
    int64_t fs_out;
    if (!last) {
      out = as<double>(z[i % 2]);
      fs_out = P;
    } else if (last_out) {
      out = last_out;
      fs_out = last_ld;
    } else {
      out = Gt.p + n_total * Gt.ld;
      fs_out = Gt.ld;
    }
    const View vout = unfolding(cols, fs_out);
    const View vUt = transposed(row_major(Ui.ld));
    const View vU = row_major(Ui.ld);

    const double occupancy = rows > 0 ? (double)r / (double)rows : 1.0;
    const bool occ_skip = use_occ && occupancy >= tau;
    // a core whose columns span its whole row space (r = rows: U_i square
    // and orthogonal) leaves a zero residual: nothing to test or append
    const bool full = r >= rows;
    const bool no_resid = occ_skip || full;
    int64_t rR = 0;
    int32_t solver = 0;
    bool again = false;  // the explicit rank check asks for another pass
    double rho2 = std::numeric_limits<double>::quiet_NaN(), tail2 = 0.0;
    double margin = std::numeric_limits<double>::infinity();

    // C = U^T Z (eq:first_resid / eq:project_further, projection part) and
    // the per-column energies of Z (level 1) and of the residual
    double* bn = nullptr;
    if (i == 0) {
      CKS(ensure(bnorm, (size_t)Ncol * sizeof(double)));
      bn = as<double>(bnorm);
    }
    // a served state's level 1 (Algorithm 1) is always fused, one column per lane
    const bool l1_served = served && i == 0 && fidx == nullptr && !profile && proj_fits((int32_t)rows, (int32_t)r);
    if (i == 0 && l1_mode == 1 && !l1_served) return kL1Plain;
    if (i == 0 && l1_mode == 2 && !l1_served) return TTICE_EDEVICE;  // the captured launch does not apply
    const bool fused = proj_fits((int32_t)rows, (int32_t)r) && (Ncol >= kFusedMinCols || l1_served);
    const int pp = proj_prec();
    // the fused FP64 pass gives the residual energies by Pythagoras, the
    // short-column kernel explicitly (one row of partials either way); in
    // reduced precision they otherwise come from the explicit residual
    // (partials per 64-row block)
    const int32_t MB_alloc = (fused && pp == kProjFP64) ? 1 : gemm_row_blocks((int32_t)rows);
    CKS(ensure(colpart, (size_t)MB_alloc * Ncol * sizeof(double)));
    CKS(ensure(fres, (size_t)N * sizeof(double)));
    CKS(ensure(rbuf, (size_t)std::max<int64_t>(1, rows * Ncol) * sizeof(double)));
    const View vr = unfolding(cols, rows * cols);
    const bool small = rows * Ncol <= ((int64_t)1 << 22);
    bool have_R = false;
    double* cp = no_resid ? nullptr : as<double>(colpart);
    // the fused pass's residual energies: in reduced precision only the
    // short-column kernel's (formed explicitly); otherwise the explicit
    // residual (below) writes them, so the pass does not
    double* rho_out = (pp == kProjFP64 || proj_short_fits(pp, (int32_t)rows, (int32_t)r)) ? cp : nullptr;
    bool rho_explicit = false;
    // one pass: ||(I - U U^T) z||^2 = ||z||^2 - ||U^T z||^2 (orthonormal U),
    // in the state's precision (pp) or in FP64
    auto fused_pass = [&](int pp, bool timed) -> hipError_t {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        if (prof_begin(&e0, &e1) != TTICE_OK) return hipErrorOutOfMemory;
        // the batch read once; the coefficients and the per-column energies written
        ev_bytes.push_back((double)N * P * sizeof(TIn) + (double)r * Ncol * sizeof(double) +
                           (double)Ncol * sizeof(double) * ((bn ? 1 : 0) + (rho_out ? 1 : 0)));
      }
      const int vmax = l1_served ? 1 : 4;
      if (zin_is_input)
        return proj_columns<TIn>(st, (int32_t)rows, (int32_t)r, (int32_t)Ncol, (const TIn*)zin, vz, Ui.p, Ui.ld, out,
                                 vout, bn, rho_out, pp, e0, e1, vmax, &rho_explicit);
      return proj_columns<double>(st, (int32_t)rows, (int32_t)r, (int32_t)Ncol, (const double*)zin, vz, Ui.p, Ui.ld,
                                  out, vout, bn, rho_out, pp, e0, e1, vmax, &rho_explicit);
    };
    // R = Z - U C with per-column energies (eq:first_resid, eq:ithresidual),
    // FP64; written to rbuf when small enough to keep for the SVD
    auto residual = [&]() -> hipError_t {
      double* rout = small ? as<double>(rbuf) : nullptr;
      have_R = small;
      if (zin_is_input)
        return gemm<double, TIn, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r, (int32_t)std::max<int64_t>(r, 1),
                                         -1.0, Ui.p, vU, out, vout, 1.0, (const TIn*)zin, vz, rout, vr, 0, cp, nullptr,
                                         gws());
      return gemm<double, double, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r, (int32_t)std::max<int64_t>(r, 1),
                                          -1.0, Ui.p, vU, out, vout, 1.0, (const double*)zin, vz, rout, vr, 0, cp,
                                          nullptr, gws());
    };
    if (fused) {
      // (reduced precision: the fused pass's energies by cancellation would
      // sit at the products' rounding level, so the residual is formed from
      // the rounded coefficients in FP64: ||Z - U C~||^2 = ||R||^2 +
      // ||C~ - C||^2, never below the true energy)
      if (l1_served && l1_mode != 0) {
        ProjDesc dsc;
        dsc.rows = (int32_t)rows;
        dsc.r = (int32_t)r;
        dsc.Ncol = (int32_t)Ncol;
        dsc.vz = vz;
        dsc.vc = vout;
        dsc.Z = zin;
        dsc.U = Ui.p;
        dsc.ldu = Ui.ld;
        dsc.C = out;
        dsc.znorm2 = bn;
        dsc.rho2 = pp == kProjFP64 ? cp : nullptr;
        if (l1_mode == 1) {
          l1_desc = dsc;
          l1_key = serve_key(pp, (int32_t)rows, (int32_t)r, sizeof(TIn) == sizeof(float));
          return kL1Captured;
        }
        // the launch made from the captured arguments must be this one
        if (!same_desc(dsc, l1_desc)) return TTICE_EDEVICE;
      } else {
        CK(fused_pass(pp, profile && i == 0));
      }
      if (pp != kProjFP64 && !no_resid && !rho_explicit) CK(residual());
    } else {
      if (zin_is_input) {
        CK((gemm<TIn, TIn, double>(st, (int32_t)r, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0, Ui.p,
                                   vUt, (const TIn*)zin, vz, 0.0, (const TIn*)nullptr, View(), out, vout,
                                   0, nullptr, bn, gws(), pp)));
      } else {
        CK((gemm<double, double, double>(st, (int32_t)r, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0,
                                         Ui.p, vUt, (const double*)zin, vz, 0.0, (const double*)nullptr,
                                         View(), out, vout, 0, nullptr, bn, gws(), pp)));
      }
      if (!no_resid) CK(residual());
    }
    const int32_t MB = (fused && (pp == kProjFP64 || rho_explicit)) ? 1 : gemm_row_blocks((int32_t)rows);

    if (i == 0 && tol2 < 0) {
      CKS(ensure(fy2, (size_t)N * sizeof(double)));
      CK(frame_sums(st, bn, 1, Ncol, (int32_t)cols, (int32_t)N, as<double>(fy2), fscratch(N)));
      CK(total_sum(st, as<double>(fy2), N, hs + 2));
    }

    if (!no_resid || (i == 0 && tol2 < 0)) {
      if (!no_resid) {
        CK(frame_sums(st, as<double>(colpart), MB, Ncol, (int32_t)cols, (int32_t)N, as<double>(fres), fscratch(N)));
        CK(total_sum(st, as<double>(fres), N, hs));
      }
      CKS(sync_scalars(4));
      if (i == 0 && tol2 < 0) {
        const double ny2 = hs[2];
        if (hs[3] != 0.0 || !isfinite(ny2)) return TTICE_EINVAL;
        if (info) info->norm_y2 = ny2;
        const double tol = eps * sqrt(ny2) / sqrt((double)d);
        tol2 = tol * tol;
        if (info) info->eps_core = tol;
      }
    }
    if (full && !occ_skip) rho2 = 0.0;
    if (!no_resid) {
      rho2 = hs[0];
      if (hs[1] != 0.0 || !isfinite(rho2)) return TTICE_EINVAL;
      rho2 = std::max(rho2, 0.0);
      tail2 = rho2;

      if (rho2 > tol2) {
        if (!have_R) {
          CK((zin_is_input
                  ? gemm<double, TIn, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r,
                                              (int32_t)std::max<int64_t>(r, 1), -1.0, Ui.p, vU, out, vout, 1.0,
                                              (const TIn*)zin, vz, as<double>(rbuf), vr, 0, nullptr, nullptr, gws())
                  : gemm<double, double, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r,
                                                 (int32_t)std::max<int64_t>(r, 1), -1.0, Ui.p, vU, out, vout,
                                                 1.0, (const double*)zin, vz, as<double>(rbuf), vr, 0, nullptr,
                                                 nullptr, gws())));
        }
        // Truncated SVD of R_cat = [R(1) ... R(N)] (eq:svdfirst) from the
        // eigenpairs of its Gram matrix: left (rows x rows) when rows <=
        // N*cols, else right (N*cols x N*cols).  A wide Gram matrix first
        // goes to the block-Lanczos solver (leading eigenpairs only); the
        // dense solver takes over when that result is not certified.
        const bool left = rows <= Ncol;
        const int64_t m = left ? rows : Ncol;
        // documented size limit of the residual's SVD, checked before any
        // workspace for it is allocated
        if (m > sym_eig_max()) return TTICE_EINVAL;
        bool have_svd = false;
        // The Gram matrix's eigenvalues carry absolute errors of about
        // m u ||R||^2 each, so its tails (sums of up to m of them) cannot
        // place a cut whose tolerance is below that floor, and the
        // directions of eigenvalues at the floor are not resolved: there
        // the candidates are the directions the Gram matrix resolves (its
        // rank at the floor), the rank among them comes from the explicit
        // residual energies below, and when those candidates leave more
        // than tol2 the level runs again on the remaining residual (whose
        // Gram matrix resolves it on its own, smaller scale).
        const double floor2 = kResolveSafety * (double)m * (double)m * DBL_EPSILON * rho2;
        const bool resolve = tol2 < floor2;
        const double tol2_sel = resolve ? floor2 : tol2;
        // the block from the core's last r_R, doubled while the result is
        // not certified
        const int32_t bmin = lz_mode == 2 ? kLzBlockForced : kLzBlockMin;
        for (int32_t b = lz_block(last_rR[i], bmin); lz_mode != 0 && !have_svd && b <= kLzBlockMax; b *= 2) {
          const int64_t basis = (int64_t)kLzSteps * b;
          if (!(m >= (lz_mode == 2 ? basis : std::max<int64_t>(kLzMinM, 2 * basis)) && last_rR[i] < basis / 2)) break;
          CKS(lanczos_svd(i, b, rows, Ncol, vr, left, tol2_sel, rows - r, &rR, &tail2, &margin, &have_svd));
        }
        if (!have_svd) CKS(dense_svd(rows, Ncol, vr, left, tol2_sel, rows - r, &rR, &tail2, &margin));
        last_rR[i] = rR;
        solver = have_svd ? 2 : 1;
        if (rR > 0) {
          double* Wp = as<double>(W);
          double* W2p = as<double>(W2);
          const View vW = row_major(rR);
          // Re-orthogonalise against U (two classical Gram-Schmidt passes)
          if (r > 0) {
            CKS(ensure(T, (size_t)std::max<int64_t>(r * rR, Ncol * rR) * sizeof(double)));
            for (int pass = 0; pass < 2; ++pass) {
              CK((gemm<double, double, double>(st, (int32_t)r, (int32_t)rR, (int32_t)rows, (int32_t)rows, 1.0,
                                               Ui.p, vUt, Wp, vW, 0.0, (const double*)nullptr, View(),
                                               as<double>(T), vW, 0, nullptr, nullptr, gws())));
              CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)rR, (int32_t)r, (int32_t)r, -1.0,
                                               Ui.p, vU, as<double>(T), vW, 1.0, Wp, vW, Wp, vW, 0, nullptr,
                                               nullptr, gws())));
            }
          }
          // ... and among themselves: Newton-Schulz steps towards the
          // orthonormal polar factor, W <- W (3I - W^T W) / 2, two at least
          // and then until max |W^T W - I| <= kOrthTol (columns built from
          // small singular values start far from orthonormal)
          CKS(ensure(S, (size_t)rR * rR * sizeof(double)));
          for (int pass = 0;; ++pass) {
            CK((gemm<double, double, double>(st, (int32_t)rR, (int32_t)rR, (int32_t)rows, (int32_t)rows, 1.0, Wp,
                                             transposed(vW), Wp, vW, 0.0, (const double*)nullptr, View(),
                                             as<double>(S), vW, 0, nullptr, nullptr, gws())));
            if (pass >= 2) {
              CK(max_off_identity(st, (int32_t)rR, as<double>(S), (int32_t)rR, hs));
              CKS(sync_scalars(2));
              if (hs[1] != 0.0) return TTICE_EDEVICE;
              if (hs[0] <= kOrthTol || pass >= kNsMaxSteps) break;
            }
            CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)rR, (int32_t)rR, (int32_t)rR, -0.5, Wp,
                                             vW, as<double>(S), vW, 1.5, Wp, vW, W2p, vW, 0, nullptr,
                                             nullptr, gws())));
            std::swap(Wp, W2p);
          }
          if (resolve) {
            // With U_R orthonormal, C = U_R^T R and the residual R - U_R C,
            // the discarded energy of keeping U_R's first r columns is
            // ||R - U_R C||^2 + sum_{j>=r} ||C_j||^2 (C_j: row j), a sum of
            // non-negative FP64 terms (eq:deltasvd without the Gram
            // matrix's cancellation); the rank is the smallest r whose
            // tail is within tol2.
            const View vC = row_major(Ncol);
            const int32_t MBr = gemm_row_blocks((int32_t)rows);
            CKS(ensure(T, (size_t)Ncol * rR * sizeof(double)));
            CKS(ensure(colpart, (size_t)MBr * Ncol * sizeof(double)));
            CKS(ensure(lam, (size_t)rR * sizeof(double)));
            CKS(ensure(tail, 2 * sizeof(double)));
            CK((gemm<double, double, double>(st, (int32_t)rR, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0, Wp,
                                             transposed(vW), as<double>(rbuf), vr, 0.0, (const double*)nullptr,
                                             View(), as<double>(T), vC, 0, nullptr, nullptr, gws())));
            CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)rR, (int32_t)rR, -1.0, Wp,
                                             vW, as<double>(T), vC, 1.0, as<double>(rbuf), vr, (double*)nullptr,
                                             View(), 0, as<double>(colpart), nullptr, gws())));
            CK(frame_sums(st, as<double>(colpart), MBr, Ncol, (int32_t)cols, (int32_t)N, as<double>(fres),
                          fscratch(N)));
            CK(total_sum(st, as<double>(fres), N, as<double>(tail)));
            CK(row_sumsq(st, (int32_t)rR, (int32_t)Ncol, Ncol, as<double>(T), as<double>(lam)));
            CK(tail_rank(st, (int32_t)rR, as<double>(lam), as<double>(tail), tol2, hs));
            CKS(sync_scalars(4));
            if (hs[3] != 0.0) return TTICE_EDEVICE;
            const int64_t rx = (int64_t)hs[0];
            tail2 = hs[1];
            margin = hs[2];
            again = rx == rR && tail2 > tol2 && !served && rounds + 1 < kResolveRounds;
            if (rx < rR) {
              // U_R's first rx columns, ld rx
              CK(gather_columns(st, (int32_t)rows, (int32_t)rx, Wp, (int32_t)rR, nullptr, nullptr, false, W2p));
              std::swap(Wp, W2p);
              rR = rx;
            }
          }
          // eq:coreexpansion: U_i <- [U_i^pad, U_R] (U_R's columns sign-fixed on
          // the way), and in the same launch the zero padding below
          CKS(grow_core(Ui, rows, r + rR, rows, r));
          double* zp = nullptr;
          int64_t zr = 0, zc = 0, zl = 0;
          // eq:ukpad: zero rows for the new rank slices of the next core
          if (!last) {
            Core& Un = U[i + 1];
            const int64_t nrow_old = rk_pend[i + 1] * dims[i + 1];
            const int64_t nrow_new = (rk_pend[i + 1] + rR) * dims[i + 1];
            CKS(grow_core(Un, nrow_new, std::max<int64_t>(rk_pend[i + 2], 1), nrow_old, rk_pend[i + 2]));
            zp = Un.p + nrow_old * Un.ld;
            zr = nrow_new - nrow_old;
            zc = Un.ld;
            zl = Un.ld;
          } else {
            // last core: new entries of the stored tensors' columns are zero
            if (!last_out) {
              CKS(grow_core(Gt, n_total + N, r + rR, n_total + N, r));
              out = Gt.p + n_total * Gt.ld;
              fs_out = Gt.ld;
              zp = Gt.p + r;
              zr = n_total;
              zc = rR;
              zl = Gt.ld;
            } else if (r + rR > last_ld) {
              return TTICE_EDEVICE;  // caller sized last_out for the maximum rank
            }
          }
          CK(sign_place(st, (int32_t)rows, (int32_t)rR, Wp, Ui.p + r, Ui.ld, zp, zr, zc, zl));
          // New rows of the next level's data (eq:project_further with the
          // appended directions): U_R^T Z below C.
          // (U_i may have been reallocated with a new leading dimension)
          const View vout2 = unfolding(cols, fs_out);
          const View vUt2 = transposed(row_major(Ui.ld));
          if (zin_is_input) {
            CK((gemm<TIn, TIn, double>(st, (int32_t)rR, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0,
                                       Ui.p + r, vUt2, (const TIn*)zin, vz, 0.0, (const TIn*)nullptr, View(),
                                       out + r * cols, vout2, 0, nullptr, nullptr, gws(), pp)));
          } else {
            CK((gemm<double, double, double>(st, (int32_t)rR, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0,
                                             Ui.p + r, vUt2, (const double*)zin, vz, 0.0,
                                             (const double*)nullptr, View(), out + r * cols, vout2, 0,
                                             nullptr, nullptr, gws(), pp)));
          }
          rk_pend[i + 1] = r + rR;
        }
      }
    }
    r_new_acc += rR;
    if (info) {
      info->r_new[i] = r_new_acc;
      info->rho2[i] = rho2;
      info->tail2[i] = occ_skip ? 0.0 : tail2;
      info->margin[i] = margin;
      info->solver[i] = solver;
    }
    if (again) {
      // the same level again with the grown core: its residual is the part
      // the appended directions left
      ++rounds;
      --i;
      continue;
    }
    r_new_acc = 0;
    rounds = 0;
    zin = out;
    zin_is_input = false;
  }
  return TTICE_OK;
}

// Push N frames through the cores with ranks rks (no update): coefficients
// into coef_out (row b = frame b, stride coef_ld), and optionally per-frame
// residual energy err2(b) = sum_i ||R_i(b)||^2 and per-frame ||Y(b)||^2.
// Every step of the chain is an orthogonal projection, so in FP64 the
// residual energy is the telescoping difference ||Y(b)||^2 - ||c(b)||^2; in
// reduced precision (pp) that cancellation would sit at the products'
// rounding level, so each level whose core is not square forms its
// residual Z - U C explicitly (energies in FP64).
template <typename TIn>
int ttice_state::chain_project(const TIn* zin0, int64_t N, const int64_t* rks, double* coef_out,
                               int64_t coef_ld, double* err2_out, double* y2_out, int* nonfinite,
                               const ChainWs* cw, int pp) {
  hipStream_t st = stream;
  const void* zin = zin0;
  bool zin_is_input = true;
  const GemmWs gw = cw ? cw->g : gws();
  const bool tele = err2_out != nullptr && pp == kProjFP64;
  double* y2p = y2_out;
  if (err2_out && !y2p) {
    if (cw) {
      y2p = cw->y2;
    } else {
      CKS(ensure(fy2, (size_t)N * sizeof(double)));
      y2p = as<double>(fy2);
    }
  }
  double* fres_p = nullptr;
  if (err2_out && !tele) CK(zero2d(st, 1, N, err2_out, N));
  for (int i = 0; i < d; ++i) {
    const int64_t rows = rks[i] * dims[i];
    const int64_t cols = this->cols(i);
    const int64_t r = rks[i + 1];
    const int64_t Ncol = N * cols;
    Core& Ui = U[i];
    const bool last = (i == d - 1);
    const View vz = unfolding(cols, P);
    double* out = last ? coef_out : (cw ? cw->z[i % 2] : as<double>(z[i % 2]));
    const int64_t fs_out = last ? coef_ld : P;
    const View vout = unfolding(cols, fs_out);
    double* bn = nullptr;
    if (i == 0 && y2p) {
      if (cw) {
        bn = cw->bnorm;
      } else {
        CKS(ensure(bnorm, (size_t)Ncol * sizeof(double)));
        bn = as<double>(bnorm);
      }
    }
    const bool fused = proj_fits((int32_t)rows, (int32_t)r) && Ncol >= kFusedMinCols;
    const bool resid = err2_out && !tele && r < rows;
    const int32_t MB = gemm_row_blocks((int32_t)rows);
    double* cp = nullptr;
    if (resid) {
      if (cw) {
        cp = cw->colpart;
        fres_p = cw->fres;
      } else {
        CKS(ensure(colpart, (size_t)MB * Ncol * sizeof(double)));
        CKS(ensure(fres, (size_t)N * sizeof(double)));
        cp = as<double>(colpart);
        fres_p = as<double>(fres);
      }
    }
    double* fsl_p = cw ? cw->fsl : fscratch(N);
    // C = U^T Z (the next level's data, eq:project_further)
    if (fused) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      // the level-1 pass in the state's arithmetic is profiled with the core loop's
      if (profile && in_update && i == 0 && pp == proj_prec()) {
        CKS(prof_begin(&e0, &e1));
        ev_bytes.push_back((double)N * P * sizeof(TIn) + (double)r * Ncol * sizeof(double) +
                           (bn ? (double)Ncol * sizeof(double) : 0.0));
      }
      if (zin_is_input)
        CK((proj_columns<TIn>(st, (int32_t)rows, (int32_t)r, (int32_t)Ncol, (const TIn*)zin, vz, Ui.p, Ui.ld, out,
                              vout, bn, nullptr, pp, e0, e1)));
      else
        CK((proj_columns<double>(st, (int32_t)rows, (int32_t)r, (int32_t)Ncol, (const double*)zin, vz, Ui.p, Ui.ld,
                                 out, vout, bn, nullptr, pp, e0, e1)));
    } else {
      if (zin_is_input)
        CK((gemm<TIn, TIn, double>(st, (int32_t)r, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0, Ui.p,
                                   transposed(row_major(Ui.ld)), (const TIn*)zin, vz, 0.0, (const TIn*)nullptr,
                                   View(), out, vout, 0, nullptr, bn, gw, pp)));
      else
        CK((gemm<double, double, double>(st, (int32_t)r, (int32_t)Ncol, (int32_t)rows, (int32_t)rows, 1.0, Ui.p,
                                         transposed(row_major(Ui.ld)), (const double*)zin, vz, 0.0,
                                         (const double*)nullptr, View(), out, vout, 0, nullptr, bn, gw, pp)));
    }
    // per-column energies of R = Z - U C (eq:ithresidual) in reduced precision
    if (resid) {
      if (zin_is_input)
        CK((gemm<double, TIn, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r, (int32_t)std::max<int64_t>(r, 1),
                                      -1.0, Ui.p, row_major(Ui.ld), out, vout, 1.0, (const TIn*)zin, vz,
                                      (double*)nullptr, View(), 0, cp, nullptr, gw, pp)));
      else
        CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r,
                                         (int32_t)std::max<int64_t>(r, 1), -1.0, Ui.p, row_major(Ui.ld), out, vout,
                                         1.0, (const double*)zin, vz, (double*)nullptr, View(), 0, cp, nullptr, gw,
                                         pp)));
      CK(frame_sums(st, cp, MB, Ncol, (int32_t)cols, (int32_t)N, fres_p, fsl_p));
      CK(accumulate(st, err2_out, fres_p, N));
    }
    if (bn) CK(frame_sums(st, bn, 1, Ncol, (int32_t)cols, (int32_t)N, y2p, fsl_p));
    zin = out;
    zin_is_input = false;
  }
  if (tele) CK(telescope(st, (int32_t)N, (int32_t)rks[d], coef_out, coef_ld, y2p, err2_out));
  if (nonfinite && y2_out) {
    CK(total_sum(st, y2_out, N, hs + 2));
    CKS(sync_scalars(4));
    *nonfinite = (hs[3] != 0.0 || !isfinite(hs[2])) ? 1 : 0;
  }
  return TTICE_OK;
}

template <typename TIn>
int ttice_state::update_impl(const TIn* batch, int64_t N, ttice_update_info* info) {
  struct InUpdate {
    bool& f;
    ~InUpdate() { f = false; }
  } in_scope{in_update};
  in_update = true;
  hipStream_t st = stream;
  CKS(ensure(z[0], (size_t)N * P * sizeof(double)));
  CKS(ensure(z[1], (size_t)N * P * sizeof(double)));
  CKS(ensure(scal, 64 * sizeof(double)));
  CKS(gemm_ws());
  CKS(grow_core(Gt, n_total + N, std::max<int64_t>(rk[d], 1), n_total, rk[d]));

  int64_t rkp[TTICE_MAX_D + 1];
  for (int i = 0; i <= d; ++i) rkp[i] = rk[i];

  if (algo == TTICE_ALG_PLAIN) {
    if (info) info->eps_upd = eps;
    CKS(core_loop<TIn>(batch, N, nullptr, -1.0, rkp, info, false, nullptr, 0));
    if (info) {
      double a = 0.0;
      for (int i = 0; i < d; ++i) a += info->tail2[i];
      info->achieved2 = a;
    }
  } else {
    // Algorithm 2: relative errors with the existing cores (eq:relerror).
    // They decide the skip and the subset D (the eps guarantee of the
    // stored tensors), so they come from an FP64 chain in every precision:
    // each step is an orthogonal projection and the residual energy of a
    // tensor is the telescoping difference ||Y(b)||^2 - ||c(b)||^2, with no
    // residual formed at any level.  (The coefficients it leaves in the
    // last core are those of a skipped increment.)
    CKS(ensure(e2acc, (size_t)N * sizeof(double)));
    CKS(ensure(fy2, (size_t)N * sizeof(double)));
    CKS(ensure(dlist, (size_t)N * sizeof(int32_t)));
    int nonfinite = 0;
    CKS(chain_project<TIn>(batch, N, rkp, Gt.p + n_total * Gt.ld, Gt.ld, as<double>(e2acc), as<double>(fy2),
                           &nonfinite, nullptr, kProjFP64));
    if (nonfinite) return TTICE_EINVAL;
    CK(star_decide(st, (int32_t)N, as<double>(e2acc), as<double>(fy2), eps, as<int32_t>(dlist),
                   hs));
    CKS(sync_scalars(7));
    const double mean_rel = hs[0], batch_rel = hs[1], sdc = hs[2], nd2 = hs[3];
    const int64_t nD = (int64_t)hs[4];
    const double ny2 = hs[5];
    if (info) {
      info->norm_y2 = ny2;
      info->achieved2 = -1.0;
      for (int i = 0; i < d; ++i) {
        info->r_new[i] = 0;
        info->rho2[i] = std::numeric_limits<double>::quiet_NaN();
        info->tail2[i] = 0.0;
        info->margin[i] = std::numeric_limits<double>::infinity();
      }
    }
    const bool skip = skip_rule == TTICE_SKIP_MEAN    ? mean_rel <= eps
                      : skip_rule == TTICE_SKIP_BATCH ? batch_rel <= eps
                                                      : false;
    if (skip || nD == 0) {
      // eq:appendupdate: the coefficients already sit in the last core
      if (info) {
        info->skipped = 1;
        info->used = 0;
        info->eps_upd = eps;
        info->eps_core = 0.0;
      }
    } else {
      // eq:subselectheuristic, eq:epsilonmodification
      const double num = std::max(0.0, eps * eps * ny2 - sdc);
      const double eps_upd = sqrt(num / nd2);
      const double tol = eps_upd * sqrt(nd2) / sqrt((double)d);
      if (info) {
        info->used = nD;
        info->eps_upd = eps_upd;
        info->eps_core = tol;
      }
      // the subset's own last-level coefficients are not kept: they go to a
      // work buffer (frame stride prod(dims) bounds any rank r_d)
      CKS(core_loop<TIn>(batch, nD, as<int32_t>(dlist), tol, rkp, info, true,
                         as<double>(z[(d - 1) % 2]), P));
      // pad the last core for the appended directions of core d (zeros for
      // the stored tensors), then re-project the whole batch (Alg. 2 project)
      const int64_t r_old = rk[d], r_new = rkp[d];
      CKS(grow_core(Gt, n_total + N, std::max<int64_t>(r_new, 1), n_total, r_old));
      if (r_new > r_old) CK(zero2d(st, n_total, r_new - r_old, Gt.p + r_old, Gt.ld));
      CKS(chain_project<TIn>(batch, N, rkp, Gt.p + n_total * Gt.ld, Gt.ld, nullptr, nullptr, nullptr, nullptr,
                             proj_prec()));
    }
  }
  CK(hipStreamSynchronize(st));
  if (profile) CKS(prof_resolve());
  // commit
  for (int i = 0; i <= d; ++i) rk[i] = rkp[i];
  n_total += N;
  return TTICE_OK;
}

template <typename TD>
int ttice_state::reconstruct_impl(int64_t first, int64_t count, TD* out) {
  hipStream_t st = stream;
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(count, ((int64_t)1 << 26) / P));
  CKS(ensure(z[0], (size_t)chunk * P * sizeof(double)));
  CKS(ensure(z[1], (size_t)chunk * P * sizeof(double)));
  CKS(gemm_ws());
  for (int64_t f0 = 0; f0 < count; f0 += chunk) {
    const int64_t cnt = std::min(chunk, count - f0);
    // level d-1 input: the last-core rows of the chosen tensors
    View vx;
    vx.rs = 1;
    vx.cs = Gt.ld;
    const double* xin = Gt.p + (first + f0) * Gt.ld;
    for (int i = d - 1; i >= 0; --i) {
      const int64_t rows = rk[i] * dims[i];
      const int64_t cols = this->cols(i);
      const int64_t r = rk[i + 1];
      const int64_t Ncol = cnt * cols;
      if (i == 0) {
        TD* o = out + f0 * P;
        CK((gemm<double, double, TD>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r, (int32_t)std::max<int64_t>(r, 1),
                                     1.0, U[i].p, row_major(U[i].ld), xin, vx, 0.0, (const double*)nullptr,
                                     View(), o, unfolding(cols, P), 0, nullptr, nullptr, gws())));
      } else {
        double* o = as<double>(z[i % 2]);
        CK((gemm<double, double, double>(st, (int32_t)rows, (int32_t)Ncol, (int32_t)r,
                                         (int32_t)std::max<int64_t>(r, 1), 1.0, U[i].p, row_major(U[i].ld), xin,
                                         vx, 0.0, (const double*)nullptr, View(), o, unfolding(cols, P), 0,
                                         nullptr, nullptr, gws())));
        xin = o;
        // next level reads per frame (r_i x cols_{i-1}) = (rk[i]) x (dims[i]*cols)
        vx = unfolding(dims[i] * cols, P);
      }
    }
  }
  CK(hipStreamSynchronize(st));
  return TTICE_OK;
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free projection
// (ttice_project_noalloc): one statically sized array in every device's
// copy of the module.  Host code never uses the array's name as an address
// (on the host it names a stand-in, not device memory): the device address
// is taken once per device, with that device current, by
// hipGetSymbolAddress, and only that address is handed to kernels.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device dev (which must be current).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return TTICE_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return TTICE_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TTICE_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI (the only symbols the library exports)
// ---------------------------------------------------------------------------
#pragma GCC visibility push(default)
extern "C" {

int ttice_create(int32_t d, const int64_t* dims, double eps, ttice_state** out) {
  if (!out) return TTICE_EINVAL;
  *out = nullptr;
  if (d < 1 || d > TTICE_MAX_D || !dims) return TTICE_EINVAL;
  if (!(eps > 0.0 && eps < 1.0)) return TTICE_EINVAL;
  int64_t P = 1;
  for (int i = 0; i < d; ++i) {
    if (dims[i] < 1) return TTICE_EINVAL;
    P *= dims[i];
    if (P >= ((int64_t)1 << 31)) return TTICE_EINVAL;
  }
  ttice_state* s = new (std::nothrow) ttice_state();
  if (!s) return TTICE_ENOMEM;
  s->d = d;
  for (int i = 0; i < d; ++i) s->dims[i] = dims[i];
  s->P = P;
  s->eps = eps;
  s->rk[0] = 1;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return TTICE_EDEVICE;
  }
  void* scr = nullptr;  // once per device: the allocation-free projection's scratch address
  if (scratch_address(s->device, &scr) != TTICE_OK) {
    delete s;
    return TTICE_EDEVICE;
  }
  if (hipHostMalloc((void**)&s->hs, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    s->hs = nullptr;
    delete s;
    return TTICE_ENOMEM;
  }
  // U_1 has n_1 rows from the start (r_0 = 1); others start with 0 rows.
  if (s->grow_core(s->U[0], dims[0], 1, 0, 0) != TTICE_OK) {
    delete s;
    return TTICE_ENOMEM;
  }
  *out = s;
  return TTICE_OK;
}

int ttice_set_option(ttice_state* st, int32_t key, const void* val) {
  if (!st) return TTICE_ESTATE;
  if (!val) return TTICE_EINVAL;
  switch (key) {
    case TTICE_OPT_PREC: {
      const int32_t v = *(const int32_t*)val;
      if (v != TTICE_PREC_FP64 && v != TTICE_PREC_FP32 && v != TTICE_PREC_BF16X3) return TTICE_EINVAL;
      st->prec = v;
      return TTICE_OK;
    }
    case TTICE_OPT_ALGO: {
      const int32_t v = *(const int32_t*)val;
      if (v != TTICE_ALG_PLAIN && v != TTICE_ALG_STAR) return TTICE_EINVAL;
      st->algo = v;
      return TTICE_OK;
    }
    case TTICE_OPT_SKIP_RULE: {
      const int32_t v = *(const int32_t*)val;
      if (v != TTICE_SKIP_MEAN && v != TTICE_SKIP_BATCH && v != TTICE_SKIP_NONE) return TTICE_EINVAL;
      st->skip_rule = v;
      return TTICE_OK;
    }
    case TTICE_OPT_TAU: {
      const double v = *(const double*)val;
      if (!(v > 0.0)) return TTICE_EINVAL;
      st->tau = v;
      return TTICE_OK;
    }
    case TTICE_OPT_STREAM:
      st->stream = *(const hipStream_t*)val;
      return TTICE_OK;
    case TTICE_OPT_SVD: {
      const int32_t v = *(const int32_t*)val;
      if (v < 0 || v > 2) return TTICE_EINVAL;
      st->lz_mode = v;
      return TTICE_OK;
    }
    case TTICE_OPT_PROFILE:
      st->profile = *(const int32_t*)val != 0;
      memset(&st->kstats[0], 0, sizeof(st->kstats[0]));
      st->ev_used = 0;
      st->ev_bytes.clear();
      return TTICE_OK;
    default:
      return TTICE_EINVAL;
  }
}

int ttice_reserve(ttice_state* st, int64_t max_batch) {
  if (!st) return TTICE_ESTATE;
  if (max_batch < 1) return TTICE_EINVAL;
  if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
  const size_t np = (size_t)max_batch * (size_t)st->P * sizeof(double);
  // level buffers, the residual and the level-1 column energies grow with the
  // batch; the column partials are sized for level 1 (one row per 64-row
  // block of its rows) and grow on demand at later levels
  CKS(st->ensure(st->z[0], np));
  CKS(st->ensure(st->z[1], np));
  CKS(st->ensure(st->rbuf, np));
  CKS(st->ensure(st->scal, 64 * sizeof(double)));
  CKS(st->gemm_ws());
  CKS(st->ensure(st->bnorm, (size_t)max_batch * st->cols(0) * sizeof(double)));
  CKS(st->ensure(st->colpart, (size_t)gemm_row_blocks((int32_t)st->dims[0]) * (size_t)max_batch * st->cols(0) *
                                  sizeof(double)));
  CKS(st->ensure(st->fres, (size_t)max_batch * sizeof(double)));
  CKS(st->ensure(st->fy2, (size_t)max_batch * sizeof(double)));
  CK(hipStreamSynchronize(st->stream));
  return TTICE_OK;
}

}  // extern "C"
#pragma GCC visibility pop

namespace {
// ttice_update with the state's level-1 mode set to l1_mode for its duration
int update_entry(ttice_state* st, const void* batch, int64_t n, int32_t dtype, ttice_update_info* info,
                 int l1_mode) {
  if (!st) return TTICE_ESTATE;
  if (n < 0 || (n > 0 && !batch)) return TTICE_EINVAL;
  if (dtype != TTICE_F32 && dtype != TTICE_F64) return TTICE_EINVAL;
  if (n * st->P >= ((int64_t)1 << 31)) return TTICE_EINVAL;  // 32-bit column indices
  struct ModeScope {
    ttice_state* s;
    ~ModeScope() { s->l1_mode = 0; }
  } scope{st};
  st->l1_mode = l1_mode;
  ttice_update_info local;
  ttice_update_info* inf = info ? info : &local;
  memset(inf, 0, sizeof(*inf));
  inf->d = st->d;
  inf->n = n;
  inf->used = n;
  inf->eps_upd = st->eps;
  int rc = TTICE_OK;
  if (n > 0) {
    if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
    rc = (dtype == TTICE_F32) ? st->update_impl<float>((const float*)batch, n, inf)
                              : st->update_impl<double>((const double*)batch, n, inf);
    if (rc == kL1Captured || rc == kL1Plain) return rc;  // nothing launched but allocations and padding
    if (rc != TTICE_OK) {
      (void)hipStreamSynchronize(st->stream);
      (void)hipGetLastError();
      st->ev_used = 0;
      st->ev_bytes.clear();
    }
  }
  inf->n_total = st->n_total;
  for (int i = 0; i <= st->d; ++i) inf->ranks[i] = st->rk[i];
  inf->ranks[st->d + 1] = 1;
  return rc;
}
}  // namespace

#pragma GCC visibility push(default)
extern "C" {
int ttice_update(ttice_state* st, const void* batch, int64_t n, int32_t dtype, ttice_update_info* info) {
  return update_entry(st, batch, n, dtype, info, 0);
}
}  // extern "C"
#pragma GCC visibility pop

// ---- serving hooks (server.hip; internal to the library)
namespace ttice {

void serve_mark(ttice_state* st) { st->served = true; }

void serve_limit(ttice_state* st, int64_t max_tensors) {
  int64_t rb[TTICE_MAX_D + 1];
  serve_rank_bounds(st->d, st->dims, max_tensors, rb);
  for (int i = 0; i < st->d; ++i) {
    st->U[i].max_rows = rb[i] * st->dims[i];
    st->U[i].max_cols = rb[i + 1];
  }
  st->Gt.max_rows = max_tensors;
  st->Gt.max_cols = rb[st->d];
}

void serve_rank_bounds(int32_t d, const int64_t* dims, int64_t T, int64_t* rb) {
  // r_i <= min(n_1 ... n_i, n_{i+1} ... n_d T): the ranks of the unfoldings of
  // the (d + 1)-way array of all T tensors; r_d <= min(prod(dims), T)
  double left = 1.0, P = 1.0;
  for (int i = 0; i < d; ++i) P *= (double)dims[i];
  rb[0] = 1;
  for (int i = 0; i < d; ++i) {
    left *= (double)dims[i];
    const double b = std::min(left, P / left * (double)T);
    rb[i + 1] = (int64_t)std::min(b, 9.0e18);
  }
}

int serve_capture(ttice_state* st, const void* batch, int64_t n, int32_t dtype, ProjDesc* desc, int32_t* key) {
  if (!st || st->algo != TTICE_ALG_PLAIN || st->d < 2 || n <= 0) return 0;
  if (update_entry(st, batch, n, dtype, nullptr, 1) != kL1Captured) return 0;  // errors: ttice_update reports them
  *desc = st->l1_desc;
  *key = st->l1_key;
  return 1;
}

int serve_update_after(ttice_state* st, const void* batch, int64_t n, int32_t dtype, ttice_update_info* info) {
  return update_entry(st, batch, n, dtype, info, 2);
}

hipError_t serve_group_launch(hipStream_t s, int32_t key, const ProjGroup& g) {
  const bool f32 = (key & 1) != 0;
  const int prec = (key >> 1) % 3;
  return f32 ? proj_group<float>(s, prec, g) : proj_group<double>(s, prec, g);
}

}  // namespace ttice

#pragma GCC visibility push(default)
extern "C" {

int ttice_reconstruct(ttice_state* st, int64_t first, int64_t count, void* out, int32_t dtype) {
  if (!st) return TTICE_ESTATE;
  if (first < 0 || count < 0 || first + count > st->n_total) return TTICE_EINVAL;
  if (dtype != TTICE_F32 && dtype != TTICE_F64) return TTICE_EINVAL;
  if (count == 0) return TTICE_OK;
  if (!out) return TTICE_EINVAL;
  if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
  int rc = (dtype == TTICE_F32) ? st->reconstruct_impl<float>(first, count, (float*)out)
                                : st->reconstruct_impl<double>(first, count, (double*)out);
  if (rc != TTICE_OK) (void)hipGetLastError();
  return rc;
}

int ttice_project(ttice_state* st, const void* batch, int64_t n, int32_t dtype, double* coef,
                  double* err2, double* y2) {
  if (!st) return TTICE_ESTATE;
  if (n < 0 || (n > 0 && (!batch || !coef))) return TTICE_EINVAL;
  if (dtype != TTICE_F32 && dtype != TTICE_F64) return TTICE_EINVAL;
  if (n == 0) return TTICE_OK;
  if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
  int rc = st->ensure(st->z[0], (size_t)n * st->P * sizeof(double));
  if (rc == TTICE_OK) rc = st->ensure(st->z[1], (size_t)n * st->P * sizeof(double));
  if (rc == TTICE_OK) rc = st->ensure(st->scal, 64 * sizeof(double));
  if (rc == TTICE_OK) rc = st->gemm_ws();
  int nonfinite = 0;
  if (rc == TTICE_OK) {
    const int64_t rd = std::max<int64_t>(st->rk[st->d], 1);
    rc = (dtype == TTICE_F32) ? st->chain_project<float>((const float*)batch, n, st->rk, coef, rd, err2, y2,
                                                         y2 ? &nonfinite : nullptr, nullptr, st->proj_prec())
                              : st->chain_project<double>((const double*)batch, n, st->rk, coef, rd, err2, y2,
                                                          y2 ? &nonfinite : nullptr, nullptr, st->proj_prec());
  }
  if (rc == TTICE_OK && hipStreamSynchronize(st->stream) != hipSuccess) rc = TTICE_EDEVICE;
  if (rc == TTICE_OK && nonfinite) rc = TTICE_EINVAL;
  if (rc != TTICE_OK) (void)hipGetLastError();
  return rc;
}

int ttice_project_noalloc(ttice_state* st, const void* batch, int64_t n, int32_t dtype, double* coef,
                          double* err2, double* y2) {
  if (!st) return TTICE_ESTATE;
  if (n < 0 || (n > 0 && (!batch || !coef))) return TTICE_EINVAL;
  if (dtype != TTICE_F32 && dtype != TTICE_F64) return TTICE_EINVAL;
  if (n == 0) return TTICE_OK;
  if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
  void* base = nullptr;
  if (scratch_address(st->device, &base) != TTICE_OK) return TTICE_EDEVICE;
  // carve the scratch (256-byte aligned pieces): level buffers, column
  // energies and partials, frame sums, product counters, then the rest for
  // K-split partials
  const int32_t d = st->d;
  int64_t cpmax = 1;
  if (err2) {
    for (int i = 0; i < d; ++i) {
      const int64_t rows = st->rk[i] * st->dims[i], Ncol = n * st->cols(i);
      cpmax = std::max<int64_t>(cpmax, (int64_t)gemm_row_blocks((int32_t)rows) * Ncol);
    }
  }
  const double nd = (double)n;
  const double need_d = 2.0 * nd * (double)st->P + nd * (double)st->cols(0) + (double)cpmax + 2.0 * nd +
                        nd * kFrameSlicesMax + (double)(kTileCounters / 2) + 7.0 * 32.0;
  if (need_d * sizeof(double) > (double)kScratchBytes) return TTICE_ESCRATCH;
  double* p = (double*)base;
  auto take = [&](int64_t count) {
    double* q = p;
    p += ((count + 31) / 32) * 32;
    return q;
  };
  ttice_state::ChainWs cw;
  cw.z[0] = take(n * st->P);
  cw.z[1] = take(n * st->P);
  cw.bnorm = take(n * st->cols(0));
  cw.colpart = take(cpmax);
  cw.fres = take(n);
  cw.fsl = take(n * kFrameSlicesMax);
  cw.y2 = take(n);
  int* cnt = (int*)take(kTileCounters / 2);
  const int64_t rest = (int64_t)(kScratchBytes / sizeof(double)) - (int64_t)(p - (double*)base);
  cw.g = GemmWs{p, std::max<int64_t>(rest, 0), cnt, kTileCounters};
  // the arrival counters of K-split products start at zero (a fill kernel,
  // not a memset: callers may capture this call)
  int rc = zero2d(st->stream, 1, kTileCounters / 2, (double*)cnt, kTileCounters / 2) == hipSuccess ? TTICE_OK
                                                                                             : TTICE_EDEVICE;
  int nonfinite = 0;
  if (rc == TTICE_OK) {
    const int64_t rd = std::max<int64_t>(st->rk[d], 1);
    rc = (dtype == TTICE_F32) ? st->chain_project<float>((const float*)batch, n, st->rk, coef, rd, err2, y2,
                                                         y2 ? &nonfinite : nullptr, &cw, st->proj_prec())
                              : st->chain_project<double>((const double*)batch, n, st->rk, coef, rd, err2, y2,
                                                          y2 ? &nonfinite : nullptr, &cw, st->proj_prec());
  }
  if (rc == TTICE_OK && hipStreamSynchronize(st->stream) != hipSuccess) rc = TTICE_EDEVICE;
  if (rc == TTICE_OK && nonfinite) rc = TTICE_EINVAL;
  if (rc != TTICE_OK) (void)hipGetLastError();
  return rc;
}

int ttice_get_kernel_stats(const ttice_state* st, int32_t kernel, struct ttice_kernel_stats* out) {
  if (!st) return TTICE_ESTATE;
  if (!out || kernel != TTICE_KERNEL_PROJ_L1) return TTICE_EINVAL;
  *out = st->kstats[kernel];
  return TTICE_OK;
}

int ttice_ranks(const ttice_state* st, int64_t* ranks, int64_t* n_total) {
  if (!st) return TTICE_ESTATE;
  if (!ranks) return TTICE_EINVAL;
  for (int i = 0; i <= st->d; ++i) ranks[i] = st->rk[i];
  ranks[st->d + 1] = 1;
  if (n_total) *n_total = st->n_total;
  return TTICE_OK;
}

int ttice_get_core(ttice_state* st, int32_t i, double* out, int64_t* rows, int64_t* cols) {
  if (!st) return TTICE_ESTATE;
  if (i < 0 || i > st->d) return TTICE_EINVAL;
  int64_t r, c;
  const Core* core;
  if (i < st->d) {
    r = st->rk[i] * st->dims[i];
    c = st->rk[i + 1];
    core = &st->U[i];
  } else {
    r = st->n_total;
    c = st->rk[st->d];
    core = &st->Gt;
  }
  if (rows) *rows = r;
  if (cols) *cols = c;
  if (!out || r == 0 || c == 0) return TTICE_OK;
  if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
  hipError_t e = hipMemcpy2DAsync(out, c * sizeof(double), core->p, core->ld * sizeof(double),
                                  c * sizeof(double), r, hipMemcpyDeviceToDevice, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return status_of(e);
}

// ---- Checkpoint image (the cores are the compressed store: a state is its
// options, ranks, cores and last core).  Layout, host byte order:
//   magic (8 bytes), d, prec, algo, skip_rule (int32 each), eps, tau
//   (double), n_total (int64), dims[d], ranks r_0..r_d (int64 each), the d
//   cores U_i packed row-major ((r_{i-1} n_i) x r_i doubles), the last core
//   transposed (n_total x r_d doubles), and the FNV-1a hash (uint64) of all
//   bytes before it.
}  // extern "C"
namespace {
constexpr char kImageMagic[8] = {'T', 'T', 'I', 'C', 'E', 'i', 'm', '1'};

uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

size_t image_header_bytes(int32_t d) { return 8 + 4 * 4 + 2 * 8 + 8 + 8 * (size_t)d + 8 * (size_t)(d + 1); }

// bytes of the whole image for dims/ranks, or 0 when it would overflow
size_t image_bytes(int32_t d, const int64_t* dims, const int64_t* rk, int64_t n_total) {
  double total = (double)image_header_bytes(d) + 8.0;
  for (int i = 0; i < d; ++i) total += 8.0 * (double)rk[i] * (double)dims[i] * (double)rk[i + 1];
  total += 8.0 * (double)n_total * (double)rk[d];
  if (total > 9.0e15) return 0;
  return (size_t)total;
}
}  // namespace
extern "C" {

int ttice_save(ttice_state* st, void* buf, int64_t cap, int64_t* size) {
  if (!st) return TTICE_ESTATE;
  if (!size) return TTICE_EINVAL;
  const int32_t d = st->d;
  const size_t need = image_bytes(d, st->dims, st->rk, st->n_total);
  if (need == 0) return TTICE_EINVAL;
  *size = (int64_t)need;
  if (!buf) return TTICE_OK;
  if (cap < (int64_t)need) return TTICE_EINVAL;
  if (hipSetDevice(st->device) != hipSuccess) return TTICE_EDEVICE;
  unsigned char* b = (unsigned char*)buf;
  size_t o = 0;
  auto put = [&](const void* v, size_t n) {
    memcpy(b + o, v, n);
    o += n;
  };
  put(kImageMagic, 8);
  put(&st->d, 4);
  put(&st->prec, 4);
  put(&st->algo, 4);
  put(&st->skip_rule, 4);
  put(&st->eps, 8);
  put(&st->tau, 8);
  put(&st->n_total, 8);
  put(st->dims, 8 * (size_t)d);
  put(st->rk, 8 * (size_t)(d + 1));
  hipError_t e = hipSuccess;
  for (int i = 0; i < d && e == hipSuccess; ++i) {
    const int64_t rows = st->rk[i] * st->dims[i], cols = st->rk[i + 1];
    if (rows > 0 && cols > 0)
      e = hipMemcpy2DAsync(b + o, cols * sizeof(double), st->U[i].p, st->U[i].ld * sizeof(double),
                           cols * sizeof(double), rows, hipMemcpyDeviceToHost, st->stream);
    o += (size_t)rows * cols * sizeof(double);
  }
  const int64_t rd = st->rk[d];
  if (e == hipSuccess && st->n_total > 0 && rd > 0)
    e = hipMemcpy2DAsync(b + o, rd * sizeof(double), st->Gt.p, st->Gt.ld * sizeof(double), rd * sizeof(double),
                         st->n_total, hipMemcpyDeviceToHost, st->stream);
  o += (size_t)st->n_total * rd * sizeof(double);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return status_of(e);
  }
  const uint64_t h = fnv1a(b, o);
  put(&h, 8);
  return o == need ? TTICE_OK : TTICE_EDEVICE;
}

int ttice_load(const void* buf, int64_t size, ttice_state** out) {
  if (!out) return TTICE_EINVAL;
  *out = nullptr;
  if (!buf || size < (int64_t)image_header_bytes(1) + 8) return TTICE_EINVAL;
  const unsigned char* b = (const unsigned char*)buf;
  if (memcmp(b, kImageMagic, 8) != 0) return TTICE_EINVAL;
  int32_t d, prec, algo, skip;
  double eps, tau;
  int64_t n_total;
  memcpy(&d, b + 8, 4);
  memcpy(&prec, b + 12, 4);
  memcpy(&algo, b + 16, 4);
  memcpy(&skip, b + 20, 4);
  memcpy(&eps, b + 24, 8);
  memcpy(&tau, b + 32, 8);
  memcpy(&n_total, b + 40, 8);
  if (d < 1 || d > TTICE_MAX_D || size < (int64_t)image_header_bytes(d) + 8) return TTICE_EINVAL;
  int64_t dims[TTICE_MAX_D], rk[TTICE_MAX_D + 1];
  memcpy(dims, b + 48, 8 * (size_t)d);
  memcpy(rk, b + 48 + 8 * (size_t)d, 8 * (size_t)(d + 1));
  // the shape rules every state satisfies: r_0 = 1 and orthonormal columns
  // (r_i <= r_{i-1} n_i), frames >= 0, options in range
  if (n_total < 0 || rk[0] != 1) return TTICE_EINVAL;
  // the dims' bounds of ttice_create first, so that r_{i-1} n_i below stays
  // far from overflow (r_i <= prod(dims) < 2^31 by induction)
  int64_t P = 1;
  for (int i = 0; i < d; ++i) {
    if (dims[i] < 1 || dims[i] >= ((int64_t)1 << 31)) return TTICE_EINVAL;
    P *= dims[i];
    if (P >= ((int64_t)1 << 31)) return TTICE_EINVAL;
  }
  for (int i = 0; i < d; ++i)
    if (rk[i + 1] < 0 || rk[i + 1] > rk[i] * dims[i]) return TTICE_EINVAL;
  if (prec != TTICE_PREC_FP64 && prec != TTICE_PREC_FP32 && prec != TTICE_PREC_BF16X3) return TTICE_EINVAL;
  if (algo != TTICE_ALG_PLAIN && algo != TTICE_ALG_STAR) return TTICE_EINVAL;
  if (skip != TTICE_SKIP_MEAN && skip != TTICE_SKIP_BATCH && skip != TTICE_SKIP_NONE) return TTICE_EINVAL;
  if (!(tau > 0.0 && tau < 1e300)) return TTICE_EINVAL;
  const size_t need = image_bytes(d, dims, rk, n_total);
  if (need == 0 || (int64_t)need != size) return TTICE_EINVAL;
  uint64_t h;
  memcpy(&h, b + need - 8, 8);
  if (h != fnv1a(b, need - 8)) return TTICE_EINVAL;

  ttice_state* s = nullptr;
  int rc = ttice_create(d, dims, eps, &s);  // checks eps and the dims' product
  if (rc != TTICE_OK) return rc;
  s->prec = prec;
  s->algo = algo;
  s->skip_rule = skip;
  s->tau = tau;
  size_t o = image_header_bytes(d);
  hipError_t e = hipSuccess;
  for (int i = 0; i < d && rc == TTICE_OK; ++i) {
    const int64_t rows = rk[i] * dims[i], cols = rk[i + 1];
    rc = s->grow_core(s->U[i], std::max<int64_t>(rows, 1), std::max<int64_t>(cols, 1), 0, 0);
    if (rc == TTICE_OK && rows > 0 && cols > 0) {
      e = hipMemcpy2DAsync(s->U[i].p, s->U[i].ld * sizeof(double), b + o, cols * sizeof(double),
                           cols * sizeof(double), rows, hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) rc = status_of(e);
    }
    o += (size_t)rows * cols * sizeof(double);
  }
  const int64_t rd = rk[d];
  if (rc == TTICE_OK) rc = s->grow_core(s->Gt, std::max<int64_t>(n_total, 1), std::max<int64_t>(rd, 1), 0, 0);
  if (rc == TTICE_OK && n_total > 0 && rd > 0) {
    e = hipMemcpy2DAsync(s->Gt.p, s->Gt.ld * sizeof(double), b + o, rd * sizeof(double), rd * sizeof(double),
                         n_total, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = status_of(e);
  }
  if (rc != TTICE_OK) {
    (void)hipGetLastError();
    ttice_destroy(s);
    return rc;
  }
  for (int i = 0; i <= d; ++i) s->rk[i] = rk[i];
  s->n_total = n_total;
  *out = s;
  return TTICE_OK;
}

int ttice_shape(const ttice_state* st, int32_t* d, int64_t* dims, double* eps) {
  if (!st) return TTICE_ESTATE;
  if (d) *d = st->d;
  if (dims)
    for (int i = 0; i < st->d; ++i) dims[i] = st->dims[i];
  if (eps) *eps = st->eps;
  return TTICE_OK;
}

void ttice_destroy(ttice_state* st) {
  if (!st) return;
  (void)hipSetDevice(st->device);
  (void)hipStreamSynchronize(st->stream);
  delete st;
}

const char* ttice_strerror(int code) {
  switch (code) {
    case TTICE_OK: return "ok";
    case TTICE_EINVAL: return "invalid argument or non-finite input";
    case TTICE_ENOMEM: return "out of memory";
    case TTICE_EDEVICE: return "HIP device or launch error";
    case TTICE_ESTATE: return "invalid state";
    case TTICE_ESCRATCH: return "request exceeds the fixed scratch of the allocation-free call";
    default: return "unknown status";
  }
}

}  // extern "C"
#pragma GCC visibility pop
