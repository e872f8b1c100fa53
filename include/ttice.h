/*
 * ttice.h - C ABI of the MI355X (gfx950) TT-ICE library, libttice.so.
 *
 * TT-ICE maintains the tensor-train (TT) decomposition of an accumulation of
 * d-way tensors Y^1, Y^2, ... of size n_1 x ... x n_d that arrive in batches
 * (increments).  Problem statement: Sec. 1, Problem 1 (keep every stored
 * tensor within eps_des relative error, ||Y^l - Yhat^l||_F <= eps_des ||Y^l||_F).
 * Algorithm 1 (TT-ICE, Sec. 3.1) expands the left-orthonormal cores with only
 * the new orthogonal directions a new increment needs; Algorithm 2 (TT-ICE*,
 * Sec. 3.3) adds the skip / subselect heuristics.
 *
 * State: unfolded cores U_i (r_{i-1} n_i x r_i), i = 1..d, r_0 = 1, and the
 * last core G_{d+1} (r_d x N_total) whose column j is the latent vector of the
 * j-th stored tensor (eq:lastcore, eq:last_core_latent).  All ranks start at 0.
 *
 * Conventions
 *  - Every tensor buffer is C-ordered (row-major), mode n_d fastest, frames
 *    outermost: a batch is [N][n_1]...[n_d].
 *  - "device pointer" = memory the HIP device can read/write (hipMalloc'd,
 *    e.g. a torch CUDA tensor's data_ptr()).  The library never frees caller
 *    memory and never keeps a pointer past the call that received it.
 *  - Every call is host-synchronous with respect to the library's stream: on
 *    return, all reads of caller buffers and all writes of outputs are done.
 *  - Status codes are negative on failure.  On ANY failure the state is left
 *    exactly as it was before the call (transactional update).
 *  - A state is not thread-safe: calls on one state must not overlap.
 */
#ifndef TTICE_H
#define TTICE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ttice_state ttice_state;

enum ttice_status {
  TTICE_OK = 0,
  TTICE_EINVAL = -1,  /* bad argument, or a non-finite batch */
  TTICE_ENOMEM = -2,  /* device or host allocation failed */
  TTICE_EDEVICE = -3, /* HIP runtime / kernel launch error */
  TTICE_ESTATE = -4,  /* null or unusable state */
  TTICE_ESCRATCH = -5 /* ttice_project_noalloc: the request needs more than
                         its fixed device scratch (32 MiB) */
};

enum ttice_dtype { TTICE_F32 = 0, TTICE_F64 = 1 };

/* Arithmetic of the level products (eq:first_resid / eq:project_further:
 * C = U_i^T Z_i, the one-pass projection of narrow cores and the large
 * products of wide ones, the new rows U_R^T Z of the next level, in the
 * update loop, in Algorithm 2's projection of the batch after an update and
 * in ttice_project): FP64 (matrix cores, or vector FMAs for unfoldings of at
 * most 8 rows); FP32 with FP32 accumulation; or split BF16 (each operand as
 * hi + lo bf16, the three products hi*hi + hi*lo + lo*hi on BF16 matrix
 * cores, FP32 accumulation).  Everything that decides the eps guarantee is
 * FP64 in all modes: ||Y||; the norm test's residual R = Z - U C~, formed
 * from the rounded coefficients in FP64 (its energy ||R||^2 + ||C~ - C||^2
 * never falls below the exact one); Algorithm 2's relative errors (an FP64
 * chain, by telescoping); the residual's SVD and the re-orthogonalisation.
 * Reconstructions agree with the FP64 path to about 1e-5 relative (FP32) or
 * 3e-4 (split BF16: its operands keep 16 significant bits). */
enum ttice_prec { TTICE_PREC_FP64 = 0, TTICE_PREC_FP32 = 1, TTICE_PREC_BF16X3 = 2 };

/* Algorithm 1 (TT-ICE) or Algorithm 2 (TT-ICE*). */
enum ttice_algo { TTICE_ALG_PLAIN = 0, TTICE_ALG_STAR = 1 };

/* TT-ICE* skip test: mean of the per-tensor relative errors (eq:relerror,
 * the rule Algorithm 2 uses), the batch relative error
 * (eq:batchrelativeerror), or none: never skip, update with the subselected
 * tensors only (the experiments' "Subselect" variant, Sec. 5; an increment
 * whose tensors are all within eps then appends their coefficients without
 * an update).  With tau above 1 the occupancy test never fires: MEAN is then
 * the experiments' "SS" variant, and MEAN with tau = 0.8 the full TT-ICE*. */
enum ttice_skip_rule { TTICE_SKIP_MEAN = 0, TTICE_SKIP_BATCH = 1, TTICE_SKIP_NONE = 2 };

enum ttice_option {
  TTICE_OPT_PREC = 1,      /* int32_t, enum ttice_prec (default FP64)          */
  TTICE_OPT_ALGO = 2,      /* int32_t, enum ttice_algo (default PLAIN)         */
  TTICE_OPT_SKIP_RULE = 3, /* int32_t, enum ttice_skip_rule (default MEAN)     */
  TTICE_OPT_TAU = 4,       /* double, occupancy threshold of Algorithm 2,
                              eq:coreoccupancy (default 1.0: skip only full
                              cores, which cannot gain a direction)            */
  TTICE_OPT_STREAM = 5,    /* hipStream_t passed as (const void*)&stream; all
                              device work of later calls runs on it (default:
                              the null stream)                                 */
  TTICE_OPT_PROFILE = 6,   /* int32_t: 1 = time the kernels listed in enum
                              ttice_kernel with HIP events carried by their
                              launches (start and end of the kernel itself, on
                              the library's stream; setting it resets the
                              counters); 0 = off                               */
  TTICE_OPT_SVD = 7        /* int32_t, solver of the residual's truncated SVD
                              (eq:svdfirst): 1 (default) = residuals whose
                              Gram matrix is wider than 256 and at least
                              twice the Krylov basis (4 blocks of 32 to 128
                              vectors, sized from the core's last r_R) first
                              try block Lanczos for the leading singular
                              pairs (the truncation rank needs only those:
                              the discarded energy is ||R||_F^2 minus their
                              sum), accepted only when the residuals of its
                              Ritz pairs certify the rank and the kept
                              subspace (else once more with twice the block,
                              then the dense eigensolver); 0 = dense only;
                              2 = as 1 for every Gram matrix wider than the
                              basis, blocks from 32 vectors                  */
};

/* Kernels whose launches TTICE_OPT_PROFILE times. */
enum ttice_kernel {
  TTICE_KERNEL_PROJ_L1 = 0 /* fused projection of level 1: one pass over each
                              increment giving U_1^T Y, ||Y(b)||^2 and the
                              residual energy (eq:first_resid); every such
                              launch of an update in the state's precision,
                              Algorithm 2's projections of the whole batch
                              included                                       */
};

/* Accumulated timing of one kernel since profiling was enabled.  bytes is
 * the algorithmic HBM traffic of the launches: the increment read once
 * (n * prod(dims) * sizeof(element)) plus the coefficients written
 * (r_1 * n * n_2...n_d FP64) and the per-column energies the launch writes
 * (n * n_2...n_d FP64 each). */
struct ttice_kernel_stats {
  int64_t launches;
  double total_ms;
  double bytes;
};

#define TTICE_MAX_D 16

/* Per-update report (all arrays indexed by core i = 0..d-1 unless noted). */
struct ttice_update_info {
  int32_t d;
  int32_t skipped;          /* Algorithm 2 took the skip branch               */
  int64_t n;                /* tensors in this increment                        */
  int64_t used;             /* tensors used to update the cores (|D| in Alg. 2) */
  int64_t n_total;          /* stored tensors after the update                  */
  double norm_y2;           /* ||Y||_F^2 of the increment (FP64)                */
  double eps_core;          /* SVD truncation tolerance used at every core      */
  double eps_upd;           /* relaxed relative tolerance (eq:epsilonmodification);
                               equals eps for Algorithm 1                        */
  int64_t ranks[TTICE_MAX_D + 2]; /* r_0 = 1, r_1..r_d, r_{d+1} = 1 after update */
  int64_t r_new[TTICE_MAX_D];     /* directions appended to core i              */
  double rho2[TTICE_MAX_D];       /* ||R_i||_F^2 (NaN when the core was skipped)  */
  double tail2[TTICE_MAX_D];      /* discarded energy ||E_i||_F^2 (eq:svdfirst)  */
  double margin[TTICE_MAX_D];     /* relative distance of the rank decision from
                                     the threshold: min over r in {r_R, r_R - 1}
                                     of |tail(r) - eps_core^2| / eps_core^2      */
  double achieved2;               /* sum_i tail2[i] = ||Y - Yhat||_F^2 for
                                     Algorithm 1 (Theorem 1's proof is a chain of
                                     Pythagorean equalities); -1 for Alg. 2     */
  int32_t solver[TTICE_MAX_D];    /* truncated SVD of core i's residual: 0 none
                                     (norm test passed or core skipped), 1 dense
                                     eigensolver, 2 block Lanczos (TTICE_OPT_SVD) */
};

/* Create an empty accumulation for d-way tensors of size dims[0..d-1] with
 * relative tolerance eps (Corollary 1: per-core tolerance eps ||Y||_F / sqrt(d)).
 * d in [1, TTICE_MAX_D], every dims[i] >= 1, eps in (0, 1), prod(dims) < 2^31.
 * Selects the current HIP device.  *out receives the new state (caller frees
 * it with ttice_destroy).  Errors: EINVAL (bad d/dims/eps/out), ENOMEM. */
int ttice_create(int32_t d, const int64_t* dims, double eps, ttice_state** out);

/* Set an option (enum ttice_option); val points to the value's type above.
 * Options may be changed between updates.  Errors: ESTATE, EINVAL. */
int ttice_set_option(ttice_state* st, int32_t key, const void* val);

/* Incorporate one increment (Algorithm 1, or Algorithm 2 per TTICE_OPT_ALGO).
 * batch: device pointer to n tensors, [n][n_1]...[n_d] C-order, element type
 * dtype (TTICE_F32 or TTICE_F64); read only.  n == 0 is a no-op.
 * info: host pointer or NULL.  Errors: EINVAL (bad args, non-finite batch,
 * or a residual whose SVD (eq:svdfirst) would exceed the eigensolver's size
 * limit: min(r_{i-1} n_i, n * n_{i+1}...n_d) above 4096 at a core that
 * grows), ENOMEM, EDEVICE, ESTATE; the state is unchanged on error. */
int ttice_update(ttice_state* st, const void* batch, int64_t n, int32_t dtype,
                 struct ttice_update_info* info);

/* Allocate now the workspace that increments of up to max_batch tensors
 * use (level buffers, residual, per-column energies, product workspace), so
 * that later ttice_update calls of that size do not allocate it on their
 * critical path.  Optional; the Gram matrix and eigen workspace still grow
 * on demand.  Errors: EINVAL (max_batch < 1), ENOMEM, EDEVICE, ESTATE. */
int ttice_reserve(ttice_state* st, int64_t max_batch);

/* Write the approximations of stored tensors first .. first+count-1
 * (eq:last_core_latent) to out: device pointer, [count][n_1]...[n_d] C-order,
 * element type dtype.  out is written on the state's stream (TTICE_OPT_STREAM)
 * and the call returns once it is written; work the caller still has queued
 * on out's memory on other streams must be complete first.  Errors: EINVAL
 * (range outside [0, n_total), bad dtype, null out with count > 0), ENOMEM,
 * EDEVICE, ESTATE. */
int ttice_reconstruct(ttice_state* st, int64_t first, int64_t count, void* out,
                      int32_t dtype);

/* Latent coefficients of new tensors under the current cores, without
 * updating anything (Sec. 4.1, relative prediction error): coef (device,
 * [n][r_d] FP64) and, if err2 != NULL, per-tensor squared residual
 * ||Y(b) - Ytilde(b)||_F^2 (device, [n] FP64) and, if y2 != NULL, ||Y(b)||_F^2
 * (device, [n] FP64).  Errors as ttice_update. */
int ttice_project(ttice_state* st, const void* batch, int64_t n, int32_t dtype,
                  double* coef, double* err2, double* y2);

/* ttice_project without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, outputs and results as
 * ttice_project (the same kernels); its workspace (level buffers, column
 * energies, K-split partials and counters) lives in one fixed 32 MiB device
 * array of the library, set up once per device when the first state is
 * created on it and held until the process ends.  The cores must already
 * exist (the state's own memory), and the outputs are caller buffers.
 * The workspace needs about (2 n prod(dims) + n n_2...n_d) doubles plus
 * the per-level column partials; a larger request returns TTICE_ESCRATCH
 * and does nothing.  Every call on a device shares that device's array:
 * calls that overlap on one device (any states, any host threads or
 * streams) race and must be serialised by the caller.  Errors: as
 * ttice_project, and TTICE_ESCRATCH. */
int ttice_project_noalloc(ttice_state* st, const void* batch, int64_t n, int32_t dtype,
                          double* coef, double* err2, double* y2);

/* Read the profile of kernel `kernel` (enum ttice_kernel) into *out (host).
 * Errors: ESTATE, EINVAL (unknown kernel or null out). */
int ttice_get_kernel_stats(const ttice_state* st, int32_t kernel, struct ttice_kernel_stats* out);

/* ranks: host array of d+2 entries (r_0 = 1, r_1..r_d, r_{d+1} = 1);
 * n_total: host pointer (may be NULL).  Errors: ESTATE, EINVAL. */
int ttice_ranks(const ttice_state* st, int64_t* ranks, int64_t* n_total);

/* Copy core i to out (device pointer, FP64, compact row-major):
 * i in [0, d): U_{i+1}, shape (r_i n_{i+1}) x r_{i+1};
 * i == d: the last core TRANSPOSED, shape N_total x r_d (row j = latent
 * vector of stored tensor j).  rows/cols (host, may be NULL) receive the
 * shape; out may be NULL to query the shape only.  out is written on the
 * state's stream and the call returns once it is written (the caller's work
 * on out's memory on other streams must be complete first).  Errors: ESTATE,
 * EINVAL, EDEVICE. */
int ttice_get_core(ttice_state* st, int32_t i, double* out, int64_t* rows, int64_t* cols);

/* Checkpoint / resume.  The cores are the compressed store of the stream
 * (the paper's storage argument, Sec. 6): a state is fully described by its
 * options (precision, algorithm, skip rule, tau), eps, dims, ranks, cores
 * and last core, and ttice_save writes exactly these into a host byte image
 * (header, cores packed row-major, last core transposed as for
 * ttice_get_core, and a 64-bit FNV-1a hash of the preceding bytes; host
 * byte order).  Updating a loaded state gives the same cores, bit for bit,
 * as updating the state that was saved.
 *
 * ttice_save: buf is a host buffer of cap bytes; *size (host) receives the
 * image size.  With buf == NULL only the size is returned (OK).  The state
 * is not changed.  Errors: ESTATE (st NULL), EINVAL (size NULL, or cap below
 * the image size: *size still receives it), EDEVICE. */
int ttice_save(ttice_state* st, void* buf, int64_t cap, int64_t* size);

/* ttice_load: a new state on the current device from an image of exactly
 * `size` bytes written by ttice_save; *out receives it (NULL on error).
 * The stream option starts at the default stream, profiling off.  Errors:
 * EINVAL (NULL arguments, wrong magic or size, hash mismatch, a shape no
 * state can have: r_0 != 1, r_i > r_{i-1} n_i, options out of range),
 * ENOMEM, EDEVICE.  The caller owns the state (ttice_destroy). */
int ttice_load(const void* buf, int64_t size, ttice_state** out);

/* Shape of a state (for one built by ttice_load): *d (host, may be NULL),
 * dims (host array of TTICE_MAX_D entries, may be NULL: n_1..n_d written),
 * *eps (host, may be NULL).  Errors: ESTATE. */
int ttice_shape(const ttice_state* st, int32_t* d, int64_t* dims, double* eps);

/* Release the state and all device memory it owns.  NULL is a no-op. */
void ttice_destroy(ttice_state* st);

/* Static description of a status code. */
const char* ttice_strerror(int code);

/* ---- Serving: many independent streams on one device --------------------
 *
 * A server owns a set of TT-ICE states (one per stream, resident in device
 * memory) and `workers` host threads, each with its own HIP stream.
 * Increments submitted to a stream are applied in submission order, one at
 * a time (Algorithm 1, or Algorithm 2 per the stream's options); increments
 * of different streams run concurrently on different workers, so the small,
 * latency-bound launches of one stream's update overlap with other streams'
 * on the device.  A free worker first continues an update whose level-1
 * projection has been made, else takes the stream that has waited longest
 * (continuous, work-conserving scheduling).
 *
 * Grouped launches: when several Algorithm 1 streams are waiting, the worker
 * that takes them makes the level-1 projection of all their increments
 * (eq:first_resid: U_1^T Z, ||z||^2 and the residual energies, the pass over
 * every element of every tensor) in one launch per launch shape, up to 16
 * streams per launch, in each stream's precision; each update then continues
 * on any worker.  A served stream's level 1 always takes that projection
 * with one column per lane, alone or grouped, and every reduction has a
 * fixed order, so a stream alone and the same stream in a mix give
 * bit-identical cores.
 *
 * Admission: each stream reserves a projected footprint for increments of
 * up to max_batch tensors and at most max_tensors tensors in all (level
 * buffers, residual, Gram and eigen workspace, and every core at its rank
 * bound with capacity doubling, the last core at max_tensors rows).  A
 * stream whose reservation exceeds the budget left waits, in order of
 * arrival, and is admitted when ttice_server_remove_stream frees enough;
 * its increments queue meanwhile.  A reservation above the whole budget is
 * refused.
 *
 * Ordering and ownership: a submitted batch (device pointer) is read after
 * all work queued on the producer stream named at submission, and must stay
 * valid and unchanged until its ticket completes.  Tickets are released once
 * their completion has been reported by ttice_server_wait or
 * ttice_server_poll. */
typedef struct ttice_server ttice_server;

/* workers in [1, 64]; budget_bytes > 0; the server runs on the current
 * device.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ttice_server_create(int32_t workers, int64_t budget_bytes, ttice_server** out);

/* New stream of order-d tensors (ttice_create's arguments) with precision
 * prec (enum ttice_prec) and algorithm algo (enum ttice_algo), for
 * increments of at most max_batch tensors and at most max_tensors tensors in
 * all (max_tensors >= max_batch); *stream_id receives its id.  The stream is
 * admitted now or waits for budget (above).  Errors: EINVAL, ENOMEM (state
 * allocation, or a reservation above the whole budget), ESTATE. */
int ttice_server_add_stream(ttice_server* srv, int32_t d, const int64_t* dims, double eps, int32_t prec,
                            int32_t algo, int64_t max_batch, int64_t max_tensors, int32_t* stream_id);

/* Queue an increment (ttice_update's batch, n, dtype) on a stream, ordered
 * after the work queued so far on `producer` (a hipStream_t of the server's
 * device; NULL: the null stream); *ticket receives its id.  Errors: EINVAL
 * (unknown stream, n < 0 or > max_batch, max_tensors exceeded, bad dtype,
 * null batch with n > 0, invalid producer), EDEVICE, ESTATE; a stream whose
 * admission failed returns that status. */
int ttice_server_submit(ttice_server* srv, int32_t stream_id, const void* batch, int64_t n, int32_t dtype,
                        void* producer, int64_t* ticket);

/* *done = 1 when the ticket has completed; then *status receives
 * ttice_update's return code, info (host, may be NULL) its report, and the
 * ticket is released.  Errors: EINVAL (unknown ticket), ESTATE. */
int ttice_server_poll(ttice_server* srv, int64_t ticket, int32_t* done, int32_t* status,
                      struct ttice_update_info* info);

/* Block until the ticket completes; as poll with done = 1. */
int ttice_server_wait(ttice_server* srv, int64_t ticket, int32_t* status, struct ttice_update_info* info);

/* Borrow a stream's state for the read-only calls (ttice_ranks,
 * ttice_reconstruct, ttice_get_core, ttice_project) once its queue has
 * drained; the server keeps ownership.  Errors: EINVAL, ESTATE (stream busy,
 * with queued increments, or not admitted). */
int ttice_server_stream_state(ttice_server* srv, int32_t stream_id, ttice_state** st);

/* Destroy an idle stream (admitted or waiting) and return its reservation,
 * then admit waiting streams that fit.  Errors: EINVAL, ESTATE (busy,
 * queued, or being admitted). */
int ttice_server_remove_stream(ttice_server* srv, int32_t stream_id);

struct ttice_server_counters {
  int64_t reserved_bytes;      /* reservations of admitted streams */
  int64_t budget_bytes;
  int64_t pending;             /* increments queued or running */
  int64_t waiting_streams;     /* streams waiting for admission */
  int64_t groups;              /* grouped level-1 launches made */
  int64_t grouped_increments;  /* increments whose level-1 projection ran in one */
};

/* The server's counters into *out (host).  Errors: EINVAL, ESTATE. */
int ttice_server_stats(ttice_server* srv, struct ttice_server_counters* out);

/* Stop the workers after the increments already running (queued ones are
 * completed with status ESTATE), then destroy every stream.  No other call
 * on the server may run concurrently with (or after) this one.  NULL is a
 * no-op. */
void ttice_server_destroy(ttice_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* TTICE_H */
