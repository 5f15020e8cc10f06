/*
 * aifmm.h — C ABI of the MI355X (gfx950) AIFMM factor/solve library.
 *
 * The library builds, factors and solves the N-body system A x = b of Sec. 2 of
 * Gujjula & Ambikasaran, "Algebraic Inverse Fast Multipole Method" (arXiv 2301.12704):
 * targets u and sources v coincide (the setting of the paper's experiments, Sec. 4), and
 * A_ij = kappa(|p_i - p_j|) + shift * delta_ij for a real, symmetric kernel kappa.
 *
 *   aifmm_build   Sec. 2.1-2.3 and 3.1: tree, lists, NNCA operators, extended sparse system.
 *   aifmm_factor  Sec. 3.2-3.3: level-by-level elimination with one-shot compression and
 *                 redirection of the accumulated well-separated fill-ins (Algorithm
 *                 "Efficient Elimination").
 *   aifmm_solve   Sec. 3.4: RHS Schur operations, level-2 multipole solve, back substitution
 *                 (Algorithm "Back Substitution"); the factor is RHS-independent (remark after
 *                 that algorithm), so solve may be called many times.
 *
 * Every entry point runs its numerical work in hand-written HIP kernels on the device
 * selected in the options; there is no CPU fallback.  All functions return an
 * aifmm_status; no exception crosses the ABI.  aifmm_last_error() gives a message.
 *
 * Layouts
 *   points  N x d, row-major (point-major), FP64, host or device memory.
 *   b, x    N x nrhs, column-major with leading dimension ldb/ldx >= N, FP64, in the caller's
 *           original point order; host or device memory (detected per call).
 * Ownership
 *   aifmm_build copies the points; the system owns all device memory it allocates and
 *   aifmm_destroy frees it.  b and x stay owned by the caller.
 * Threading
 *   One thread per system at a time.  Calls are stream-ordered on opt.stream (NULL = the
 *   default stream) and return after the work has completed.
 */
#ifndef AIFMM_H
#define AIFMM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AIFMM_OK = 0,
  AIFMM_ERR_ARG = 1,       /* invalid argument (null pointer, bad size, bad kernel) */
  AIFMM_ERR_NOMEM = 2,     /* device allocation failed */
  AIFMM_ERR_SINGULAR = 3,  /* exactly singular self-block or top-level system */
  AIFMM_ERR_STATE = 4,     /* call out of order (e.g. solve before factor) */
  AIFMM_ERR_DEVICE = 5,    /* HIP runtime error */
  AIFMM_ERR_NOCONV = 6,    /* iterative refinement did not reach the requested residual */
  AIFMM_ERR_CAPACITY = 7,  /* a rank exceeded its preallocated capacity */
  AIFMM_ERR_BUSY = 8       /* serving: no slot or memory for the request right now */
} aifmm_status;

typedef enum {
  AIFMM_K_EXP = 0,   /* kappa(r) = exp(-r / scale)            */
  AIFMM_K_INVMQ = 1  /* kappa(r) = 1 / sqrt(r^2 + scale^2)    */
} aifmm_kernel_kind;

typedef struct {
  aifmm_kernel_kind kind;
  double scale;  /* > 0 */
  double shift;  /* added on the diagonal */
} aifmm_kernel;

/* Arithmetic of the Schur fill-in updates and of the compressions (RRQRs, bases, basis
 * changes).  The block store, the NNCA, the pivot-block LU, the solves, the matvec and GMRES
 * are FP64 in both.  AIFMM_FP32 is the precision form: an approximate factorization used as
 * the preconditioner of FP64 GMRES (Sec. 4, Exp. 5 uses AIFMM as a preconditioner). */
typedef enum { AIFMM_FP64 = 0, AIFMM_FP32 = 1 } aifmm_precision;

typedef struct {
  int32_t dim;         /* 2 or 3 */
  int32_t leaf_size;   /* n_max: mean points per leaf used by the depth rule (default 64) */
  int32_t depth;       /* 0: L = max(2, ceil(log_{2^d}(N / leaf_size))), else the tree depth */
  int32_t device;      /* HIP device ordinal */
  void* stream;        /* hipStream_t, NULL = default stream */
  int32_t prec;        /* aifmm_precision (default AIFMM_FP64) */
  double matvec_tol;   /* eps_G of the H^2 operator (aifmm_matvec_h2, the operator of aifmm_gmres):
                          0 (default) = the NNCA at tol itself; otherwise aifmm_build also builds a
                          second NNCA of the same tree at this tolerance for the product (Sec. 4:
                          the GMRES products use the NNCA-based H^2 product at tolerance eps_G) */
} aifmm_options;

typedef struct aifmm_system aifmm_system;

/* Fill *opt with defaults (dim 2, leaf 64, depth auto, device 0, default stream, FP64, no
 * separate matvec tolerance). */
aifmm_status aifmm_options_default(aifmm_options* opt);

/* Build the tree (Sec. 2.1), neighbour and interaction lists (Sec. 2.2, eta = sqrt(d)), the
 * NNCA operators with tolerance tol (Sec. 2.3) and the extended system (Sec. 3.1).
 * points: N x opt->dim row-major.  On success *out owns a new system. */
aifmm_status aifmm_build(const double* points, int64_t n, aifmm_kernel kernel, double tol,
                         const aifmm_options* opt, aifmm_system** out);

/* Eliminate levels L..2 with compression of the pending well-separated fill-ins before each
 * box elimination (Algorithm "Efficient Elimination", Sec. 3.3), then factor the level-2
 * multipole system densely.  AIFMM_ERR_SINGULAR names the level and box in the message. */
aifmm_status aifmm_factor(aifmm_system* s);

/* x = (factored A)^{-1} b for nrhs right-hand sides (Sec. 3.4). */
aifmm_status aifmm_solve(aifmm_system* s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): aifmm_solve with b and x in device memory and every
 * work buffer of the solve carved from one fixed scratch array per GPU (64 MiB, a static device
 * array that the GPU holds until the process ends).  No allocation and no graph: only kernel
 * launches and a stream synchronization.  Same layouts and result as aifmm_solve.  Errors:
 * AIFMM_ERR_ARG for a host pointer or bad sizes, AIFMM_ERR_STATE before aifmm_factor,
 * AIFMM_ERR_CAPACITY when N, the tree and nrhs need more scratch than the maximum (about
 * 8 bytes x nrhs x (N + the ranks' and pivot blocks' rows); the message states both sizes).
 * Every call on a GPU shares that GPU's scratch array, which keeps the last call's contents:
 * calls that overlap on one GPU (other systems, other threads or streams) race and must be
 * serialized by the caller. */
aifmm_status aifmm_solve_noalloc(aifmm_system* s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx);

/* y = A x with every kernel entry evaluated in FP64 (exact product, O(N^2) work; used for
 * residuals, and the operator of aifmm_gmres when op is NULL).  Same layouts as aifmm_solve. */
aifmm_status aifmm_matvec(aifmm_system* s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy);

/* y = A~ x with the NNCA-based H^2 product (Sec. 2.3, the operator table: P2M, M2M, M2L, L2L, L2P
 * over the interaction lists of every level, P2P of the leaf neighbours evaluated exactly) at the
 * system's matvec tolerance (opt.matvec_tol, else tol).  Valid after aifmm_build (independent of
 * aifmm_factor).  Same layouts as aifmm_solve.  O(N) work per column. */
aifmm_status aifmm_matvec_h2(aifmm_system* s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy);

/* Solve A x = b to relative residual ||A x - b|| / ||b|| <= rtol for every column with
 * right-preconditioned flexible GMRES(restart) in FP64 (AIFMM as a preconditioner, Sec. 4,
 * Experiment 5): preconditioner the factored system prec (its aifmm_solve), operator the H^2
 * product of op (aifmm_matvec_h2 of op: its NNCA at its matvec tolerance eps_G) or, when op is
 * NULL, prec's exact product (aifmm_matvec).  op may be prec itself (a system built with
 * matvec_tol and factored) or another system built from the same points, kernel and options
 * (AIFMM_ERR_ARG otherwise).  The iteration stops on the operator's residual, recomputed from
 * b - A x at every restart.  With an H^2 operator the result is then checked with the exact
 * product, whose residual the H^2 product's error (about eps_G |A|) hides: while a column's exact
 * residual is above rtol, the exact residual is solved for with the same FGMRES and added (at
 * most three times), so the returned residuals are exact ones.  x is an output (the iteration
 * starts from 0).  iters[nrhs] and relres[nrhs] (may be NULL) receive per-column iteration counts
 * (all FGMRES steps) and final relative residuals under the exact product (op NULL: the
 * operator is the exact product).
 * AIFMM_ERR_NOCONV if some column is above rtol after maxit iterations (x then holds the last
 * iterate).  Calls on the two systems are serialized with their other calls. */
aifmm_status aifmm_gmres(aifmm_system* op, aifmm_system* prec, const double* b, int64_t nrhs, int64_t ldb, double rtol,
                         int32_t restart, int32_t maxit, double* x, int64_t ldx, int32_t* iters, double* relres);

/* Tree depth L. */
aifmm_status aifmm_get_depth(const aifmm_system* s, int32_t* L);
/* Ranks of the 2^(d*level) boxes of a level (2 <= level <= L): the NNCA ranks before
 * factor, the ranks at elimination time after it. */
aifmm_status aifmm_get_ranks(const aifmm_system* s, int32_t level, int32_t* ranks);
/* Statistics, filled into an array of doubles (see AIFMM_STAT_* for the slots). */
enum {
  AIFMM_STAT_BUILD_S = 0, AIFMM_STAT_FACTOR_S = 1, AIFMM_STAT_SOLVE_S = 2,
  AIFMM_STAT_SCHUR_FLOPS = 3,     /* counted Schur-update GEMM flops of the last factor */
  AIFMM_STAT_SCHUR_BYTES = 4,     /* minimum HBM bytes of those GEMMs                 */
  AIFMM_STAT_TRSM_FLOPS = 5, AIFMM_STAT_LU_FLOPS = 6,
  AIFMM_STAT_DEVICE_BYTES = 7,    /* device bytes held by the system                  */
  AIFMM_STAT_SCHUR_KERNEL_S = 8,  /* summed device time of the Schur-update launches (HIP events) */
  AIFMM_STAT_SCHUR_LAUNCHES = 9,
  AIFMM_STAT_COMPRESS_KERNEL_S = 10, /* summed device time of the compression launches */
  AIFMM_STAT_COMPRESS_LAUNCHES = 11,
  AIFMM_STAT_GMRES_S = 12,        /* wall time of the last aifmm_gmres call */
  AIFMM_STAT_TRSM_KERNEL_S = 13,  /* summed device time of the pivot-block solve launches (HIP events) */
  AIFMM_STAT_TRSM_LAUNCHES = 14,
  AIFMM_STAT_SOLVE_BYTES = 15,    /* factor-store bytes the products of one solve read (any nrhs) */
  AIFMM_STAT_COUNT = 16
};
aifmm_status aifmm_get_stats(const aifmm_system* s, double* stats /* AIFMM_STAT_COUNT */);
/* Figures of one level (2 <= level <= L) of the last factorization, into an array of doubles
 * (AIFMM_LSTAT_COUNT slots).  Device times are HIP-event times of the level's launches on the
 * system's stream.  Flop and byte counts are the algorithmic ones of the elimination per box
 * (R coupled rows, C coupled columns, n = x size, m = n + k): Schur update 2 R n C flops and
 * 8 (R n + n C + 2 R C) bytes, pivot-block solve 2 m^2 C (as executed 2 m^2 (C + n): W also holds
 * Piv^{-1}[:, x_b] for the solve phase), pivot-block LU (2/3) m^3; the compressions' pivoted QRs
 * (4 (rows - s)(cols - s) per pivot step s), Q formations (4 rows q rank) and coefficient products.
 * CRIT_STEPS sums over the compression rounds the longest pivot-step chain of the round (the
 * dependent barrier steps), PIVOT_STEPS counts all pivot steps.  AIFMM_ERR_STATE before
 * aifmm_factor. */
enum {
  AIFMM_LSTAT_FACTOR_S = 0, AIFMM_LSTAT_SCHUR_FLOPS = 1, AIFMM_LSTAT_SCHUR_BYTES = 2, AIFMM_LSTAT_TRSM_FLOPS = 3,
  AIFMM_LSTAT_TRSM_FLOPS_IMPL = 4, AIFMM_LSTAT_LU_FLOPS = 5, AIFMM_LSTAT_SCHUR_KERNEL_S = 6,
  AIFMM_LSTAT_TRSM_KERNEL_S = 7, AIFMM_LSTAT_COMPRESS_KERNEL_S = 8, AIFMM_LSTAT_COMPRESS_FLOPS = 9,
  AIFMM_LSTAT_COMPRESSIONS = 10, AIFMM_LSTAT_ROUNDS = 11, AIFMM_LSTAT_CRIT_STEPS = 12, AIFMM_LSTAT_PIVOT_STEPS = 13,
  AIFMM_LSTAT_BOXES = 14, AIFMM_LSTAT_COUNT = 16
};
aifmm_status aifmm_get_level_stats(const aifmm_system* s, int32_t level, double* out /* AIFMM_LSTAT_COUNT */);
/* Decision log of the last factorization (the decision-margin record of the compressions):
 * one record per compression of the static schedule, in launch order.  rec gets 10 ints per
 * compression: level, box i being eliminated, kind (0 = P2P pair (i, j), 1 = P2L pair (r, i)),
 * partner, then the RRQR ranks r1 r2 r3 r4 and the new ranks k_i' k_j' (P2L: r5 r6 0 0 k_i' 0);
 * ratio gets 8 doubles: for each RRQR |R_kk| / (tol |R_11|) of the last kept and of the first
 * rejected pivot (0 when none).  At most cap records are written; *count gets the total.
 * rec / ratio may be NULL.  AIFMM_ERR_STATE before aifmm_factor. */
aifmm_status aifmm_get_trace(const aifmm_system* s, int32_t* rec, double* ratio, int64_t cap, int64_t* count);
/* NNCA output of one box (Sec. 2.3, eq. NCA and the operator table): the k_B incoming pivots
 * t^{B,i} and s^{B,i} as original point indices (arrays of at least k_B, may be NULL), and
 * U_B = A[T_B, s^{B,i}] (A[t^{B,i}, s^{B,i}])^{-1} (rows x k_B row-major, may be NULL) where
 * T_B is the box's points at the leaf and its children's incoming pivots above.  *k and
 * *rows receive k_B and |T_B|.  Valid after aifmm_build. */
aifmm_status aifmm_get_nnca(const aifmm_system* s, int32_t level, int32_t box, int64_t* t_i, int64_t* s_i, double* U,
                            int32_t* k, int32_t* rows);
/* Message of the last error on this system (s != NULL) or of the calling thread (s == NULL). */
const char* aifmm_last_error(const aifmm_system* s);
/* Free every resource of the system; NULL is accepted. */
void aifmm_destroy(aifmm_system* s);

/* Batching: factor n independent built systems (each as aifmm_factor would, with the same
 * results) in lockstep groups of up to `group` systems of one device and precision, taken in
 * order.  A group runs on its first system's stream: step t handles level L_s - t of every
 * system s of the group, and each launch of the step (a round of compressions of the
 * efficient elimination, Sec. 3.3, its basis changes, the elimination phases of a colour,
 * Sec. 3.2) carries the work of all of the group's systems, so many small systems fill the
 * device together.  Groups run one after another; each system's own stream is restored.
 * A failure fails its whole group (every system of it reports the error through
 * aifmm_last_error); returns AIFMM_OK or the first failing status.  AIFMM_ERR_ARG for NULL,
 * n <= 0, group <= 0 or a system listed twice; AIFMM_ERR_STATE if one is already factored. */
aifmm_status aifmm_factor_batch(aifmm_system* const* systems, int32_t n, int32_t group);

/* ---- Serving: resident factorizations, continuously batched solve requests ----------------
 * The factorization does not depend on the right-hand side (Sec. 3.4: the solve reuses the
 * stored factors), so factored systems stay on the device and answer any number of requests.
 * Each system gets a worker thread and a stream of its own (its previous stream is restored by
 * aifmm_server_destroy); requests for a system that arrive while a batch of it runs are merged,
 * FIFO and up to max_cols right-hand sides, into its next batch; batches of different systems
 * run concurrently.  Memory admission charges what the systems hold: each system's right-hand-
 * side workspaces stay allocated at the size of its largest batch and are charged to hbm_budget
 * while it is resident (0 = 90% of the free device memory at creation plus what the systems
 * already hold).  A batch needs the growth of its system's workspaces (estimated as N x cols x
 * 8 bytes x (8 + 60 when rtol > 0), less what the system holds); it is admitted when that
 * growth fits in the device's free memory, read at every decision, and in the budget next to
 * everything charged (a batch with no other batch running may exceed the budget).  When the
 * growth does not fit in the free memory and no other batch runs, the batch's requests
 * complete with AIFMM_ERR_BUSY (aifmm_server_wait returns it; x is left unchanged) and may be
 * submitted again.  rtol > 0 solves every
 * request to that relative residual with flexible GMRES(30) preconditioned by the factors
 * (aifmm_gmres with the system's own operator: its H^2 product when it was built with a
 * matvec tolerance, else the exact product); rtol = 0 uses the direct solve (aifmm_solve).  While served, the systems
 * must not be used through other calls.
 * Errors: AIFMM_ERR_ARG (NULL, nsys <= 0, a system listed twice, max_cols <= 0, rtol < 0),
 * AIFMM_ERR_STATE (a system not factored), AIFMM_ERR_DEVICE (stream creation failed). */
typedef struct aifmm_server aifmm_server;
aifmm_status aifmm_server_create(aifmm_system* const* systems, int32_t nsys, size_t hbm_budget, double rtol,
                                 int32_t max_cols, aifmm_server** out);
/* Queue a request: b is N x nrhs column-major in the system's original point order, host
 * memory, copied before the call returns (1 <= nrhs <= max_cols, ldb >= N).  *ticket
 * identifies it for aifmm_server_wait.  AIFMM_ERR_STATE once the server is shutting down. */
aifmm_status aifmm_server_submit(aifmm_server* srv, int32_t sys, const double* b, int64_t nrhs, int64_t ldb,
                                 int64_t* ticket);
/* Block until the request is done and copy its solution to x (host, N x nrhs, ldx >= N).
 * *latency_s gets submission-to-completion seconds, *batch_cols the right-hand sides of the
 * batch that served it, iters / relres (nrhs entries each) the GMRES iterations and final
 * relative residuals (0 for direct solves); each may be NULL.  Returns the status of that
 * batch's solve.  A ticket is waited for once, by one thread. */
aifmm_status aifmm_server_wait(aifmm_server* srv, int64_t ticket, double* x, int64_t ldx, double* latency_s,
                               int32_t* batch_cols, int32_t* iters, double* relres);
/* Batches run so far, requests they served, and the peak charged device bytes (the systems'
 * retained right-hand-side workspaces plus admitted growth). */
aifmm_status aifmm_server_stats(aifmm_server* srv, int64_t* batches, int64_t* requests, size_t* peak_bytes);
/* Finish the queued requests, stop the workers and restore the systems' streams. */
void aifmm_server_destroy(aifmm_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* AIFMM_H */
