/*
 * AIFMM CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 reference of the Algebraic Inverse FMM (Gujjula &
 * Ambikasaran, arXiv 2301.12704): uniform 2^d tree (Sec. 2.1), strong
 * admissibility lists (Sec. 2.2), NNCA operators (Sec. 2.3, eq. NCA and the
 * operator table), the extended sparse system (Sec. 3.1), the efficient
 * elimination with one-shot compression and redirection of the accumulated
 * well-separated fill-ins (Sec. 3.2-3.3, Algorithm "Efficient Elimination"),
 * and the back substitution (Sec. 3.4, Algorithm "Back Substitution").
 *
 * Only the test suite, the smoke entry and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP library.
 *
 * Dense ground truth (partial-pivot LU of the full N x N matrix) and a
 * brute-force O(N^2) matvec are included for residual / forward-error checks.
 *
 * Conventions: all matrices are row-major unless stated; b and x are
 * N x nrhs column-major in the caller's original point order.
 */
#ifndef AIFMM_ORACLE_H
#define AIFMM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* kernel kinds: 0 = exp(-r/scale), 1 = 1/sqrt(r^2 + scale^2); shift*delta_ij is added */
void   oracle_kernel_block(const double* pts, int d, int kind, double scale, double shift,
                           const int64_t* rows, int64_t nr, const int64_t* cols, int64_t nc,
                           double* out /* nr x nc row-major */);
/* y = A x (brute force, every entry evaluated), x,y: N x nrhs column-major */
void   oracle_matvec(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                     const double* x, int64_t nrhs, double* y);
/* rows subset: y[r, :] = A[rows[r], :] x   (nsel x nrhs column-major) */
void   oracle_matvec_rows(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                          const int64_t* rows, int64_t nsel, const double* x, int64_t nrhs, double* y);
/* dense partial-pivot LU solve of A X = B (A n x n row-major, B,X n x nrhs column-major);
   returns 0, or 1+k if the k-th pivot is exactly zero */
int    oracle_dense_solve(int64_t n, const double* A, int64_t nrhs, const double* B, double* X);

/* unit pieces, exposed for pin tests */
/* ACA with partial pivoting on an explicit m x n matrix; returns rank k and fills
   I[k], J[k] (pivot rows / cols in pivot order), U (m x k col-major), V (k x n row-major) */
int    oracle_aca(const double* M, int m, int n, double tol, int* I, int* J, double* U, double* V);
/* Householder QR with column pivoting truncated at |R_{k+1,k+1}| <= tol |R_11|;
   returns k; Q gets the first qcols columns of H_1..H_k (m x qcols row-major),
   perm (n) the column order, R (k x n row-major, in pivoted column order) */
int    oracle_cpqr(const double* M, int m, int n, double tol, int qcols, double* Q, int* perm, double* R);

/* full AIFMM */
typedef struct oracle_sys oracle_sys;
oracle_sys* oracle_create(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                          double tol, int leaf_size, int depth);
/* Readings where the paper fixes no operation order or arithmetic routine.  Mode 0 (the
   default) takes the orders the device uses; the flags switch each to its textbook form:
     ORACLE_MODE_STD_EXP     e^x of the exponential kernel from the C library (exp) instead of
                             the Cody-Waite / Taylor routine;
     ORACLE_MODE_ASC_SUMS    row sums of the pivoted QRs and Q formations as one ascending
                             chain instead of sixteen interleaved chains and a tree;
     ORACLE_MODE_ASC_BACK    the pivot-block solve W = Piv^{-1} [rhs] as substitution on the
                             right-hand sides with ascending back substitution, instead of the
                             product of the explicit inverse (formed by substitution on the
                             identity's columns, column-oriented back substitution) with them;
     ORACLE_MODE_SEQUENTIAL  the Algorithm's order box by box (each compression applied in full,
                             then the elimination) instead of colour rounds.
   ORACLE_MODE_TEXTBOOK = all four. */
#define ORACLE_MODE_STD_EXP 1
#define ORACLE_MODE_ASC_SUMS 2
#define ORACLE_MODE_ASC_BACK 4
#define ORACLE_MODE_SEQUENTIAL 8
#define ORACLE_MODE_TEXTBOOK 15
oracle_sys* oracle_create_mode(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                               double tol, int leaf_size, int depth, int mode);
const char* oracle_error(oracle_sys* s);
int    oracle_depth(oracle_sys* s);
int    oracle_box_count(oracle_sys* s, int level, int* nb /* 2^(d*level) */);   /* n_b (x size) */
int    oracle_nnca_ranks(oracle_sys* s, int level, int* k);                   /* k_b from NNCA */
int    oracle_final_ranks(oracle_sys* s, int level, int* k);                  /* k_b at elimination */
int    oracle_xsize(oracle_sys* s, int level, int* n);                         /* n_b at elimination */
int    oracle_pivots(oracle_sys* s, int level, int box, int64_t* t_i, int64_t* s_i); /* returns k */
int    oracle_perm(oracle_sys* s, int64_t* perm);
/* NNCA interpolation operator of a box, |T_B| x k_B row-major; returns |T_B| */
int    oracle_nnca_U(oracle_sys* s, int level, int box, double* out);   /* tree order -> original index */
int    oracle_elim_order(oracle_sys* s, int level, int* order);
/* dense extended matrix before elimination (small problems only). Writes dim into *dim;
   if out != NULL fills the dim x dim matrix and xcols[N] = column of x_m for original point m */
int    oracle_dense_extended(oracle_sys* s, int64_t* dim, double* out, int64_t* xcols);
/* NNCA-based H^2 product y = A~ x with the system's NNCA operators at its tolerance (P2M,
   M2M, M2L, L2L, L2P over the interaction lists, P2P over the leaf neighbours); x, y: N x nrhs
   column-major, original order.  Valid after create (independent of factor); 0 on success */
int    oracle_h2_matvec(oracle_sys* s, const double* x, int64_t nrhs, double* y);
int    oracle_factor(oracle_sys* s);
int    oracle_solve(oracle_sys* s, const double* b, int64_t nrhs, double* x);
/* compression trace: rows of 4 ints (level, box being eliminated, kind 0=P2P 1=P2L, partner) */
int64_t oracle_trace(oracle_sys* s, int* out, int64_t cap);
/* per compression of the trace: 6 ranks (r1,r2,r3,r4,k_i',k_j' for P2P; r5,r6,0,0,k_i',0 for
   P2L) and 8 decision ratios |R_kk|/(tol |R_11|) (last kept, first rejected) per RRQR */
int64_t oracle_trace_ranks(oracle_sys* s, int* ranks, double* ratio, int64_t cap);
/* number of blocks ever created outside dist_inf <= 2 (must be 0) */
int64_t oracle_far_fill_count(oracle_sys* s);
/* number of compressions that transformed a row (Z by a left factor, Y by a new basis) whose
   right-hand side may already be nonzero (must be 0: compressions never touch the RHS) */
int64_t oracle_rhs_violations(oracle_sys* s);
/* row set T_B of the NNCA of a box (original indices; the box's points at the leaf, the
   children's incoming pivots above); returns |T_B| */
int    oracle_row_set(oracle_sys* s, int level, int box, int64_t* out);
/* the exponential kernel's e^x routine, elementwise */
void   oracle_kexp(const double* x, int64_t n, double* out);
/* N(box) and IL(box) at a level; returns 1000*|N| + |IL| */
int    oracle_lists(oracle_sys* s, int level, int box, int* nbr, int* il);
/* decision margins: min over all CPQR calls of |log(ratio)| where ratio = |R_kk|/(tol|R_11|)
   for the last kept and first rejected pivot; and min ACA argmax relative gap */
void   oracle_margins(oracle_sys* s, double* cpqr_margin, double* aca_stop_margin, double* aca_gap);
/* flop counters: [0]=LU [1]=TRSM [2]=Schur GEMM [3]=RRQR [4]=basis change */
void   oracle_flops(oracle_sys* s, double* f5);
void   oracle_destroy(oracle_sys* s);

#ifdef __cplusplus
}
#endif
#endif
