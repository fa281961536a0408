/*
 * icpcg.h — C ABI of an MI355X (gfx950) library for incomplete-Cholesky
 * preconditioned conjugate gradients on sparse symmetric positive definite
 * matrices.
 *
 * The problem follows Li, Wang, Wang, "Deep Learning-Enhanced Preconditioning
 * for Efficient Conjugate Gradient Solvers in Large-Scale PDE Systems":
 *   - solve A x = b, A sparse SPD (Introduction);
 *   - preconditioner P = L L^T with L lower triangular on the pattern of
 *     tril(A) (Model Architecture section, IC(0); supplementary section 2);
 *     L comes from icpcg_factor() or from the caller (for example a learned
 *     correction L = L_IC + GNN(A), Eq. (2));
 *   - PCG iteration of supplementary Algorithm 1, stopped on the relative
 *     residual (Evaluation Metrics section);
 *   - P-time (factor) and CG-time (solve) are separate calls (supplementary
 *     section 2, total time T_p + l * t_cg).
 *
 * Conventions for every call
 *   - Matrices are CSR: row_ptr int64[n+1] (row_ptr[0] = 0), col int32[nnz]
 *     strictly ascending inside each row, values in the stated type. Every
 *     row stores its diagonal. A lower factor keeps its diagonal last in each
 *     row.
 *   - Multi-column blocks (nrhs columns) are row-major n x nrhs: entry (i, k)
 *     at i * nrhs + k. One column is a plain vector.
 *   - Every matrix, vector and block pointer is a DEVICE pointer owned by the
 *     caller; the caller keeps it alive until the call returns. Handles are
 *     owned by the library and released by the matching *_destroy call.
 *   - All work is enqueued on the context's HIP stream. Calls that return
 *     information (icpcg_factor, icpcg_solve, icpcg_tril_nnz, ...) synchronize
 *     that stream before returning; pure kernels (icpcg_spmv, icpcg_apply,
 *     icpcg_apply_backward, icpcg_trsv) return without synchronizing.
 *   - Errors are reported as status codes; nothing aborts or throws across the
 *     boundary. icpcg_last_error() gives a message for the last failing call on
 *     a context.
 *   - A context is not thread-safe; use one per host thread.
 *
 * Tuning knobs (environment, read when a context is created or a kernel is
 * first chosen; the defaults are the measured best on MI355X):
 *   ICPCG_TRSV_WAVES_PER_CU  cap on the resident waves per CU of the
 *                            triangular solves (default: all that fit; for
 *                            16 columns with an FP32 / BF16 factor at most
 *                            about 2.8 supernode levels' worth, e.g. 16 at
 *                            100^3; a value above what fits means all that
 *                            fit)
 *   ICPCG_SPMVG_SLOTS        entry slots per row group of the grouped SpMV
 *                            (16 or 32; default 32 below 8 columns, else 16)
 *   ICPCG_SPMVG_ITERS        row groups per lane group and block of the grouped
 *                            SpMV (default 1, 1, 2, 8, 1 at 1, 2, 4, 8, 16
 *                            columns)
 *   ICPCG_SPMV_SLOTS         entry slots per row of the plain SpMV (default 16)
 *   ICPCG_NO_ROW_GROUPS      when set, analysed matrices use the plain SpMV
 *   ICPCG_IC0_SYNC_FREE      when set to a nonzero integer, icpcg_factor runs
 *                            each shift attempt as one sync-free launch
 *                            instead of one launch per level of tril(A) (same
 *                            bits; slower on the elasticity workloads)
 *   ICPCG_FUSE_RZ            0: the backward solve of a PCG step never forms
 *                            r^T z itself (a separate pass does, as for FP64
 *                            factors and one column); default 1 (fused for
 *                            FP32 / BF16 factors on 2-16 columns)
 *   ICPCG_FUSE_XR            0: a PCG step updates x and r (x += alpha p,
 *                            r -= alpha w, ||r||^2) in a pass of its own;
 *                            default 1: for FP32 / BF16 factors on 2-16
 *                            columns the next step's forward solve applies the
 *                            update ahead of its solve (same values; ||r||^2
 *                            summed in another order)
 *   ICPCG_WAIT_LIMIT_US      time limit of one device-side dependency wait
 *                            (default 4 s); a wait that reaches it gives up,
 *                            the kernel finishes with a NaN in that place and
 *                            the call (or the next icpcg_sync) reports
 *                            ICPCG_E_DEVICE
 */
#ifndef ICPCG_H
#define ICPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ICPCG_OK = 0,
  ICPCG_E_INVALID = 1,       /* bad argument or malformed matrix */
  ICPCG_E_PIVOT = 2,         /* IC(0) pivot <= 0 after all allowed shifts */
  ICPCG_E_BREAKDOWN = 3,     /* PCG: r^T z <= 0 or p^T A p <= 0 */
  ICPCG_E_MAXITER = 4,       /* PCG: iteration cap reached (x is the last iterate) */
  ICPCG_E_NONFINITE = 5,     /* PCG: NaN or Inf met */
  ICPCG_E_DEVICE = 6,        /* HIP runtime error or device-side wait limit hit */
  ICPCG_E_NOMEM = 7,         /* device allocation failed */
  ICPCG_E_TRUE_RESIDUAL = 8  /* recurrence converged but ||b - A x|| stayed above
                                rtol ||b|| after the allowed residual replacements */
} icpcg_status;

/* Storage / arithmetic precision of the factor when it is applied. */
typedef enum {
  ICPCG_F64 = 0,  /* FP64 values, FP64 arithmetic */
  ICPCG_F32 = 1,  /* FP32 values (round-to-nearest-even of FP64), FP32 arithmetic */
  ICPCG_BF16 = 2  /* bfloat16 values (RNE of the FP32 copy), FP32 arithmetic */
} icpcg_dtype;

/* A square CSR matrix with FP64 values (device pointers). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t *row_ptr;
  const int32_t *col;
  const double *val;
} icpcg_csr;

typedef struct icpcg_ctx icpcg_ctx;    /* stream, workspace, device properties */
typedef struct icpcg_mat icpcg_mat;    /* A with its row-group analysis */
typedef struct icpcg_gnn icpcg_gnn;    /* A prepared for the learned factor correction */
typedef struct icpcg_prec icpcg_prec;  /* L, L^T, schedules, reduced-precision copies */

/* ---------------------------------------------------------------- context */

/* Create a context bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL means the null stream). */
icpcg_status icpcg_create(icpcg_ctx **ctx, void *hip_stream);
icpcg_status icpcg_destroy(icpcg_ctx *ctx);
/* Rebind the context to another stream of the same device. */
icpcg_status icpcg_set_stream(icpcg_ctx *ctx, void *hip_stream);
const char *icpcg_last_error(const icpcg_ctx *ctx);
const char *icpcg_status_string(icpcg_status st);

/* -------------------------------------------------------------- factor */

/* Number of stored entries of tril(A) (diagonal included, explicit zeros
 * counted): the size of the factor buffers icpcg_factor() fills. */
icpcg_status icpcg_tril_nnz(icpcg_ctx *ctx, const icpcg_csr *A, int64_t *nnz_lower);

typedef struct {
  int max_restarts;    /* shifts tried after alpha = 0 (default 30 when < 0) */
  double alpha_min;    /* first nonzero shift (default 1e-3 when <= 0) */
} icpcg_factor_opts;

typedef struct {
  double alpha;        /* shift used: factor of A + alpha diag(A) */
  int restarts;        /* number of shifted restarts */
  double min_pivot;    /* smallest squared pivot of the successful attempt */
  int64_t nlevels;     /* steps of the row schedule of tril(A): supernode level
                          x 3 + position in the supernode (empty steps included) */
} icpcg_factor_info;

/* IC(0): lower L on the pattern of tril(A) with (L L^T)_ij = A_ij on that
 * pattern (Model Architecture section; zero fill). Computed in FP64 on the
 * GPU, one wave per row, one launch per step of tril(A)'s row schedule (rows
 * ordered by the level of their supernode, then their position in it), or one
 * sync-free launch per shift attempt (see ICPCG_IC0_SYNC_FREE); the result does
 * not depend on the schedule. A pivot that is not > 0 restarts on
 * A + alpha diag(A) with alpha = 0, alpha_min, 2 alpha_min, 4 alpha_min, ...
 * (the paper uses IC(0) as a black box; this global shift is this library's
 * rule). Outputs L_row_ptr[n+1], L_col[nnz_lower], L_val[nnz_lower] (caller
 * buffers sized by icpcg_tril_nnz). opts and info may be NULL.
 * Errors: ICPCG_E_INVALID (malformed A, row of tril(A) longer than 1024),
 * ICPCG_E_PIVOT (every shift failed; L holds the last attempt, with NaN or
 * pending entries where that attempt stopped), ICPCG_E_DEVICE (a dependency
 * wait reached its time limit). */
icpcg_status icpcg_factor(icpcg_ctx *ctx, const icpcg_csr *A, int64_t *L_row_ptr,
                          int32_t *L_col, double *L_val, const icpcg_factor_opts *opts,
                          icpcg_factor_info *info);

/* ------------------------------------------------------- preconditioner */

/* Build a preconditioner from a lower-triangular CSR factor L (any lower
 * pattern with a stored, positive diagonal; values FP64). The library copies
 * what it needs (transpose L^T, supernode schedules, the FP32 or BF16 copy
 * when apply_dtype asks for one), so L's buffers may be released afterwards.
 * Errors: ICPCG_E_INVALID (not lower triangular, unsorted, missing or
 * non-positive diagonal, non-finite value). */
icpcg_status icpcg_prec_create(icpcg_ctx *ctx, const icpcg_csr *L, icpcg_dtype apply_dtype,
                               icpcg_prec **P);

typedef enum {
  ICPCG_PREC_FACTOR = 0,  /* P = L L^T (icpcg_prec_create) */
  ICPCG_PREC_JACOBI = 1,  /* P = diag(A): z_i = r_i / a_ii (Baseline Methods, Table 1) */
  ICPCG_PREC_NONE = 2     /* P = I: plain CG (Table 1) */
} icpcg_prec_kind;

/* The baselines of Table 1 as preconditioners for icpcg_solve: Jacobi keeps
 * a copy of A's diagonal (which must be stored and positive); none keeps only
 * n. They apply in FP64; calls that need a triangular factor (trsv, apply,
 * apply_backward, levels, transpose, update_values, gnn_create) reject them
 * with ICPCG_E_INVALID. */
icpcg_status icpcg_prec_create_simple(icpcg_ctx *ctx, const icpcg_csr *A, icpcg_prec_kind kind,
                                      icpcg_prec **P);
icpcg_status icpcg_prec_destroy(icpcg_prec *P);

/* Fill-in dropout of Eq. 10 (supplementary Additional Results): every
 * off-diagonal entry of the lower factor L with |l_ij| <= eps becomes a
 * structural zero and is removed; the diagonal is always kept, and kept
 * entries keep their order and values. eps >= 0 is absolute (the caller
 * scales it, e.g. by sqrt(s) to threshold in the network's scaled units).
 * Outputs are caller-owned device buffers sized for L (row_ptr n + 1, col and
 * val nnz(L)); *nnz_out (host) receives the kept count. Synchronizes the
 * stream. Errors: ICPCG_E_INVALID (L not a valid lower factor, eps < 0). */
icpcg_status icpcg_dropout(icpcg_ctx *ctx, const icpcg_csr *L, double eps, int64_t *row_ptr,
                           int32_t *col, double *val, int64_t *nnz_out);

/* Replace the factor's values (same pattern, FP64, CSR order of L) and
 * refresh L^T and the reduced-precision copy. */
icpcg_status icpcg_prec_update_values(icpcg_ctx *ctx, icpcg_prec *P, const double *L_val);

typedef struct {
  int64_t n, nnz;          /* of L */
  int64_t nlevels_L;       /* row levels of forward substitution */
  int64_t nlevels_U;       /* row levels of backward substitution */
  int64_t nsupernodes_L;   /* schedule units of forward substitution */
  int64_t nsupernodes_U;   /* schedule units of backward substitution */
  int64_t nsn_levels_L;    /* dependent steps of the forward schedule */
  int64_t nsn_levels_U;    /* dependent steps of the backward schedule */
  int dtype;               /* icpcg_dtype of application */
  int kind;                /* icpcg_prec_kind (0 for a factor; other kinds report n only) */
} icpcg_prec_info;

icpcg_status icpcg_prec_get_info(icpcg_ctx *ctx, const icpcg_prec *P, icpcg_prec_info *info);

/* Row level sets (supplementary section 5: substitution is sequential row
 * by row; rows of one level are independent). level_L[i] = 0 if row i of L
 * has no off-diagonal entry, else 1 + max level_L[j] over stored j < i;
 * level_U likewise on L^T. perm_* lists rows sorted by (level, row);
 * level_ptr_*[l] .. level_ptr_*[l+1] delimits level l. All outputs are
 * device int32 buffers: level and perm sized n, level_ptr sized nlevels + 1
 * (nlevels from icpcg_prec_get_info). Any pointer may be NULL. */
icpcg_status icpcg_prec_levels(icpcg_ctx *ctx, const icpcg_prec *P, int32_t *level_L,
                               int32_t *perm_L, int32_t *level_ptr_L, int32_t *level_U,
                               int32_t *perm_U, int32_t *level_ptr_U);

/* L^T as CSR (diagonal first in each row): U_row_ptr[n+1], U_col[nnz],
 * U_val[nnz] FP64 device buffers. */
icpcg_status icpcg_prec_transpose(icpcg_ctx *ctx, const icpcg_prec *P, int64_t *U_row_ptr,
                                  int32_t *U_col, double *U_val);

/* ------------------------------------------------------------ kernels */

/* W = A X for nrhs columns (supplementary Algorithm 1, w = A p). X, W are
 * FP64 n x nrhs blocks. */
icpcg_status icpcg_spmv(icpcg_ctx *ctx, const icpcg_csr *A, const double *X, double *W,
                        int64_t nrhs);

/* One triangular solve with the preconditioner's factor: transpose = 0
 * solves L Y = R (forward substitution), 1 solves L^T Y = R (backward),
 * Eq. (11) read as standard substitution. R and Y are n x nrhs blocks of
 * FP64 (dtype F64 preconditioner) or FP32 (F32/BF16 preconditioner), except
 * that the forward solve of a reduced-precision preconditioner takes FP64 R
 * when r_is_f64 = 1 (rounded to FP32 on load). */
icpcg_status icpcg_trsv(icpcg_ctx *ctx, const icpcg_prec *P, int transpose, const void *R,
                        int r_is_f64, void *Y, int64_t nrhs);

/* Preconditioner solve P Z = R, P = L L^T (supplementary Algorithm 1, the two
 * triangle solves): Y = L^-1 R, Z = L^-T Y. Blocks are FP64 for an F64
 * preconditioner and FP32 otherwise (R may be FP64 with r_is_f64 = 1). Y is
 * kept for icpcg_apply_backward and may not be NULL. */
icpcg_status icpcg_apply(icpcg_ctx *ctx, const icpcg_prec *P, const void *R, int r_is_f64,
                         void *Y, void *Z, int64_t nrhs);

/* The preconditioner solve as a PCG step runs it (supplementary Algorithm 1:
 * the two triangle solves, then r^T z for beta): Y = L^-1 R and Z = L^-T Y
 * with R an FP64 block, Y and Z in the factor's block type (FP64, or FP32 for
 * an FP32 / BF16 factor, R rounded to FP32 on load), and rz[k] = sum_i
 * R_ik Z_ik accumulated in FP64 for every column k (rz: device, nrhs FP64
 * values). For FP32 / BF16 factors on 2-16 columns the backward solve forms
 * r^T z from the rows it publishes (the fused form icpcg_solve uses; see
 * ICPCG_FUSE_RZ); otherwise a separate pass over R and Z does. The sum order
 * is fixed by the launch shape (deterministic). Uses the context's reduction
 * workspace; stream-ordered. Errors: ICPCG_E_INVALID, ICPCG_E_NOMEM. */
icpcg_status icpcg_apply_rz(icpcg_ctx *ctx, const icpcg_prec *P, const double *R, void *Y, void *Z,
                            double *rz, int64_t nrhs);

/* The backward half of icpcg_apply_rz alone, as a PCG step launches it
 * (supplementary Algorithm 1: the solve with L^T, then r^T z for beta): Z =
 * L^-T Y and rz[k] = sum_i R_ik Z_ik (FP64). Y and Z are blocks of the
 * factor's type (FP64, or FP32 for an FP32 / BF16 factor), R is FP64, all
 * n x nrhs. Like icpcg_trsv it first fills Z with the marker its dependency
 * waits poll (a PCG step re-arms z in its p update instead). r^T z is fused
 * into the solve for FP32 / BF16 factors on 2-16 columns (see
 * ICPCG_FUSE_RZ), else a separate pass forms it. Uses the context's reduction
 * workspace; stream-ordered. Errors: ICPCG_E_INVALID, ICPCG_E_NOMEM. */
icpcg_status icpcg_trsv_rz(icpcg_ctx *ctx, const icpcg_prec *P, const void *Y, const double *R, void *Z,
                           double *rz, int64_t nrhs);

/* icpcg_apply_rz for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results (bit for bit) as icpcg_apply_rz, but the
 * reduction partials live in a static device array of the library (65,536
 * FP64 values, 512 KiB per GPU, held until the process ends) instead of the
 * context's workspace, and the call makes no allocation of any kind. The
 * array's address is taken when a context is created (icpcg_create, with its
 * device current). Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two contexts, two threads) race and must be
 * ordered by the caller. Stream-ordered, no synchronization; a dependency
 * wait that reaches its time limit is reported by the next icpcg_sync on the
 * context. Errors: ICPCG_E_INVALID (bad arguments, or a device with so many
 * CUs that nrhs columns of partials would not fit the array), ICPCG_E_DEVICE
 * (the array's address could not be taken). */
icpcg_status icpcg_apply_rz_noalloc(icpcg_ctx *ctx, const icpcg_prec *P, const double *R, void *Y, void *Z,
                                    double *rz, int64_t nrhs);

/* Reverse-mode derivative of Z = L^-T L^-1 R (not in the paper; what training
 * a learned correction of L needs). Given G = dl/dZ and the Y, Z of the
 * forward call: Ybar = L^-1 G, dR = L^-T Ybar, and for every stored (a, b) of
 * L: dL_val[q] = -sum_k (Z_ak Ybar_bk + dR_ak Y_bk), in L's CSR order. Types
 * follow icpcg_apply (FP64 or FP32 blocks, dL in the same type). Ybar is a
 * caller scratch block of the same shape. */
icpcg_status icpcg_apply_backward(icpcg_ctx *ctx, const icpcg_prec *P, const void *G,
                                  const void *Y, const void *Z, void *Ybar, void *dR,
                                  void *dL_val, int64_t nrhs);

/* ------------------------------------------------------ analyzed matrix */

/* Analyze A once for repeated products: consecutive rows with identical
 * column lists (the rows of one multi-DOF node) form groups of up to 3 that
 * the SpMV reads as a unit (each column index and each gathered x row once
 * per group). The handle keeps A's pointers: A's buffers must stay valid and
 * unchanged while it is used. Errors: ICPCG_E_INVALID (malformed A). */
icpcg_status icpcg_mat_create(icpcg_ctx *ctx, const icpcg_csr *A, icpcg_mat **M);
icpcg_status icpcg_mat_destroy(icpcg_mat *M);

/* W = A X through the row-group kernel (same result as icpcg_spmv up to the
 * order of the additions inside a row). */
icpcg_status icpcg_mat_spmv(icpcg_ctx *ctx, const icpcg_mat *M, const double *X, double *W,
                            int64_t nrhs);

/* ----------------------------------------------------------------- PCG */

typedef struct {
  double rtol;           /* stop when ||r_k|| <= rtol ||b|| (per column) */
  int64_t max_iter;      /* products A p per column; <= 0: min(n, max(10, 10 sqrt n)) */
  int max_replace;       /* true-residual replacements per column (default 3 when < 0) */
  int block_width;       /* columns per pass: 0 = the autotuner's choice (icpcg_autotune),
                            else 1, 2, 4, 8 or 16. A column's iterates round differently
                            at different widths (the order of the additions inside a
                            triangular-solve row follows the lane layout): pass an explicit
                            width for bitwise-reproducible runs across contexts */
  int check_every;       /* host polls the convergence flags every k steps (<= 0: 8); steps
                            queued after every column stopped return at once */
  int use_graph;         /* 1: the check_every steps between two polls are captured once as a
                            hipGraph (on a private stream of the context) and replayed; the
                            graph is kept in the context and reused by later solves while the
                            operands' pointers, sizes and width are unchanged. Same kernels,
                            same order, so the same results as use_graph = 0 */
} icpcg_solve_opts;

typedef struct {
  int64_t iters;         /* products A p performed for this column */
  int replacements;      /* residual replacements performed */
  int status;            /* icpcg_status of this column */
  double relres;         /* recurrence ||r|| / ||b|| at exit */
  double true_relres;    /* ||b - A x|| / ||b|| at exit (FP64) */
} icpcg_col_info;

/* PCG of supplementary Algorithm 1 for nrhs right-hand sides at once
 * (columns advance in lockstep and freeze when they converge; each column is
 * the same iteration as a one-column solve). B is FP64 n x nrhs; X holds x_0
 * on entry and the solution on exit. The stop test is the relative
 * recurrence residual, then the true residual b - A x is checked and, when it
 * is above the tolerance, r is replaced by it and the iteration continues
 * (at most max_replace times). Iterations count the products A p; b = 0
 * gives x = 0 after 0 iterations. info (nullable) receives nrhs entries.
 * Returns the worst column status. opts may be NULL (rtol 1e-8). A is
 * analyzed on each call (see icpcg_mat_create). */
icpcg_status icpcg_solve(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P,
                         const double *B, double *X, int64_t nrhs, const icpcg_solve_opts *opts,
                         icpcg_col_info *info);

typedef struct {
  int block_width;       /* chosen columns per pass */
  double ms_per_step[5]; /* measured time of the step's SpMV and two triangular solves at widths
                            1, 2, 4, 8, 16 (0 where not tried) */
  double ms_per_rhs;     /* the chosen width's step time per column of the nrhs */
} icpcg_tune_info;

/* Block-width autotuner for a multi-RHS solve of nrhs columns with (M, P): it
 * times one step's bandwidth-heavy kernels (both triangular solves with their
 * re-arming, and the SpMV) at every width w in 1, 2, 4, ... up to the
 * smallest power of two >= nrhs (at most 16) on the real operands, and picks
 * the w with the least time for ceil(nrhs / w) passes. The choice is cached in
 * the context per (operands, nrhs); icpcg_solve with block_width = 0 uses it.
 * The timing runs on the context's stream and synchronizes it; the
 * workspace's r, p, w, y and z are overwritten. Errors: ICPCG_E_INVALID,
 * ICPCG_E_NOMEM, ICPCG_E_DEVICE. */
icpcg_status icpcg_autotune(icpcg_ctx *ctx, const icpcg_mat *M, const icpcg_prec *P,
                            int64_t nrhs, icpcg_tune_info *info);

/* icpcg_solve on an analyzed matrix (skips the per-call analysis). */
icpcg_status icpcg_solve_mat(icpcg_ctx *ctx, const icpcg_mat *M, const icpcg_prec *P,
                             const double *B, double *X, int64_t nrhs,
                             const icpcg_solve_opts *opts, icpcg_col_info *info);

/* Per-phase timing of PCG steps (the CG part of supplementary section 2's
 * time model T = T_p + l t_cg, split by phase). With enable != 0 the context
 * records events on its stream at the phase boundaries of the next eager
 * steps (use_graph = 0; graph-replayed steps are not timed), up to 64 steps
 * from the call on; enable = 0 stops recording. icpcg_step_timing_get
 * synchronizes the stream and writes ms[6] (host), the mean over the recorded
 * steps of each phase in ms: the forward solve; the backward solve (with r^T z
 * and beta where the solve forms them, else with their pass); the p update
 * (with the re-arming of y and z); w = A p; p^T w and alpha (empty where the
 * SpMV forms p^T w); the x and r update with ||r|| (empty where the next
 * step's forward solve applies the update, see ICPCG_FUSE_XR; that solve's
 * phase then includes it). *steps (host) receives the number of steps
 * recorded (0: ms all 0): every eager step queued while recording, also those
 * queued after the last column stopped, which return at once. Errors:
 * ICPCG_E_INVALID (null arguments), ICPCG_E_DEVICE. */
icpcg_status icpcg_step_timing(icpcg_ctx *ctx, int enable);
icpcg_status icpcg_step_timing_get(icpcg_ctx *ctx, double *ms, int64_t *steps);

/* ------------------------------------------------ multicolour ordering */

/* A symmetric permutation that exposes parallelism to the triangular solves
 * (the layout direction of supplementary Additional Results). Nodes are the
 * row groups of A (consecutive rows with identical column lists, at most 3);
 * node v (key: SplitMix64(seed + v), then v) takes the smallest colour not
 * used by its neighbours of higher key (neighbours: the nodes of the columns
 * its rows store), which is a proper colouring for a structurally symmetric
 * A. perm (device, n int32, new row -> old row) lists the nodes by (colour,
 * id), each node's rows in order; *ncolours (host) receives the count.
 * Factorizing P A P^T then gives at most (colours x rows per node) row
 * levels. Synchronizes the stream. Errors: ICPCG_E_INVALID (malformed A,
 * more than 256 colours), ICPCG_E_NOMEM. */
icpcg_status icpcg_color_order(icpcg_ctx *ctx, const icpcg_csr *A, uint64_t seed, int32_t *perm,
                               int32_t *ncolours);

/* Block multicolour order (the block variant of the ordering above): the
 * caller partitions the rows into blocks (block: device, n int32, values in
 * [0, nblocks); for instance blocks of mesh nodes, a node's rows in one
 * block). Blocks coupled by a stored entry of A are neighbours; block b takes
 * the smallest colour not used by its neighbours of lower id (sequential first
 * fit in id order; on a grid of blocks numbered like its nodes this gives the
 * 8-colour parity pattern), and perm (device, n int32, new row -> old row)
 * lists the rows by (colour of their block, block, row). Blocks keep the
 * locality of the original order inside them while the colours cut the
 * dependency chains of the triangular solves; *ncolours (host) receives the
 * colour count. Synchronizes the stream. Errors: ICPCG_E_INVALID (malformed
 * A, a block id out of range, more than 256 colours), ICPCG_E_NOMEM. */
icpcg_status icpcg_block_color_order(icpcg_ctx *ctx, const icpcg_csr *A, const int32_t *block,
                                     int32_t nblocks, int32_t *perm, int32_t *ncolours);

/* B = P A P^T (entry (i, j) = A[perm[i], perm[j]]) into caller-owned device
 * buffers (row_ptr n + 1, col and val nnz(A)), rows with ascending columns.
 * Synchronizes the stream. Errors: ICPCG_E_INVALID (perm not a permutation,
 * malformed A). */
icpcg_status icpcg_permute_matrix(icpcg_ctx *ctx, const icpcg_csr *A, const int32_t *perm,
                                  int64_t *row_ptr, int32_t *col, double *val);

/* Row-major n x nrhs FP64 blocks: Y[i] = X[perm[i]] (inverse = 0) or
 * Y[perm[i]] = X[i] (inverse = 1). Stream-ordered; X and Y must not alias. */
icpcg_status icpcg_permute_rows(icpcg_ctx *ctx, const int32_t *perm, int64_t n, int64_t nrhs,
                                const double *X, double *Y, int inverse);

/* ------------------------------------------- learned factor correction */

/* The correction of Eq. 2, L_pred = L_IC + GNN(A), with the network of the
 * Model Architecture section: node features of supplementary Table 2
 * (degree; max, min, mean and variance of the neighbours' degrees; diagonal
 * dominance |a_ii| / sum_j |a_ij|; diagonal decay max_{j != i} |a_ij| / |a_ii|;
 * sin and cos of pi i / n), edge input a_ij / s with s the population
 * standard deviation of tril(A)'s entries, graph normalization of the node
 * features, and three message-passing blocks (supplementary Eqs. 7-9): an
 * edge updater (two layers, hidden 8, tanh) on [e, x_row, x_col], sum and
 * mean aggregation over the edges at a node (an edge counts at both of its
 * nodes, the diagonal once), a node updater (two layers, hidden 8, tanh) on
 * [x, sum, mean]; blocks 2 and 3 take [e_input, e_previous] as edge input.
 * The last block's edge value g gives L = L_IC + sqrt(s) g off the diagonal
 * and L = L_IC exp(g / 2) on it. Everything is FP64.
 *
 * Parameters are one FP64 device vector of icpcg_gnn_num_params() values in
 * this order: normalization alpha[9], gamma[9], beta[9]; then edge block 1,
 * node block 1, edge block 2, node block 2, edge block 3, where an edge block
 * is W1[8][d] (row-major, d = 19 in block 1, 20 after), b1[8], w2[8], b2[1]
 * and a node block is W1[8][11], b1[8], W2[9][8], b2[9]. */
int64_t icpcg_gnn_num_params(void);

/* Prepare A (full symmetric CSR, FP64, device) for the network, with the
 * pattern of P's factor, which must be exactly tril(A)'s. P must be an FP64
 * preconditioner holding L_IC; its values are copied (later updates of P do
 * not change L_IC here) but its pattern arrays are used in place: P, and A's
 * buffers, must outlive G. The handle keeps the activations of its last pass:
 * calls on one handle must not overlap. Errors: ICPCG_E_INVALID (pattern
 * mismatch, P not FP64, tril(A) with zero spread), ICPCG_E_NOMEM. */
icpcg_status icpcg_gnn_create(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P,
                              icpcg_gnn **G);
icpcg_status icpcg_gnn_destroy(icpcg_gnn *G);

/* The network's inputs (device): node features x[n][9] (nullable), edge
 * inputs e[nnz] in the factor's CSR order (nullable); *scale (host, nullable)
 * receives s. */
icpcg_status icpcg_gnn_inputs(icpcg_ctx *ctx, const icpcg_gnn *G, double *x, double *e,
                              double *scale);

/* L_pred values (device, FP64, the factor's CSR order) for parameters theta
 * (device). Stream-ordered. */
icpcg_status icpcg_gnn_forward(icpcg_ctx *ctx, icpcg_gnn *G, const double *theta, double *L_val);

/* Loss of Eq. 5 with one probe z (device, n values, normally +-1, drawn by
 * the caller): ||L L^T z - A z||^2 / ||A z||^2 with L = L_pred(theta), and
 * its gradient with respect to theta. loss (device, 1 value) and grad
 * (device, num_params values) are overwritten, or added to when accumulate
 * is nonzero (to sum over a batch of matrices). Stream-ordered. */
icpcg_status icpcg_gnn_loss_grad(icpcg_ctx *ctx, icpcg_gnn *G, const double *theta,
                                 const double *z, double *loss, double *grad, int accumulate);

/* One Adam step on count FP64 device values: m and v (device) are the
 * moment estimates, t >= 1 the step number (bias corrections 1 - beta^t).
 * theta -= lr * m_hat / (sqrt(v_hat) + eps). Stream-ordered. */
icpcg_status icpcg_adam_step(icpcg_ctx *ctx, double *theta, const double *grad, double *m, double *v,
                             int64_t count, int64_t t, double lr, double beta1, double beta2,
                             double eps);

/* Synchronize the context's stream and report a device-side failure of the
 * non-synchronizing calls (a dependency wait that hit its time limit). */
icpcg_status icpcg_sync(icpcg_ctx *ctx);

/* Library description (static string). */
const char *icpcg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ICPCG_H */
