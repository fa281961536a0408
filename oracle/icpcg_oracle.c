/*
 * Plain, slow, sequential FP64 CPU reference of the IC(0)-preconditioned
 * conjugate gradient path. TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the benchmark's CPU-baseline leg use it to judge the GPU library;
 * the GPU library never calls, links or includes it, and it shares no code,
 * header or table with the GPU library.
 *
 * Source of every step (Li, Wang, Wang, "Deep Learning-Enhanced
 * Preconditioning for Efficient Conjugate Gradient Solvers in Large-Scale PDE
 * Systems"):
 *   - PCG loop ..................... supplementary Algorithm 1 (IC-PCG)
 *   - P = L L^T, forward/backward
 *     substitution .................. supplementary section 2 and Eq. (11)
 *   - IC(0): L on the pattern of
 *     tril(A), no fill-in ........... Model Architecture section; Eq. (2)
 *   - relative-residual stop ....... Evaluation Metrics section
 * Readings where the paper is silent or garbled are stated at each function.
 *
 * Conventions: CSR with int64 row pointers, int32 column indices ascending in
 * every row, FP64 values. Triangular factors store the diagonal in every row:
 * last in a lower row, first in an upper row. Every sum runs sequentially in
 * ascending index order (inner products with compensation, see orc_dot).
 * Build with -ffp-contract=off (no fused multiply-add)
 * and without fast-math so each operation is one IEEE-754 rounding.
 *
 * Threads: the product A x and the element-wise vector updates of the PCG
 * loop split their rows over OpenMP threads (every output element is still
 * computed by the same sequential code, so results do not depend on the
 * thread count); inner products, the factorization and the triangular solves
 * are sequential.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_PIVOT 2
#define ORC_BREAKDOWN 3
#define ORC_MAXITER 4
#define ORC_NONFINITE 5
#define ORC_TRUE_RESIDUAL 8

/* ---------------------------------------------------------------- basics */

/* w = A x, row by row, ascending column order (sparse matrix-vector product
 * of supplementary Algorithm 1). */
void orc_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *x, double *w) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) s += v[q] * x[ci[q]];
    w[i] = s;
  }
}

/* Threads used by the row-parallel loops (<= 0 leaves the OpenMP default). */
void orc_set_threads(int t) {
  if (t > 0) omp_set_num_threads(t);
}

int orc_max_threads(void) { return omp_get_max_threads(); }

/* Inner product sum_i a_i b_i (the r^T z, p^T w and ||r||^2 of supplementary
 * Algorithm 1). The paper fixes no summation order; the products are summed in
 * ascending index order with Neumaier's compensation, so the result is close
 * to the exactly rounded inner product (plain running sums over 1e5+ terms
 * carry enough error to move the iteration at which CG crosses the
 * tolerance). */
double orc_dot(int64_t n, const double *a, const double *b) {
  double s = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double x = a[i] * b[i];
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  return s + c;
}

/* Checks the CSR invariants the solver relies on: row pointers
 * non-decreasing, columns in range and strictly ascending, a stored diagonal.
 * Returns ORC_OK or ORC_INVALID. */
int orc_check_csr(int64_t n, const int64_t *rp, const int32_t *ci) {
  if (rp[0] != 0) return ORC_INVALID;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return ORC_INVALID;
    int has_diag = 0;
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
      if (ci[q] < 0 || ci[q] >= n) return ORC_INVALID;
      if (q > rp[i] && ci[q] <= ci[q - 1]) return ORC_INVALID;
      if (ci[q] == i) has_diag = 1;
    }
    if (!has_diag) return ORC_INVALID;
  }
  return ORC_OK;
}

/* Number of stored entries of tril(A) (structural: explicit zeros count). */
int64_t orc_tril_nnz(int64_t n, const int64_t *rp, const int32_t *ci) {
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
      if (ci[q] <= i) ++c;
  return c;
}

/* tril(A): the pattern IC(0) keeps (no fill-in, Model Architecture section). */
void orc_tril(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              int64_t *lrp, int32_t *lci, double *lv) {
  int64_t c = 0;
  lrp[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
      if (ci[q] <= i) {
        lci[c] = ci[q];
        if (lv) lv[c] = v[q];
        ++c;
      }
    lrp[i + 1] = c;
  }
}

/* U = L^T in CSR by a stable counting sort on the column index: row j of U
 * lists the rows i >= j with a stored L_ij, ascending (diagonal first). */
void orc_transpose(int64_t n, const int64_t *lrp, const int32_t *lci, const double *lv,
                   int64_t *urp, int32_t *uci, double *uv) {
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t q = 0; q < lrp[n]; ++q) cnt[lci[q] + 1]++;
  urp[0] = 0;
  for (int64_t j = 0; j < n; ++j) urp[j + 1] = urp[j] + cnt[j + 1];
  for (int64_t j = 0; j < n; ++j) cnt[j] = urp[j];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = lrp[i]; q < lrp[i + 1]; ++q) {
      int64_t d = cnt[lci[q]]++;
      uci[d] = (int32_t)i;
      if (uv) uv[d] = lv[q];
    }
  free(cnt);
}

/* ---------------------------------------------------------------- IC(0) */

/* Incomplete Cholesky with zero fill on the pattern S of the lower factor:
 * the lower L on S with (L L^T)_ij = A_ij for every (i, j) in S, computed row by
 * row ("up-looking"): for each stored j < i in ascending order
 *     L_ij = (A_ij - sum_{k in S(i) and S(j), k < j} L_ik L_jk) / L_jj
 * and then L_ii = sqrt(A_ii - sum_{k < i} L_ik^2). The diagonal is read as
 * A_ii + alpha * A_ii (the shifted matrix A + alpha diag(A)).
 * On entry lv holds the values of tril(A) on S (diagonal unshifted); on exit the
 * factor. A squared pivot that is not > 0 stops the factorization: returns
 * ORC_PIVOT and the failing row. min_pivot receives the smallest squared pivot
 * seen. */
int orc_ic0(int64_t n, const int64_t *lrp, const int32_t *lci, double *lv, double alpha,
            int64_t *fail_row, double *min_pivot) {
  double mp = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t rs = lrp[i], re = lrp[i + 1];
    if (re <= rs || lci[re - 1] != i) return ORC_INVALID;
    for (int64_t q = rs; q < re - 1; ++q) {
      const int32_t j = lci[q];
      double s = lv[q];
      /* merge the prefix of row i (positions rs..q-1, columns < j) with row j
         without its diagonal (columns < j) */
      int64_t a = rs, b = lrp[j];
      const int64_t be = lrp[j + 1] - 1;
      while (a < q && b < be) {
        if (lci[a] == lci[b]) { s -= lv[a] * lv[b]; ++a; ++b; }
        else if (lci[a] < lci[b]) ++a;
        else ++b;
      }
      lv[q] = s / lv[be];
    }
    double d = lv[re - 1] + alpha * lv[re - 1];
    for (int64_t q = rs; q < re - 1; ++q) d -= lv[q] * lv[q];
    if (d < mp) mp = d;
    if (!(d > 0.0)) {
      if (fail_row) *fail_row = i;
      if (min_pivot) *min_pivot = mp;
      return ORC_PIVOT;
    }
    lv[re - 1] = sqrt(d);
  }
  if (min_pivot) *min_pivot = mp;
  return ORC_OK;
}

/* IC(0) with a global diagonal shift on breakdown (reading of "diagonal shift
 * on nonpositive pivots": the paper treats IC(0) as a black box). Try alpha = 0;
 * while a pivot fails, restart from tril(A) with alpha <- max(1e-3, 2 alpha), at
 * most max_restarts times. Returns the status; alpha and restart count out. */
int orc_ic0_shifted(int64_t n, const int64_t *arp, const int32_t *aci, const double *av,
                    int64_t *lrp, int32_t *lci, double *lv, int max_restarts,
                    double *alpha_out, int *restarts_out, double *min_pivot) {
  orc_tril(n, arp, aci, av, lrp, lci, lv);
  const int64_t nnzl = lrp[n];
  double *a0 = (double *)malloc((size_t)nnzl * sizeof(double));
  memcpy(a0, lv, (size_t)nnzl * sizeof(double));
  double alpha = 0.0;
  int st = ORC_PIVOT, r = 0;
  for (r = 0; r <= max_restarts; ++r) {
    if (r > 0) {
      alpha = alpha * 2.0 > 1e-3 ? alpha * 2.0 : 1e-3;
      memcpy(lv, a0, (size_t)nnzl * sizeof(double));
    }
    int64_t fr = -1;
    st = orc_ic0(n, lrp, lci, lv, alpha, &fr, min_pivot);
    if (st != ORC_PIVOT) break;
  }
  free(a0);
  if (alpha_out) *alpha_out = alpha;
  if (restarts_out) *restarts_out = r > max_restarts ? max_restarts : r;
  return st;
}

/* ---------------------------------------------------------------- levels */

/* Level of each row of a lower-triangular pattern: 0 without off-diagonal
 * entries, else 1 + the largest level among the stored columns j < i. Rows of
 * one level are independent in forward substitution. Returns the count. */
int64_t orc_levels_lower(int64_t n, const int64_t *lrp, const int32_t *lci, int32_t *level) {
  int32_t mx = -1;
  for (int64_t i = 0; i < n; ++i) {
    int32_t l = 0;
    for (int64_t q = lrp[i]; q < lrp[i + 1]; ++q) {
      const int32_t j = lci[q];
      if (j < i && level[j] + 1 > l) l = level[j] + 1;
    }
    level[i] = l;
    if (l > mx) mx = l;
  }
  return (int64_t)mx + 1;
}

/* Level of each row of U = L^T for backward substitution, from L's pattern:
 * 1 + the largest level among rows j > i with a stored L_ji, 0 if none.
 * Rows are visited in descending order and push their level to the columns
 * of their off-diagonal entries. */
int64_t orc_levels_upper(int64_t n, const int64_t *lrp, const int32_t *lci, int32_t *level) {
  for (int64_t i = 0; i < n; ++i) level[i] = 0;
  int32_t mx = n > 0 ? 0 : -1;
  for (int64_t j = n - 1; j >= 0; --j) {
    if (level[j] > mx) mx = level[j];
    for (int64_t q = lrp[j]; q < lrp[j + 1]; ++q) {
      const int32_t i = lci[q];
      if (i < j && level[j] + 1 > level[i]) level[i] = level[j] + 1;
    }
  }
  return (int64_t)mx + 1;
}

/* Counting sort of rows by level, rows ascending inside a level:
 * perm[level_ptr[l] .. level_ptr[l+1]) are the rows of level l. */
void orc_level_sort(int64_t n, const int32_t *level, int64_t nlev, int32_t *perm,
                    int32_t *level_ptr) {
  for (int64_t l = 0; l <= nlev; ++l) level_ptr[l] = 0;
  for (int64_t i = 0; i < n; ++i) level_ptr[level[i] + 1]++;
  for (int64_t l = 0; l < nlev; ++l) level_ptr[l + 1] += level_ptr[l];
  int32_t *cur = (int32_t *)malloc(((size_t)nlev + 1) * sizeof(int32_t));
  memcpy(cur, level_ptr, ((size_t)nlev + 1) * sizeof(int32_t));
  for (int64_t i = 0; i < n; ++i) perm[cur[level[i]]++] = (int32_t)i;
  free(cur);
}

/* ------------------------------------------------------- triangular solves */

/* Forward substitution L y = r (Eq. (11) read as standard substitution:
 * y_i = (r_i - sum_{j < i} L_ij y_j) / L_ii, rows ascending). */
void orc_trsv_lower(int64_t n, const int64_t *lrp, const int32_t *lci, const double *lv,
                    const double *r, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double s = r[i];
    const int64_t re = lrp[i + 1] - 1;
    for (int64_t q = lrp[i]; q < re; ++q) s -= lv[q] * y[lci[q]];
    y[i] = s / lv[re];
  }
}

/* Backward substitution L^T z = y with U = L^T stored as CSR (diagonal first):
 * z_i = (y_i - sum_{j > i} U_ij z_j) / U_ii, rows descending. */
void orc_trsv_upper(int64_t n, const int64_t *urp, const int32_t *uci, const double *uv,
                    const double *y, double *z) {
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = y[i];
    const int64_t rs = urp[i];
    for (int64_t q = rs + 1; q < urp[i + 1]; ++q) s -= uv[q] * z[uci[q]];
    z[i] = s / uv[rs];
  }
}

/* ---- reduced-precision application of the factor (not in the paper) ---- */

/* float -> bfloat16 -> float with round-to-nearest-even on the upper 16 bits
 * (NaN kept quiet). */
float orc_round_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    u |= 0x00400000u;
    u &= 0xffff0000u;
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
  }
  float g;
  memcpy(&g, &u, 4);
  return g;
}

/* Lower-precision copy of factor values: prec 1 = float (RNE from double),
 * prec 2 = bfloat16 (RNE from that float), both held as float. */
void orc_cast_values(int64_t m, const double *v, int prec, float *out) {
  for (int64_t q = 0; q < m; ++q) {
    float f = (float)v[q];
    out[q] = prec == 2 ? orc_round_bf16(f) : f;
  }
}

/* z = L^-T L^-1 r with the factor in float: r rounded to float on load, y kept
 * in float, z accumulated in float and widened to double on store. */
void orc_apply_f32(int64_t n, const int64_t *lrp, const int32_t *lci, const float *lv,
                   const int64_t *urp, const int32_t *uci, const float *uv,
                   const double *r, double *z, float *y32, float *z32) {
  for (int64_t i = 0; i < n; ++i) {
    float s = (float)r[i];
    const int64_t re = lrp[i + 1] - 1;
    for (int64_t q = lrp[i]; q < re; ++q) s -= lv[q] * y32[lci[q]];
    y32[i] = s / lv[re];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    float s = y32[i];
    const int64_t rs = urp[i];
    for (int64_t q = rs + 1; q < urp[i + 1]; ++q) s -= uv[q] * z32[uci[q]];
    z32[i] = s / uv[rs];
    z[i] = (double)z32[i];
  }
}

/* ------------------------------------------------------------------- PCG */

typedef struct {
  int64_t n;
  const int64_t *lrp, *urp;
  const int32_t *lci, *uci;
  const double *lv, *uv;
  const float *lv32, *uv32; /* non-null: apply the factor in float */
  double *y;
  float *y32, *z32;
  int kind;                  /* 0: L L^T; 1: Jacobi (diag); 2: none */
  const double *diag;        /* kind 1: a_ii */
} orc_prec;

static void prec_apply(const orc_prec *P, const double *r, double *z) {
  if (P->kind == 1) {
    /* Jacobi: the reciprocal of A's diagonal as the inverse (Baseline Methods) */
    for (int64_t i = 0; i < P->n; ++i) z[i] = r[i] / P->diag[i];
  } else if (P->kind == 2) {
    for (int64_t i = 0; i < P->n; ++i) z[i] = r[i];
  } else if (P->lv32) {
    orc_apply_f32(P->n, P->lrp, P->lci, P->lv32, P->urp, P->uci, P->uv32, r, z, P->y32, P->z32);
  } else {
    orc_trsv_lower(P->n, P->lrp, P->lci, P->lv, r, P->y);
    orc_trsv_upper(P->n, P->urp, P->uci, P->uv, P->y, z);
  }
}

/* Preconditioned CG, supplementary Algorithm 1, with these readings:
 *  - stop when ||r_k||_2 <= rtol ||b||_2 (the text's relative residual; the
 *    listing's absolute epsilon becomes rtol ||b||), r_k the recurrence
 *    residual; then the true residual b - A x is checked and, if it is above
 *    the tolerance, r is replaced by it and the iteration continues with the
 *    same search direction (at most max_replace times);
 *  - the iteration count is the number of products A p; the listing's step
 *    before the loop is iteration 1 (it equals a loop pass with beta = 0);
 *  - b = 0 returns x = 0 after 0 iterations; ||r_0|| <= rtol ||b|| returns
 *    after 0 iterations;
 *  - r^T z <= 0 or p^T A p <= 0 stops with ORC_BREAKDOWN, a non-finite value
 *    with ORC_NONFINITE, max_iter products with ORC_MAXITER (x is the last
 *    iterate);
 *  - a converged recurrence whose true residual is still above the tolerance
 *    after max_replace replacements returns ORC_TRUE_RESIDUAL.
 * x holds x_0 on entry and the solution on exit. hist (nullable, max_iter + 1
 * entries) receives ||r_k|| / ||b|| per iteration. snap (nullable) records
 * the iterate on a few entries at a range of steps (a copy only; it changes
 * no arithmetic). */
typedef struct {
  int64_t k_from, k_count;  /* steps k_from .. k_from + k_count - 1 */
  int64_t nidx;
  const int64_t *idx;       /* entries recorded */
  double *out;              /* k_count x nidx, row (k - k_from) */
} orc_snap;

static void snap_take(const orc_snap *sn, int64_t k, const double *x) {
  if (!sn || k < sn->k_from || k >= sn->k_from + sn->k_count) return;
  double *row = sn->out + (k - sn->k_from) * sn->nidx;
  for (int64_t t = 0; t < sn->nidx; ++t) row[t] = x[sn->idx[t]];
}

int orc_pcg_run(const orc_prec *P, int64_t n, const int64_t *rp, const int32_t *ci,
                const double *v, const double *b, double *x, double rtol, int64_t max_iter,
                int max_replace, int64_t *iters_out, int *repl_out, double *relres_out,
                double *true_relres_out, double *hist, const orc_snap *snap) {
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *z = (double *)malloc((size_t)n * sizeof(double));
  double *p = (double *)calloc((size_t)n, sizeof(double));
  double *w = (double *)malloc((size_t)n * sizeof(double));
  int st = ORC_OK, repl = 0;
  int64_t k = 0;
  const double bb = orc_dot(n, b, b);
  double rr = 0.0, rz = 0.0, trr = 0.0;
  const double tol2 = rtol * rtol * bb;
  if (bb == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    goto done;
  }
  orc_spmv(n, rp, ci, v, x, w);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
  rr = orc_dot(n, r, r);
  if (hist) hist[0] = sqrt(rr / bb);
  if (!isfinite(rr)) { st = ORC_NONFINITE; goto done; }
  for (;;) {
    while (rr > tol2) {
      if (k >= max_iter) { st = ORC_MAXITER; break; }
      prec_apply(P, r, z);
      const double rz_new = orc_dot(n, r, z);
      if (!isfinite(rz_new)) { st = ORC_NONFINITE; break; }
      if (!(rz_new > 0.0)) { st = ORC_BREAKDOWN; break; }
      const double beta = k == 0 ? 0.0 : rz_new / rz;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      orc_spmv(n, rp, ci, v, p, w);
      const double pw = orc_dot(n, p, w);
      if (!isfinite(pw)) { st = ORC_NONFINITE; break; }
      if (!(pw > 0.0)) { st = ORC_BREAKDOWN; break; }
      const double alpha = rz_new / pw;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * w[i];
      rz = rz_new;
      ++k;
      snap_take(snap, k, x);
      rr = orc_dot(n, r, r);
      if (hist) hist[k] = sqrt(rr / bb);
      if (!isfinite(rr)) { st = ORC_NONFINITE; break; }
    }
    /* true residual */
    orc_spmv(n, rp, ci, v, x, w);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) w[i] = b[i] - w[i];
    trr = orc_dot(n, w, w);
    if (st != ORC_OK || trr <= tol2) break;
    if (repl >= max_replace) { st = ORC_TRUE_RESIDUAL; break; }
    memcpy(r, w, (size_t)n * sizeof(double));
    rr = trr;
    ++repl;
  }
done:
  if (iters_out) *iters_out = k;
  if (repl_out) *repl_out = repl;
  if (relres_out) *relres_out = bb > 0 ? sqrt(rr / bb) : 0.0;
  if (true_relres_out) *true_relres_out = bb > 0 ? sqrt(trr / bb) : 0.0;
  free(r); free(z); free(p); free(w);
  return st;
}

/* PCG with the factor L (lower CSR) and its transpose U. prec: 0 = apply in
 * FP64; 1 = factor rounded to float; 2 = factor rounded to bfloat16 (both
 * applied with float arithmetic, recurrences FP64). */
int orc_pcg(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
            const int64_t *lrp, const int32_t *lci, const double *lv,
            const int64_t *urp, const int32_t *uci, const double *uv,
            const double *b, double *x, double rtol, int64_t max_iter, int max_replace,
            int prec, int64_t *iters_out, int *repl_out, double *relres_out,
            double *true_relres_out, double *hist, int64_t snap_from, int64_t snap_count,
            int64_t snap_nidx, const int64_t *snap_idx, double *snap_out) {
  orc_snap sn = {snap_from, snap_count, snap_nidx, snap_idx, snap_out};
  const orc_snap *snap = (snap_out && snap_count > 0 && snap_nidx > 0) ? &sn : NULL;
  orc_prec P;
  memset(&P, 0, sizeof(P));
  P.n = n; P.lrp = lrp; P.lci = lci; P.lv = lv; P.urp = urp; P.uci = uci; P.uv = uv;
  float *l32 = NULL, *u32 = NULL;
  if (prec == 1 || prec == 2) {
    l32 = (float *)malloc((size_t)lrp[n] * sizeof(float));
    u32 = (float *)malloc((size_t)urp[n] * sizeof(float));
    orc_cast_values(lrp[n], lv, prec, l32);
    orc_cast_values(urp[n], uv, prec, u32);
    P.lv32 = l32; P.uv32 = u32;
    P.y32 = (float *)malloc((size_t)n * sizeof(float));
    P.z32 = (float *)malloc((size_t)n * sizeof(float));
  } else {
    P.y = (double *)malloc((size_t)n * sizeof(double));
  }
  int st = orc_pcg_run(&P, n, rp, ci, v, b, x, rtol, max_iter, max_replace, iters_out,
                       repl_out, relres_out, true_relres_out, hist, snap);
  free(l32); free(u32); free(P.y32); free(P.z32); free(P.y);
  return st;
}

/* z = L^-T L^-1 r in FP64 (the preconditioner solve P z = r, P = L L^T). */
void orc_apply(int64_t n, const int64_t *lrp, const int32_t *lci, const double *lv,
               const int64_t *urp, const int32_t *uci, const double *uv,
               const double *r, double *y, double *z) {
  orc_trsv_lower(n, lrp, lci, lv, r, y);
  orc_trsv_upper(n, urp, uci, uv, y, z);
}

/* --------------------------------------------------------------- adjoint */

/* Reverse-mode derivative of Z = L^-T L^-1 R (columns independent; not in the
 * paper, derived from L Y = R and L^T Z = Y): with G = dl/dZ,
 *   Ybar = L^-1 G,  Rbar = L^-T Ybar  (= dl/dR),
 *   dl/dL_ab = -sum_k (Z_ak Ybar_bk + Rbar_ak Y_bk)  for (a, b) stored in L.
 * Blocks are n x m, row-major (entry (i, k) at i*m + k). */
void orc_apply_adjoint(int64_t n, const int64_t *lrp, const int32_t *lci, const double *lv,
                       const int64_t *urp, const int32_t *uci, const double *uv, int64_t m,
                       const double *R, const double *G, double *Y, double *Z,
                       double *Ybar, double *Rbar, double *dL) {
  double *c0 = (double *)malloc((size_t)n * sizeof(double));
  double *c1 = (double *)malloc((size_t)n * sizeof(double));
  double *c2 = (double *)malloc((size_t)n * sizeof(double));
  for (int64_t k = 0; k < m; ++k) {
    for (int64_t i = 0; i < n; ++i) c0[i] = R[i * m + k];
    orc_trsv_lower(n, lrp, lci, lv, c0, c1);
    for (int64_t i = 0; i < n; ++i) Y[i * m + k] = c1[i];
    orc_trsv_upper(n, urp, uci, uv, c1, c2);
    for (int64_t i = 0; i < n; ++i) Z[i * m + k] = c2[i];
    for (int64_t i = 0; i < n; ++i) c0[i] = G[i * m + k];
    orc_trsv_lower(n, lrp, lci, lv, c0, c1);
    for (int64_t i = 0; i < n; ++i) Ybar[i * m + k] = c1[i];
    orc_trsv_upper(n, urp, uci, uv, c1, c2);
    for (int64_t i = 0; i < n; ++i) Rbar[i * m + k] = c2[i];
  }
  for (int64_t a = 0; a < n; ++a)
    for (int64_t q = lrp[a]; q < lrp[a + 1]; ++q) {
      const int64_t bcol = lci[q];
      double s = 0.0;
      for (int64_t k = 0; k < m; ++k)
        s += Z[a * m + k] * Ybar[bcol * m + k] + Rbar[a * m + k] * Y[bcol * m + k];
      dL[q] = -s;
    }
  free(c0); free(c1); free(c2);
}

/* The same PCG with the two baselines of Table 1: kind 1 = Jacobi (z_i =
 * r_i / a_ii), kind 2 = no preconditioner (z = r, plain CG). A must store
 * its diagonal. */
int orc_pcg_simple(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, int kind,
                   const double *b, double *x, double rtol, int64_t max_iter, int max_replace,
                   int64_t *iters_out, int *repl_out, double *relres_out, double *true_relres_out,
                   double *hist) {
  orc_prec P;
  memset(&P, 0, sizeof(P));
  P.n = n;
  P.kind = kind;
  double *d = NULL;
  if (kind == 1) {
    d = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
      d[i] = 0.0;
      for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
        if (ci[q] == i) d[i] = v[q];
    }
    P.diag = d;
  }
  int st = orc_pcg_run(&P, n, rp, ci, v, b, x, rtol, max_iter, max_replace, iters_out,
                       repl_out, relres_out, true_relres_out, hist, NULL);
  free(d);
  return st;
}
