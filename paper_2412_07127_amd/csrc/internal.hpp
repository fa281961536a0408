// Host-side internals of the library: device buffers, the context and
// preconditioner objects, and the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/icpcg.h"
#include "common.hpp"

namespace icpcg {

// Largest supernode (rows solved together by one wave) of the triangular
// solve schedules.
constexpr int kSupernodeMax = 3;

// Last error text of the calling thread; the ABI layer copies it into the
// context that made the call.
void set_error(const std::string &msg);
const std::string &get_error();

// Owning device buffer (hipMalloc / hipFree).
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // (Re)allocate to at least `b` bytes; returns ICPCG_OK or ICPCG_E_NOMEM.
  int reserve(size_t b);
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct Device {
  int id = 0;
  int num_cu = 256;
  int trsv_waves_per_cu = 0;  // 0: as many as fit
  bool ic0_sync_free = false;  // IC(0) in one sync-free launch instead of level launches
  bool fuse_rz = true;         // backward solves of a PCG step form r^T z where that pays
  bool fuse_xr = true;         // forward solves of a PCG step apply the previous step's x, r update
  long long wall_hz = 100000000;  // wall_clock64 rate
  long long wait_ticks = 400000000;  // device-side wait limit (4 s)
};

// Per-column PCG state kept on the device.
struct ColState {
  double bb, tol2, rr, rz, pw, alpha, beta, trr;
  int active;   // still iterating
  int conv;     // recurrence converged, true residual pending
  int status;   // icpcg_status
  int iters;    // products A p
  int repl;     // residual replacements
  int replace;  // replace r by the true residual on the next pass
  int zero_x;   // b = 0: x is set to 0
  int upd;      // alpha is set and x, r still await their update with it
};

struct SolveFlags {
  int n_active;
  int n_conv;
  int err;
  int pad;
};

// Work buffers of a context (grow monotonically).
struct Workspace {
  DevBuf r, p, w, y, z, partials, cols, flags, tmp0, tmp1;
  void *host_flags = nullptr;  // pinned SolveFlags
};

}  // namespace icpcg

struct icpcg_ctx {
  hipStream_t stream = nullptr;
  icpcg::Device dev;
  icpcg::Workspace ws;
  std::string last_error;
  // PCG steps captured as one graph on a private stream (default priority),
  // replayed while every launch argument (step_key) is unchanged
  hipStream_t capture = nullptr;
  hipGraphExec_t step_exec = nullptr;
  std::vector<uintptr_t> step_key;
  // block widths picked by the autotuner, keyed by the operands' identity
  struct Tune {
    std::vector<uintptr_t> key;
    int width;
    double ms[5];
  };
  std::vector<Tune> tunes;
  // per-phase timing of eager PCG steps (icpcg_step_timing): events recorded
  // at the kPhaseMarks phase boundaries of the first kTimedSteps steps
  static constexpr int kPhaseMarks = 7, kTimedSteps = 64;
  bool timing = false;
  std::vector<hipEvent_t> tev;
  int64_t tsteps = 0;
};

// One schedule position of a triangular solve: the supernode's first row a,
// the start of that row in the CSR arrays, and (m << 3) | size with m the
// number of shared off-block entries.
struct SnItem {
  int64_t ro0;
  int32_t a;
  int32_t m_sz;
};

// One triangular factor's schedule: supernodes (row ranges solved together)
// ordered by level.
struct TriSchedule {
  icpcg::DevBuf sn_ptr;    // int32[nsn + 1]
  icpcg::DevBuf sn_order;  // int32[nsn]: supernodes sorted by (level, id)
  icpcg::DevBuf items;     // SnItem[nsn] in schedule order
  int64_t nsn = 0;
  int64_t nlev = 0;
};

struct icpcg_mat {
  icpcg_csr A;
  icpcg::DevBuf gptr;   // int32[ngroups + 1] row groups
  icpcg::DevBuf grec;   // SpGroup[ngroups]
  int64_t ngroups = 0;
  bool grouped = false;
};

struct icpcg_prec {
  int64_t n = 0, nnz = 0;
  icpcg_dtype dtype = ICPCG_F64;
  int kind = ICPCG_PREC_FACTOR;      // icpcg_prec_kind
  icpcg::DevBuf diag;                // f64[n]: A's diagonal (Jacobi)
  icpcg::DevBuf lrp, lci, lval;      // L (int64, int32, f64)
  icpcg::DevBuf urp, uci, uval;      // U = L^T (int64, int32, f64)
  icpcg::DevBuf upos;                // int32: L position of each U entry
  icpcg::DevBuf lval_lo, uval_lo;    // f32 or bf16 copies
  TriSchedule sl, su;                // forward / backward schedules
  int64_t nlev_rows_L = -1, nlev_rows_U = -1;  // row level counts (on demand)
};

// A matrix prepared for the learned correction: pattern and transpose map of
// the preconditioner it was made from (which must outlive it), a copy of
// L_IC, node features, edge inputs and their scale, and the activations and
// gradients of the last pass.
struct icpcg_gnn {
  int64_t n = 0, nnz = 0;
  icpcg_csr A{};
  const icpcg_prec *P = nullptr;
  icpcg::DevBuf erow, aedge, lic, deg, x, e0, red, flag, tmp, part, pp;
  double scale = 0.0;
  icpcg::DevBuf d, mu, sd, h[3], e[3], q[3], nin[2], Q[2], L;
  icpcg::DevBuf az, u, llz, r, ltr, sq2, sums, dout, de, deprev, dhr, dhc, dp, dh, direct, ds, dP, rows3, dd;
};

namespace icpcg {

// ------------------------------------------------------------ primitives
// All launchers enqueue on `s` and return an icpcg_status value.
int scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, int64_t *total_host);
int scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, int32_t *total_host);
int scan_inclusive_max_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
int reduce_max_i32(const int32_t *in, int64_t n, hipStream_t s, int32_t *host_out);
int reduce_min_f64(const double *in, int64_t n, hipStream_t s, double *host_out);
// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
// Inputs are preserved; sorted results land in keys_out / vals_out.
int radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                     uint32_t *vals_out, int64_t n, int bits, hipStream_t s);
int fill_iota_u32(uint32_t *out, int64_t n, hipStream_t s);
int fill_i32(int32_t *out, int32_t v, int64_t n, hipStream_t s);
int fill_u64(uint64_t *out, uint64_t v, int64_t n, hipStream_t s);
int fill_u32(uint32_t *out, uint32_t v, int64_t n, hipStream_t s);

// ------------------------------------------------------------ setup
int check_csr(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, int mode,
              const double *val, hipStream_t s, int *bad_row_host);
int tril_count(const int64_t *rp, const int32_t *ci, int64_t n, int64_t *cnt, hipStream_t s);
int tril_copy(const int64_t *rp, const int32_t *ci, const double *v, int64_t n,
              const int64_t *lrp, int32_t *lci, double *lv, hipStream_t s);
int build_transpose(icpcg_prec *P, hipStream_t s);
// Fill-in dropout of a lower CSR factor into (orp, oci, ov); *nnz_host gets the kept count.
int dropout(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, double eps, int64_t *orp,
            int32_t *oci, double *ov, int64_t *nnz_host, hipStream_t s);
int refresh_values(icpcg_prec *P, hipStream_t s);
int build_schedule(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, int smax,
                   TriSchedule &out, hipStream_t s, const Device &dev);
// Most blocks of a kernel that writes per-block reduction partials (the
// solve's partials buffer holds kMaxDotBlocks * R * 2 doubles).
constexpr int64_t kMaxDotBlocks = 32768;

// One row group of A for the SpMV: its first row r0, the CSR offset `base`
// of that row (the group's rows follow at base + u * m) and (m << 3) | size.
struct SpGroup {
  int64_t base;
  int32_t r0;
  int32_t m_sz;
};

// Groups of up to gmax consecutive rows with identical column lists (gptr)
// and their SpGroup records (rows must have fewer than 2^28 entries).
int build_row_groups(const int64_t *rp, const int32_t *ci, int64_t n, int gmax, DevBuf &gptr, DevBuf &grec,
                     int64_t *ngroups, hipStream_t s);
// Row schedule of a lower pattern from its supernode levels (key = supernode
// level * kSupernodeMax + position in the supernode); key_ptr needs room for
// kSupernodeMax * n + 1 entries.
int supernode_row_order(const int64_t *rp, const int32_t *ci, int64_t n, int32_t *perm, int32_t *key_ptr,
                        int64_t *nkeys_host, hipStream_t s, const Device &dev);
int row_levels(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, int32_t *level,
               int32_t *perm, int32_t *level_ptr, int64_t *nlev_host, hipStream_t s,
               const Device &dev);

// ------------------------------------------------------------ kernels
// IC(0) with one launch per level of tril(A)'s row schedule (level_ptr on the
// host), or in one sync-free launch over the rows in level order (lv filled
// with the pending pattern and *ticket zeroed first; err raised when a wait
// reaches its limit).
int ic0_factor_levels(const int64_t *lrp, const int32_t *lci, double *lv, const double *a_lower,
                      int64_t n, const int32_t *perm, const std::vector<int32_t> &level_ptr,
                      double alpha, int *fail_flag, double *pivots, hipStream_t s, int max_row_len,
                      const Device &dev);
int ic0_factor_sync(const int64_t *lrp, const int32_t *lci, double *lv, const double *a_lower, int64_t n,
                    const int32_t *order, double alpha, int *fail_flag, int *err, int *ticket, double *pivots,
                    hipStream_t s, int max_row_len, const Device &dev);
int ic0_max_row();

// multicolour ordering (order.hip)
int color_order(const int64_t *rp, const int32_t *ci, int64_t n, uint64_t seed, int32_t *perm, int32_t *ncolours,
                hipStream_t s);
int block_color_order(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, const int32_t *blk, int32_t nblk,
                      int32_t *perm, int32_t *ncolours, hipStream_t s);
int permute_matrix(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t nnz, const int32_t *perm,
                   int64_t *orp, int32_t *oci, double *ov, hipStream_t s);
int permute_rows(const int32_t *perm, int64_t n, int64_t R, const double *x, double *y, bool inverse, hipStream_t s);

// learned correction of the factor (gnn.hip)
int gnn_num_params();
int gnn_setup(icpcg_gnn *G, const icpcg_csr *A, const icpcg_prec *P, hipStream_t s);
int gnn_inputs(const icpcg_gnn *G, double *x, double *e, hipStream_t s);
int gnn_forward(icpcg_gnn *G, const double *theta, double *L_out, bool keep, hipStream_t s);
int gnn_loss_grad(icpcg_gnn *G, const double *theta, const double *z, double *loss, double *grad, bool accumulate,
                  hipStream_t s);
int adam_step(double *th, const double *g, double *m, double *v, int64_t count, int64_t t, double lr, double b1,
              double b2, double eps, hipStream_t s);
int spmv_default_slots(int R);

// partials/cols non-null: also p^T w and the alpha update, fused into the row
// kernel (active must then point at the solve's SolveFlags); active (nullable)
// as for trsv.
int spmv(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x,
         double *y, int R, int slots, hipStream_t s, double *partials = nullptr,
         ColState *cols = nullptr, const int *active = nullptr);

// partials (nullable): also p^T w -> alpha of each column, in a second pass
// over x = p and y = w (n rows).
int spmv_grouped(const int32_t *ci, const double *v, int64_t ngroups, const SpGroup *grec, int64_t n,
                 const double *x, double *y, int R, int slots, hipStream_t s, double *partials = nullptr,
                 ColState *cols = nullptr, const int *active = nullptr);
int spmv_grouped_default_slots(int R);

// active (nullable): the solve's count of iterating columns; when it reads 0
// the launch returns at once (steps queued past convergence cost a launch).
// rz.partials (nullable, backward solves of a PCG step): also r^T z of every
// column with r = rz.r (n x R, FP64), folded into beta by k_rz_fin, or, when
// rz.out is set, into out[c] (FP64, one value per column).
struct RzDot {
  const double *r = nullptr;
  double *partials = nullptr;
  ColState *cols = nullptr;
  SolveFlags *flags = nullptr;
  double *out = nullptr;
  // doubles available at `partials` (< 0: sized by the caller for any grid);
  // a launch whose grid needs more is refused with ICPCG_E_INVALID
  int64_t partials_cap = -1;
  // the solve also re-arms its right-hand side as pending once read (the
  // next step's forward solve writes it), in place of the p update
  bool rearm_rhs = false;
};
// xr.X (nullable, forward solves of a PCG step): first the previous step's
// update of every column c with cols[c].upd set, x += alpha p and r -= alpha w
// (X, r, p, w: n x R, FP64; the solve's right-hand side is then the updated r,
// read through `rhs`, which must be xr.r), with ||r||^2 of those columns into
// block partials folded by k_rr_fin (iteration count and stop tests, as the
// update_xr step does), which also clears upd.
struct XrUpd {
  double *X = nullptr;
  double *r = nullptr;
  const double *p = nullptr;
  const double *w = nullptr;
  ColState *cols = nullptr;
  double *partials = nullptr;
  int64_t partials_cap = -1;  // as in RzDot
  int64_t max_iter = 0;
  SolveFlags *flags = nullptr;
};
int trsv(const icpcg_prec *P, bool upper, const void *rhs, bool rhs_f64, void *out, int R,
         int64_t ld, hipStream_t s, const Device &dev, int *err, const int *active = nullptr,
         const RzDot &rz = RzDot{}, const XrUpd &xr = XrUpd{});
// whether the backward solve of a PCG step with this factor and width forms r^T z
bool trsv_fuses_rz(const icpcg_prec *P, int R, const Device &dev);
// whether the forward solve of a PCG step with this factor and width applies
// the previous step's x, r update
bool trsv_fuses_xr(const icpcg_prec *P, int R, const Device &dev);

int prec_dL(const icpcg_prec *P, const void *Z, const void *Yb, const void *Rb, const void *Y,
            void *dL, int R, hipStream_t s);

// PCG vector steps (vec.hip); each reduction is a compute kernel plus a
// one-block finalize kernel.
int pcg_init(int64_t n, int R, const double *B, const double *W, double *r, double *p,
             void *y, void *z, bool f32, double rtol, double *partials, ColState *cols,
             int64_t max_iter, SolveFlags *flags, hipStream_t s);
int pcg_zero_x(int64_t n, int R, double *X, const ColState *cols, hipStream_t s);
int pcg_dot_rz(int64_t n, int R, const double *r, const void *z, bool f32, double *partials,
               ColState *cols, SolveFlags *flags, hipStream_t s);
// p = z + beta p; then z (read in place) and y are re-armed as pending (y
// null: y was re-armed by the backward solve)
int pcg_update_p(int64_t n, int R, void *z, bool f32, double *p, void *y, const ColState *cols,
                 const SolveFlags *flags, hipStream_t s);
int pcg_pw_finalize(int R, const double *partials, int nb, ColState *cols, const SolveFlags *flags,
                    hipStream_t s);
int pcg_dot_pw(int64_t n, int R, const double *p, const double *w, double *partials, ColState *cols,
               const SolveFlags *flags, hipStream_t s);
int pcg_rz_finalize(int R, const double *partials, int nb, ColState *cols, SolveFlags *flags, hipStream_t s);
// out[c] = column c's sum of the nb block partials (fixed order)
int dot_finalize_out(int R, const double *partials, int nb, double *out, hipStream_t s);
// out[c] = sum_i r[i, c] z[i, c] (FP64; z FP64 or FP32), deterministic
int col_dot_out(int64_t n, int R, const double *r, const void *z, bool f32, double *partials, double *out,
                hipStream_t s);
int pcg_update_xr(int64_t n, int R, double *X, double *r, const double *p, const double *w,
                  double *partials, ColState *cols, int64_t max_iter, SolveFlags *flags,
                  hipStream_t s);
// The stop tests of update_xr from ||r||^2 block partials formed elsewhere
// (the forward solve that applies the update): columns with upd set only.
int pcg_rr_finalize(int R, const double *partials, int nb, ColState *cols, int64_t max_iter, SolveFlags *flags,
                    hipStream_t s);
int pcg_true_residual(int64_t n, int R, const double *B, double *W, double *partials,
                      ColState *cols, int64_t max_iter, int max_replace, int final_pass,
                      SolveFlags *flags, hipStream_t s);
// z = r / d (Jacobi, d non-null) or z = r (no preconditioner) for an n x R
// block; returns at once when *active == 0.
int pcg_diag_apply(int64_t n, int R, const double *r, const double *d, double *z, const int *active, hipStream_t s);
int pcg_replace_r(int64_t n, int R, const double *W, double *r, ColState *cols, hipStream_t s);
int gather_cols(int64_t n, int R, const double *src, int64_t lds, int64_t c0, int nc, double *dst,
                hipStream_t s);
int scatter_cols(int64_t n, int R, const double *src, double *dst, int64_t ldd, int64_t c0, int nc,
                 hipStream_t s);
int fill_pending(void *p, int64_t count, bool f32, hipStream_t s);

}  // namespace icpcg
