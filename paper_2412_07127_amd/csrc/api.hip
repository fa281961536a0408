// C ABI entry points (include/icpcg.h): argument checks, object lifetime, the
// IC(0) shift loop and the PCG driver. Every numerical step runs in the
// library's own kernels; the host only sequences launches and reads the
// per-column flags.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace icpcg {

namespace {
thread_local std::string g_err;

__global__ void k_row_len(const int64_t *rp, int64_t n, int32_t *len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    len[i] = (int32_t)(rp[i + 1] - rp[i]);
}
__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }
// d_i = a_ii (0 when row i stores no diagonal)
__global__ void k_extract_diag(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, double *d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double x = 0.0;
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t)
      if (ci[t] == i) x = v[t];
    d[i] = x;
  }
}
}  // namespace

void set_error(const std::string &msg) { g_err = msg; }
const std::string &get_error() { return g_err; }

}  // namespace icpcg

using namespace icpcg;

// Reduction partials of icpcg_apply_rz_noalloc, for callers that cannot
// allocate: every call on a device shares that device's copy, which lives
// until the process ends. Each launch that reads partials first writes all it
// reads (one value per block and column), so nothing needs clearing between
// calls. 16 blocks per CU on 256 CUs at 16 columns; the fused backward solve
// uses at most its resident blocks and the separate r^T z pass at most 1024.
constexpr int64_t kScratchDoubles = 16 * 256 * 16;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Device address of `scratch` per device (the host symbol is only a stand-in
// for it), taken once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

int scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device id out of range for the no-allocation scratch table");
    return ICPCG_E_DEVICE;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_dev[dev]) return ICPCG_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return ICPCG_E_DEVICE;
  }
  g_scratch_dev[dev] = static_cast<double *>(ptr);
  return ICPCG_OK;
}

double *scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_dev[dev];
}

constexpr int kSmax = kSupernodeMax;

icpcg_status finish(icpcg_ctx *ctx, int st) {
  if (ctx && st != ICPCG_OK) ctx->last_error = get_error();
  return (icpcg_status)st;
}

icpcg_status fail(icpcg_ctx *ctx, icpcg_status st, const std::string &msg) {
  set_error(msg);
  return finish(ctx, st);
}

bool valid_csr_args(const icpcg_csr *A) {
  return A && A->n >= 0 && A->nnz >= 0 && A->n < INT32_MAX && (A->n == 0 || (A->row_ptr && A->col && A->val));
}

// Calls that need the triangular factor reject the baseline kinds.
bool not_factor(icpcg_ctx *ctx, const icpcg_prec *P, const char *what) {
  if (P && P->kind != ICPCG_PREC_FACTOR) {
    set_error(std::string(what) + ": the preconditioner has no triangular factor (Jacobi or none)");
    finish(ctx, ICPCG_E_INVALID);
    return true;
  }
  return false;
}

bool pow2_width(int64_t r) { return r == 1 || r == 2 || r == 4 || r == 8 || r == 16; }

int64_t default_max_iter(int64_t n) {
  int64_t m = (int64_t)(10.0 * std::sqrt((double)n));
  if (m < 10) m = 10;
  if (m > n) m = n;
  if (m < 1) m = 1;
  return m;
}

int check_matrix(icpcg_ctx *ctx, const icpcg_csr *A, int mode) {
  if (A->n == 0) return ICPCG_OK;
  int bad = -1;
  int st = check_csr(A->row_ptr, A->col, A->n, A->nnz, mode, A->val, ctx->stream, &bad);
  if (st) return st;
  if (bad >= 0) {
    set_error(std::string(mode == 1 ? "factor" : "matrix") + " row " + std::to_string(bad) +
              (mode == 1 ? " is not lower triangular with a positive finite diagonal last, sorted columns, "
                           "in-range indices and finite values"
                         : " has unsorted, duplicate or out-of-range columns, no diagonal, or a non-finite value"));
    return ICPCG_E_INVALID;
  }
  return ICPCG_OK;
}

// Device-side error flag of the dependency waits (shared SolveFlags buffer).
int ensure_flags(icpcg_ctx *ctx) {
  Workspace &ws = ctx->ws;
  if (!ws.flags.p) {
    int st = ws.flags.reserve(sizeof(SolveFlags) + 64);
    if (st) return st;
    ICPCG_HIP_TRY(hipMemsetAsync(ws.flags.p, 0, sizeof(SolveFlags) + 64, ctx->stream));
  }
  if (!ws.host_flags) ICPCG_HIP_TRY(hipHostMalloc(&ws.host_flags, sizeof(SolveFlags) + 64, hipHostMallocDefault));
  return ICPCG_OK;
}

SolveFlags *dev_flags(icpcg_ctx *ctx) { return ctx->ws.flags.as<SolveFlags>(); }

int read_flags(icpcg_ctx *ctx, SolveFlags *h) {
  ICPCG_HIP_TRY(hipMemcpyAsync(ctx->ws.host_flags, ctx->ws.flags.p, sizeof(SolveFlags), hipMemcpyDeviceToHost,
                               ctx->stream));
  ICPCG_HIP_TRY(hipStreamSynchronize(ctx->stream));
  std::memcpy(h, ctx->ws.host_flags, sizeof(SolveFlags));
  return ICPCG_OK;
}

int take_wait_error(icpcg_ctx *ctx) {
  SolveFlags h;
  int st = read_flags(ctx, &h);
  if (st) return st;
  if (h.err) {
    ICPCG_HIP_TRY(hipMemsetAsync(&dev_flags(ctx)->err, 0, sizeof(int), ctx->stream));
    set_error("a device-side dependency wait exceeded its time limit");
    return ICPCG_E_DEVICE;
  }
  return ICPCG_OK;
}

}  // namespace

extern "C" {

const char *icpcg_version(void) {
  return "icpcg 0.1 (gfx950; IC(0)-PCG with sync-free supernodal triangular solves)";
}

const char *icpcg_status_string(icpcg_status st) {
  switch (st) {
    case ICPCG_OK: return "ok";
    case ICPCG_E_INVALID: return "invalid argument";
    case ICPCG_E_PIVOT: return "IC(0) pivot breakdown";
    case ICPCG_E_BREAKDOWN: return "PCG breakdown";
    case ICPCG_E_MAXITER: return "maximum iterations reached";
    case ICPCG_E_NONFINITE: return "non-finite value";
    case ICPCG_E_DEVICE: return "device error";
    case ICPCG_E_NOMEM: return "out of device memory";
    case ICPCG_E_TRUE_RESIDUAL: return "true residual above tolerance";
  }
  return "unknown status";
}

icpcg_status icpcg_create(icpcg_ctx **out, void *stream) {
  if (!out) return ICPCG_E_INVALID;
  *out = nullptr;
  icpcg_ctx *ctx = new (std::nothrow) icpcg_ctx();
  if (!ctx) return ICPCG_E_NOMEM;
  ctx->stream = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete ctx;
    return ICPCG_E_DEVICE;
  }
  ctx->dev.id = dev;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    ctx->dev.num_cu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) == hipSuccess && v > 0)
    ctx->dev.wall_hz = (long long)v * 1000LL;  // attribute is in kHz
  ctx->dev.wait_ticks = ctx->dev.wall_hz * 4;  // 4 s
  if (const char *e = std::getenv("ICPCG_WAIT_LIMIT_US")) {
    const long long us = std::atoll(e);
    if (us >= 0) ctx->dev.wait_ticks = ctx->dev.wall_hz / 1000000 * us;
  }
  if (const char *e = std::getenv("ICPCG_TRSV_WAVES_PER_CU")) ctx->dev.trsv_waves_per_cu = std::atoi(e);
  if (const char *e = std::getenv("ICPCG_IC0_SYNC_FREE")) ctx->dev.ic0_sync_free = std::atoi(e) != 0;
  if (const char *e = std::getenv("ICPCG_FUSE_RZ")) ctx->dev.fuse_rz = std::atoi(e) != 0;
  if (const char *e = std::getenv("ICPCG_FUSE_XR")) ctx->dev.fuse_xr = std::atoi(e) != 0;
  if (ensure_flags(ctx) != ICPCG_OK) {
    delete ctx;
    return ICPCG_E_NOMEM;
  }
  if (scratch_init(dev) != ICPCG_OK) {
    delete ctx;
    return ICPCG_E_DEVICE;
  }
  *out = ctx;
  return ICPCG_OK;
}

icpcg_status icpcg_destroy(icpcg_ctx *ctx) {
  if (!ctx) return ICPCG_OK;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->step_exec) (void)hipGraphExecDestroy(ctx->step_exec);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
  if (ctx->ws.host_flags) (void)hipHostFree(ctx->ws.host_flags);
  delete ctx;
  return ICPCG_OK;
}

icpcg_status icpcg_set_stream(icpcg_ctx *ctx, void *stream) {
  if (!ctx) return ICPCG_E_INVALID;
  ctx->stream = (hipStream_t)stream;
  return ICPCG_OK;
}

const char *icpcg_last_error(const icpcg_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

icpcg_status icpcg_step_timing(icpcg_ctx *ctx, int enable) {
  if (!ctx) return ICPCG_E_INVALID;
  if (enable && ctx->tev.empty()) {
    ctx->tev.resize((size_t)icpcg_ctx::kPhaseMarks * icpcg_ctx::kTimedSteps, nullptr);
    for (hipEvent_t &e : ctx->tev) {
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return fail(ctx, ICPCG_E_DEVICE, std::string("step_timing: ") + hipGetErrorString(r));
    }
  }
  ctx->timing = enable != 0;
  if (enable) ctx->tsteps = 0;
  return ICPCG_OK;
}

icpcg_status icpcg_step_timing_get(icpcg_ctx *ctx, double *ms, int64_t *steps) {
  if (!ctx || !ms || !steps) return ICPCG_E_INVALID;
  constexpr int NP = icpcg_ctx::kPhaseMarks - 1;
  for (int m = 0; m < NP; ++m) ms[m] = 0.0;
  *steps = ctx->tsteps;
  if (ctx->tsteps == 0) return ICPCG_OK;
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, ICPCG_E_DEVICE, std::string("step_timing_get: ") + hipGetErrorString(e));
  for (int64_t k = 0; k < ctx->tsteps; ++k) {
    for (int m = 0; m < NP; ++m) {
      float t = 0.f;
      const hipError_t r = hipEventElapsedTime(&t, ctx->tev[k * icpcg_ctx::kPhaseMarks + m],
                                               ctx->tev[k * icpcg_ctx::kPhaseMarks + m + 1]);
      if (r != hipSuccess) return fail(ctx, ICPCG_E_DEVICE, std::string("step_timing_get: ") + hipGetErrorString(r));
      ms[m] += t;
    }
  }
  for (int m = 0; m < NP; ++m) ms[m] /= (double)ctx->tsteps;
  return ICPCG_OK;
}

icpcg_status icpcg_tril_nnz(icpcg_ctx *ctx, const icpcg_csr *A, int64_t *nnz_lower) {
  if (!ctx || !valid_csr_args(A) || !nnz_lower) return fail(ctx, ICPCG_E_INVALID, "tril_nnz: bad arguments");
  if (A->n == 0) { *nnz_lower = 0; return ICPCG_OK; }
  int st = check_matrix(ctx, A, 0);
  if (st) return finish(ctx, st);
  DevBuf cnt, ex;
  if (cnt.reserve(A->n * 8) || ex.reserve(A->n * 8)) return finish(ctx, ICPCG_E_NOMEM);
  if ((st = tril_count(A->row_ptr, A->col, A->n, cnt.as<int64_t>(), ctx->stream))) return finish(ctx, st);
  int64_t total = 0;
  if ((st = scan_exclusive_i64(cnt.as<int64_t>(), ex.as<int64_t>(), A->n, ctx->stream, &total)))
    return finish(ctx, st);
  *nnz_lower = total;
  return ICPCG_OK;
}

icpcg_status icpcg_factor(icpcg_ctx *ctx, const icpcg_csr *A, int64_t *L_row_ptr, int32_t *L_col, double *L_val,
                          const icpcg_factor_opts *opts, icpcg_factor_info *info) {
  if (!ctx || !valid_csr_args(A) || (A->n > 0 && (!L_row_ptr || !L_col || !L_val)))
    return fail(ctx, ICPCG_E_INVALID, "factor: bad arguments");
  const int64_t n = A->n;
  const int max_restarts = opts && opts->max_restarts >= 0 ? opts->max_restarts : 30;
  const double alpha_min = opts && opts->alpha_min > 0 ? opts->alpha_min : 1e-3;
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return ICPCG_OK;
  hipStream_t s = ctx->stream;
  int st = check_matrix(ctx, A, 0);
  if (st) return finish(ctx, st);
  // pattern of tril(A)
  DevBuf cnt;
  if (cnt.reserve(n * 8)) return finish(ctx, ICPCG_E_NOMEM);
  if ((st = tril_count(A->row_ptr, A->col, n, cnt.as<int64_t>(), s))) return finish(ctx, st);
  int64_t nnzl = 0;
  if ((st = scan_exclusive_i64(cnt.as<int64_t>(), L_row_ptr, n, s, &nnzl))) return finish(ctx, st);
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, L_row_ptr + n, nnzl);
  DevBuf a_low, pivots, lens, perm, lptr, fl;
  if (a_low.reserve(nnzl * 8) || pivots.reserve(n * 8) || lens.reserve(n * 4) || perm.reserve(n * 4) ||
      lptr.reserve((kSupernodeMax * n + 1) * 4) || fl.reserve(12))
    return finish(ctx, ICPCG_E_NOMEM);
  if ((st = tril_copy(A->row_ptr, A->col, A->val, n, L_row_ptr, L_col, a_low.as<double>(), s))) return finish(ctx, st);
  // longest row (LDS staging limit)
  hipLaunchKernelGGL(k_row_len, dim3(1024), dim3(256), 0, s, L_row_ptr, n, lens.as<int32_t>());
  int32_t maxlen = 0;
  if ((st = reduce_max_i32(lens.as<int32_t>(), n, s, &maxlen))) return finish(ctx, st);
  if (maxlen > ic0_max_row())
    return fail(ctx, ICPCG_E_INVALID, "factor: a row of tril(A) has " + std::to_string(maxlen) +
                                          " entries (limit " + std::to_string(ic0_max_row()) + ")");
  // row schedule of tril(A), from its supernode levels
  int64_t nlev = 0;
  if ((st = supernode_row_order(L_row_ptr, L_col, n, perm.as<int32_t>(), lptr.as<int32_t>(), &nlev, s, ctx->dev)))
    return finish(ctx, st);
  const bool by_levels = !ctx->dev.ic0_sync_free;
  std::vector<int32_t> hlp;
  if (by_levels) {
    hlp.resize((size_t)nlev + 1);
    if (hipMemcpyAsync(hlp.data(), lptr.p, (nlev + 1) * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(ctx, ICPCG_E_DEVICE, "factor: level copy failed");
  }
  double alpha = 0.0;
  int restarts = 0;
  int ok = 0;
  for (restarts = 0; restarts <= max_restarts; ++restarts) {
    if (restarts > 0) alpha = std::max(alpha_min, 2.0 * alpha);
    if ((st = fill_i32(fl.as<int32_t>(), 0, 3, s))) return finish(ctx, st);  // failure flag, wait error, ticket
    if (by_levels) {
      st = ic0_factor_levels(L_row_ptr, L_col, L_val, a_low.as<double>(), n, perm.as<int32_t>(), hlp, alpha,
                             fl.as<int>(), pivots.as<double>(), s, maxlen, ctx->dev);
    } else if (!(st = fill_pending(L_val, nnzl, false, s))) {
      st = ic0_factor_sync(L_row_ptr, L_col, L_val, a_low.as<double>(), n, perm.as<int32_t>(), alpha, fl.as<int>(),
                           fl.as<int>() + 1, fl.as<int>() + 2, pivots.as<double>(), s, maxlen, ctx->dev);
    }
    if (st) return finish(ctx, st);
    int hfl[2] = {0, 0};
    if (hipMemcpyAsync(hfl, fl.p, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return fail(ctx, ICPCG_E_DEVICE, "factor: flag copy failed");
    if (hfl[1])
      return fail(ctx, ICPCG_E_DEVICE, "factor: a dependency wait reached its time limit");
    if (!hfl[0]) { ok = 1; break; }
  }
  if (restarts > max_restarts) restarts = max_restarts;
  double minp = 0.0;
  if ((st = reduce_min_f64(pivots.as<double>(), n, s, &minp))) return finish(ctx, st);
  if (info) {
    info->alpha = alpha;
    info->restarts = restarts;
    info->min_pivot = minp;
    info->nlevels = nlev;
  }
  if (!ok) return fail(ctx, ICPCG_E_PIVOT, "factor: IC(0) broke down for every shift tried");
  return ICPCG_OK;
}

icpcg_status icpcg_prec_create(icpcg_ctx *ctx, const icpcg_csr *L, icpcg_dtype dt, icpcg_prec **out) {
  if (!ctx || !valid_csr_args(L) || !out || (dt != ICPCG_F64 && dt != ICPCG_F32 && dt != ICPCG_BF16) || L->n == 0)
    return fail(ctx, ICPCG_E_INVALID, "prec_create: bad arguments");
  *out = nullptr;
  hipStream_t s = ctx->stream;
  int st = check_matrix(ctx, L, 1);
  if (st) return finish(ctx, st);
  if (L->nnz >= ((int64_t)1 << 31)) return fail(ctx, ICPCG_E_INVALID, "prec_create: factor has 2^31 or more entries");
  {
    DevBuf lens;
    if (lens.reserve(L->n * 4)) return finish(ctx, ICPCG_E_NOMEM);
    hipLaunchKernelGGL(k_row_len, dim3(1024), dim3(256), 0, s, L->row_ptr, L->n, lens.as<int32_t>());
    int32_t maxlen = 0;
    if ((st = reduce_max_i32(lens.as<int32_t>(), L->n, s, &maxlen))) return finish(ctx, st);
    if (maxlen >= (1 << 27))
      return fail(ctx, ICPCG_E_INVALID, "prec_create: a factor row has 2^27 or more entries");
  }
  icpcg_prec *P = new (std::nothrow) icpcg_prec();
  if (!P) return finish(ctx, ICPCG_E_NOMEM);
  P->n = L->n;
  P->nnz = L->nnz;
  P->dtype = dt;
  auto bail = [&](int code) { delete P; return finish(ctx, code); };
  if (P->lrp.reserve((P->n + 1) * 8) || P->lci.reserve(P->nnz * 4) || P->lval.reserve(P->nnz * 8))
    return bail(ICPCG_E_NOMEM);
  if (hipMemcpyAsync(P->lrp.p, L->row_ptr, (P->n + 1) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(P->lci.p, L->col, P->nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(P->lval.p, L->val, P->nnz * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return bail(host_error(hipGetLastError(), "copy factor", __FILE__, __LINE__));
  if ((st = build_transpose(P, s))) return bail(st);
  if ((st = build_schedule(P->lrp.as<int64_t>(), P->lci.as<int32_t>(), P->n, false, kSmax, P->sl, s, ctx->dev)))
    return bail(st);
  if ((st = build_schedule(P->urp.as<int64_t>(), P->uci.as<int32_t>(), P->n, true, kSmax, P->su, s, ctx->dev)))
    return bail(st);
  if (hipStreamSynchronize(s) != hipSuccess) return bail(host_error(hipGetLastError(), "sync", __FILE__, __LINE__));
  *out = P;
  return ICPCG_OK;
}

icpcg_status icpcg_prec_create_simple(icpcg_ctx *ctx, const icpcg_csr *A, icpcg_prec_kind kind, icpcg_prec **out) {
  if (!ctx || !valid_csr_args(A) || !out || (kind != ICPCG_PREC_JACOBI && kind != ICPCG_PREC_NONE))
    return fail(ctx, ICPCG_E_INVALID, "prec_create_simple: bad arguments");
  *out = nullptr;
  icpcg_prec *P = new (std::nothrow) icpcg_prec();
  if (!P) return finish(ctx, ICPCG_E_NOMEM);
  P->n = A->n;
  P->kind = kind;
  if (kind == ICPCG_PREC_JACOBI && A->n > 0) {
    int st = check_matrix(ctx, A, 0);
    if (!st && P->diag.reserve(A->n * 8)) st = ICPCG_E_NOMEM;
    if (st) {
      delete P;
      return finish(ctx, st);
    }
    hipLaunchKernelGGL(k_extract_diag, dim3(1024), dim3(256), 0, ctx->stream, A->row_ptr, A->col,
                       (const double *)A->val, A->n, P->diag.as<double>());
    double dmin = 0.0;
    if (hipGetLastError() != hipSuccess || reduce_min_f64(P->diag.as<double>(), A->n, ctx->stream, &dmin) != ICPCG_OK) {
      delete P;
      return fail(ctx, ICPCG_E_DEVICE, "prec_create_simple: diagonal extraction failed");
    }
    if (!(dmin > 0.0)) {
      delete P;
      return fail(ctx, ICPCG_E_INVALID, "prec_create_simple: Jacobi needs a positive diagonal");
    }
  }
  *out = P;
  return ICPCG_OK;
}

icpcg_status icpcg_dropout(icpcg_ctx *ctx, const icpcg_csr *L, double eps, int64_t *row_ptr, int32_t *col,
                           double *val, int64_t *nnz_out) {
  if (!ctx || !valid_csr_args(L) || !(eps >= 0.0) || !nnz_out || (L->n > 0 && (!row_ptr || !col || !val)))
    return fail(ctx, ICPCG_E_INVALID, "dropout: bad arguments");
  *nnz_out = 0;
  if (L->n == 0) return ICPCG_OK;
  int st = check_matrix(ctx, L, 1);
  if (st) return finish(ctx, st);
  return finish(ctx, dropout(L->row_ptr, L->col, (const double *)L->val, L->n, eps, row_ptr, col, val, nnz_out,
                             ctx->stream));
}

icpcg_status icpcg_prec_destroy(icpcg_prec *P) {
  delete P;
  return ICPCG_OK;
}

icpcg_status icpcg_prec_update_values(icpcg_ctx *ctx, icpcg_prec *P, const double *L_val) {
  if (!ctx || !P || !L_val) return fail(ctx, ICPCG_E_INVALID, "prec_update_values: bad arguments");
  if (not_factor(ctx, P, "prec_update_values")) return ICPCG_E_INVALID;
  icpcg_csr L{P->n, P->nnz, P->lrp.as<int64_t>(), P->lci.as<int32_t>(), L_val};
  int st = check_matrix(ctx, &L, 1);
  if (st) return finish(ctx, st);
  if (hipMemcpyAsync(P->lval.p, L_val, P->nnz * 8, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
    return finish(ctx, host_error(hipGetLastError(), "copy values", __FILE__, __LINE__));
  return finish(ctx, refresh_values(P, ctx->stream));
}

icpcg_status icpcg_prec_get_info(icpcg_ctx *ctx, const icpcg_prec *Pc, icpcg_prec_info *info) {
  if (!ctx || !Pc || !info) return fail(ctx, ICPCG_E_INVALID, "prec_get_info: bad arguments");
  icpcg_prec *P = const_cast<icpcg_prec *>(Pc);
  if (P->kind != ICPCG_PREC_FACTOR) {
    *info = icpcg_prec_info{};
    info->n = P->n;
    info->dtype = ICPCG_F64;
    info->kind = P->kind;
    return ICPCG_OK;
  }
  int st;
  if (P->nlev_rows_L < 0) {
    if ((st = row_levels(P->lrp.as<int64_t>(), P->lci.as<int32_t>(), P->n, false, nullptr, nullptr, nullptr,
                         &P->nlev_rows_L, ctx->stream, ctx->dev)))
      return finish(ctx, st);
  }
  if (P->nlev_rows_U < 0) {
    if ((st = row_levels(P->urp.as<int64_t>(), P->uci.as<int32_t>(), P->n, true, nullptr, nullptr, nullptr,
                         &P->nlev_rows_U, ctx->stream, ctx->dev)))
      return finish(ctx, st);
  }
  info->n = P->n;
  info->nnz = P->nnz;
  info->nlevels_L = P->nlev_rows_L;
  info->nlevels_U = P->nlev_rows_U;
  info->nsupernodes_L = P->sl.nsn;
  info->nsupernodes_U = P->su.nsn;
  info->nsn_levels_L = P->sl.nlev;
  info->nsn_levels_U = P->su.nlev;
  info->dtype = (int)P->dtype;
  info->kind = P->kind;
  return ICPCG_OK;
}

icpcg_status icpcg_prec_levels(icpcg_ctx *ctx, const icpcg_prec *Pc, int32_t *level_L, int32_t *perm_L,
                               int32_t *level_ptr_L, int32_t *level_U, int32_t *perm_U, int32_t *level_ptr_U) {
  if (!ctx || !Pc) return fail(ctx, ICPCG_E_INVALID, "prec_levels: bad arguments");
  if (not_factor(ctx, Pc, "prec_levels")) return ICPCG_E_INVALID;
  icpcg_prec *P = const_cast<icpcg_prec *>(Pc);
  int st;
  if (level_L || perm_L || level_ptr_L) {
    if ((st = row_levels(P->lrp.as<int64_t>(), P->lci.as<int32_t>(), P->n, false, level_L, perm_L, level_ptr_L,
                         &P->nlev_rows_L, ctx->stream, ctx->dev)))
      return finish(ctx, st);
  }
  if (level_U || perm_U || level_ptr_U) {
    if ((st = row_levels(P->urp.as<int64_t>(), P->uci.as<int32_t>(), P->n, true, level_U, perm_U, level_ptr_U,
                         &P->nlev_rows_U, ctx->stream, ctx->dev)))
      return finish(ctx, st);
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess)
    return finish(ctx, host_error(hipGetLastError(), "sync", __FILE__, __LINE__));
  return ICPCG_OK;
}

icpcg_status icpcg_prec_transpose(icpcg_ctx *ctx, const icpcg_prec *P, int64_t *urp, int32_t *uci, double *uval) {
  if (!ctx || !P) return fail(ctx, ICPCG_E_INVALID, "prec_transpose: bad arguments");
  if (not_factor(ctx, P, "prec_transpose")) return ICPCG_E_INVALID;
  hipStream_t s = ctx->stream;
  if ((urp && hipMemcpyAsync(urp, P->urp.p, (P->n + 1) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
      (uci && hipMemcpyAsync(uci, P->uci.p, P->nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
      (uval && hipMemcpyAsync(uval, P->uval.p, P->nnz * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return finish(ctx, host_error(hipGetLastError(), "copy transpose", __FILE__, __LINE__));
  return ICPCG_OK;
}

icpcg_status icpcg_spmv(icpcg_ctx *ctx, const icpcg_csr *A, const double *X, double *W, int64_t nrhs) {
  if (!ctx || !valid_csr_args(A) || !pow2_width(nrhs) || (A->n > 0 && (!X || !W)))
    return fail(ctx, ICPCG_E_INVALID, "spmv: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  return finish(ctx, spmv(A->row_ptr, A->col, A->val, A->n, X, W, (int)nrhs, spmv_default_slots((int)nrhs),
                          ctx->stream));
}

icpcg_status icpcg_trsv(icpcg_ctx *ctx, const icpcg_prec *P, int transpose, const void *R, int r_is_f64, void *Y,
                        int64_t nrhs) {
  if (!ctx || !P || !R || !Y || !pow2_width(nrhs))
    return fail(ctx, ICPCG_E_INVALID, "trsv: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  if (not_factor(ctx, P, "trsv")) return ICPCG_E_INVALID;
  const bool lo = P->dtype != ICPCG_F64;
  int st = fill_pending(Y, P->n * nrhs, lo, ctx->stream);
  if (st) return finish(ctx, st);
  return finish(ctx, trsv(P, transpose != 0, R, lo ? r_is_f64 != 0 : true, Y, (int)nrhs, nrhs, ctx->stream, ctx->dev,
                          &dev_flags(ctx)->err));
}

icpcg_status icpcg_apply(icpcg_ctx *ctx, const icpcg_prec *P, const void *R, int r_is_f64, void *Y, void *Z,
                         int64_t nrhs) {
  if (!ctx || !P || !R || !Y || !Z || !pow2_width(nrhs))
    return fail(ctx, ICPCG_E_INVALID, "apply: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  if (not_factor(ctx, P, "apply")) return ICPCG_E_INVALID;
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  int st;
  if ((st = fill_pending(Y, P->n * nrhs, lo, s))) return finish(ctx, st);
  if ((st = trsv(P, false, R, lo ? r_is_f64 != 0 : true, Y, (int)nrhs, nrhs, s, ctx->dev, &dev_flags(ctx)->err)))
    return finish(ctx, st);
  if ((st = fill_pending(Z, P->n * nrhs, lo, s))) return finish(ctx, st);
  return finish(ctx, trsv(P, true, Y, !lo, Z, (int)nrhs, nrhs, s, ctx->dev, &dev_flags(ctx)->err));
}

icpcg_status icpcg_apply_rz(icpcg_ctx *ctx, const icpcg_prec *P, const double *R, void *Y, void *Z, double *rz,
                            int64_t nrhs) {
  if (!ctx || !P || !R || !Y || !Z || !rz || !pow2_width(nrhs))
    return fail(ctx, ICPCG_E_INVALID, "apply_rz: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  if (not_factor(ctx, P, "apply_rz")) return ICPCG_E_INVALID;
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  Workspace &ws = ctx->ws;
  if (ws.partials.reserve((size_t)kMaxDotBlocks * nrhs * 2 * 8)) return finish(ctx, ICPCG_E_NOMEM);
  double *part = ws.partials.as<double>();
  int *err = &dev_flags(ctx)->err;
  const int Rw = (int)nrhs;
  int st;
  if ((st = fill_pending(Y, P->n * nrhs, lo, s))) return finish(ctx, st);
  if ((st = trsv(P, false, R, true, Y, Rw, nrhs, s, ctx->dev, err))) return finish(ctx, st);
  if ((st = fill_pending(Z, P->n * nrhs, lo, s))) return finish(ctx, st);
  if (trsv_fuses_rz(P, Rw, ctx->dev)) {
    RzDot d{R, part, nullptr, nullptr, rz};
    return finish(ctx, trsv(P, true, Y, !lo, Z, Rw, nrhs, s, ctx->dev, err, nullptr, d));
  }
  if ((st = trsv(P, true, Y, !lo, Z, Rw, nrhs, s, ctx->dev, err))) return finish(ctx, st);
  return finish(ctx, col_dot_out(P->n, Rw, R, Z, lo, part, rz, s));
}

icpcg_status icpcg_trsv_rz(icpcg_ctx *ctx, const icpcg_prec *P, const void *Y, const double *R, void *Z, double *rz,
                           int64_t nrhs) {
  if (!ctx || !P || !Y || !R || !Z || !rz || !pow2_width(nrhs))
    return fail(ctx, ICPCG_E_INVALID, "trsv_rz: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  if (not_factor(ctx, P, "trsv_rz")) return ICPCG_E_INVALID;
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  Workspace &ws = ctx->ws;
  if (ws.partials.reserve((size_t)kMaxDotBlocks * nrhs * 2 * 8)) return finish(ctx, ICPCG_E_NOMEM);
  double *part = ws.partials.as<double>();
  int *err = &dev_flags(ctx)->err;
  const int Rw = (int)nrhs;
  int st;
  if ((st = fill_pending(Z, P->n * nrhs, lo, s))) return finish(ctx, st);
  if (trsv_fuses_rz(P, Rw, ctx->dev)) {
    RzDot d{R, part, nullptr, nullptr, rz};
    return finish(ctx, trsv(P, true, Y, !lo, Z, Rw, nrhs, s, ctx->dev, err, nullptr, d));
  }
  if ((st = trsv(P, true, Y, !lo, Z, Rw, nrhs, s, ctx->dev, err))) return finish(ctx, st);
  return finish(ctx, col_dot_out(P->n, Rw, R, Z, lo, part, rz, s));
}

icpcg_status icpcg_apply_rz_noalloc(icpcg_ctx *ctx, const icpcg_prec *P, const double *R, void *Y, void *Z,
                                    double *rz, int64_t nrhs) {
  if (!ctx || !P || !R || !Y || !Z || !rz || !pow2_width(nrhs))
    return fail(ctx, ICPCG_E_INVALID, "apply_rz_noalloc: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  if (not_factor(ctx, P, "apply_rz_noalloc")) return ICPCG_E_INVALID;
  double *part = scratch_ptr(ctx->dev.id);
  if (!part) {
    int st = scratch_init(ctx->dev.id);  // context created on another device than this one
    if (st) return finish(ctx, st);
    part = scratch_ptr(ctx->dev.id);
  }
  // bound on the blocks either reduction launches (16 per CU, or the separate
  // pass's 1024), checked before any work is queued
  const int64_t blocks = std::max<int64_t>(16 * (int64_t)ctx->dev.num_cu, 1024);
  if (blocks * nrhs > kScratchDoubles)
    return fail(ctx, ICPCG_E_INVALID,
                "apply_rz_noalloc: " + std::to_string(nrhs) + " columns on " + std::to_string(ctx->dev.num_cu) +
                    " CUs need more than the " + std::to_string(kScratchDoubles) + " partials of the static scratch");
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  int *err = &dev_flags(ctx)->err;
  const int Rw = (int)nrhs;
  int st;
  if ((st = fill_pending(Y, P->n * nrhs, lo, s))) return finish(ctx, st);
  if ((st = trsv(P, false, R, true, Y, Rw, nrhs, s, ctx->dev, err))) return finish(ctx, st);
  if ((st = fill_pending(Z, P->n * nrhs, lo, s))) return finish(ctx, st);
  if (trsv_fuses_rz(P, Rw, ctx->dev)) {
    RzDot d{R, part, nullptr, nullptr, rz, kScratchDoubles};
    return finish(ctx, trsv(P, true, Y, !lo, Z, Rw, nrhs, s, ctx->dev, err, nullptr, d));
  }
  if ((st = trsv(P, true, Y, !lo, Z, Rw, nrhs, s, ctx->dev, err))) return finish(ctx, st);
  return finish(ctx, col_dot_out(P->n, Rw, R, Z, lo, part, rz, s));
}

icpcg_status icpcg_apply_backward(icpcg_ctx *ctx, const icpcg_prec *P, const void *G, const void *Y, const void *Z,
                                  void *Ybar, void *dR, void *dL, int64_t nrhs) {
  if (!ctx || !P || !G || !Y || !Z || !Ybar || !dR || !dL || !pow2_width(nrhs))
    return fail(ctx, ICPCG_E_INVALID, "apply_backward: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  if (not_factor(ctx, P, "apply_backward")) return ICPCG_E_INVALID;
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  int st;
  if ((st = fill_pending(Ybar, P->n * nrhs, lo, s))) return finish(ctx, st);
  if ((st = trsv(P, false, G, !lo, Ybar, (int)nrhs, nrhs, s, ctx->dev, &dev_flags(ctx)->err))) return finish(ctx, st);
  if ((st = fill_pending(dR, P->n * nrhs, lo, s))) return finish(ctx, st);
  if ((st = trsv(P, true, Ybar, !lo, dR, (int)nrhs, nrhs, s, ctx->dev, &dev_flags(ctx)->err))) return finish(ctx, st);
  return finish(ctx, prec_dL(P, Z, Ybar, dR, Y, dL, (int)nrhs, s));
}

icpcg_status icpcg_sync(icpcg_ctx *ctx) {
  if (!ctx) return ICPCG_E_INVALID;
  return finish(ctx, take_wait_error(ctx));
}

}  // extern "C"

// ------------------------------------------------------------------ PCG

namespace {

struct PassBuffers {
  double *r, *p, *w, *B, *X;
  void *y, *z;
  double *partials;
  ColState *cols;
  const SpGroup *grec;  // row groups of A (identical column lists)
  int64_t ngroups;
};

// w = A x (optionally with p^T w and alpha) through the row-group
// kernel when groups are available.
int spmv_pass(const icpcg_csr *A, const PassBuffers &b, const double *x, double *y, int R, hipStream_t s,
              double *partials = nullptr, ColState *cols = nullptr, const int *active = nullptr) {
  if (b.grec)
    return spmv_grouped(A->col, A->val, b.ngroups, b.grec, A->n, x, y, R, spmv_grouped_default_slots(R), s,
                        partials, cols, active);
  return spmv(A->row_ptr, A->col, A->val, A->n, x, y, R, spmv_default_slots(R), s, partials, cols, active);
}

// `count` PCG steps of supplementary Algorithm 1 on stream s: z = L^-T L^-1 r,
// r'z and beta (formed by the backward solve for FP32 / BF16 factors on several
// columns), p = z + beta p, w = A p with p'w, then alpha, x, r and ||r|| (for
// those factors formed by the next step's forward solve, ahead of its solve).
// Queued steps return at once when no column is active.
int enqueue_steps(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P, const PassBuffers &b, int R,
                  int64_t max_iter, int count, hipStream_t s, bool timed = false) {
  const int64_t n = A->n;
  const bool lo = P->dtype != ICPCG_F64;
  SolveFlags *fl = dev_flags(ctx);
  int *err = &fl->err;
  const int *act = &fl->n_active;
  int st;
  // phase boundaries of the step (icpcg_step_timing; eager steps only)
  auto mark = [&](int m) -> int {
    if (!timed || ctx->tsteps >= icpcg_ctx::kTimedSteps) return ICPCG_OK;
    ICPCG_HIP_TRY(hipEventRecord(ctx->tev[ctx->tsteps * icpcg_ctx::kPhaseMarks + m], s));
    return ICPCG_OK;
  };
  // the x, r update of a step applied by the next step's forward solve, whose
  // ||r||^2 then drives the stop tests (the updated x and r, and the tests,
  // are those of the separate pass; the queued forward solve of a column that
  // stops there goes unused)
  const bool fxr = P->kind == ICPCG_PREC_FACTOR && trsv_fuses_xr(P, R, ctx->dev);
  XrUpd xr{};
  if (fxr) {
    xr.X = b.X;
    xr.r = b.r;
    xr.p = b.p;
    xr.w = b.w;
    xr.cols = b.cols;
    xr.partials = b.partials;
    xr.max_iter = max_iter;
    xr.flags = fl;
  }
  for (int k = 0; k < count; ++k) {
    if ((st = mark(0))) return st;
    if (P->kind != ICPCG_PREC_FACTOR) {
      if ((st = pcg_diag_apply(n, R, b.r, P->kind == ICPCG_PREC_JACOBI ? P->diag.as<double>() : nullptr,
                               static_cast<double *>(b.z), act, s)))
        return st;
    } else {
      if ((st = trsv(P, false, b.r, true, b.y, R, R, s, ctx->dev, err, act, RzDot{}, xr))) return st;
      if ((st = mark(1))) return st;
      // the backward solve also forms r^T z and beta where that pays, and then
      // re-arms y (its right-hand side) for the next step's forward solve
      RzDot rz{};
      if (trsv_fuses_rz(P, R, ctx->dev)) {
        rz.r = b.r;
        rz.partials = b.partials;
        rz.cols = b.cols;
        rz.flags = fl;
        rz.rearm_rhs = true;
      }
      if ((st = trsv(P, true, b.y, !lo, b.z, R, R, s, ctx->dev, err, act, rz))) return st;
    }
    if (P->kind != ICPCG_PREC_FACTOR && (st = mark(1))) return st;
    if (!(P->kind == ICPCG_PREC_FACTOR && trsv_fuses_rz(P, R, ctx->dev)) &&
        (st = pcg_dot_rz(n, R, b.r, b.z, lo, b.partials, b.cols, fl, s)))
      return st;
    if ((st = mark(2))) return st;
    const bool y_rearmed = P->kind == ICPCG_PREC_FACTOR && trsv_fuses_rz(P, R, ctx->dev);
    if ((st = pcg_update_p(n, R, b.z, lo, b.p, y_rearmed ? nullptr : b.y, b.cols, fl, s))) return st;
    if ((st = mark(3))) return st;
    if (b.grec) {
      // w = A p, then p^T w and alpha in their own pass (what the grouped
      // SpMV launch does with partials, split here at a phase boundary)
      if ((st = spmv_grouped(A->col, A->val, b.ngroups, b.grec, n, b.p, b.w, R, spmv_grouped_default_slots(R), s,
                             nullptr, nullptr, act)))
        return st;
      if ((st = mark(4))) return st;
      if ((st = pcg_dot_pw(n, R, b.p, b.w, b.partials, b.cols, fl, s))) return st;
    } else {
      // the row kernel forms p^T w in its epilogue (the p^T w phase is empty)
      if ((st = spmv_pass(A, b, b.p, b.w, R, s, b.partials, b.cols, act))) return st;
      if ((st = mark(4))) return st;
    }
    if ((st = mark(5))) return st;
    if (!fxr && (st = pcg_update_xr(n, R, b.X, b.r, b.p, b.w, b.partials, b.cols, max_iter, fl, s))) return st;
    if ((st = mark(6))) return st;
    if (timed && ctx->tsteps < icpcg_ctx::kTimedSteps) ++ctx->tsteps;
  }
  return ICPCG_OK;
}

// The graph of `count` steps: captured on the context's private stream the
// first time, then reused while every pointer and size the launches bake in
// is the same (the values behind the pointers may change freely).
int step_graph(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P, const PassBuffers &b, int R,
               int64_t max_iter, int count, hipGraphExec_t *out) {
  auto u = [](const void *p) { return (uintptr_t)p; };
  const std::vector<uintptr_t> key = {
      u(A->row_ptr), u(A->col), u(A->val), (uintptr_t)A->n, u(b.grec), (uintptr_t)b.ngroups, u(P),
      (uintptr_t)P->dtype, u(P->lci.p), u(P->uci.p), u(P->lval.p), u(P->uval.p), u(P->lval_lo.p),
      u(P->uval_lo.p), u(P->sl.items.p), u(P->su.items.p), (uintptr_t)P->sl.nsn, (uintptr_t)P->su.nsn,
      (uintptr_t)P->kind, u(P->diag.p),
      u(b.r), u(b.p), u(b.w), u(b.y), u(b.z), u(b.X), u(b.partials), u(b.cols), u(dev_flags(ctx)),
      (uintptr_t)R, (uintptr_t)max_iter, (uintptr_t)count, (uintptr_t)ctx->dev.wait_ticks,
      (uintptr_t)ctx->dev.trsv_waves_per_cu, (uintptr_t)spmv_grouped_default_slots(R),
      (uintptr_t)spmv_default_slots(R)};
  if (ctx->step_exec && key == ctx->step_key) {
    *out = ctx->step_exec;
    return ICPCG_OK;
  }
  if (ctx->step_exec) {
    ICPCG_HIP_TRY(hipGraphExecDestroy(ctx->step_exec));
    ctx->step_exec = nullptr;
    ctx->step_key.clear();
  }
  if (!ctx->capture) ICPCG_HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  ICPCG_HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed));
  const int st = enqueue_steps(ctx, A, P, b, R, max_iter, count, ctx->capture);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->capture, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return host_error(e, "hipStreamEndCapture", __FILE__, __LINE__);
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return host_error(ei, "hipGraphInstantiate", __FILE__, __LINE__);
  ctx->step_exec = ex;
  ctx->step_key = key;
  *out = ex;
  return ICPCG_OK;
}

// One block of R columns through supplementary Algorithm 1 with the stop,
// replacement and failure rules stated in icpcg.h.
int run_pass(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P, const PassBuffers &b, int R,
             const icpcg_solve_opts &o, int64_t max_iter) {
  hipStream_t s = ctx->stream;
  const int64_t n = A->n;
  const bool lo = P->dtype != ICPCG_F64;
  SolveFlags *fl = dev_flags(ctx);
  int st;
  ICPCG_HIP_TRY(hipMemsetAsync(fl, 0, sizeof(SolveFlags), s));
  if ((st = spmv_pass(A, b, b.X, b.w, R, s))) return st;
  if ((st = pcg_init(n, R, b.B, b.w, b.r, b.p, b.y, b.z, lo, o.rtol, b.partials, b.cols, max_iter, fl, s))) return st;
  if ((st = pcg_zero_x(n, R, b.X, b.cols, s))) return st;
  const int every = o.check_every > 0 ? o.check_every : 8;
  hipGraphExec_t exec = nullptr;
  if (o.use_graph && (st = step_graph(ctx, A, P, b, R, max_iter, every, &exec))) return st;
  const int64_t guard = max_iter * (int64_t)(o.max_replace + 1) + 16;
  int64_t steps = 0;
  for (;;) {
    SolveFlags h;
    if ((st = read_flags(ctx, &h))) return st;
    if (h.err) {
      set_error("a device-side dependency wait exceeded its time limit");
      return ICPCG_E_DEVICE;
    }
    if (h.n_active == 0) {
      if (h.n_conv == 0) break;
      if ((st = spmv_pass(A, b, b.X, b.w, R, s))) return st;
      if ((st = pcg_true_residual(n, R, b.B, b.w, b.partials, b.cols, max_iter, o.max_replace, 0, fl, s))) return st;
      if ((st = pcg_replace_r(n, R, b.w, b.r, b.cols, s))) return st;
      // The step that stopped the last active column may have ended before its
      // p update (a breakdown of r^T z), which is where y and z are re-armed for
      // the next solves: re-arm them here, so a column that a replacement
      // re-activates never reads an earlier step's values as published.
      if (P->kind == ICPCG_PREC_FACTOR &&
          ((st = fill_pending(b.y, n * R, lo, s)) || (st = fill_pending(b.z, n * R, lo, s))))
        return st;
      continue;
    }
    if (steps > guard) {
      set_error("solve: step guard exceeded");
      return ICPCG_E_DEVICE;
    }
    if (exec)
      ICPCG_HIP_TRY(hipGraphLaunch(exec, s));
    else if ((st = enqueue_steps(ctx, A, P, b, R, max_iter, every, s, ctx->timing)))
      return st;
    steps += every;
  }
  // final true residual of every column (reported)
  if ((st = spmv_pass(A, b, b.X, b.w, R, s))) return st;
  if ((st = pcg_true_residual(n, R, b.B, b.w, b.partials, b.cols, max_iter, o.max_replace, 1, fl, s))) return st;
  return ICPCG_OK;
}

}  // namespace

namespace {

int reserve_pass(Workspace &ws, int64_t n, int Rb, bool lo, bool gathered) {
  const size_t vec8 = (size_t)n * Rb * 8, vecy = (size_t)n * Rb * (lo ? 4 : 8);
  if (ws.r.reserve(vec8) || ws.p.reserve(vec8) || ws.w.reserve(vec8) || ws.y.reserve(vecy) || ws.z.reserve(vecy) ||
      ws.partials.reserve((size_t)kMaxDotBlocks * Rb * 2 * 8) || ws.cols.reserve(sizeof(ColState) * Rb))
    return ICPCG_E_NOMEM;
  if (gathered && (ws.tmp0.reserve(vec8) || ws.tmp1.reserve(vec8))) return ICPCG_E_NOMEM;
  return ICPCG_OK;
}

int width_slot(int w) { return w == 1 ? 0 : w == 2 ? 1 : w == 4 ? 2 : w == 8 ? 3 : 4; }

// Block-width autotuner: for each width w up to the smallest power of two
// >= nrhs (at most 16) it times the bandwidth-heavy part of one PCG step at
// that width on the real operands (re-arming y and z, both triangular
// solves, the SpMV) and picks the width with the least time for all nrhs
// columns, ceil(nrhs / w) passes of it. Decisions are cached per context.
int tune_width(icpcg_ctx *ctx, const icpcg_mat *M, const icpcg_prec *P, int64_t nrhs, int *width, double ms[5]) {
  const icpcg_csr *A = &M->A;
  const int64_t n = A->n;
  const std::vector<uintptr_t> key = {(uintptr_t)A->row_ptr, (uintptr_t)A->col, (uintptr_t)A->val, (uintptr_t)n,
                                      (uintptr_t)A->nnz,     (uintptr_t)P,      (uintptr_t)P->dtype,
                                      (uintptr_t)P->nnz,     (uintptr_t)std::min<int64_t>(nrhs, 1 << 20)};
  for (const auto &t : ctx->tunes)
    if (t.key == key) {
      *width = t.width;
      for (int i = 0; i < 5; ++i) ms[i] = t.ms[i];
      return ICPCG_OK;
    }
  for (int i = 0; i < 5; ++i) ms[i] = 0.0;
  int wmax = 1;
  while (wmax < nrhs && wmax < 16) wmax <<= 1;
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  int st = reserve_pass(ctx->ws, n, wmax, lo, false);
  if (st) return st;
  Workspace &ws = ctx->ws;
  ICPCG_HIP_TRY(hipMemsetAsync(ws.r.p, 0, (size_t)n * wmax * 8, s));
  ICPCG_HIP_TRY(hipMemsetAsync(ws.p.p, 0, (size_t)n * wmax * 8, s));
  PassBuffers b{};
  b.grec = M->grouped ? M->grec.as<SpGroup>() : nullptr;
  b.ngroups = M->ngroups;
  int *err = &dev_flags(ctx)->err;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ICPCG_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return host_error(hipGetLastError(), "hipEventCreate", __FILE__, __LINE__);
  }
  auto one_step = [&](int w) -> int {
    int r;
    if (P->kind != ICPCG_PREC_FACTOR) {
      if ((r = pcg_diag_apply(n, w, ws.r.as<double>(), P->kind == ICPCG_PREC_JACOBI ? P->diag.as<double>() : nullptr,
                              ws.z.as<double>(), nullptr, s)))
        return r;
      return spmv_pass(A, b, ws.p.as<double>(), ws.w.as<double>(), w, s);
    }
    if ((r = fill_pending(ws.y.p, n * w, lo, s))) return r;
    if ((r = trsv(P, false, ws.r.p, true, ws.y.p, w, w, s, ctx->dev, err))) return r;
    if ((r = fill_pending(ws.z.p, n * w, lo, s))) return r;
    if ((r = trsv(P, true, ws.y.p, !lo, ws.z.p, w, w, s, ctx->dev, err))) return r;
    return spmv_pass(A, b, ws.p.as<double>(), ws.w.as<double>(), w, s);
  };
  constexpr int kReps = 3;
  double best = 0.0;
  int best_w = 1;
  for (int w = 1; w <= wmax && !st; w <<= 1) {
    if ((st = one_step(w))) break;  // warm-up (code objects, caches)
    if (hipEventRecord(e0, s) != hipSuccess) { st = host_error(hipGetLastError(), "hipEventRecord", __FILE__, __LINE__); break; }
    for (int k = 0; k < kReps && !st; ++k) st = one_step(w);
    if (st) break;
    float t = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      st = host_error(hipGetLastError(), "autotune timing", __FILE__, __LINE__);
      break;
    }
    const double step = (double)t / kReps;
    ms[width_slot(w)] = step;
    const double total = step * (double)((nrhs + w - 1) / w);
    if (w == 1 || total < best) {
      best = total;
      best_w = w;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if ((st = take_wait_error(ctx))) return st;
  ctx->tunes.push_back(icpcg_ctx::Tune{key, best_w, {ms[0], ms[1], ms[2], ms[3], ms[4]}});
  *width = best_w;
  return ICPCG_OK;
}

}  // namespace

static icpcg_status solve_impl(icpcg_ctx *ctx, const icpcg_mat *M, const icpcg_prec *P, const double *B, double *X,
                               int64_t nrhs, const icpcg_solve_opts *opts, icpcg_col_info *info) {
  const icpcg_csr *A = &M->A;
  if (!valid_csr_args(A) || !P || nrhs < 1 || A->n != P->n || (A->n > 0 && (!B || !X)))
    return fail(ctx, ICPCG_E_INVALID, "solve: bad arguments");
  icpcg_solve_opts o{1e-8, 0, 3, 0, 8, 0};
  if (opts) o = *opts;
  if (!(o.rtol >= 0.0)) return fail(ctx, ICPCG_E_INVALID, "solve: rtol must be >= 0");
  if (o.max_replace < 0) o.max_replace = 3;
  const int64_t n = A->n;
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : default_max_iter(n);
  if (n == 0) {
    if (info)
      for (int64_t c = 0; c < nrhs; ++c) info[c] = icpcg_col_info{0, 0, ICPCG_OK, 0.0, 0.0};
    return ICPCG_OK;
  }
  int Rb = o.block_width;
  if (Rb != 0 && !pow2_width(Rb)) return fail(ctx, ICPCG_E_INVALID, "solve: block_width must be 0, 1, 2, 4, 8 or 16");
  if (Rb == 0) {
    double ms[5];
    const int st = nrhs == 1 ? (Rb = 1, ICPCG_OK) : tune_width(ctx, M, P, nrhs, &Rb, ms);
    if (st) return finish(ctx, st);
  }
  const bool lo = P->dtype != ICPCG_F64;
  hipStream_t s = ctx->stream;
  Workspace &ws = ctx->ws;
  const bool gathered = nrhs != Rb;
  if (reserve_pass(ws, n, Rb, lo, gathered)) return finish(ctx, ICPCG_E_NOMEM);
  int worst = ICPCG_OK;
  std::vector<ColState> hc(Rb);
  for (int64_t c0 = 0; c0 < nrhs; c0 += Rb) {
    const int nc = (int)std::min<int64_t>(Rb, nrhs - c0);
    PassBuffers b;
    b.r = ws.r.as<double>();
    b.p = ws.p.as<double>();
    b.w = ws.w.as<double>();
    b.y = ws.y.p;
    b.z = ws.z.p;
    b.partials = ws.partials.as<double>();
    b.cols = ws.cols.as<ColState>();
    b.grec = M->grouped ? M->grec.as<SpGroup>() : nullptr;
    b.ngroups = M->ngroups;
    int st;
    if (gathered) {
      b.B = ws.tmp0.as<double>();
      b.X = ws.tmp1.as<double>();
      if ((st = gather_cols(n, Rb, B, nrhs, c0, nc, b.B, s)) || (st = gather_cols(n, Rb, X, nrhs, c0, nc, b.X, s)))
        return finish(ctx, st);
    } else {
      b.B = const_cast<double *>(B);
      b.X = X;
    }
    if ((st = run_pass(ctx, A, P, b, Rb, o, max_iter))) return finish(ctx, st);
    if (gathered && (st = scatter_cols(n, Rb, b.X, X, nrhs, c0, nc, s))) return finish(ctx, st);
    if (hipMemcpyAsync(hc.data(), b.cols, sizeof(ColState) * Rb, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return finish(ctx, host_error(hipGetLastError(), "copy column states", __FILE__, __LINE__));
    for (int c = 0; c < nc; ++c) {
      const ColState &cs = hc[c];
      if (info) {
        info[c0 + c].iters = cs.iters;
        info[c0 + c].replacements = cs.repl;
        info[c0 + c].status = cs.status;
        info[c0 + c].relres = cs.bb > 0 ? std::sqrt(cs.rr / cs.bb) : 0.0;
        info[c0 + c].true_relres = cs.bb > 0 ? std::sqrt(cs.trr / cs.bb) : 0.0;
      }
      if (cs.status > worst) worst = cs.status;
    }
  }
  if (worst != ICPCG_OK) {
    set_error(std::string("solve: at least one column ended with status '") +
              icpcg_status_string((icpcg_status)worst) + "'");
    return finish(ctx, worst);
  }
  return ICPCG_OK;
}

namespace {
int mat_init(icpcg_ctx *ctx, const icpcg_csr *A, icpcg_mat *M) {
  M->A = *A;
  if (A->n == 0) return ICPCG_OK;
  int st = check_matrix(ctx, A, 0);
  if (st) return st;
  // the group records hold row lengths in 28 bits
  bool short_rows = A->nnz < (int64_t{1} << 28);
  if (!short_rows) {
    DevBuf lens;
    if (lens.reserve(A->n * 4)) return ICPCG_E_NOMEM;
    hipLaunchKernelGGL(k_row_len, dim3(256), dim3(256), 0, ctx->stream, A->row_ptr, A->n, lens.as<int32_t>());
    ICPCG_HIP_TRY(hipGetLastError());
    int32_t maxlen = 0;
    if ((st = reduce_max_i32(lens.as<int32_t>(), A->n, ctx->stream, &maxlen))) return st;
    short_rows = maxlen < (1 << 28);
  }
  if (!short_rows || std::getenv("ICPCG_NO_ROW_GROUPS")) return ICPCG_OK;
  if ((st = build_row_groups(A->row_ptr, A->col, A->n, kSupernodeMax, M->gptr, M->grec, &M->ngroups, ctx->stream)))
    return st;
  M->grouped = M->ngroups < A->n;
  return ICPCG_OK;
}
}  // namespace

extern "C" icpcg_status icpcg_mat_create(icpcg_ctx *ctx, const icpcg_csr *A, icpcg_mat **out) {
  if (!ctx || !valid_csr_args(A) || !out) return fail(ctx, ICPCG_E_INVALID, "mat_create: bad arguments");
  *out = nullptr;
  icpcg_mat *M = new (std::nothrow) icpcg_mat();
  if (!M) return finish(ctx, ICPCG_E_NOMEM);
  const int st = mat_init(ctx, A, M);
  if (st) {
    delete M;
    return finish(ctx, st);
  }
  *out = M;
  return ICPCG_OK;
}

extern "C" icpcg_status icpcg_mat_destroy(icpcg_mat *M) {
  delete M;
  return ICPCG_OK;
}

extern "C" icpcg_status icpcg_mat_spmv(icpcg_ctx *ctx, const icpcg_mat *M, const double *X, double *W, int64_t nrhs) {
  if (!ctx || !M || !pow2_width(nrhs) || (M->A.n > 0 && (!X || !W)))
    return fail(ctx, ICPCG_E_INVALID, "mat_spmv: bad arguments (nrhs must be 1, 2, 4, 8 or 16)");
  const icpcg_csr *A = &M->A;
  if (!M->grouped)
    return finish(ctx, spmv(A->row_ptr, A->col, A->val, A->n, X, W, (int)nrhs, spmv_default_slots((int)nrhs),
                            ctx->stream));
  return finish(ctx, spmv_grouped(A->col, A->val, M->ngroups, M->grec.as<SpGroup>(), A->n, X, W, (int)nrhs,
                                  spmv_grouped_default_slots((int)nrhs), ctx->stream));
}

extern "C" icpcg_status icpcg_autotune(icpcg_ctx *ctx, const icpcg_mat *M, const icpcg_prec *P, int64_t nrhs,
                                       icpcg_tune_info *info) {
  if (!ctx || !M || !P || nrhs < 1 || M->A.n != P->n || !info) return fail(ctx, ICPCG_E_INVALID, "autotune: bad arguments");
  *info = icpcg_tune_info{};
  if (M->A.n == 0) {
    info->block_width = 1;
    return ICPCG_OK;
  }
  int w = 1;
  const int st = tune_width(ctx, M, P, nrhs, &w, info->ms_per_step);
  if (st) return finish(ctx, st);
  info->block_width = w;
  info->ms_per_rhs = info->ms_per_step[width_slot(w)] * (double)((nrhs + w - 1) / w) / (double)nrhs;
  return ICPCG_OK;
}

extern "C" icpcg_status icpcg_solve_mat(icpcg_ctx *ctx, const icpcg_mat *M, const icpcg_prec *P, const double *B,
                                        double *X, int64_t nrhs, const icpcg_solve_opts *opts, icpcg_col_info *info) {
  if (!ctx || !M) return fail(ctx, ICPCG_E_INVALID, "solve: bad arguments");
  return solve_impl(ctx, M, P, B, X, nrhs, opts, info);
}

extern "C" icpcg_status icpcg_solve(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P, const double *B,
                                    double *X, int64_t nrhs, const icpcg_solve_opts *opts, icpcg_col_info *info) {
  if (!ctx || !valid_csr_args(A)) return fail(ctx, ICPCG_E_INVALID, "solve: bad arguments");
  icpcg_mat M;
  const int st = mat_init(ctx, A, &M);
  if (st) return finish(ctx, st);
  return solve_impl(ctx, &M, P, B, X, nrhs, opts, info);
}

// ------------------------------------------------- learned factor correction

extern "C" int64_t icpcg_gnn_num_params(void) { return gnn_num_params(); }

extern "C" icpcg_status icpcg_gnn_create(icpcg_ctx *ctx, const icpcg_csr *A, const icpcg_prec *P, icpcg_gnn **out) {
  if (!ctx || !valid_csr_args(A) || !P || !out || A->n != P->n || A->n == 0)
    return fail(ctx, ICPCG_E_INVALID, "gnn_create: bad arguments");
  *out = nullptr;
  if (not_factor(ctx, P, "gnn_create")) return ICPCG_E_INVALID;
  if (P->dtype != ICPCG_F64) return fail(ctx, ICPCG_E_INVALID, "gnn_create: the preconditioner must be FP64 (L_IC)");
  int st = check_matrix(ctx, A, 0);
  if (st) return finish(ctx, st);
  icpcg_gnn *G = new (std::nothrow) icpcg_gnn();
  if (!G) return finish(ctx, ICPCG_E_NOMEM);
  if ((st = gnn_setup(G, A, P, ctx->stream))) {
    delete G;
    return finish(ctx, st);
  }
  *out = G;
  return ICPCG_OK;
}

extern "C" icpcg_status icpcg_gnn_destroy(icpcg_gnn *G) {
  delete G;
  return ICPCG_OK;
}

extern "C" icpcg_status icpcg_gnn_inputs(icpcg_ctx *ctx, const icpcg_gnn *G, double *x, double *e, double *scale) {
  if (!ctx || !G) return fail(ctx, ICPCG_E_INVALID, "gnn_inputs: bad arguments");
  if (scale) *scale = G->scale;
  return finish(ctx, gnn_inputs(G, x, e, ctx->stream));
}

extern "C" icpcg_status icpcg_gnn_forward(icpcg_ctx *ctx, icpcg_gnn *G, const double *theta, double *L_val) {
  if (!ctx || !G || !theta || !L_val) return fail(ctx, ICPCG_E_INVALID, "gnn_forward: bad arguments");
  return finish(ctx, gnn_forward(G, theta, L_val, false, ctx->stream));
}

extern "C" icpcg_status icpcg_gnn_loss_grad(icpcg_ctx *ctx, icpcg_gnn *G, const double *theta, const double *z,
                                            double *loss, double *grad, int accumulate) {
  if (!ctx || !G || !theta || !z || !loss || !grad) return fail(ctx, ICPCG_E_INVALID, "gnn_loss_grad: bad arguments");
  return finish(ctx, gnn_loss_grad(G, theta, z, loss, grad, accumulate != 0, ctx->stream));
}

extern "C" icpcg_status icpcg_adam_step(icpcg_ctx *ctx, double *theta, const double *grad, double *m, double *v,
                                        int64_t count, int64_t t, double lr, double beta1, double beta2, double eps) {
  if (!ctx || count < 0 || t < 1 || (count > 0 && (!theta || !grad || !m || !v)))
    return fail(ctx, ICPCG_E_INVALID, "adam_step: bad arguments");
  if (count == 0) return ICPCG_OK;
  return finish(ctx, adam_step(theta, grad, m, v, count, t, lr, beta1, beta2, eps, ctx->stream));
}

// ------------------------------------------------------ multicolour ordering

extern "C" icpcg_status icpcg_color_order(icpcg_ctx *ctx, const icpcg_csr *A, uint64_t seed, int32_t *perm,
                                          int32_t *ncolours) {
  if (!ctx || !valid_csr_args(A) || !ncolours || (A->n > 0 && !perm))
    return fail(ctx, ICPCG_E_INVALID, "color_order: bad arguments");
  *ncolours = 0;
  if (A->n == 0) return ICPCG_OK;
  int st = check_matrix(ctx, A, 0);
  if (st) return finish(ctx, st);
  return finish(ctx, color_order(A->row_ptr, A->col, A->n, seed, perm, ncolours, ctx->stream));
}

extern "C" icpcg_status icpcg_block_color_order(icpcg_ctx *ctx, const icpcg_csr *A, const int32_t *block,
                                                int32_t nblocks, int32_t *perm, int32_t *ncolours) {
  if (!ctx || !valid_csr_args(A) || !ncolours || (A->n > 0 && (!perm || !block || nblocks < 1)) ||
      A->nnz >= (int64_t{1} << 32))
    return fail(ctx, ICPCG_E_INVALID, "block_color_order: bad arguments");
  *ncolours = 0;
  if (A->n == 0) return ICPCG_OK;
  int st = check_matrix(ctx, A, 0);
  if (st) return finish(ctx, st);
  return finish(ctx, block_color_order(A->row_ptr, A->col, A->n, A->nnz, block, nblocks, perm, ncolours, ctx->stream));
}

extern "C" icpcg_status icpcg_permute_matrix(icpcg_ctx *ctx, const icpcg_csr *A, const int32_t *perm,
                                             int64_t *row_ptr, int32_t *col, double *val) {
  if (!ctx || !valid_csr_args(A) || (A->n > 0 && (!perm || !row_ptr || !col || !val)) || A->nnz >= (int64_t{1} << 32))
    return fail(ctx, ICPCG_E_INVALID, "permute_matrix: bad arguments");
  if (A->n == 0) return ICPCG_OK;
  int st = check_matrix(ctx, A, 0);
  if (st) return finish(ctx, st);
  return finish(ctx, permute_matrix(A->row_ptr, A->col, (const double *)A->val, A->n, A->nnz, perm, row_ptr, col, val,
                                    ctx->stream));
}

extern "C" icpcg_status icpcg_permute_rows(icpcg_ctx *ctx, const int32_t *perm, int64_t n, int64_t nrhs,
                                           const double *X, double *Y, int inverse) {
  if (!ctx || n < 0 || nrhs < 1 || (n > 0 && (!perm || !X || !Y)) || X == Y)
    return fail(ctx, ICPCG_E_INVALID, "permute_rows: bad arguments");
  if (n == 0) return ICPCG_OK;
  return finish(ctx, permute_rows(perm, n, nrhs, X, Y, inverse != 0, ctx->stream));
}
