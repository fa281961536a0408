// Vector steps of the PCG loop (supplementary Algorithm 1) for an R-column
// block. Each step that needs a grid-wide reduction is a compute kernel that
// writes per-block partials plus a one-block finalize kernel that folds them in
// fixed order and updates the per-column state:
//   init          r = b - A x0, ||b||^2, ||r||^2           -> tolerance, start flags
//   dot_rz        r^T z (formed by the backward triangular
//                 solve for FP32 / BF16 factors on several
//                 columns, k_rz_fin alone then)             -> beta = r_k^T z_k / r_{k-1}^T z_{k-1}
//   update_p      p = z + beta p (also re-arms z, and y where the backward solve
//                 did not, as pending for the next solves)
//   dot_pw        p^T w, after the SpMV (fused in the plain
//                 row kernel)                               -> alpha = r^T z / p^T w
//   update_xr     x += alpha p, r -= alpha w, ||r||^2        -> iteration count, stop test
//                 (for FP32 / BF16 factors on several columns applied by the
//                 next step's forward solve, k_rr_fin alone then)
//   true_residual b - A x, ||b - A x||^2                     -> accept / replace / give up
// Converged or failed columns are frozen (their x, r, p are no longer touched).
// Steps queued after every column stopped return at once (n_active == 0).
#include "reduce.hpp"

namespace icpcg {

namespace {

constexpr int kBlock = kRedBlock;

inline unsigned vec_grid(int64_t n, int R) {
  int64_t g = (n * R + kBlock - 1) / kBlock;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (unsigned)g;
}

#define ICPCG_GRID_LOOP(e, total) \
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < (total); e += (int64_t)gridDim.x * kBlock)

template <typename T> struct Pending;
template <> struct Pending<double> {
  static __device__ __forceinline__ double get() { return bitcast<double>(Flag<double>::kPending); }
};
template <> struct Pending<float> {
  static __device__ __forceinline__ float get() { return bitcast<float>(Flag<float>::kPending); }
};

// ------------------------------------------------------------------ init

template <int R, typename TZ>
__global__ __launch_bounds__(kBlock) void k_init(int64_t n, const double *__restrict__ B, const double *__restrict__ W,
                                                 double *__restrict__ r, double *__restrict__ p, TZ *__restrict__ y,
                                                 TZ *__restrict__ z, double *partials) {
  __shared__ double smem[2 * kRedBlock];
  double bb = 0.0, rr = 0.0;
  ICPCG_GRID_LOOP(e, n * R) {
    const double b = B[e];
    const double ri = b - W[e];
    r[e] = ri;
    p[e] = 0.0;
    y[e] = Pending<TZ>::get();
    z[e] = Pending<TZ>::get();
    bb += b * b;
    rr += ri * ri;
  }
  const double v[2] = {bb, rr};
  block_partials<R, 2>(v, partials, smem);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_init_fin(const double *partials, int nb, double rtol, ColState *cols,
                                                     int64_t max_iter, SolveFlags *flags) {
  __shared__ double smem[2 * kRedBlock];
  __shared__ double out[2 * R];
  fold_partials<R, 2>(partials, nb, smem, out);
  const int t = threadIdx.x;
  if (t < R) {
    ColState cs;
    cs.bb = out[t];
    cs.rr = out[R + t];
    cs.tol2 = rtol * rtol * cs.bb;
    cs.rz = cs.pw = cs.alpha = cs.beta = 0.0;
    cs.trr = cs.rr;
    cs.iters = cs.repl = cs.replace = cs.zero_x = 0;
    cs.status = ICPCG_OK;
    cs.conv = 0;
    cs.active = 0;
    cs.upd = 0;
    if (cs.bb == 0.0) {
      cs.zero_x = 1;  // b = 0: x = 0 after 0 iterations
      cs.rr = cs.trr = 0.0;
    } else if (!isfinite(cs.rr) || !isfinite(cs.bb)) {
      cs.status = ICPCG_E_NONFINITE;
    } else if (cs.rr <= cs.tol2) {
      cs.conv = 1;
    } else if (max_iter <= 0) {
      cs.status = ICPCG_E_MAXITER;
    } else {
      cs.active = 1;
    }
    cols[t] = cs;
  }
  __syncthreads();
  count_flags<R>(cols, flags);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_zero_x(int64_t n, double *__restrict__ X, const ColState *__restrict__ cols) {
  ICPCG_GRID_LOOP(e, n * R) {
    if (cols[e % R].zero_x) X[e] = 0.0;
  }
}

// ------------------------------------------------------- r^T z and p^T w

// Per-column dot of two n x R blocks into block partials.
template <int R, typename TZ>
__global__ __launch_bounds__(kBlock) void k_col_dot(int64_t n, const double *__restrict__ r, const TZ *__restrict__ z,
                                                    double *partials, const SolveFlags *flags) {
  if (flags && flags->n_active == 0) return;
  __shared__ double smem[kRedBlock];
  double acc = 0.0;
  ICPCG_GRID_LOOP(e, n * R) acc += r[e] * (double)z[e];
  const double v[1] = {acc};
  block_partials<R, 1>(v, partials, smem);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_rz_fin(const double *partials, int nb, ColState *cols, SolveFlags *flags) {
  if (flags->n_active == 0) return;
  __shared__ double smem[kRedBlock];
  __shared__ double out[R];
  fold_partials<R, 1>(partials, nb, smem, out);
  const int t = threadIdx.x;
  if (t < R) {
    ColState &cs = cols[t];
    cs.replace = 0;
    if (cs.active) {
      const double rz = out[t];
      if (!isfinite(rz)) { cs.status = ICPCG_E_NONFINITE; cs.active = 0; }
      else if (!(rz > 0.0)) { cs.status = ICPCG_E_BREAKDOWN; cs.active = 0; }
      else {
        cs.beta = cs.iters == 0 ? 0.0 : rz / cs.rz;
        cs.rz = rz;
      }
    }
  }
  __syncthreads();
  count_flags<R>(cols, flags);
}

// Plain per-column sums of block partials (icpcg_apply_rz).
template <int R>
__global__ __launch_bounds__(kBlock) void k_dot_out(const double *partials, int nb, double *out) {
  __shared__ double smem[kRedBlock];
  __shared__ double res[R];
  fold_partials<R, 1>(partials, nb, smem, res);
  if (threadIdx.x < R) out[threadIdx.x] = res[threadIdx.x];
}

// ------------------------------------------------------------- update p

// z is read and then re-armed as pending in place (one pointer, so the
// compiler keeps each read before the store to the same element). Y: y is
// re-armed here too (else the backward solve did it).
template <int R, typename TZ, bool Y>
__global__ __launch_bounds__(kBlock) void k_update_p(int64_t n, TZ *z, double *__restrict__ p, TZ *__restrict__ y,
                                                     const ColState *__restrict__ cols, const SolveFlags *flags) {
  if (flags->n_active == 0) return;
  __shared__ double beta[R];
  __shared__ int act[R];
  if (threadIdx.x < R) {
    beta[threadIdx.x] = cols[threadIdx.x].beta;
    act[threadIdx.x] = cols[threadIdx.x].active;
  }
  __syncthreads();
  ICPCG_GRID_LOOP(e, n * R) {
    const int c = (int)(e % R);
    if (act[c]) p[e] = (double)z[e] + beta[c] * p[e];
    if (Y) y[e] = Pending<TZ>::get();
    z[e] = Pending<TZ>::get();
  }
}

// ------------------------------------------------------------ p^T w -> alpha

template <int R>
__global__ __launch_bounds__(kBlock) void k_pw_fin(const double *partials, int nb, ColState *cols,
                                                   const SolveFlags *flags) {
  if (flags->n_active == 0) return;
  __shared__ double smem[kRedBlock];
  __shared__ double out[R];
  fold_partials<R, 1>(partials, nb, smem, out);
  const int t = threadIdx.x;
  if (t < R) {
    ColState &cs = cols[t];
    if (cs.active) {
      const double pw = out[t];
      cs.pw = pw;
      if (!isfinite(pw)) { cs.status = ICPCG_E_NONFINITE; cs.active = 0; }
      else if (!(pw > 0.0)) { cs.status = ICPCG_E_BREAKDOWN; cs.active = 0; }
      else {
        cs.alpha = cs.rz / pw;
        cs.upd = 1;
      }
    }
  }
}

// --------------------------------------------------------- update x, r

template <int R>
__global__ __launch_bounds__(kBlock) void k_update_xr(int64_t n, double *__restrict__ X, double *__restrict__ r,
                                                      const double *__restrict__ p, const double *__restrict__ w,
                                                      const ColState *__restrict__ cols, double *partials,
                                                      const SolveFlags *flags) {
  if (flags->n_active == 0) return;
  __shared__ double smem[kRedBlock];
  __shared__ double alpha[R];
  __shared__ int act[R];
  if (threadIdx.x < R) {
    alpha[threadIdx.x] = cols[threadIdx.x].alpha;
    act[threadIdx.x] = cols[threadIdx.x].active;
  }
  __syncthreads();
  double acc = 0.0;
  ICPCG_GRID_LOOP(e, n * R) {
    const int c = (int)(e % R);
    if (act[c]) {
      X[e] = fma(alpha[c], p[e], X[e]);
      const double ri = fma(-alpha[c], w[e], r[e]);
      r[e] = ri;
      acc += ri * ri;
    }
  }
  const double v[1] = {acc};
  block_partials<R, 1>(v, partials, smem);
}

// FUSED: the partials come from the forward solve that applied the update,
// which covers the columns with upd set (the others kept their x and r).
template <int R, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_rr_fin(const double *partials, int nb, ColState *cols, int64_t max_iter,
                                                   SolveFlags *flags) {
  if (flags->n_active == 0) return;
  __shared__ double smem[kRedBlock];
  __shared__ double out[R];
  fold_partials<R, 1>(partials, nb, smem, out);
  const int t = threadIdx.x;
  if (t < R) {
    ColState &cs = cols[t];
    const bool updated = FUSED ? cs.upd != 0 : cs.active != 0;
    cs.upd = 0;
    if (cs.active && updated) {
      cs.iters += 1;
      cs.rr = out[t];
      if (!isfinite(cs.rr)) { cs.status = ICPCG_E_NONFINITE; cs.active = 0; }
      else if (cs.rr <= cs.tol2) { cs.conv = 1; cs.active = 0; }
      else if (cs.iters >= max_iter) { cs.status = ICPCG_E_MAXITER; cs.active = 0; }
    }
  }
  __syncthreads();
  count_flags<R>(cols, flags);
}

// ---------------------------------------------------------- true residual

// W holds A x on entry and b - A x on exit.
template <int R>
__global__ __launch_bounds__(kBlock) void k_true_residual(int64_t n, const double *__restrict__ B, double *__restrict__ W,
                                                          double *partials) {
  __shared__ double smem[kRedBlock];
  double acc = 0.0;
  ICPCG_GRID_LOOP(e, n * R) {
    const double t = B[e] - W[e];
    W[e] = t;
    acc += t * t;
  }
  const double v[1] = {acc};
  block_partials<R, 1>(v, partials, smem);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_tr_fin(const double *partials, int nb, ColState *cols, int64_t max_iter,
                                                   int max_replace, int final_pass, SolveFlags *flags) {
  __shared__ double smem[kRedBlock];
  __shared__ double out[R];
  fold_partials<R, 1>(partials, nb, smem, out);
  const int t = threadIdx.x;
  if (t < R) {
    ColState &cs = cols[t];
    cs.trr = out[t];
    if (!final_pass && cs.conv) {
      cs.conv = 0;
      if (cs.trr <= cs.tol2) {
        // converged: status stays OK
      } else if (cs.repl < max_replace) {
        cs.repl += 1;
        cs.rr = cs.trr;
        if (cs.iters >= max_iter) {
          cs.status = ICPCG_E_MAXITER;
        } else {
          cs.replace = 1;
          cs.active = 1;
        }
      } else {
        cs.status = ICPCG_E_TRUE_RESIDUAL;
      }
    }
  }
  __syncthreads();
  count_flags<R>(cols, flags);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_replace_r(int64_t n, const double *__restrict__ W, double *__restrict__ r,
                                                      const ColState *__restrict__ cols) {
  ICPCG_GRID_LOOP(e, n * R) {
    if (cols[e % R].replace) r[e] = W[e];
  }
}

// z = r / d_i (Jacobi: the reciprocal of A's diagonal as the inverse) or z = r
// (no preconditioner) for an n x R block.
__global__ __launch_bounds__(kBlock) void k_diag_apply(int64_t n, int R, const double *__restrict__ r,
                                                       const double *__restrict__ d, double *__restrict__ z,
                                                       const int *__restrict__ active) {
  if (active && *active == 0) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * R; e += (int64_t)gridDim.x * blockDim.x)
    z[e] = d ? r[e] / d[e / R] : r[e];
}

__global__ void k_gather_cols(int64_t n, int R, const double *__restrict__ src, int64_t lds, int64_t c0, int nc,
                              double *__restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * R; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R;
    const int c = (int)(e % R);
    dst[e] = c < nc ? src[i * lds + c0 + c] : 0.0;
  }
}

__global__ void k_scatter_cols(int64_t n, int R, const double *__restrict__ src, double *__restrict__ dst, int64_t ldd,
                               int64_t c0, int nc) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * R; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R;
    const int c = (int)(e % R);
    if (c < nc) dst[i * ldd + c0 + c] = src[e];
  }
}

template <typename T>
__global__ void k_fill_pending(T *p, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = Pending<T>::get();
}

}  // namespace

#define ICPCG_R_SWITCH(R, CALL)                                          \
  switch (R) {                                                           \
    case 1: { constexpr int RR = 1; CALL; } break;                       \
    case 2: { constexpr int RR = 2; CALL; } break;                       \
    case 4: { constexpr int RR = 4; CALL; } break;                       \
    case 8: { constexpr int RR = 8; CALL; } break;                       \
    case 16: { constexpr int RR = 16; CALL; } break;                     \
    default: set_error("unsupported block width"); return ICPCG_E_INVALID; \
  }

int pcg_init(int64_t n, int R, const double *B, const double *W, double *r, double *p, void *y, void *z, bool f32,
             double rtol, double *partials, ColState *cols, int64_t max_iter, SolveFlags *flags, hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  if (f32) {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_init<RR, float>), dim3(g), dim3(kBlock), 0, s, n, B, W, r, p, (float *)y,
                                         (float *)z, partials));
  } else {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_init<RR, double>), dim3(g), dim3(kBlock), 0, s, n, B, W, r, p,
                                         (double *)y, (double *)z, partials));
  }
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_init_fin<RR>, dim3(1), dim3(kBlock), 0, s, partials, (int)g, rtol, cols,
                                       max_iter, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_zero_x(int64_t n, int R, double *X, const ColState *cols, hipStream_t s) {
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_zero_x<RR>, dim3(vec_grid(n, R)), dim3(kBlock), 0, s, n, X, cols));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_dot_rz(int64_t n, int R, const double *r, const void *z, bool f32, double *partials, ColState *cols,
               SolveFlags *flags, hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  if (f32) {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_col_dot<RR, float>), dim3(g), dim3(kBlock), 0, s, n, r, (const float *)z,
                                         partials, flags));
  } else {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_col_dot<RR, double>), dim3(g), dim3(kBlock), 0, s, n, r,
                                         (const double *)z, partials, flags));
  }
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_rz_fin<RR>, dim3(1), dim3(kBlock), 0, s, partials, (int)g, cols, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_rz_finalize(int R, const double *partials, int nb, ColState *cols, SolveFlags *flags, hipStream_t s) {
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_rz_fin<RR>, dim3(1), dim3(kBlock), 0, s, partials, nb, cols, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int dot_finalize_out(int R, const double *partials, int nb, double *out, hipStream_t s) {
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_dot_out<RR>, dim3(1), dim3(kBlock), 0, s, partials, nb, out));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int col_dot_out(int64_t n, int R, const double *r, const void *z, bool f32, double *partials, double *out,
                hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  if (f32) {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_col_dot<RR, float>), dim3(g), dim3(kBlock), 0, s, n, r, (const float *)z,
                                         partials, nullptr));
  } else {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_col_dot<RR, double>), dim3(g), dim3(kBlock), 0, s, n, r,
                                         (const double *)z, partials, nullptr));
  }
  ICPCG_HIP_TRY(hipGetLastError());
  return dot_finalize_out(R, partials, (int)g, out, s);
}

int pcg_update_p(int64_t n, int R, void *z, bool f32, double *p, void *y, const ColState *cols,
                 const SolveFlags *flags, hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  if (f32 && y) {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_update_p<RR, float, true>), dim3(g), dim3(kBlock), 0, s, n, (float *)z,
                                         p, (float *)y, cols, flags));
  } else if (f32) {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_update_p<RR, float, false>), dim3(g), dim3(kBlock), 0, s, n, (float *)z,
                                         p, (float *)y, cols, flags));
  } else if (y) {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_update_p<RR, double, true>), dim3(g), dim3(kBlock), 0, s, n,
                                         (double *)z, p, (double *)y, cols, flags));
  } else {
    ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_update_p<RR, double, false>), dim3(g), dim3(kBlock), 0, s, n,
                                         (double *)z, p, (double *)y, cols, flags));
  }
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_pw_finalize(int R, const double *partials, int nb, ColState *cols, const SolveFlags *flags, hipStream_t s) {
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_pw_fin<RR>, dim3(1), dim3(kBlock), 0, s, partials, nb, cols, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_dot_pw(int64_t n, int R, const double *p, const double *w, double *partials, ColState *cols,
               const SolveFlags *flags, hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_col_dot<RR, double>), dim3(g), dim3(kBlock), 0, s, n, p, w, partials, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return pcg_pw_finalize(R, partials, (int)g, cols, flags, s);
}

int pcg_update_xr(int64_t n, int R, double *X, double *r, const double *p, const double *w, double *partials,
                  ColState *cols, int64_t max_iter, SolveFlags *flags, hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_update_xr<RR>, dim3(g), dim3(kBlock), 0, s, n, X, r, p, w, cols, partials,
                                       flags));
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_rr_fin<RR, false>), dim3(1), dim3(kBlock), 0, s, partials, (int)g, cols,
                                       max_iter, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_rr_finalize(int R, const double *partials, int nb, ColState *cols, int64_t max_iter, SolveFlags *flags,
                    hipStream_t s) {
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL((k_rr_fin<RR, true>), dim3(1), dim3(kBlock), 0, s, partials, nb, cols,
                                       max_iter, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_true_residual(int64_t n, int R, const double *B, double *W, double *partials, ColState *cols,
                      int64_t max_iter, int max_replace, int final_pass, SolveFlags *flags, hipStream_t s) {
  const unsigned g = vec_grid(n, R);
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_true_residual<RR>, dim3(g), dim3(kBlock), 0, s, n, B, W, partials));
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_tr_fin<RR>, dim3(1), dim3(kBlock), 0, s, partials, (int)g, cols, max_iter,
                                       max_replace, final_pass, flags));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_replace_r(int64_t n, int R, const double *W, double *r, ColState *cols, hipStream_t s) {
  ICPCG_R_SWITCH(R, hipLaunchKernelGGL(k_replace_r<RR>, dim3(vec_grid(n, R)), dim3(kBlock), 0, s, n, W, r, cols));
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int pcg_diag_apply(int64_t n, int R, const double *r, const double *d, double *z, const int *active, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_apply, dim3(vec_grid(n, R)), dim3(kBlock), 0, s, n, R, r, d, z, active);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int gather_cols(int64_t n, int R, const double *src, int64_t lds, int64_t c0, int nc, double *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3(vec_grid(n, R)), dim3(kBlock), 0, s, n, R, src, lds, c0, nc, dst);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int scatter_cols(int64_t n, int R, const double *src, double *dst, int64_t ldd, int64_t c0, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_cols, dim3(vec_grid(n, R)), dim3(kBlock), 0, s, n, R, src, dst, ldd, c0, nc);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int fill_pending(void *p, int64_t count, bool f32, hipStream_t s) {
  int64_t g = (count + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  if (f32)
    hipLaunchKernelGGL(k_fill_pending<float>, dim3((unsigned)g), dim3(kBlock), 0, s, (float *)p, count);
  else
    hipLaunchKernelGGL(k_fill_pending<double>, dim3((unsigned)g), dim3(kBlock), 0, s, (double *)p, count);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace icpcg
