// Deterministic grid-wide reductions for R-column blocks in two launches:
// every 256-thread block folds its threads' partials per column in a fixed
// tree and writes one partial per (block, quantity, column); a one-block
// finalize kernel then folds the partials in block order and runs the
// per-column finalizer. The kernel boundary makes the partials visible, so no
// device-scope fence (an L2 write-back on gfx950) is needed per block. The
// result depends only on the grid shape, never on scheduling.
#pragma once

#include "internal.hpp"

namespace icpcg {

constexpr int kRedBlock = 256;

// Tree over threads t of the block that share t % R, for K quantities held in
// smem[k * 256 + t]; afterwards smem[k * 256 + c] (c < R) holds the sums.
template <int R, int K>
__device__ __forceinline__ void block_fold(double *smem) {
  const int t = threadIdx.x;
#pragma unroll
  for (int st = kRedBlock / 2; st >= R; st >>= 1) {
    if (t < st) {
#pragma unroll
      for (int k = 0; k < K; ++k) smem[k * kRedBlock + t] += smem[k * kRedBlock + t + st];
    }
    __syncthreads();
  }
}

// Block partials: thread t contributes v[k] to column t % R.
// partials[(block * K + k) * R + c]. Must be called by every thread.
template <int R, int K>
__device__ __forceinline__ void block_partials(const double (&v)[K], double *partials, double *smem) {
  static_assert(kRedBlock % R == 0, "R must divide the block");
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) smem[k * kRedBlock + t] = v[k];
  __syncthreads();
  block_fold<R, K>(smem);
  if (t < R) {
#pragma unroll
    for (int k = 0; k < K; ++k) partials[((int64_t)blockIdx.x * K + k) * R + t] = smem[k * kRedBlock + t];
  }
}

// Same, for the lane layout where a thread holds CPL consecutive columns
// starting at ((t % (R / CPL)) * CPL); K = 1.
template <int R, int CPL>
__device__ __forceinline__ void block_partials_cpl(const double (&v)[CPL], double *partials, double *smem) {
  constexpr int LPR = R / CPL;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < CPL; ++k) smem[k * kRedBlock + t] = v[k];
  __syncthreads();
  block_fold<LPR, CPL>(smem);
  if (t < LPR) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) partials[(int64_t)blockIdx.x * R + t * CPL + k] = smem[k * kRedBlock + t];
  }
}

// In the one-block finalize kernel: out[k * R + c] = sum over the nb blocks'
// partials in a fixed order: thread t takes blocks t / R + j * (256 / R), into
// 8 accumulators by j mod 8 (8 independent loads in flight), combined in
// order, then the block tree. Must be called by every thread.
template <int R, int K>
__device__ __forceinline__ void fold_partials(const double *partials, int nb, double *smem, double *out) {
  const int t = threadIdx.x;
  const int c = t % R;
  constexpr int STEP = kRedBlock / R;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a8[j] = 0.0;
    int b = t / R;
    for (; b + 7 * STEP < nb; b += 8 * STEP) {
#pragma unroll
      for (int j = 0; j < 8; ++j) a8[j] += partials[((int64_t)(b + j * STEP) * K + k) * R + c];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (b + j * STEP < nb) a8[j] += partials[((int64_t)(b + j * STEP) * K + k) * R + c];
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += a8[j];
    smem[k * kRedBlock + t] = acc;
  }
  __syncthreads();
  block_fold<R, K>(smem);
  if (t < R) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k * R + t] = smem[k * kRedBlock + t];
  }
  __syncthreads();
}

// Refresh the host-visible counters from the column states (finalize kernel,
// after its finalizer has run).
template <int R>
__device__ __forceinline__ void count_flags(const ColState *cols, SolveFlags *flags) {
  if (threadIdx.x == 0) {
    int na = 0, nc = 0;
    for (int c = 0; c < R; ++c) {
      na += cols[c].active;
      nc += cols[c].conv;
    }
    flags->n_active = na;
    flags->n_conv = nc;
  }
}

}  // namespace icpcg
