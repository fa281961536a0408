// Deterministic grid-wide reduction for R-column blocks: each 256-thread block
// folds its threads' partials per column in a fixed tree, writes them to a
// partials buffer, and the last block to arrive (ticket counter) folds the
// blocks' partials in block order. The result depends only on the grid shape,
// never on scheduling.
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

// Returns true in the last block only; then out[k * R + c] holds the grid sum
// of quantity k for column c (out lives in the caller's shared memory).
// Thread t contributes v[k] to column t % R. Must be called by every thread.
template <int R, int K>
__device__ bool grid_reduce(const double (&v)[K], double *partials, unsigned *counter, double *smem,
                            double *out) {
  static_assert(kRedBlock % R == 0, "R must divide the block");
  __shared__ unsigned ticket;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) smem[k * kRedBlock + t] = v[k];
  __syncthreads();
  block_fold<R, K>(smem);
  if (t < R) {
#pragma unroll
    for (int k = 0; k < K; ++k) partials[((int64_t)blockIdx.x * K + k) * R + t] = smem[k * kRedBlock + t];
  }
  __threadfence();
  __syncthreads();
  if (t == 0) ticket = atomicAdd(counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return false;
  __threadfence();
  const int c = t % R;
  const int nb = (int)gridDim.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int b = t / R; b < nb; b += kRedBlock / R) acc += partials[((int64_t)b * K + k) * R + c];
    smem[k * kRedBlock + t] = acc;
  }
  __syncthreads();
  block_fold<R, K>(smem);
  if (t < R) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k * R + t] = smem[k * kRedBlock + t];
  }
  if (t == 0) *counter = 0u;
  __syncthreads();
  return true;
}

// Same as grid_reduce<R, 1>, for the lane layout where a thread holds CPL
// consecutive columns starting at ((t % (R / CPL)) * CPL).
template <int R, int CPL>
__device__ bool grid_reduce_cpl(const double (&v)[CPL], double *partials, unsigned *counter, double *smem,
                                double *out) {
  constexpr int LPR = R / CPL;
  __shared__ unsigned ticket;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < CPL; ++k) smem[k * kRedBlock + t] = v[k];
  __syncthreads();
  block_fold<LPR, CPL>(smem);
  if (t < LPR) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) partials[(int64_t)blockIdx.x * R + t * CPL + k] = smem[k * kRedBlock + t];
  }
  __threadfence();
  __syncthreads();
  if (t == 0) ticket = atomicAdd(counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return false;
  __threadfence();
  const int c = t % R;
  const int nb = (int)gridDim.x;
  double acc = 0.0;
  for (int b = t / R; b < nb; b += kRedBlock / R) acc += partials[(int64_t)b * R + c];
  smem[t] = acc;
  __syncthreads();
  block_fold<R, 1>(smem);
  if (t < R) out[t] = smem[t];
  if (t == 0) *counter = 0u;
  __syncthreads();
  return true;
}

// Refresh the host-visible counters from the column states (last block only,
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
