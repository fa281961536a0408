// IC(0) factorization in FP64 (incomplete Cholesky with zero fill: L keeps
// the pattern of tril(A); Model Architecture section), row-oriented:
//   for each stored j < i, ascending:
//     L_ij = (A_ij - sum_{k in S(i) and S(j), k < j} L_ik L_jk) / L_jj
//   L_ii = sqrt(A_ii + alpha A_ii - sum_{k < i} L_ik^2)
// Rows of one level (all their j are on lower levels) are factorized by one
// kernel launch, one wave per row. The row being built lives in LDS, and the
// rows j it depends on (final, from earlier launches) are staged there too in
// one batch of independent loads when they fit, so the sequential chain over
// j runs from LDS; for each j the wave walks row j in parallel, looks each
// column up in the row's sorted prefix by binary search, and folds the
// products in a fixed butterfly. Once a pivot fails, the remaining levels of
// that attempt return at once.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kMaxRow = 4096;
constexpr size_t kLdsLimit = 60 * 1024;  // dynamic LDS per block

// Entries of the rows j that one row depends on which fit next to the row
// itself in the LDS budget (0: always walk the rows j in global memory).
int stage_budget(int max_row_len) {
  const size_t row = (size_t)max_row_len * (2 * sizeof(double) + 2 * sizeof(int32_t)) + 16;
  if (row >= kLdsLimit) return 0;
  const size_t b = (kLdsLimit - row) / (sizeof(double) + sizeof(int32_t));
  return b >= 64 ? (int)std::min<size_t>(b, 2048) : 0;
}

__global__ __launch_bounds__(64) void k_ic0_rows(const int32_t *__restrict__ rows, const int64_t *__restrict__ lrp,
                                                 const int32_t *__restrict__ lci, double *lv,
                                                 const double *__restrict__ a_low, double alpha, int *fail,
                                                 double *__restrict__ pivots, int max_len, int budget) {
  if (*fail) return;  // an earlier level broke down: this attempt is discarded
  extern __shared__ double smem_d[];
  const int lane = threadIdx.x;
  const int i = rows[blockIdx.x];
  const int64_t rs = lrp[i];
  const int len = (int)(lrp[i + 1] - rs);
  // LDS: row i (values, columns), then per entry q of row i the start of row
  // j = cols[q] in the staged arrays and its diagonal, then the staged rows
  double *vals = smem_d;
  double *jdiag = vals + max_len;
  double *jv = jdiag + max_len;
  int32_t *cols = reinterpret_cast<int32_t *>(jv + budget);
  int32_t *off = cols + max_len;
  int32_t *jc = off + max_len + 1;
  for (int q = lane; q < len; q += 64) {
    cols[q] = lci[rs + q];
    vals[q] = a_low[rs + q];
  }
  __syncthreads();
  // lengths of the rows j (without their diagonal), scanned into offsets
  int carry = 0;
  for (int q0 = 0; q0 < len - 1; q0 += 64) {
    const int q = q0 + lane;
    int l = 0;
    if (q < len - 1) {
      const int j = cols[q];
      const int64_t je = lrp[j + 1];
      l = (int)(je - lrp[j]) - 1;
      jdiag[q] = lv[je - 1];
    }
    int x = l;  // inclusive wave scan
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (q < len - 1) off[q] = carry + x - l;
    carry += __shfl(x, 63, 64);
  }
  if (lane == 0) off[len - 1 > 0 ? len - 1 : 0] = carry;
  const bool staged = carry <= budget;
  __syncthreads();
  if (staged) {
    // every entry of every row j in one batch of independent loads
    for (int e0 = 0; e0 < carry; e0 += 4 * 64) {
      int32_t c4[4];
      double v4[4];
      int d4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * 64 + lane;
        d4[u] = -1;
        if (e < carry) {
          int lo = 0, hi = len - 1;  // q with off[q] <= e < off[q + 1]
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= e) lo = mid; else hi = mid - 1;
          }
          const int64_t src = lrp[cols[lo]] + (e - off[lo]);
          c4[u] = lci[src];
          v4[u] = lv[src];
          d4[u] = e;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (d4[u] >= 0) {
          jc[d4[u]] = c4[u];
          jv[d4[u]] = v4[u];
        }
    }
    __syncthreads();
  }
  for (int q = 0; q < len - 1; ++q) {
    double part = 0.0;
    if (staged) {
      const int b = off[q], jl = off[q + 1] - b;
      for (int p = lane; p < jl; p += 64) {
        const int k = jc[b + p];
        int lo = 0, hi = q;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (cols[mid] < k) lo = mid + 1; else hi = mid;
        }
        if (lo < q && cols[lo] == k) part += vals[lo] * jv[b + p];
      }
    } else {
      const int j = cols[q];
      const int64_t js = lrp[j];
      const int jlen = (int)(lrp[j + 1] - js);
      for (int p = lane; p < jlen - 1; p += 64) {
        const int k = lci[js + p];
        int lo = 0, hi = q;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (cols[mid] < k) lo = mid + 1; else hi = mid;
        }
        if (lo < q && cols[lo] == k) part += vals[lo] * lv[js + p];
      }
    }
    const double sum = wave_sum(part);
    if (lane == 0) vals[q] = (vals[q] - sum) / jdiag[q];
    __syncthreads();
  }
  double dp = 0.0;
  for (int q = lane; q < len - 1; q += 64) dp += vals[q] * vals[q];
  dp = wave_sum(dp);
  if (lane == 0) {
    const double aii = vals[len - 1];
    const double d = aii + alpha * aii - dp;
    pivots[i] = d;
    if (!(d > 0.0)) atomicOr(fail, 1);
    vals[len - 1] = d > 0.0 ? sqrt(d) : (double)NAN;
  }
  __syncthreads();
  for (int q = lane; q < len; q += 64) lv[rs + q] = vals[q];
}

}  // namespace

int ic0_max_row() { return kMaxRow; }

// One launch per level of the row schedule of tril(A).
int ic0_factor_levels(const int64_t *lrp, const int32_t *lci, double *lv, const double *a_low, int64_t,
                      const int32_t *perm, const std::vector<int32_t> &level_ptr, double alpha, int *fail,
                      double *pivots, hipStream_t s, int max_row_len, int num_cu) {
  // Staging pays on narrow levels (each row's chain is latency-bound); on
  // levels wider than one resident round of staged blocks the smaller
  // footprint (more resident rows) wins.
  const int budget = stage_budget(max_row_len);
  const size_t row_lds = (size_t)max_row_len * (2 * sizeof(double) + 2 * sizeof(int32_t)) + 16;
  const size_t lds_staged = row_lds + (size_t)budget * (sizeof(double) + sizeof(int32_t));
  const int64_t staged_round = (int64_t)num_cu * (int64_t)std::max<size_t>(1, (160 * 1024) / lds_staged);
  for (size_t l = 0; l + 1 < level_ptr.size(); ++l) {
    const int32_t b = level_ptr[l], e = level_ptr[l + 1];
    if (e <= b) continue;
    const bool stage = budget > 0 && (int64_t)(e - b) <= staged_round;
    hipLaunchKernelGGL(k_ic0_rows, dim3((unsigned)(e - b)), dim3(64), stage ? lds_staged : row_lds, s, perm + b, lrp,
                       lci, lv, a_low, alpha, fail, pivots, max_row_len, stage ? budget : 0);
  }
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace icpcg
