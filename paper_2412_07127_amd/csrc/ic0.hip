// IC(0) factorization in FP64 (incomplete Cholesky with zero fill: L keeps
// the pattern of tril(A); Model Architecture section), row-oriented:
//   for each stored j < i, ascending:
//     L_ij = (A_ij - sum_{k in S(i) and S(j), k < j} L_ik L_jk) / L_jj
//   L_ii = sqrt(A_ii + alpha A_ii - sum_{k < i} L_ik^2)
// Rows of one level (all their j are on lower levels) are factorized by one
// kernel launch, one wave per row. The row being built lives in LDS; for
// each j the wave walks row j (final, from earlier launches) in parallel and
// looks each column up in the row's sorted prefix by binary search, then
// folds the products in a fixed butterfly.
#include <cmath>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kMaxRow = 4096;

__global__ __launch_bounds__(64) void k_ic0_rows(const int32_t *__restrict__ rows, const int64_t *__restrict__ lrp,
                                                 const int32_t *__restrict__ lci, double *lv,
                                                 const double *__restrict__ a_low, double alpha, int *fail,
                                                 double *__restrict__ pivots) {
  extern __shared__ double smem_d[];
  const int lane = threadIdx.x;
  const int i = rows[blockIdx.x];
  const int64_t rs = lrp[i];
  const int len = (int)(lrp[i + 1] - rs);
  double *vals = smem_d;
  int32_t *cols = reinterpret_cast<int32_t *>(smem_d + len);
  for (int q = lane; q < len; q += 64) {
    cols[q] = lci[rs + q];
    vals[q] = a_low[rs + q];
  }
  __syncthreads();
  for (int q = 0; q < len - 1; ++q) {
    const int j = cols[q];
    const int64_t js = lrp[j];
    const int jlen = (int)(lrp[j + 1] - js);
    double part = 0.0;
    for (int p = lane; p < jlen - 1; p += 64) {
      const int k = lci[js + p];
      int lo = 0, hi = q;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < k) lo = mid + 1; else hi = mid;
      }
      if (lo < q && cols[lo] == k) part += vals[lo] * lv[js + p];
    }
    const double sum = wave_sum(part);
    if (lane == 0) vals[q] = (vals[q] - sum) / lv[js + jlen - 1];
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
                      double *pivots, hipStream_t s, int max_row_len) {
  const size_t lds = (size_t)max_row_len * (sizeof(double) + sizeof(int32_t)) + 16;
  for (size_t l = 0; l + 1 < level_ptr.size(); ++l) {
    const int32_t b = level_ptr[l], e = level_ptr[l + 1];
    if (e <= b) continue;
    hipLaunchKernelGGL(k_ic0_rows, dim3((unsigned)(e - b)), dim3(64), lds, s, perm + b, lrp, lci, lv, a_low, alpha,
                       fail, pivots);
  }
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace icpcg
