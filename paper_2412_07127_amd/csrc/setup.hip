// One-time analysis of matrices and factors: validation, tril(A), the
// transpose L -> L^T, row level sets and the supernode schedules of the
// triangular solves.
#include <climits>
#include <cmath>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_rows(int64_t rows, int rows_per_block) {
  int64_t g = (rows + rows_per_block - 1) / rows_per_block;
  if (g < 1) g = 1;
  if (g > 262144) g = 262144;
  return (unsigned)g;
}

// ------------------------------------------------------------ validation

// mode 0: general square CSR with a stored diagonal; mode 1: lower factor
// (every column <= row, diagonal last and > 0). Values (when given) must be
// finite. The smallest offending row lands in *bad (INT_MAX if none).
__global__ __launch_bounds__(kBlock) void k_check_csr(const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const double *__restrict__ val, int64_t n,
                                                      int64_t nnz, int mode, int *bad) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    const int64_t s = rp[i], e = rp[i + 1];
    bool ok = (e >= s) && s >= 0 && e <= nnz && (i > 0 || s == 0) && (i < n - 1 || e == nnz);
    bool has_diag = false;
    if (ok) {
      for (int64_t q = s + lane; q < e; q += 64) {
        const int32_t c = ci[q];
        bool g = c >= 0 && c < n;
        if (q > s) g = g && ci[q - 1] < c;
        if (mode == 1) g = g && c <= i;
        if (val) {
          const double v = val[q];
          g = g && isfinite(v);
          if (mode == 1 && c == i) g = g && v > 0.0;
        }
        if (c == i) has_diag = true;
        ok = ok && g;
      }
      if (mode == 1 && e > s && lane == 0) ok = ok && ci[e - 1] == i;
    }
    const bool all_ok = __ballot(!ok) == 0ull;
    const bool diag_ok = __ballot(has_diag) != 0ull;
    if (lane == 0 && !(all_ok && diag_ok)) atomicMin(bad, (int)i);
  }
}

// Number of entries with column <= row (a prefix of each sorted row).
__global__ __launch_bounds__(kBlock) void k_tril_count(const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, int64_t n,
                                                       int64_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    const int64_t s = rp[i], e = rp[i + 1];
    int c = 0;
    for (int64_t q = s + lane; q < e; q += 64) c += ci[q] <= i ? 1 : 0;
    c = wave_sum(c);
    if (lane == 0) cnt[i] = c;
  }
}

__global__ __launch_bounds__(kBlock) void k_tril_copy(const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const double *__restrict__ v, int64_t n,
                                                      const int64_t *__restrict__ lrp,
                                                      int32_t *__restrict__ lci, double *__restrict__ lv) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    const int64_t s = rp[i], d = lrp[i], len = lrp[i + 1] - lrp[i];
    for (int64_t q = lane; q < len; q += 64) {
      if (lci) lci[d + q] = ci[s + q];
      if (lv) lv[d + q] = v[s + q];
    }
  }
}

// Row id of every stored entry.
__global__ __launch_bounds__(kBlock) void k_row_of_entry(const int64_t *__restrict__ rp, int64_t n,
                                                         uint32_t *__restrict__ rowid) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t i = w0; i < n; i += nw)
    for (int64_t q = rp[i] + lane; q < rp[i + 1]; q += 64) rowid[q] = (uint32_t)i;
}

__global__ void k_col_count(const int32_t *__restrict__ ci, int64_t nnz, unsigned long long *cnt) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[ci[q]], 1ull);
}

__global__ void k_transpose_gather(const uint32_t *__restrict__ perm, const uint32_t *__restrict__ rowid,
                                   int64_t nnz, int32_t *__restrict__ uci, int32_t *__restrict__ upos) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < nnz; d += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t q = perm[d];
    uci[d] = (int32_t)rowid[q];
    upos[d] = (int32_t)q;
  }
}

__global__ void k_set_last_i64(int64_t *p, int64_t idx, int64_t v) { p[idx] = v; }
__global__ void k_set_last_i32(int32_t *p, int64_t idx, int32_t v) { p[idx] = v; }

// Value refresh: U values gathered from L, reduced-precision copies.
__global__ void k_gather_f64(const double *__restrict__ src, const int32_t *__restrict__ pos, int64_t m,
                             double *__restrict__ dst) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < m; d += (int64_t)gridDim.x * blockDim.x)
    dst[d] = src[pos[d]];
}
__global__ void k_cast_f32(const double *__restrict__ src, int64_t m, float *__restrict__ dst) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < m; d += (int64_t)gridDim.x * blockDim.x)
    dst[d] = (float)src[d];
}
__global__ void k_cast_bf16(const double *__restrict__ src, int64_t m, unsigned short *__restrict__ dst) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < m; d += (int64_t)gridDim.x * blockDim.x)
    dst[d] = f32_to_bf16_rne((float)src[d]);
}

// ------------------------------------------------------------- supernodes

// begin[i] = 1 when row i cannot extend row i-1's supernode. Lower pattern:
// row i must be row i-1 followed by the diagonal i. Upper pattern (diagonal
// first): row i must be row i-1 without its diagonal.
template <bool UPPER>
__global__ __launch_bounds__(kBlock) void k_sn_begin(const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, int64_t n,
                                                     int32_t *__restrict__ begin) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    if (i == 0) {
      if (lane == 0) begin[0] = 1;
      continue;
    }
    const int64_t sp = rp[i - 1], lp = rp[i] - rp[i - 1];
    const int64_t si = rp[i], li = rp[i + 1] - rp[i];
    bool ok;
    if (!UPPER) {
      ok = (li == lp + 1);
      if (ok) {
        bool g = true;
        for (int64_t q = lane; q < lp; q += 64) g = g && (ci[si + q] == ci[sp + q]);
        if (lane == 0) g = g && ci[si + li - 1] == (int32_t)i;
        ok = __ballot(!g) == 0ull;
      }
    } else {
      ok = (li == lp - 1) && li > 0;
      if (ok) {
        bool g = true;
        for (int64_t q = lane; q < li; q += 64) g = g && (ci[si + q] == ci[sp + 1 + q]);
        ok = __ballot(!g) == 0ull;
      }
    }
    if (lane == 0) begin[i] = ok ? 0 : 1;
  }
}

// begin[i] = 1 unless row i has exactly the columns of row i-1 (rows of one
// 3-DOF node in a stiffness matrix).
__global__ __launch_bounds__(kBlock) void k_same_begin(const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, int64_t n,
                                                       int32_t *__restrict__ begin) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    if (i == 0) {
      if (lane == 0) begin[0] = 1;
      continue;
    }
    const int64_t sp = rp[i - 1], lp = rp[i] - rp[i - 1];
    const int64_t si = rp[i], li = rp[i + 1] - rp[i];
    bool ok = li == lp;
    if (ok) {
      bool g = true;
      for (int64_t q = lane; q < li; q += 64) g = g && (ci[si + q] == ci[sp + q]);
      ok = __ballot(!g) == 0ull;
    }
    if (lane == 0) begin[i] = ok ? 0 : 1;
  }
}

__global__ void k_begin_key(const int32_t *__restrict__ begin, int64_t n, int32_t *__restrict__ key) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = begin[i] ? (int32_t)i : 0;
}

// Split runs into supernodes of at most smax rows.
__global__ void k_split(const int32_t *__restrict__ begin, const int32_t *__restrict__ run_start,
                        int64_t n, int smax, int32_t *__restrict__ fb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    fb[i] = (begin[i] || ((i - run_start[i]) % smax) == 0) ? 1 : 0;
}

__global__ void k_sn_index(const int32_t *__restrict__ fb, const int32_t *__restrict__ ex, int64_t n,
                           int32_t *__restrict__ sn_ptr, int32_t *__restrict__ sn_of_row) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (fb[i]) sn_ptr[ex[i]] = (int32_t)i;
    sn_of_row[i] = ex[i] + fb[i] - 1;
  }
}

// ------------------------------------------------------------------ levels

// Level of each schedule unit (a row, or a supernode of rows) as the longest
// dependency chain below it. One wave per unit; units are visited in an order
// where every dependency comes earlier (ascending for the lower pattern,
// descending for the upper one), spread round-robin over all resident waves,
// and a wave waits for each dependency's level to be published. Because the
// smallest unfinished position is always held by a running wave whose
// dependencies are finished, the grid (sized to be fully resident) always
// makes progress.
template <bool UPPER, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_levels(const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, int64_t nitems,
                                                   const int32_t *__restrict__ sn_ptr,
                                                   const int32_t *__restrict__ sn_of_row, int *level,
                                                   int *err, long long limit) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t t = w0; t < nitems; t += nw) {
    const int64_t item = UPPER ? nitems - 1 - t : t;
    const int64_t a = IDENT ? item : sn_ptr[item];
    const int64_t b = IDENT ? item + 1 : sn_ptr[item + 1];
    const int64_t row = UPPER ? b - 1 : a;
    const int64_t s = rp[row], e = rp[row + 1];
    const int64_t lo = UPPER ? s + 1 : s, hi = UPPER ? e : e - 1;
    // one lane waits for the nearest dependency (usually the last to finish)
    if (hi > lo && lane == 0) {
      const int32_t j = ci[UPPER ? lo : hi - 1];
      (void)wait_int(level + (IDENT ? j : sn_of_row[j]), err, limit);
    }
    int mx = -1;
    for (int64_t q = lo + lane; q < hi; q += 64) {
      const int32_t j = ci[q];
      const int dep = IDENT ? j : sn_of_row[j];
      const int lv = wait_int(level + dep, err, limit);
      mx = lv > mx ? lv : mx;
    }
    mx = wave_max_int(mx);
    if (lane == 0) st_agent(level + item, mx + 1);
  }
}

// Schedule records in level order (see SnItem).
__global__ void k_sched_items(const int32_t *__restrict__ order, const int32_t *__restrict__ sn_ptr,
                              const int64_t *__restrict__ rp, int64_t nsn, bool upper, SnItem *__restrict__ items) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nsn; t += (int64_t)gridDim.x * blockDim.x) {
    const int s = order[t];
    const int a = sn_ptr[s], sz = sn_ptr[s + 1] - a;
    const int64_t m = upper ? rp[a + sz] - rp[a + sz - 1] - 1 : rp[a + 1] - rp[a] - 1;
    SnItem it;
    it.ro0 = rp[a];
    it.a = a;
    it.m_sz = (int32_t)((m << 3) | sz);
    items[t] = it;
  }
}

__global__ void k_level_hist(const int32_t *__restrict__ level, int64_t n, int32_t *cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[level[i]], 1);
}

template <typename K>
int resident_grid(K kernel, int block, const Device &dev, int64_t want_waves) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  int64_t g = (int64_t)per_cu * dev.num_cu;
  const int64_t need = (want_waves * 64 + block - 1) / block;
  if (need < g) g = need;
  if (g < 1) g = 1;
  return (int)g;
}

int bits_for(int64_t maxval) {
  int b = 1;
  while (b < 32 && ((int64_t)1 << b) <= maxval) ++b;
  return b;
}

// level[] of nitems units -> (nlev, order sorted by (level, id), optional level_ptr)
int sort_by_level(const int32_t *level, int64_t nitems, int32_t *order, int32_t *level_ptr,
                  int64_t *nlev_host, hipStream_t s) {
  int32_t mx = -1;
  int st = reduce_max_i32(level, nitems, s, &mx);
  if (st) return st;
  const int64_t nlev = nitems > 0 ? (int64_t)mx + 1 : 0;
  *nlev_host = nlev;
  if (order) {
    DevBuf iota, kout;
    if (iota.reserve(nitems * 4) || kout.reserve(nitems * 4)) return ICPCG_E_NOMEM;
    if ((st = fill_iota_u32(iota.as<uint32_t>(), nitems, s))) return st;
    if ((st = radix_sort_pairs(reinterpret_cast<const uint32_t *>(level), iota.as<uint32_t>(),
                               kout.as<uint32_t>(), reinterpret_cast<uint32_t *>(order), nitems,
                               bits_for(nlev), s)))
      return st;
  }
  if (level_ptr) {
    DevBuf cnt;
    if (cnt.reserve((nlev + 1) * 4)) return ICPCG_E_NOMEM;
    if ((st = fill_i32(cnt.as<int32_t>(), 0, nlev + 1, s))) return st;
    hipLaunchKernelGGL(k_level_hist, dim3(grid_rows(nitems, kBlock)), dim3(kBlock), 0, s, level, nitems,
                       cnt.as<int32_t>());
    ICPCG_HIP_TRY(hipGetLastError());
    if ((st = scan_exclusive_i32(cnt.as<int32_t>(), level_ptr, nlev + 1, s, nullptr))) return st;
    ICPCG_HIP_TRY(hipStreamSynchronize(s));
  }
  return ICPCG_OK;
}

int check_err_flag(DevBuf &err, hipStream_t s, const char *what) {
  int h = 0;
  ICPCG_HIP_TRY(hipMemcpyAsync(&h, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  if (h) {
    set_error(std::string(what) + ": device-side dependency wait timed out");
    return ICPCG_E_DEVICE;
  }
  return ICPCG_OK;
}

}  // namespace

// -------------------------------------------------------------- launchers

int check_csr(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, int mode, const double *val,
              hipStream_t s, int *bad_row_host) {
  DevBuf bad;
  if (bad.reserve(sizeof(int))) return ICPCG_E_NOMEM;
  int st;
  if ((st = fill_i32(bad.as<int32_t>(), INT_MAX, 1, s))) return st;
  hipLaunchKernelGGL(k_check_csr, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, val, n, nnz, mode,
                     bad.as<int>());
  ICPCG_HIP_TRY(hipGetLastError());
  int h = INT_MAX;
  ICPCG_HIP_TRY(hipMemcpyAsync(&h, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  *bad_row_host = h == INT_MAX ? -1 : h;
  return ICPCG_OK;
}

int tril_count(const int64_t *rp, const int32_t *ci, int64_t n, int64_t *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_tril_count, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, n, cnt);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int tril_copy(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const int64_t *lrp,
              int32_t *lci, double *lv, hipStream_t s) {
  hipLaunchKernelGGL(k_tril_copy, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, v, n, lrp, lci, lv);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

// U = L^T by a stable radix sort of L's entries on their column index: rows
// of U list the rows of L in ascending order, so every U row starts with its
// diagonal. upos keeps, for each U entry, its position in L (used to refresh
// values without re-sorting).
int build_transpose(icpcg_prec *P, hipStream_t s) {
  const int64_t n = P->n, nnz = P->nnz;
  int st;
  if ((st = P->urp.reserve((n + 1) * 8)) || (st = P->uci.reserve(nnz * 4)) ||
      (st = P->upos.reserve(nnz * 4)) || (st = P->uval.reserve(nnz * 8)))
    return st;
  DevBuf rowid, iota, kout, perm, cnt;
  if (rowid.reserve(nnz * 4) || iota.reserve(nnz * 4) || kout.reserve(nnz * 4) || perm.reserve(nnz * 4) ||
      cnt.reserve((n + 1) * 8))
    return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_row_of_entry, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, P->lrp.as<int64_t>(), n,
                     rowid.as<uint32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = fill_iota_u32(iota.as<uint32_t>(), nnz, s))) return st;
  if ((st = radix_sort_pairs(P->lci.as<uint32_t>(), iota.as<uint32_t>(), kout.as<uint32_t>(),
                             perm.as<uint32_t>(), nnz, bits_for(n - 1), s)))
    return st;
  if ((st = fill_u64(cnt.as<uint64_t>(), 0, n + 1, s))) return st;
  hipLaunchKernelGGL(k_col_count, dim3(grid_rows(nnz, kBlock)), dim3(kBlock), 0, s, P->lci.as<int32_t>(), nnz,
                     cnt.as<unsigned long long>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t total = 0;
  if ((st = scan_exclusive_i64(cnt.as<int64_t>(), P->urp.as<int64_t>(), n, s, &total))) return st;
  hipLaunchKernelGGL(k_set_last_i64, dim3(1), dim3(1), 0, s, P->urp.as<int64_t>(), n, nnz);
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_transpose_gather, dim3(grid_rows(nnz, kBlock)), dim3(kBlock), 0, s, perm.as<uint32_t>(),
                     rowid.as<uint32_t>(), nnz, P->uci.as<int32_t>(), P->upos.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return refresh_values(P, s);
}

int refresh_values(icpcg_prec *P, hipStream_t s) {
  const int64_t nnz = P->nnz;
  const unsigned g = grid_rows(nnz, kBlock);
  hipLaunchKernelGGL(k_gather_f64, dim3(g), dim3(kBlock), 0, s, P->lval.as<double>(), P->upos.as<int32_t>(), nnz,
                     P->uval.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  if (P->dtype == ICPCG_F32) {
    if (P->lval_lo.reserve(nnz * 4) || P->uval_lo.reserve(nnz * 4)) return ICPCG_E_NOMEM;
    hipLaunchKernelGGL(k_cast_f32, dim3(g), dim3(kBlock), 0, s, P->lval.as<double>(), nnz, P->lval_lo.as<float>());
    hipLaunchKernelGGL(k_cast_f32, dim3(g), dim3(kBlock), 0, s, P->uval.as<double>(), nnz, P->uval_lo.as<float>());
    ICPCG_HIP_TRY(hipGetLastError());
  } else if (P->dtype == ICPCG_BF16) {
    if (P->lval_lo.reserve(nnz * 2) || P->uval_lo.reserve(nnz * 2)) return ICPCG_E_NOMEM;
    hipLaunchKernelGGL(k_cast_bf16, dim3(g), dim3(kBlock), 0, s, P->lval.as<double>(), nnz,
                       P->lval_lo.as<unsigned short>());
    hipLaunchKernelGGL(k_cast_bf16, dim3(g), dim3(kBlock), 0, s, P->uval.as<double>(), nnz,
                       P->uval_lo.as<unsigned short>());
    ICPCG_HIP_TRY(hipGetLastError());
  }
  return ICPCG_OK;
}

// Runs of rows flagged by begin[] (1 = starts a new run) split into pieces of
// at most smax rows: ptr[0..count] row ranges, and (optionally) the piece of
// every row.
int runs_to_pieces(const int32_t *begin, int64_t n, int smax, DevBuf &ptr, int32_t *piece_of_row, int64_t *count,
                   hipStream_t s) {
  int st;
  DevBuf key, rs, fb, ex, pr;
  if (key.reserve(n * 4) || rs.reserve(n * 4) || fb.reserve(n * 4) || ex.reserve(n * 4)) return ICPCG_E_NOMEM;
  if (!piece_of_row) {
    if (pr.reserve(n * 4)) return ICPCG_E_NOMEM;
    piece_of_row = pr.as<int32_t>();
  }
  const unsigned g = grid_rows(n, kBlock);
  hipLaunchKernelGGL(k_begin_key, dim3(g), dim3(kBlock), 0, s, begin, n, key.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = scan_inclusive_max_i32(key.as<int32_t>(), rs.as<int32_t>(), n, s))) return st;
  hipLaunchKernelGGL(k_split, dim3(g), dim3(kBlock), 0, s, begin, rs.as<int32_t>(), n, smax, fb.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int32_t np = 0;
  if ((st = scan_exclusive_i32(fb.as<int32_t>(), ex.as<int32_t>(), n, s, &np))) return st;
  *count = np;
  if (ptr.reserve(((size_t)np + 1) * 4)) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_sn_index, dim3(g), dim3(kBlock), 0, s, fb.as<int32_t>(), ex.as<int32_t>(), n,
                     ptr.as<int32_t>(), piece_of_row);
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_set_last_i32, dim3(1), dim3(1), 0, s, ptr.as<int32_t>(), (int64_t)np, (int32_t)n);
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

// Groups of up to gmax consecutive rows with identical column lists (used by
// the grouped SpMV, which then reads each column index and gathers each x row
// once per group).
__global__ void k_group_records(const int64_t *__restrict__ rp, const int32_t *__restrict__ gptr, int64_t ngroups,
                                SpGroup *__restrict__ rec) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r0 = gptr[g];
    const int64_t base = rp[r0];
    SpGroup G;
    G.base = base;
    G.r0 = r0;
    G.m_sz = (int32_t)((rp[r0 + 1] - base) << 3) | (gptr[g + 1] - r0);
    rec[g] = G;
  }
}

int build_row_groups(const int64_t *rp, const int32_t *ci, int64_t n, int gmax, DevBuf &gptr, DevBuf &grec,
                     int64_t *ngroups, hipStream_t s) {
  DevBuf begin;
  if (begin.reserve(n * 4)) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_same_begin, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, n, begin.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int st = runs_to_pieces(begin.as<int32_t>(), n, gmax, gptr, nullptr, ngroups, s);
  if (st) return st;
  if (grec.reserve(*ngroups * sizeof(SpGroup))) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_group_records, dim3(grid_rows(*ngroups, 4)), dim3(kBlock), 0, s, rp, gptr.as<int32_t>(),
                     *ngroups, grec.as<SpGroup>());
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

// Fill-in dropout (Eq. 10): per row, the diagonal and the entries with
// |l_ij| > eps are kept.
__global__ void k_drop_count(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, int64_t n, double eps, int64_t *__restrict__ cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t c = 0;
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) c += (ci[t] == i || fabs(v[t]) > eps) ? 1 : 0;
    cnt[i] = c;
  }
}

__global__ void k_drop_copy(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const double *__restrict__ v, int64_t n, double eps, const int64_t *__restrict__ orp,
                            int32_t *__restrict__ oci, double *__restrict__ ov) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = orp[i];
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      if (ci[t] == i || fabs(v[t]) > eps) {
        oci[o] = ci[t];
        ov[o] = v[t];
        ++o;
      }
    }
  }
}

int dropout(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, double eps, int64_t *orp,
            int32_t *oci, double *ov, int64_t *nnz_host, hipStream_t s) {
  DevBuf cnt;
  if (cnt.reserve((n + 1) * 8)) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_drop_count, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, v, n, eps, cnt.as<int64_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t total = 0;
  int st = scan_exclusive_i64(cnt.as<int64_t>(), orp, n, s, &total);
  if (st) return st;
  hipLaunchKernelGGL(k_set_last_i64, dim3(1), dim3(1), 0, s, orp, n, total);
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_drop_copy, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, v, n, eps, orp, oci, ov);
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  *nnz_host = total;
  return ICPCG_OK;
}

// Supernode schedule of a triangular pattern: maximal runs of consecutive
// rows that share their off-block columns (split into pieces of at most smax
// rows), with the level of each supernode in the quotient dependency graph
// and the supernodes sorted by (level, id).
int build_schedule(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, int smax, TriSchedule &out,
                   hipStream_t s, const Device &dev) {
  int st;
  DevBuf begin, sn_of_row, level, err;
  if (begin.reserve(n * 4) || sn_of_row.reserve(n * 4) || err.reserve(4)) return ICPCG_E_NOMEM;
  const unsigned gw = grid_rows(n, 4);
  if (upper)
    hipLaunchKernelGGL(k_sn_begin<true>, dim3(gw), dim3(kBlock), 0, s, rp, ci, n, begin.as<int32_t>());
  else
    hipLaunchKernelGGL(k_sn_begin<false>, dim3(gw), dim3(kBlock), 0, s, rp, ci, n, begin.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t nsn = 0;
  if ((st = runs_to_pieces(begin.as<int32_t>(), n, smax, out.sn_ptr, sn_of_row.as<int32_t>(), &nsn, s))) return st;
  out.nsn = nsn;
  if (out.sn_order.reserve(nsn * 4) || level.reserve(nsn * 4)) return ICPCG_E_NOMEM;
  if ((st = fill_i32(level.as<int32_t>(), -1, nsn, s)) || (st = fill_i32(err.as<int32_t>(), 0, 1, s))) return st;
  if (upper) {
    auto k = k_levels<true, false>;
    const int grid = resident_grid(k, kBlock, dev, nsn);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, rp, ci, (int64_t)nsn, out.sn_ptr.as<int32_t>(),
                       sn_of_row.as<int32_t>(), level.as<int>(), err.as<int>(), dev.wait_ticks);
  } else {
    auto k = k_levels<false, false>;
    const int grid = resident_grid(k, kBlock, dev, nsn);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, rp, ci, (int64_t)nsn, out.sn_ptr.as<int32_t>(),
                       sn_of_row.as<int32_t>(), level.as<int>(), err.as<int>(), dev.wait_ticks);
  }
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = check_err_flag(err, s, "supernode level analysis"))) return st;
  if ((st = sort_by_level(level.as<int32_t>(), nsn, out.sn_order.as<int32_t>(), nullptr, &out.nlev, s))) return st;
  if (out.items.reserve((size_t)nsn * sizeof(SnItem))) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_sched_items, dim3(grid_rows(nsn, kBlock)), dim3(kBlock), 0, s, out.sn_order.as<int32_t>(),
                     out.sn_ptr.as<int32_t>(), rp, (int64_t)nsn, upper, out.items.as<SnItem>());
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

// Row schedule of a lower pattern derived from its supernode levels: row r of
// supernode S (position p in it) gets the key level(S) * kSupernodeMax + p.
// Every dependency of r lies in a supernode of a lower level or earlier in S,
// so ordering rows by key is a valid schedule; it has about as many steps as
// the row levels on node-structured matrices (3-DOF nodes) but the analysis
// walks supernodes, not rows. Outputs the rows sorted by (key, row), the key
// pointer array (kSupernodeMax * n + 1 entries at most) and its length.
__global__ void k_sn_row_keys(const int32_t *__restrict__ sn_of_row, const int32_t *__restrict__ sn_ptr,
                              const int32_t *__restrict__ level, int64_t n, int32_t *__restrict__ key) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t sn = sn_of_row[r];
    key[r] = level[sn] * kSupernodeMax + (int32_t)(r - sn_ptr[sn]);
  }
}

int supernode_row_order(const int64_t *rp, const int32_t *ci, int64_t n, int32_t *perm, int32_t *key_ptr,
                        int64_t *nkeys_host, hipStream_t s, const Device &dev) {
  int st;
  DevBuf begin, sn_of_row, sn_ptr, level, err, key;
  if (begin.reserve(n * 4) || sn_of_row.reserve(n * 4) || err.reserve(4) || key.reserve(n * 4))
    return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_sn_begin<false>, dim3(grid_rows(n, 4)), dim3(kBlock), 0, s, rp, ci, n, begin.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t nsn = 0;
  if ((st = runs_to_pieces(begin.as<int32_t>(), n, kSupernodeMax, sn_ptr, sn_of_row.as<int32_t>(), &nsn, s)))
    return st;
  if (level.reserve(nsn * 4)) return ICPCG_E_NOMEM;
  if ((st = fill_i32(level.as<int32_t>(), -1, nsn, s)) || (st = fill_i32(err.as<int32_t>(), 0, 1, s))) return st;
  auto k = k_levels<false, false>;
  const int grid = resident_grid(k, kBlock, dev, nsn);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, rp, ci, (int64_t)nsn, sn_ptr.as<int32_t>(),
                     sn_of_row.as<int32_t>(), level.as<int>(), err.as<int>(), dev.wait_ticks);
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = check_err_flag(err, s, "supernode level analysis"))) return st;
  hipLaunchKernelGGL(k_sn_row_keys, dim3(grid_rows(n, kBlock)), dim3(kBlock), 0, s, sn_of_row.as<int32_t>(),
                     sn_ptr.as<int32_t>(), level.as<int32_t>(), n, key.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  return sort_by_level(key.as<int32_t>(), n, perm, key_ptr, nkeys_host, s);
}

// Row level sets (bit-exact integers): level, rows sorted by (level, row) and
// the level pointer array.
int row_levels(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, int32_t *level, int32_t *perm,
               int32_t *level_ptr, int64_t *nlev_host, hipStream_t s, const Device &dev) {
  int st;
  DevBuf err, lev_own;
  if (err.reserve(4)) return ICPCG_E_NOMEM;
  int32_t *lev = level;
  if (!lev) {
    if (lev_own.reserve(n * 4)) return ICPCG_E_NOMEM;
    lev = lev_own.as<int32_t>();
  }
  if ((st = fill_i32(lev, -1, n, s)) || (st = fill_i32(err.as<int32_t>(), 0, 1, s))) return st;
  if (upper) {
    auto k = k_levels<true, true>;
    const int grid = resident_grid(k, kBlock, dev, n);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, rp, ci, n, nullptr, nullptr, lev, err.as<int>(),
                       dev.wait_ticks);
  } else {
    auto k = k_levels<false, true>;
    const int grid = resident_grid(k, kBlock, dev, n);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, rp, ci, n, nullptr, nullptr, lev, err.as<int>(),
                       dev.wait_ticks);
  }
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = check_err_flag(err, s, "row level analysis"))) return st;
  return sort_by_level(lev, n, perm, level_ptr, nlev_host, s);
}

}  // namespace icpcg
