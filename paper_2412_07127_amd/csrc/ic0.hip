// IC(0) factorization in FP64 (incomplete Cholesky with zero fill: L keeps
// the pattern of tril(A); Model Architecture section), row-oriented:
//   for each stored j < i, ascending:
//     L_ij = (A_ij - sum_{k in S(i) and S(j), k < j} L_ik L_jk) / L_jj
//   L_ii = sqrt(A_ii + alpha A_ii - sum_{k < i} L_ik^2)
// One wave computes one row i:
//  * Row i lives in LDS. The rows j it depends on are read once, in one batch
//    of independent loads; each entry L_jk is matched against row i's pattern
//    (binary search) while the batch is in flight, and only the entries that
//    meet it are kept in LDS with the position of k in row i (a wave-ballot
//    compaction that keeps them grouped by j). For 3-DOF elasticity about a
//    third of the entries of the rows j meet row i, so the staged data is a
//    few KB per wave.
//  * Rows with at most 64 off-diagonal entries run a right-looking chain:
//    lane q' owns L_iq' and accumulates A_iq' - sum_{q < q'} L_iq L_{j'k_q}
//    (ascending q); at step q, L_iq = acc_q / L_jj is broadcast from lane q and
//    every lane whose next staged entry sits at position q folds it in. A step
//    is one division, one broadcast and one FMA.
//  * Longer rows pull instead: per step q, the lanes cover the staged entries
//    of row j = cols[q] and meet in a fixed butterfly; rows whose matched
//    entries exceed the LDS budget walk the rows j in global memory.
// Two schedules run that row routine:
//  * level launches (default): one launch per level of tril(A)'s row
//    schedule, one wave per row; a level wider than one resident round of
//    staged waves runs without staging (more rows in flight); a failed shift
//    attempt's remaining levels return at once;
//  * sync-free: one launch per shift attempt. Waves take rows in level order
//    from a ticket counter (fetched one row ahead); the factor values start as
//    a reserved NaN pattern and every row is published with device-scope
//    stores. A row first waits for all the entries it uses (one lane polls the
//    last pending row's diagonal with backoff, then all lanes reload once). A
//    row is taken only by a running wave, so the smallest unfinished row is
//    always held by a running wave whose inputs are done and the launch
//    progresses however many of its blocks are resident. A failed pivot stops
//    the attempt everywhere and a wall-clock limit turns an impossible wait
//    into an error. On the elasticity workloads it is slower than the level
//    launches (waiting rows hold waves and their polls contend for memory).
// The two give bit-identical factors whenever every level is narrow enough to
// be staged (then each row takes the same path in both).
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kMaxRow = 1024;   // entries of one row of tril(A)
constexpr int kMatchCap = 576;  // staged entries of the rows j that meet row i (at most)
using U64 = unsigned long long;

// Dynamic LDS of one wave: vals, jdiag, jstart (8 B x L), staged values (8 B x
// M), cols (4 B x L), off and coff (4 B x (L + 1)), staged positions (4 B x M),
// for rows of at most L entries and a staging budget of M entries.
size_t row_lds_bytes(int L, int M) { return (size_t)L * 36 + 8 + (size_t)M * 12; }

template <bool SYNC>
__device__ __forceinline__ U64 load_val(const double *p) {
  if constexpr (SYNC) return ld_agent(reinterpret_cast<const U64 *>(p));
  return *reinterpret_cast<const U64 *>(p);
}

// First position of k in the sorted cols[0, q), or -1.
__device__ __forceinline__ int find_col(const int32_t *cols, int q, int k) {
  int lo = 0, hi = q;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cols[mid] < k) lo = mid + 1; else hi = mid;
  }
  return (lo < q && cols[lo] == k) ? lo : -1;
}

__device__ __forceinline__ bool attempt_failed(const int *fail) {
  return __builtin_amdgcn_readfirstlane(ld_agent(fail)) != 0;
}

// Factor row i. Returns false when a sync-free attempt is abandoned (another
// row failed, or a wait reached its time limit).
template <bool SYNC>
__device__ bool factor_row(int i, const int64_t *__restrict__ lrp, const int32_t *__restrict__ lci, double *lv,
                           const double *__restrict__ a_low, double alpha, int *fail, int *err, long long limit,
                           double *__restrict__ pivots, int L, int mcap, double *smem) {
  const int lane = threadIdx.x;
  double *vals = smem;
  double *jdiag = vals + L;
  double *mv = jdiag + L;
  int64_t *jstart = reinterpret_cast<int64_t *>(mv + mcap);
  int32_t *cols = reinterpret_cast<int32_t *>(jstart + L);
  int32_t *off = cols + L;
  int32_t *coff = off + L + 1;
  uint32_t *mpp = reinterpret_cast<uint32_t *>(coff + L + 1);

  const int64_t rs = lrp[i];
  const int len = (int)(lrp[i + 1] - rs);
  for (int q = lane; q < len; q += 64) {
    cols[q] = lci[rs + q];
    vals[q] = a_low[rs + q];
  }
  __syncthreads();
  // rows j: start, diagonal, and lengths (without the diagonal) scanned into
  // offsets of the concatenated entry list
  int carry = 0;
  for (int q0 = 0; q0 < len - 1; q0 += 64) {
    const int q = q0 + lane;
    int l = 0;
    if (q < len - 1) {
      const int j = cols[q];
      const int64_t js = lrp[j], je = lrp[j + 1];
      l = (int)(je - js) - 1;
      jstart[q] = js;
      jdiag[q] = bitcast<double>(load_val<SYNC>(lv + je - 1));
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
  if (lane == 0) off[len - 1] = carry;
  __syncthreads();
  // stage the entries of the rows j that meet row i, grouped by j, with the
  // position of their column in row i and their offset in row j
  int base = 0;
  for (int e0 = 0; mcap > 0 && e0 < carry; e0 += 4 * 64) {
    int qq[4], pp[4], kk[4];
    U64 raw[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * 64 + lane;
      qq[u] = -1;
      pp[u] = 0;
      kk[u] = 0;
      raw[u] = 0;
      if (e < carry) {
        int lo = 0, hi = len - 1;  // q with off[q] <= e < off[q + 1]
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int p = e - off[lo];
        const int64_t src = jstart[lo] + p;
        kk[u] = lci[src];
        raw[u] = load_val<SYNC>(lv + src);
        qq[u] = lo;
        pp[u] = p;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int pos = qq[u] >= 0 ? find_col(cols, qq[u], kk[u]) : -1;
      const U64 mask = __ballot(pos >= 0);
      const int before =
          base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
      if (pos >= 0 && before < mcap) {
        mv[before] = bitcast<double>(raw[u]);
        mpp[before] = (uint32_t)pos | ((uint32_t)pp[u] << 16);
      }
      if (qq[u] >= 0 && pp[u] == 0) {  // first entry of row j: its staged offset
        const int e = e0 + u * 64 + lane;
        coff[qq[u]] = before;
        for (int q2 = qq[u] - 1; q2 >= 0 && off[q2] == e; --q2) coff[q2] = before;  // empty rows j before it
      }
      base += __popcll(mask);
    }
  }
  for (int q = lane; q < len; q += 64)
    if (off[q] == carry) coff[q] = base;
  // without a staging budget only rows with no entries in their rows j count
  // as staged (the fast chain then folds nothing)
  const bool staged = mcap > 0 ? base <= mcap : carry == 0;
  __syncthreads();

  const int nq = len - 1;  // off-diagonal entries of row i
  if (staged && nq <= 64) {
    // Right-looking chain, lane q' owning L_iq'. Lane q' keeps
    // A_iq' - sum_{q < q'} L_iq L_{j'k_q} in acc: at step q, L_iq = acc_q / L_jj
    // is broadcast from lane q and every lane whose next staged entry sits at
    // position q folds it in. A step is one division, one broadcast and one
    // FMA; the staged entries stream through a register window.
    if constexpr (SYNC) {
      // all inputs of the row first: staged entries and diagonals of the rows
      // j. While some are pending, one lane polls the diagonal of the last
      // pending row j (rows finish roughly in order), then every lane reloads
      // its pending entries once.
      const long long t0 = wall_clock64();
      while (true) {
        bool pend = false;
        if (lane < nq) {
          for (int t = coff[lane]; t < coff[lane + 1]; ++t) pend |= bitcast<U64>(mv[t]) == Flag<double>::kPending;
          pend |= bitcast<U64>(jdiag[lane]) == Flag<double>::kPending;
        }
        const U64 mask = __ballot(pend);
        if (!mask) break;
        const int sl = 63 - __builtin_clzll(mask);  // last pending entry of row i
        if (lane == 0) {
          const bool ok = poll_f64(lv + jstart[sl] + (off[sl + 1] - off[sl]), err, limit, fail);
          if (!ok && !ld_agent(fail)) __hip_atomic_fetch_or(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (attempt_failed(fail)) return false;
        if (pend) {
          const U64 *src = reinterpret_cast<const U64 *>(lv + jstart[lane]);
          for (int t = coff[lane]; t < coff[lane + 1]; ++t)
            if (bitcast<U64>(mv[t]) == Flag<double>::kPending) mv[t] = bitcast<double>(ld_agent(src + (mpp[t] >> 16)));
          if (bitcast<U64>(jdiag[lane]) == Flag<double>::kPending)
            jdiag[lane] = bitcast<double>(ld_agent(src + (off[lane + 1] - off[lane])));
        }
        if (wall_clock64() - t0 > limit) {
          if (lane == 0) {
            __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          return false;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    double acc = 0.0, dj = 1.0, fin = 0.0;
    int ptr = 0, end = 0;
    if (lane < nq) {
      acc = vals[lane];
      dj = jdiag[lane];
      ptr = coff[lane];
      end = coff[lane + 1];
    }
    int p0 = 64, p1 = 64, p2 = 64;  // positions in row i of the next three entries
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (ptr < end) { p0 = (int)(mpp[ptr] & 0xFFFFu); v0 = mv[ptr]; }
    if (ptr + 1 < end) { p1 = (int)(mpp[ptr + 1] & 0xFFFFu); v1 = mv[ptr + 1]; }
    if (ptr + 2 < end) { p2 = (int)(mpp[ptr + 2] & 0xFFFFu); v2 = mv[ptr + 2]; }
    for (int q = 0; q < nq; ++q) {
      const double lq = acc / dj;  // final on lane q
      const U64 u = bitcast<U64>(lq);
      const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, q);
      const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), q);
      const double x = bitcast<double>(((U64)hi << 32) | lo);
      if (lane == q) fin = x;
      if (p0 == q) {
        acc = fma(-x, v0, acc);
        p0 = p1; v0 = v1;
        p1 = p2; v1 = v2;
        ++ptr;
        p2 = 64;
        if (ptr + 2 < end) { p2 = (int)(mpp[ptr + 2] & 0xFFFFu); v2 = mv[ptr + 2]; }
      }
    }
    if (lane < nq) vals[lane] = fin;
    __syncthreads();
  } else {
    // per step: lanes over the entries of row j = cols[q], one butterfly
    for (int q = 0; q < len - 1; ++q) {
      double part = 0.0;
      if (staged) {
        const int b = coff[q], cnt = coff[q + 1] - b;
        if constexpr (SYNC) {
          // wait until the entries of row j used here and its diagonal are final
          bool pend = false;
          for (int p = lane; p < cnt; p += 64) pend |= bitcast<U64>(mv[b + p]) == Flag<double>::kPending;
          if (lane == 0) pend |= bitcast<U64>(jdiag[q]) == Flag<double>::kPending;
          if (__ballot(pend)) {
            const long long t0 = wall_clock64();
            int backoff = 1;
            while (true) {
              for (int t = 0; t < backoff; ++t) __builtin_amdgcn_s_sleep(1);
              if (backoff < 8) backoff <<= 1;
              pend = false;
              for (int p = lane; p < cnt; p += 64)
                if (bitcast<U64>(mv[b + p]) == Flag<double>::kPending) {
                  const U64 v = ld_agent(reinterpret_cast<const U64 *>(lv + jstart[q] + (mpp[b + p] >> 16)));
                  mv[b + p] = bitcast<double>(v);
                  pend |= v == Flag<double>::kPending;
                }
              if (lane == 0 && bitcast<U64>(jdiag[q]) == Flag<double>::kPending) {
                const U64 v = ld_agent(reinterpret_cast<const U64 *>(lv + jstart[q] + (off[q + 1] - off[q])));
                jdiag[q] = bitcast<double>(v);
                pend |= v == Flag<double>::kPending;
              }
              if (!__ballot(pend)) break;
              if (attempt_failed(fail)) return false;
              if (wall_clock64() - t0 > limit) {
                if (lane == 0) {
                  __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                  __hip_atomic_fetch_or(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return false;
              }
            }
          }
        }
        for (int p = lane; p < cnt; p += 64) part += vals[mpp[b + p] & 0xFFFFu] * mv[b + p];
      } else {
        // row j walked in global memory
        const int64_t js = jstart[q];
        const int jl = off[q + 1] - off[q];
        bool gone = false;
        if constexpr (SYNC) {
          if (lane == 0) {
            U64 v = bitcast<U64>(jdiag[q]);
            const long long t0 = wall_clock64();
            while (v == Flag<double>::kPending) {
              __builtin_amdgcn_s_sleep(1);
              v = ld_agent(reinterpret_cast<const U64 *>(lv + js + jl));
              if (v != Flag<double>::kPending) break;
              if (ld_agent(fail) || wall_clock64() - t0 > limit) { gone = true; break; }
            }
            jdiag[q] = bitcast<double>(v);
          }
        }
        for (int p = lane; p < jl && !gone; p += 64) {
          const int pos = find_col(cols, q, lci[js + p]);
          if (pos < 0) continue;
          U64 v = load_val<SYNC>(lv + js + p);
          if constexpr (SYNC) {
            const long long t0 = wall_clock64();
            while (v == Flag<double>::kPending) {
              __builtin_amdgcn_s_sleep(1);
              v = ld_agent(reinterpret_cast<const U64 *>(lv + js + p));
              if (v != Flag<double>::kPending) break;
              if (ld_agent(fail) || wall_clock64() - t0 > limit) { gone = true; break; }
            }
          }
          part += vals[pos] * bitcast<double>(v);
        }
        if constexpr (SYNC) {
          if (__ballot(gone)) {
            if (lane == 0 && !ld_agent(fail)) {  // time limit, not another row's failure
              __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              __hip_atomic_fetch_or(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return false;
          }
        }
      }
      const double sum = wave_sum(part);
      if (lane == 0) vals[q] = (vals[q] - sum) / jdiag[q];
      __syncthreads();
    }
  }
  double dp = 0.0;
  for (int q = lane; q < len - 1; q += 64) dp += vals[q] * vals[q];
  dp = wave_sum(dp);
  if (lane == 0) {
    const double aii = vals[len - 1];
    const double d = aii + alpha * aii - dp;
    pivots[i] = d;
    if (!(d > 0.0)) __hip_atomic_fetch_or(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    vals[len - 1] = d > 0.0 ? sqrt(d) : (double)NAN;
  }
  __syncthreads();
  for (int q = lane; q < len; q += 64) {
    if constexpr (SYNC) publish_value(lv + rs + q, vals[q]);
    else lv[rs + q] = vals[q];
  }
  __syncthreads();  // LDS is reused by the next row
  return true;
}

// One level of the row schedule: one wave per row, rows j final.
__global__ __launch_bounds__(64) void k_ic0_rows(const int32_t *__restrict__ rows, const int64_t *__restrict__ lrp,
                                                 const int32_t *__restrict__ lci, double *lv,
                                                 const double *__restrict__ a_low, double alpha, int *fail,
                                                 double *__restrict__ pivots, int L, int mcap) {
  if (*fail) return;  // an earlier level broke down: this attempt is discarded
  extern __shared__ double smem_d[];
  factor_row<false>(rows[blockIdx.x], lrp, lci, lv, a_low, alpha, fail, nullptr, 0, pivots, L, mcap, smem_d);
}

// Whole factor in one launch (lv filled with the pending pattern, *ticket 0).
__global__ __launch_bounds__(64) void k_ic0_sync(const int32_t *__restrict__ order, int n,
                                                 const int64_t *__restrict__ lrp, const int32_t *__restrict__ lci,
                                                 double *lv, const double *__restrict__ a_low, double alpha, int *fail,
                                                 int *err, unsigned *ticket, long long limit,
                                                 double *__restrict__ pivots, int L) {
  extern __shared__ double smem_d[];
  const unsigned nu = (unsigned)n;
  unsigned it = take_ticket(ticket);
  while (it < nu) {
    const unsigned next = take_ticket(ticket);  // tickets rise, so holding one ahead keeps the order
    if (attempt_failed(fail)) return;
    if (!factor_row<true>(order[it], lrp, lci, lv, a_low, alpha, fail, err, limit, pivots, L, kMatchCap, smem_d))
      return;
    it = next;
  }
}

}  // namespace

int ic0_max_row() { return kMaxRow; }

int ic0_factor_levels(const int64_t *lrp, const int32_t *lci, double *lv, const double *a_low, int64_t,
                      const int32_t *perm, const std::vector<int32_t> &level_ptr, double alpha, int *fail,
                      double *pivots, hipStream_t s, int max_row_len, const Device &dev) {
  // Staging pays while a level's rows are resident at once (each row is a
  // latency-bound chain); a level wider than one resident round of staged
  // waves runs without staging, where the smaller footprint keeps more rows
  // in flight (rows whose matched entries exceed the budget walk the rows j in
  // global memory either way).
  const size_t lds_staged = row_lds_bytes(max_row_len, kMatchCap);
  const size_t lds_plain = row_lds_bytes(max_row_len, 0);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ic0_rows, 64, lds_staged) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  const int64_t staged_round = (int64_t)per_cu * dev.num_cu;
  // A failed attempt's remaining launches return at once, but launching them
  // still costs time: every kBatch levels the failure flag is copied to pinned
  // memory behind an event, and before the next batch is queued the host looks
  // at the previous batch's copy (one batch stays queued, so the GPU does not
  // wait for the host) and stops queueing once the attempt has failed.
  constexpr size_t kBatch = 256;
  int *hflag = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int st = ICPCG_OK;
  if (hipHostMalloc(reinterpret_cast<void **>(&hflag), 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    st = ICPCG_E_DEVICE;
  }
  const size_t nlev = level_ptr.empty() ? 0 : level_ptr.size() - 1;
  for (size_t l0 = 0, bt = 0; st == ICPCG_OK && l0 < nlev; l0 += kBatch, ++bt) {
    for (size_t l = l0; l < std::min(nlev, l0 + kBatch); ++l) {
      const int32_t b = level_ptr[l], e = level_ptr[l + 1];
      if (e <= b) continue;
      const bool stage = (int64_t)(e - b) <= staged_round;
      hipLaunchKernelGGL(k_ic0_rows, dim3((unsigned)(e - b)), dim3(64), stage ? lds_staged : lds_plain, s, perm + b,
                         lrp, lci, lv, a_low, alpha, fail, pivots, max_row_len, stage ? kMatchCap : 0);
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hflag + (bt & 1), fail, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(ev[bt & 1], s) != hipSuccess) {
      st = ICPCG_E_DEVICE;
      break;
    }
    if (bt > 0) {
      if (hipEventSynchronize(ev[(bt - 1) & 1]) != hipSuccess) {
        st = ICPCG_E_DEVICE;
        break;
      }
      if (hflag[(bt - 1) & 1]) break;  // the caller reads the flag after the stream drains
    }
  }
  if (st) set_error("factor: level launch or failure-flag copy failed");
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (hflag) {
    (void)hipStreamSynchronize(s);  // the last copy into the pinned flags has landed
    (void)hipHostFree(hflag);
  }
  return st;
}

int ic0_factor_sync(const int64_t *lrp, const int32_t *lci, double *lv, const double *a_low, int64_t n,
                    const int32_t *order, double alpha, int *fail, int *err, int *ticket, double *pivots,
                    hipStream_t s, int max_row_len, const Device &dev) {
  if (n == 0) return ICPCG_OK;
  const size_t lds = row_lds_bytes(max_row_len, kMatchCap);
  int q = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_ic0_sync, 64, lds) != hipSuccess || q < 1) {
    (void)hipGetLastError();
    q = 1;
  }
  // one wave per row slot the device holds; blocks that do not fit start
  // when others finish and simply take later tickets
  const int64_t grid = std::min<int64_t>((int64_t)q * dev.num_cu, n);
  hipLaunchKernelGGL(k_ic0_sync, dim3((unsigned)grid), dim3(64), lds, s, order, (int)n, lrp, lci, lv, a_low, alpha,
                     fail, err, reinterpret_cast<unsigned *>(ticket), dev.wait_ticks, pivots, max_row_len);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace icpcg
