// Sparse triangular solves with the factor of P = L L^T (the two "triangle
// solving" steps of supplementary Algorithm 1; Eq. (11) read as standard
// substitution), for R right-hand sides at once.
//
// Design (gfx950, wave64):
//  * Schedule unit = supernode: consecutive rows sharing their off-block
//    columns (for 3-DOF elasticity nodes, the 3 rows of a node). One wave owns
//    one supernode, gathers each shared x_j once for all its rows, and solves
//    the small dense diagonal block in registers. This cuts the dependent
//    steps by the supernode size relative to row levels.
//  * Sync-free: supernodes are sorted by level and dealt round-robin to all
//    resident waves. A wave does not wait for a whole level, only for the
//    x_j it reads: the output array starts filled with a reserved NaN
//    pattern, every result is published with a device-scope store, and a
//    reader checks each value with a device-scope load (the value is its own
//    flag, so no fences are needed). The smallest unfinished position is
//    always held by a running wave whose inputs are done, so the co-resident
//    grid always progresses; a wall-clock limit turns an impossible wait into
//    an error instead of a hang.
//  * Latency: every item's metadata is one 16-byte record in schedule order,
//    fetched one item ahead; indices, factor values, the diagonal block and
//    the right-hand side are loaded before any wait; all dependencies are
//    gathered in one round. While some are still pending, the 16-column
//    FP32 / BF16 solves load every pending one again each round (the round
//    that sees the last input ends the wait), pausing between rounds while
//    many inputs are still missing; the others let the lanes
//    covering one pending row poll it (with a short backoff) before the
//    pending ones are loaded again, which keeps their memory traffic lower
//    (measured: faster for the FP64 solves, slower for the 16-column FP32
//    ones).
//  * Lanes of a wave are (slot, column group): a lane owns CPL consecutive
//    columns (1, or 2 from 8 columns up) and R / CPL lanes cover one gathered
//    row of the row-major block, so every device-scope load and every publish
//    is one contiguous row per instruction (full-line requests, no
//    partial-line writes); the slots stride over the off-block entries.
//    Partial sums meet in a fixed butterfly (deterministic).
//  * Factor values may be FP64, FP32 or bfloat16 (widened to FP32); FP32 and
//    bfloat16 factors run FP32 arithmetic.
//  * Inside a PCG step with an FP32 or bfloat16 factor on several columns the
//    solves carry the step's streaming work: the forward solve first applies
//    the previous step's x, r update to its rows (XR) and the backward solve
//    forms r^T z (RZ), each summed into block partials in a fixed order.
#include <algorithm>
#include <cmath>
#include <utility>

#include "reduce.hpp"

namespace icpcg {

namespace {

constexpr int kBlock = 256;
constexpr int kSmax = kSupernodeMax;

template <int LO, typename T>
__device__ __forceinline__ T xor_sum_hi(T v) {
#pragma unroll
  for (int b = 32; b >= (1 << LO); b >>= 1) v += __shfl_xor(v, b, ICPCG_WAVE);
  return v;
}

// Lane K of each 16-lane row of the wave, to every lane of that row (DPP
// row_newbcast). Source lanes are in the reader's own row, so a row that is
// active as a whole reads defined values.
template <int K>
__device__ __forceinline__ float row_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x150 + K, 0xf, 0xf, true));
}
template <int K>
__device__ __forceinline__ int row_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xf, 0xf, true);
}

// f(integral_constant<int, K>) for K = 0 .. N-1 in order (DPP controls must be
// compile-time constants).
template <typename F, int... K>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Row start of row a+u of a supernode from the first row's start: lower rows
// grow by one diagonal-block entry per row, upper rows shrink by one.
template <bool UPPER>
__device__ __forceinline__ int64_t row_start(int64_t ro0, int u, int m, int sz) {
  return UPPER ? ro0 + (int64_t)u * (sz + m) - (int64_t)u * (u - 1) / 2
               : ro0 + (int64_t)u * (m + 1) + (int64_t)u * (u - 1) / 2;
}

// CPL consecutive elements of a row at p, each read with a device-scope load
// (a pair of FP32 values in one 8-byte load). Each element keeps its own
// pending pattern, so a reader never needs the pair to change at once.
template <typename TA, int CPL>
__device__ __forceinline__ void load_elems(const TA *p, typename Flag<TA>::U (&e)[CPL]) {
  using U = typename Flag<TA>::U;
  if constexpr (CPL == 2 && sizeof(U) == 4) {
    const unsigned long long v = ld_agent(reinterpret_cast<const unsigned long long *>(p));
    e[0] = (U)v;
    e[1] = (U)(v >> 32);
  } else {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) e[cc] = ld_agent(reinterpret_cast<const U *>(p) + cc);
  }
}

template <typename TA, int CPL>
__device__ __forceinline__ bool any_pending(const typename Flag<TA>::U (&e)[CPL]) {
  bool pd = false;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) pd |= e[cc] == Flag<TA>::kPending;
  return pd;
}

template <typename TA, int CPL>
__device__ __forceinline__ void publish_elems(TA *p, const TA (&x)[CPL]) {
  using U = typename Flag<TA>::U;
  if constexpr (CPL == 2 && sizeof(U) == 4) {
    U lo = bitcast<U>(x[0]), hi = bitcast<U>(x[1]);
    if (lo == Flag<TA>::kPending) lo = Flag<TA>::kCanonNaN;
    if (hi == Flag<TA>::kPending) hi = Flag<TA>::kCanonNaN;
    st_agent(reinterpret_cast<unsigned long long *>(p), (unsigned long long)lo | ((unsigned long long)hi << 32));
  } else {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) publish_value<TA>(p + cc, x[cc]);
  }
}

// The previous PCG step's x and r update, for the forward solve that applies it.
struct XrArgs {
  double *X;
  double *r;
  const double *p;
  const double *w;
  const ColState *cols;
};

// RZ (backward solves inside the PCG loop): also r^T z of every column, from
// the residual rows loaded with the right-hand side and each published row,
// into block partials (a fixed per-lane order over the lane's items, then the
// block tree).
// XR (forward solves inside the PCG loop): the right-hand side is r after the
// previous step's update r -= alpha w of the columns with upd set. The lanes
// of slot 0 (which solve the diagonal block) form it from r and w loaded with
// the right-hand side, store it with their published rows and sum it as
// ||r||^2 into block partials like RZ; the lanes of slot 1 + u form
// x += alpha p of row u. Each element of r is read once, by the lane that
// then writes it, so reading it through the restrict-qualified rhs is sound.
template <typename TV, typename TA, typename TR, int R, bool UPPER, int QD, int CPL, bool RZ, bool XR>
__global__ __launch_bounds__(kBlock) void k_trsv(const int32_t *__restrict__ ci, const TV *__restrict__ val,
                                                 const SnItem *__restrict__ sched, int64_t nsn,
                                                 const TR *__restrict__ rhs, TA *out, int *err, long long limit,
                                                 const int *__restrict__ active, const double *__restrict__ rres,
                                                 double *rz_partials, XrArgs xr,
                                                 typename Flag<TR>::U *rhs_rearm) {
  static_assert(!(XR && (UPPER || RZ || R == 1 || CPL != 1 || 64 / R <= kSmax)),
                "the x, r update goes with multi-column FP32 forward solves");
  if (active && *active == 0) return;  // every column of the solve has stopped
  using U = typename Flag<TA>::U;
  constexpr int LPR = R / CPL;                   // lanes per gathered row
  constexpr int SLOTS = 64 / LPR;                // entry slots per wave
  constexpr int NDB = kSmax * (kSmax + 1) / 2;  // stored entries of a dense diagonal block
  constexpr unsigned long long kRowMask = LPR >= 64 ? ~0ull : ((1ull << LPR) - 1);
  // Window by broadcast (16 columns of 4-byte values: a slot's lanes form one
  // 16-lane DPP row): each lane loads one window entry (its column index and
  // its values in the supernode's rows) and the row's lanes take entry k from
  // lane k by row broadcast, instead of every lane loading and holding all QD
  // entries (about 30 fewer registers per lane, one more resident wave per SIMD).
  constexpr bool kBC = LPR == 16 && CPL == 1 && sizeof(TA) == 4 && QD <= 16;
  constexpr bool kBCJ = false;  // column indices by broadcast
  constexpr bool kBCV = kBC;    // factor values by broadcast
  const int lane = threadIdx.x & 63, slot = lane / LPR, c0 = (lane % LPR) * CPL;
  // kBC kernels: the wave index as a wave-uniform value, so the item records
  // come through the scalar unit, whose count (lgkmcnt) a wave waits on at the
  // top of each item instead of the vector count, which on this architecture
  // also holds the acknowledgements of the previous item's published rows
  const int64_t wl = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t w0 = kBC ? (int64_t)__builtin_amdgcn_readfirstlane((int)wl) : wl;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  double dot[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) dot[cc] = 0.0;
  double alx[CPL];  // XR: alpha of the lane's columns, 0 where there is no update
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) alx[cc] = 0.0;
  bool upx[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) upx[cc] = false;
  if constexpr (XR) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      upx[cc] = xr.cols[c0 + cc].upd != 0;
      alx[cc] = xr.cols[c0 + cc].alpha;
    }
  }
  SnItem nxt;
  if (w0 < nsn) nxt = sched[w0];
  for (int64_t t = w0; t < nsn; t += nw) {
    const SnItem it = nxt;
    if (t + nw < nsn) nxt = sched[t + nw];  // next item's record arrives while this one runs
    const int a = it.a, sz = it.m_sz & 7, m = it.m_sz >> 3;
    int64_t ro[kSmax];
#pragma unroll
    for (int u = 0; u < kSmax; ++u) ro[u] = row_start<UPPER>(it.ro0, u, m, sz);
    // off-block columns as listed in the first row: after its sz diagonal-block
    // entries (upper) or before its diagonal (lower)
    const int64_t pcol = UPPER ? ro[0] + sz : ro[0];
    // Everything that does not depend on other waves is loaded first.
    // Several columns (R > 1): the factor values unconditionally from a clamped
    // place in the same row (its diagonal when the supernode has no off-block
    // entry), the diagonal block and the right-hand side by every lane (a wave
    // issues the same instructions either way; slot 0 uses them), all kept raw
    // and converted only where used. A load behind a branch, or converted at
    // the join, makes the compiler wait for it there, one row at a time,
    // before the dependencies are even requested, and a wide solve is bound by
    // each item's round trips. A slot past the window gathers x = 0 and the
    // factor's values are finite (checked when the preconditioner is made), so
    // such a product is exactly 0; rows u >= sz are never read. One column: a
    // wave waits on its dependencies anyway (the solve is bound by their
    // depth), so the loads stay behind their branches with the conversions
    // done before the wait, which keeps the path after it shortest
    // (measured: 2-7% faster at one column, 11% slower at sixteen).
    constexpr bool kRaw = R > 1;
    int jj[kBCJ ? 1 : QD];
    TV vv[kBCV ? 1 : QD][kSmax];  // raw (R > 1)
    TA vw[kBCV ? 1 : QD][kSmax];  // widened (R == 1)
    // broadcast forms: lane (slot, c) holds the slot's window entry c
    // (q = slot + c * SLOTS)
    int jown = 0;
    TV vown[kSmax];
    {
      const int qo = slot + c0 * SLOTS;
      const int qoc = qo < m ? qo : m - 1;
      if constexpr (kBCJ) jown = ci[m > 0 ? pcol + qoc : ro[0]];
      if constexpr (kBCV) {
#pragma unroll
        for (int u = 0; u < kSmax; ++u) {
          const int uc = u < sz ? u : sz - 1;
          vown[u] = val[m > 0 ? (UPPER ? ro[uc] + (sz - uc) + qoc : ro[uc] + qoc) : ro[uc]];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int q = slot + k * SLOTS;
      const int qc = q < m ? q : m - 1;
      // kBC kernels: from a clamped in-row place, no branch (the gather of a
      // place past the row is skipped; a supernode with no off-block entry
      // reads its own first entry)
      if constexpr (!kBCJ) jj[k] = kBC ? ci[m > 0 ? pcol + qc : ro[0]] : (q < m ? ci[pcol + q] : 0);
      if constexpr (!kBCV) {
#pragma unroll
        for (int u = 0; u < kSmax; ++u) {
          if constexpr (kRaw) {
            const int uc = u < sz ? u : sz - 1;
            vv[k][u] = val[m > 0 ? (UPPER ? ro[uc] + (sz - uc) + qc : ro[uc] + qc) : ro[uc]];
          } else {
            vw[k][u] = (q < m && u < sz) ? widen<TA>(val[UPPER ? ro[u] + (sz - u) + q : ro[u] + q]) : TA(0);
          }
        }
      }
    }
    auto fval = [&](int k, int u) -> TA {
      if constexpr (kRaw) return widen<TA>(vv[k][u]);
      else return vw[k][u];
    };
    // the diagonal block (row by row; lower: columns a..a+u, upper:
    // a+u..a+sz-1; row a+u of the upper factor holds a+u..a+sz-1 first, so
    // (u, u+w) sits at u*kSmax - u*(u-1)/2 + w) and the right-hand side
    TV dr[NDB];
    TR br[kSmax][CPL];
    TA dv[NDB];
    TA bv[kSmax][CPL];
    double rr[kSmax][CPL];  // residual rows (RZ)
    double tx[kSmax];       // XR: w of the item's rows (slot 0); x and p of row slot - 1
    if constexpr (kRaw) {
#pragma unroll
      for (int u = 0; u < kSmax; ++u) {
        const int uc = u < sz ? u : sz - 1;
        if (!UPPER) {
#pragma unroll
          for (int w = 0; w <= u; ++w) dr[u * (u + 1) / 2 + w] = val[ro[uc] + m + (w < uc ? w : uc)];
        } else {
#pragma unroll
          for (int w = 0; w < kSmax - u; ++w)
            dr[u * kSmax - u * (u - 1) / 2 + w] = val[ro[uc] + (w < sz - uc ? w : sz - 1 - uc)];
        }
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) br[u][cc] = rhs[(int64_t)(a + uc) * R + c0 + cc];
        if constexpr (XR) {
          // one load per register in every lane, its address chosen by slot
          const int ux = slot >= 1 && slot <= kSmax && slot - 1 < sz ? slot - 1 : 0;
          const int64_t ex = (int64_t)(a + ux) * R + c0;
          const double *src = slot == 0 ? xr.w + (int64_t)(a + uc) * R + c0 : u == 0 ? xr.X + ex : xr.p + ex;
          tx[u] = *src;
        }
        if constexpr (RZ) {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) rr[u][cc] = rres[(int64_t)(a + uc) * R + c0 + cc];
        }
      }
    } else if (slot == 0) {
#pragma unroll
      for (int u = 0; u < kSmax; ++u) {
        if (!UPPER) {
#pragma unroll
          for (int w = 0; w <= u; ++w) dv[u * (u + 1) / 2 + w] = u < sz ? widen<TA>(val[ro[u] + m + w]) : TA(1);
        } else {
#pragma unroll
          for (int w = 0; w < kSmax - u; ++w)
            dv[u * kSmax - u * (u - 1) / 2 + w] = (u < sz && w < sz - u) ? widen<TA>(val[ro[u] + w]) : TA(1);
        }
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) bv[u][cc] = u < sz ? (TA)rhs[(int64_t)(a + u) * R + c0 + cc] : TA(0);
        if constexpr (RZ) {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) rr[u][cc] = u < sz ? rres[(int64_t)(a + u) * R + c0 + cc] : 0.0;
        }
      }
    }
    auto dval = [&](int i) -> TA {
      if constexpr (kRaw) return widen<TA>(dr[i]);
      else return dv[i];
    };
    auto bval = [&](int u, int cc) -> TA {
      if constexpr (kRaw) return (TA)br[u][cc];
      else return bv[u][cc];
    };
    // gather the dependencies: one attempt for all, then while any is still
    // pending the lanes covering one pending row poll it together (one
    // contiguous row per load) and the pending ones are loaded again
    U xb[QD][CPL];
    static_for<QD>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      int jk;
      if constexpr (kBCJ) jk = row_bcast<k>(jown);
      else jk = jj[k];
      if (slot + k * SLOTS < m) {
        load_elems<TA, CPL>(out + (int64_t)jk * R + c0, xb[k]);
      } else {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) xb[k][cc] = 0;
      }
    });
    // XR: the update, formed here, where its loads (issued before the gathers)
    // have arrived by the time the first gather is waited for, and stored with
    // the published rows (measured: 0.6% faster than storing it here)
    double xn = 0.0;
    if constexpr (XR) {
#pragma unroll
      for (int u = 0; u < kSmax; ++u) {
        const double rn = fma(-alx[0], tx[u], br[u][0]);
        br[u][0] = upx[0] ? rn : br[u][0];  // meaningful in slot 0
      }
      xn = fma(alx[0], tx[1], tx[0]);  // meaningful in slots 1 .. kSmax
    }
    if constexpr (kBC) {
      // every pending entry is loaded again each round (one round trip per
      // round, no sleep): the first round that sees the last input ends the
      // wait, where polling one row and then reloading the rest costs a
      // second round trip per dependency level
      const long long t0w = wall_clock64();
      for (;;) {
        bool pend = false;
#pragma unroll
        for (int k = 0; k < QD; ++k) pend |= any_pending<TA, CPL>(xb[k]);
        if (!__ballot(pend)) break;
        {
          // pacing: a wave still waiting for more than four nodes' rows is
          // several levels from ready; it sleeps about 1.7 us (64 x 64
          // clocks) between its rounds, which leaves the memory system to the waves
          // near the front (measured at 100^3: forward 1.60 -> 1.51 ms,
          // backward with r^T z 1.54 -> 1.48 ms; shorter sleeps or a lower
          // threshold gained less, longer ones lost)
          int np = 0;
#pragma unroll
          for (int k = 0; k < QD; ++k) np += __popcll(__ballot(any_pending<TA, CPL>(xb[k])));
          if (np > 12 * LPR) __builtin_amdgcn_s_sleep(64);
        }
        const bool late = wall_clock64() - t0w > limit;
        static_for<QD>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          if (any_pending<TA, CPL>(xb[k])) {
            if (late) {
              __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
              for (int cc = 0; cc < CPL; ++cc)
                if (xb[k][cc] == Flag<TA>::kPending) xb[k][cc] = Flag<TA>::kCanonNaN;
            } else {
              load_elems<TA, CPL>(out + (int64_t)jj[k] * R + c0, xb[k]);
            }
          }
        });
      }
    }
    for (; !kBC;) {
      bool pend = false;
      int pk = 0;
#pragma unroll
      for (int k = QD - 1; k >= 0; --k)
        if (any_pending<TA, CPL>(xb[k])) { pend = true; pk = k; }
      const unsigned long long mask = __ballot(pend);
      if (!mask) break;
      const int leader = 63 - __clzll(mask);  // the nearest rows sit last
      const int pslot = __shfl(slot, leader, ICPCG_WAVE);
      const int pkk = __shfl(pk, leader, ICPCG_WAVE);
      int jp = 0;
      if constexpr (kBCJ) {
        jp = __shfl(jown, pslot * LPR + pkk, ICPCG_WAVE);  // every lane active here
      } else {
#pragma unroll
        for (int k = 0; k < QD; ++k)
          if (k == pkk) jp = jj[k];
      }
      if (slot == pslot) {
        const TA *p = out + (int64_t)jp * R + c0;
        U v[CPL];
        load_elems<TA, CPL>(p, v);
        const long long t0 = wall_clock64();
        int backoff = 1;
        while (__ballot(any_pending<TA, CPL>(v)) & (kRowMask << (pslot * LPR))) {
          for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(1);
          if (backoff < 4) backoff <<= 1;
          if (any_pending<TA, CPL>(v)) load_elems<TA, CPL>(p, v);
          if (wall_clock64() - t0 > limit && any_pending<TA, CPL>(v)) {
            __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc)
              if (v[cc] == Flag<TA>::kPending) v[cc] = Flag<TA>::kCanonNaN;
          }
        }
#pragma unroll
        for (int k = 0; k < QD; ++k)
          if (k == pkk) {
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc) xb[k][cc] = v[cc];
          }
      }
      static_for<QD>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        int jk;
        if constexpr (kBCJ) jk = row_bcast<k>(jown);
        else jk = jj[k];
        if (any_pending<TA, CPL>(xb[k])) load_elems<TA, CPL>(out + (int64_t)jk * R + c0, xb[k]);
      });
    }
    TA acc[kSmax][CPL];
#pragma unroll
    for (int u = 0; u < kSmax; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[u][cc] = TA(0);
    if constexpr (kBCV) {
      // entries past the row gathered x = 0 and their (clamped) factor values
      // are finite, so their products are exactly 0: no branch
      TA vwn[kSmax];
#pragma unroll
      for (int u = 0; u < kSmax; ++u) vwn[u] = widen<TA>(vown[u]);
      static_for<QD>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const TA x = bitcast<TA>(xb[k][0]);
#pragma unroll
        for (int u = 0; u < kSmax; ++u) acc[u][0] += row_bcast<k>(vwn[u]) * x;
      });
    } else {
#pragma unroll
      for (int k = 0; k < QD; ++k) {
        const int q = slot + k * SLOTS;
        if (q < m) {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) {
            const TA x = bitcast<TA>(xb[k][cc]);
#pragma unroll
            for (int u = 0; u < kSmax; ++u) acc[u][cc] += fval(k, u) * x;
          }
        }
      }
    }
    // rows longer than the prefetch window
    for (int q = slot + QD * SLOTS; q < m; q += SLOTS) {
      const int64_t jr = (int64_t)ci[pcol + q] * R + c0;
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const TA x = wait_value<TA>(out + jr + cc, err, limit);
#pragma unroll
        for (int u = 0; u < kSmax; ++u)
          if (u < sz) acc[u][cc] += widen<TA>(val[UPPER ? ro[u] + (sz - u) + q : ro[u] + q]) * x;
      }
    }
#pragma unroll
    for (int u = 0; u < kSmax; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[u][cc] = xor_sum_hi<Log2<LPR>::v>(acc[u][cc]);
    if (slot == 0) {
      TA xs[kSmax][CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        if (!UPPER) {
#pragma unroll
          for (int u = 0; u < kSmax; ++u) {
            if (u < sz) {
              TA sum = bval(u, cc) - acc[u][cc];
#pragma unroll
              for (int w = 0; w < u; ++w) sum -= dval(u * (u + 1) / 2 + w) * xs[w][cc];
              xs[u][cc] = sum / dval(u * (u + 1) / 2 + u);
            }
          }
        } else {
#pragma unroll
          for (int uu = kSmax - 1; uu >= 0; --uu) {
            if (uu < sz) {
              const int base = uu * kSmax - uu * (uu - 1) / 2;  // (uu, uu) in the upper storage
              TA sum = bval(uu, cc) - acc[uu][cc];
#pragma unroll
              for (int w = uu + 1; w < kSmax; ++w)
                if (w < sz) sum -= dval(base + (w - uu)) * xs[w][cc];
              xs[uu][cc] = sum / dval(base);
            }
          }
        }
      }
      // one contiguous row of R values per store instruction
#pragma unroll
      for (int u = 0; u < kSmax; ++u)
        if (u < sz) publish_elems<TA, CPL>(out + (int64_t)(a + u) * R + c0, xs[u]);
      if constexpr (RZ) {
#pragma unroll
        for (int u = 0; u < kSmax; ++u)
          if (u < sz) {
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc) dot[cc] += rr[u][cc] * (double)xs[u][cc];
          }
        // the right-hand side rows were read once, by this item: re-armed as
        // pending for the next step's forward solve, which writes them
        if (rhs_rearm) {
#pragma unroll
          for (int u = 0; u < kSmax; ++u)
            if (u < sz) {
#pragma unroll
              for (int cc = 0; cc < CPL; ++cc) rhs_rearm[(int64_t)(a + u) * R + c0 + cc] = Flag<TR>::kPending;
            }
        }
      }
      if constexpr (XR) {
        if (upx[0]) {
#pragma unroll
          for (int u = 0; u < kSmax; ++u)
            if (u < sz) {
              xr.r[(int64_t)(a + u) * R + c0] = br[u][0];
              dot[0] += br[u][0] * br[u][0];
            }
        }
      }
    }
    if constexpr (XR) {
      if (upx[0] && slot >= 1 && slot <= kSmax && slot - 1 < sz) xr.X[(int64_t)(a + slot - 1) * R + c0] = xn;
    }
  }
  if constexpr (RZ || XR) {
    __shared__ double smem[CPL * kRedBlock];
    block_partials_cpl<R, CPL>(dot, rz_partials, smem);
  }
}

// Waves the solve keeps resident (the static round-robin needs the whole grid
// resident): all that fit, at most `cap` per CU where the kernel has a
// measured best (cap > 0), or the number ICPCG_TRSV_WAVES_PER_CU asks.
template <typename K>
int64_t resident_blocks(K kernel, const Device &dev, int &cached, int cap = 0) {
  if (cached <= 0) {
    int q = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, kernel, kBlock, 0) != hipSuccess || q < 1) {
      (void)hipGetLastError();
      q = 1;
    }
    cached = q;
  }
  int per_cu = cached;
  if (dev.trsv_waves_per_cu > 0) cap = dev.trsv_waves_per_cu;
  if (cap > 0) {
    const int want = (cap + 3) / 4;
    if (want < per_cu) per_cu = want;
  }
  return (int64_t)per_cu * dev.num_cu;
}

// Columns per lane: two for FP64 solves from 8 columns up, which halves the
// prefetch arrays (3 instead of 2 resident waves per SIMD for this
// latency-bound kernel) while R / 2 lanes still cover a gathered row with one
// contiguous request; FP32 solves keep one (measured: the pair layout
// streams faster but lengthens each dependency hop more than it gains).
template <typename TA, int R> struct Cpl { static constexpr int v = (sizeof(TA) == 8 && R >= 8) ? 2 : 1; };
// Prefetch window (entries per lane) so that slots x depth >= 40 covers the 39
// shared off-block entries of a 3-DOF elasticity node; longer rows go
// through the (slower) remainder loop.
template <typename TA, int R> struct Depth {
  static constexpr int slots = 64 / (R / Cpl<TA, R>::v);
  static constexpr int v = (40 + slots - 1) / slots;
};

template <typename TV, typename TA, typename TR, int R, bool UPPER, bool RZ, bool XR>
int launch(const TriSchedule &S, const int32_t *ci, const TV *val, const TR *rhs, TA *out, hipStream_t s,
           const Device &dev, int *err, const int *active, const RzDot &rz, const XrUpd &xr) {
  if constexpr ((RZ || XR) && R == 1) {  // not fused at one column (trsv_fuses_rz, trsv_fuses_xr)
    return ICPCG_E_INVALID;
  } else {
  if (S.nsn == 0) return ICPCG_OK;
  auto k = k_trsv<TV, TA, TR, R, UPPER, Depth<TA, R>::v, Cpl<TA, R>::v, RZ, XR>;
  static int per_cu = 0;  // occupancy of this instantiation (same on every MI355X)
  // 16 columns in FP32 arithmetic: as many resident waves as about 2.8 levels
  // of supernodes, where that is fewer than fit (measured in the PCG step at
  // 100^3, 1464 supernodes per level: 16 waves per CU beat 8, 12 and all that
  // fit, 20 (forward solve with the x, r update 1.68 -> 1.63 ms, backward with
  // r^T z 1.49 -> 1.46 ms); at 150^3 and in the multicolour orders, with more
  // supernodes per level, fewer waves than fit were slower)
  int wave_cap = 0;
  if constexpr (R == 16 && sizeof(TA) == 4) {
    if (S.nlev > 0) {
      const double waves = 2.8 * (double)S.nsn / (double)S.nlev;
      const long blocks = std::lround(waves / (4.0 * dev.num_cu));
      wave_cap = 4 * (int)std::max(1L, std::min(blocks, 64L));
    }
  }
  int64_t grid = resident_blocks(k, dev, per_cu, wave_cap);
  const int64_t need = (S.nsn + 3) / 4;
  if (need < grid) grid = need;
  if (grid < 1) grid = 1;
  const int64_t cap = RZ ? rz.partials_cap : xr.partials_cap;
  if ((RZ || XR) && cap >= 0 && grid * R > cap) {
    set_error(std::string("trsv: the ") + (RZ ? "r^T z" : "||r||^2") + " partials of " + std::to_string(grid) +
              " blocks x " + std::to_string(R) + " columns exceed the " + std::to_string(cap) +
              " values of the given buffer");
    return ICPCG_E_INVALID;
  }
  const XrArgs xa{xr.X, xr.r, xr.p, xr.w, xr.cols};
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kBlock), 0, s, ci, val, S.items.as<SnItem>(), S.nsn, rhs, out,
                     err, dev.wait_ticks, active, rz.r, RZ ? rz.partials : xr.partials, xa,
                     RZ && rz.rearm_rhs ? reinterpret_cast<typename Flag<TR>::U *>(const_cast<TR *>(rhs)) : nullptr);
  ICPCG_HIP_TRY(hipGetLastError());
  if constexpr (RZ) {
    if (rz.out) return dot_finalize_out(R, rz.partials, (int)grid, rz.out, s);
    return pcg_rz_finalize(R, rz.partials, (int)grid, rz.cols, rz.flags, s);
  }
  if constexpr (XR) return pcg_rr_finalize(R, xr.partials, (int)grid, xr.cols, xr.max_iter, xr.flags, s);
  return ICPCG_OK;
  }
}

template <typename TV, typename TA, typename TR, bool UPPER, bool RZ = false, bool XR = false>
int dispatch_r(int R, const TriSchedule &S, const int32_t *ci, const TV *val, const TR *rhs, TA *out, hipStream_t s,
               const Device &dev, int *err, const int *active, const RzDot &rz = RzDot{},
               const XrUpd &xr = XrUpd{}) {
  switch (R) {
    case 1: return launch<TV, TA, TR, 1, UPPER, RZ, XR>(S, ci, val, rhs, out, s, dev, err, active, rz, xr);
    case 2: return launch<TV, TA, TR, 2, UPPER, RZ, XR>(S, ci, val, rhs, out, s, dev, err, active, rz, xr);
    case 4: return launch<TV, TA, TR, 4, UPPER, RZ, XR>(S, ci, val, rhs, out, s, dev, err, active, rz, xr);
    case 8: return launch<TV, TA, TR, 8, UPPER, RZ, XR>(S, ci, val, rhs, out, s, dev, err, active, rz, xr);
    case 16: return launch<TV, TA, TR, 16, UPPER, RZ, XR>(S, ci, val, rhs, out, s, dev, err, active, rz, xr);
    default:
      set_error("trsv: unsupported block width " + std::to_string(R));
      return ICPCG_E_INVALID;
  }
}

}  // namespace

// The fused r^T z costs registers: FP64 solves would lose resident waves
// (16 columns: 3 -> 2 per SIMD; one column: 7 -> 5) and one-column solves are
// bound by their dependency depth, so those keep the separate pass (about 10 us
// at one column), while FP32 arithmetic on 2-16 columns saves its pass over r
// and z (about 0.1 ms at 16 columns) at no cost in waves.
bool trsv_fuses_rz(const icpcg_prec *P, int R, const Device &dev) {
  return dev.fuse_rz && P->dtype != ICPCG_F64 && R > 1;
}

// The x, r update rides on the forward solve where the solve has registers to
// spare for its operands and is bound by its dependency chain, not by memory:
// FP32 arithmetic on 2-16 columns. Its separate pass streams x, r, p and w
// (48 bytes per entry, about 0.43 ms per step at 16 columns of 3.06M rows).
bool trsv_fuses_xr(const icpcg_prec *P, int R, const Device &dev) {
  return dev.fuse_xr && P->dtype != ICPCG_F64 && R > 1;
}

// `out` must hold the pending pattern in every entry on entry.
int trsv(const icpcg_prec *P, bool upper, const void *rhs, bool rhs_f64, void *out, int R, int64_t, hipStream_t s,
         const Device &dev, int *err, const int *active, const RzDot &rz, const XrUpd &xr) {
  const int32_t *ci = upper ? P->uci.as<int32_t>() : P->lci.as<int32_t>();
  const TriSchedule &S = upper ? P->su : P->sl;
  if (xr.X) {
    // the forward solve of a PCG step with the previous step's x, r update
    if (upper || !rhs_f64 || rz.partials || rhs != xr.r || !xr.r || !xr.p || !xr.w || !xr.cols || !xr.partials ||
        !xr.flags || !trsv_fuses_xr(P, R, dev)) {
      set_error("trsv: the x, r update only with the forward solve of a PCG step (FP32 or BF16 factor, 2-16 "
                "columns, right-hand side r)");
      return ICPCG_E_INVALID;
    }
    if (P->dtype == ICPCG_F32)
      return dispatch_r<float, float, double, false, false, true>(R, S, ci, P->lval_lo.as<float>(),
                                                                  (const double *)rhs, (float *)out, s, dev, err,
                                                                  active, RzDot{}, xr);
    return dispatch_r<unsigned short, float, double, false, false, true>(
        R, S, ci, P->lval_lo.as<unsigned short>(), (const double *)rhs, (float *)out, s, dev, err, active, RzDot{},
        xr);
  }
  if (rz.partials) {
    // the backward solve of a PCG step (right-hand side in the factor's precision)
    if (!upper || rhs_f64 || !trsv_fuses_rz(P, R, dev)) {
      set_error("trsv: r^T z only with the backward solve of a PCG step (FP32 or BF16 factor, 2-16 columns)");
      return ICPCG_E_INVALID;
    }
    if (P->dtype == ICPCG_F32)
      return dispatch_r<float, float, float, true, true>(R, S, ci, P->uval_lo.as<float>(), (const float *)rhs,
                                                         (float *)out, s, dev, err, active, rz);
    return dispatch_r<unsigned short, float, float, true, true>(R, S, ci, P->uval_lo.as<unsigned short>(),
                                                                (const float *)rhs, (float *)out, s, dev, err,
                                                                active, rz);
  }
  if (P->dtype == ICPCG_F64) {
    const double *v = upper ? P->uval.as<double>() : P->lval.as<double>();
    if (upper)
      return dispatch_r<double, double, double, true>(R, S, ci, v, (const double *)rhs, (double *)out, s, dev, err, active);
    return dispatch_r<double, double, double, false>(R, S, ci, v, (const double *)rhs, (double *)out, s, dev, err, active);
  }
  if (P->dtype == ICPCG_F32) {
    const float *v = upper ? P->uval_lo.as<float>() : P->lval_lo.as<float>();
    if (upper) {
      if (rhs_f64)
        return dispatch_r<float, float, double, true>(R, S, ci, v, (const double *)rhs, (float *)out, s, dev, err, active);
      return dispatch_r<float, float, float, true>(R, S, ci, v, (const float *)rhs, (float *)out, s, dev, err, active);
    }
    if (rhs_f64)
      return dispatch_r<float, float, double, false>(R, S, ci, v, (const double *)rhs, (float *)out, s, dev, err, active);
    return dispatch_r<float, float, float, false>(R, S, ci, v, (const float *)rhs, (float *)out, s, dev, err, active);
  }
  const unsigned short *v = upper ? P->uval_lo.as<unsigned short>() : P->lval_lo.as<unsigned short>();
  if (upper) {
    if (rhs_f64)
      return dispatch_r<unsigned short, float, double, true>(R, S, ci, v, (const double *)rhs, (float *)out, s, dev, err, active);
    return dispatch_r<unsigned short, float, float, true>(R, S, ci, v, (const float *)rhs, (float *)out, s, dev, err, active);
  }
  if (rhs_f64)
    return dispatch_r<unsigned short, float, double, false>(R, S, ci, v, (const double *)rhs, (float *)out, s, dev, err, active);
  return dispatch_r<unsigned short, float, float, false>(R, S, ci, v, (const float *)rhs, (float *)out, s, dev, err, active);
}

}  // namespace icpcg
