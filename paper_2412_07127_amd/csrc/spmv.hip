// CSR sparse matrix times an R-column block, FP64 (w = A p of supplementary
// Algorithm 1), with p^T w for alpha = r^T z / p^T w when the solver asks
// (deterministic block partials, folded by a one-block finalize kernel). The
// plain kernel fuses that dot, taking p of each row from the x gathered for
// its diagonal column (passed through LDS); the row-group kernel leaves it to
// one pass over p and w.
//
// Mapping (wave64): a group of SLOTS * R / CPL lanes owns one row (one row
// group in the grouped kernel); a lane owns CPL consecutive columns (min(R, 4)
// in the plain kernel, min(R, 8) in the grouped one) and strides over the
// row's entries slot, slot + SLOTS, ... Each lane first loads the indices and
// values of up to QD of its entries, with no load behind a branch, then
// issues their x gathers (each one contiguous piece of a row of the row-major
// block), so every wave keeps many loads in flight. Partial sums meet in a
// fixed butterfly. Each block owns a contiguous row range; block ids are
// remapped so that each XCD works on one contiguous part of the matrix and its
// L2 serves the neighbouring gathers.
#include <cstdlib>

#include "reduce.hpp"

namespace icpcg {

namespace {

constexpr int kBlock = 256;

template <int LO, int HI, typename T>
__device__ __forceinline__ T xor_sum_bits(T v) {
#pragma unroll
  for (int b = 1 << (HI - 1); b >= (1 << LO); b >>= 1) v += __shfl_xor(v, b, ICPCG_WAVE);
  return v;
}

// The same butterfly over lane bits LO..HI-1 (highest first) applied to NV
// values at once, exchanging only what is still needed: while the count held
// is even and at least 2 * MIN, the lane with the bit clear keeps the lower
// half and its partner the upper half, each sending the other the half it
// gives up; the remaining rounds exchange all that is left. Each sum is
// formed by the same pairwise additions as xor_sum_bits applied to every
// value, so the results are bit-identical to it, at about a third of the
// exchanges for 24 values over 16 lanes. Afterwards a[0 .. held) holds the
// values first .. first + held of the lanes' common sums, where first is
// returned and held and the lane bits of the full rounds are given by RsPlan.
template <int LO, int HI, int NV, int MIN> struct RsPlan {
  static constexpr bool halves(int k) { return k % 2 == 0 && k >= 2 * MIN; }
  static constexpr int held() {
    int k = NV;
    for (int b = HI - 1; b >= LO; --b)
      if (halves(k)) k /= 2;
    return k;
  }
  static constexpr int full_bits() {
    int k = NV, m = 0;
    for (int b = HI - 1; b >= LO; --b) {
      if (halves(k))
        k /= 2;
      else
        m |= 1 << b;
    }
    return m;
  }
};

template <int LO, int B, int K, int NV, int MIN>
__device__ __forceinline__ int xor_reduce_scatter(double (&a)[NV], int lane, int first) {
  if constexpr (B < LO) {
    return first;
  } else {
    constexpr int bit = 1 << B;
    if constexpr (RsPlan<LO, B + 1, NV, MIN>::halves(K)) {
      constexpr int H = K / 2;
      const bool up = (lane & bit) != 0;
      // all exchanges of the round are issued before the first sum waits
      double got[H];
#pragma unroll
      for (int j = 0; j < H; ++j) got[j] = __shfl_xor(up ? a[j] : a[j + H], bit, ICPCG_WAVE);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < H; ++j) a[j] = (up ? a[j + H] : a[j]) + got[j];
      return xor_reduce_scatter<LO, B - 1, H, NV, MIN>(a, lane, first + (up ? H : 0));
    } else {
      double got[K];
#pragma unroll
      for (int j = 0; j < K; ++j) got[j] = __shfl_xor(a[j], bit, ICPCG_WAVE);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < K; ++j) a[j] += got[j];
      return xor_reduce_scatter<LO, B - 1, K, NV, MIN>(a, lane, first);
    }
  }
}

template <int SLOTS> struct SpmvDepth { static constexpr int v = 128 / SLOTS > 8 ? 8 : 128 / SLOTS; };

template <int R, int SLOTS, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const double *__restrict__ v, int64_t n,
                                                 const double *__restrict__ x, double *__restrict__ y,
                                                 int64_t chunk, double *partials, const int *__restrict__ active) {
  if (DOT && active && *active == 0) return;
  constexpr int CPL = R >= 4 ? 4 : R;
  constexpr int LPR = R / CPL;
  constexpr int GROUP = SLOTS * LPR;
  static_assert(GROUP <= 64 && 64 % GROUP == 0, "group must tile a wave");
  constexpr int GPB = kBlock / GROUP;
  constexpr int QD = SpmvDepth<SLOTS>::v;
  const int t = threadIdx.x;
  const int g = t / GROUP, lg = t % GROUP, slot = lg / LPR, c0 = (lg % LPR) * CPL;
  (void)t;
  // for the fused p^T w: p of the row is the x gathered for its diagonal (every
  // row stores it); the lane that gathers it leaves it in the group's LDS slot
  __shared__ double pdiag[DOT ? GPB * R : 1];
  double *pd = pdiag + (DOT ? g * R : 0);
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t r0 = lb * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  double dot[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) dot[cc] = 0.0;
  for (int64_t row = r0 + g; row < r1; row += GPB) {
    const int64_t s = rp[row], e = rp[row + 1];
    double acc[CPL];
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) acc[cc] = 0.0;
    if (e > s) {  // an empty row sums to zero
      // no load behind a per-entry branch (see the grouped kernel): a slot
      // past the row's end reloads the row's last entry with its value scaled
      // by 0 (a non-finite value or x there makes the row non-finite either way)
      int jj[QD];
      bool ok[QD];
      double vv[QD];
#pragma unroll
      for (int k = 0; k < QD; ++k) {
        const int64_t q = s + slot + k * SLOTS;
        ok[k] = q < e;
        const int64_t qc = ok[k] ? q : e - 1;
        jj[k] = ci[qc];
        vv[k] = v[qc] * (ok[k] ? 1.0 : 0.0);
      }
#pragma unroll
      for (int k = 0; k < QD; ++k) {
        const double *xr = x + (int64_t)jj[k] * R + c0;
        double xv[CPL];
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) xv[cc] = xr[cc];
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) acc[cc] += vv[k] * xv[cc];
        if (DOT && ok[k] && jj[k] == row) {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) pd[c0 + cc] = xv[cc];
        }
      }
    }
    for (int64_t q = s + slot + QD * SLOTS; q < e; q += SLOTS) {
      const int32_t j = ci[q];
      const double *xr = x + (int64_t)j * R + c0;
      const double vq = v[q];
      double xv[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) xv[cc] = xr[cc];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[cc] += vq * xv[cc];
      if (DOT && j == row) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) pd[c0 + cc] = xv[cc];
      }
    }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) acc[cc] = xor_sum_bits<Log2<LPR>::v, Log2<GROUP>::v>(acc[cc]);
    if (slot == 0) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        y[row * R + c0 + cc] = acc[cc];
        if (DOT) dot[cc] += pd[c0 + cc] * acc[cc];
      }
    }
  }
  if (DOT) {
    __shared__ double smem[CPL * kRedBlock];
    block_partials_cpl<R, CPL>(dot, partials, smem);
  }
}

// Row-group variant: a lane group owns up to GMAX consecutive rows with
// identical column lists (the rows of one node), reads each column index once
// and gathers each x row once for all of them. Each group's record is loaded
// one iteration ahead. The load order is fixed in the source, not left to the
// compiler: all index and value loads of a lane's QD entries first, then the
// x gathers in batches of KB entries, each batch issued whole before its
// products (scheduling barriers), so a group costs about one trip for the
// indices and one per batch. No load sits behind a branch, since the compiler
// waits for such a load (or one whose result is selected) at the join: a slot
// past the group's columns reloads its last column with its value scaled by
// 0. Every group has a column and finite values (each row stores its
// diagonal, checked when the matrix handle is made), and that column is one
// of the group's own, so a non-finite x there makes the rows non-finite
// either way. The solver's p^T w is a separate pass over p and w (below):
// keeping p of each row for it inside this kernel costs more registers than
// the pass costs time.
template <int SLOTS> struct GrpDepth {
  static constexpr int v = (88 + SLOTS - 1) / SLOTS > 11 ? 11 : (88 + SLOTS - 1) / SLOTS;
};

// At least three waves per SIMD (at most 168 VGPRs). NT: A's values are
// loaded nontemporal, so the stream of A (read once) does not push the x rows
// out of the L2 between their gathers.
template <int R, int SLOTS, int CPL, bool NT, int QD = GrpDepth<SLOTS>::v>
__global__ __launch_bounds__(kBlock, 3) void k_spmv_grp(const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                     int64_t ngroups, const SpGroup *__restrict__ grec,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     int64_t chunk, const int *__restrict__ active) {
  if (active && *active == 0) return;
  constexpr int GMAX = kSupernodeMax;
  constexpr int LPR = R / CPL;
  constexpr int GROUP = SLOTS * LPR;
  static_assert(GROUP <= 64 && 64 % GROUP == 0, "group must tile a wave");
  constexpr int GPB = kBlock / GROUP;
  // entries per gather batch: about 48 registers of x in flight per lane
  constexpr int KB = 24 / CPL > QD ? QD : 24 / CPL;
  const int t = threadIdx.x;
  const int g = t / GROUP, lg = t % GROUP, slot = lg / LPR, c0 = (lg % LPR) * CPL;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t g0 = lb * chunk;
  const int64_t g1 = g0 + chunk < ngroups ? g0 + chunk : ngroups;
  SpGroup nxt{};
  if (g0 + g < g1) nxt = grec[g0 + g];
  for (int64_t gi = g0 + g; gi < g1; gi += GPB) {
    const SpGroup G = nxt;
    if (gi + GPB < g1) nxt = grec[gi + GPB];
    const int64_t r0 = G.r0;
    const int sz = G.m_sz & 7;
    const int64_t base = G.base;
    const int64_t m = G.m_sz >> 3;
    int jj[QD];
    double vv[QD][GMAX];
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int64_t q = slot + k * SLOTS;
      const bool ok = q < m;
      const int64_t qc = ok ? q : m - 1;
      const double keep = ok ? 1.0 : 0.0;
      jj[k] = ci[base + qc];
#pragma unroll
      for (int u = 0; u < GMAX; ++u)  // rows >= sz: unused
        vv[k][u] = (NT ? __builtin_nontemporal_load(v + base + (u < sz ? u : sz - 1) * m + qc)
                       : v[base + (u < sz ? u : sz - 1) * m + qc]) * keep;
    }
    __builtin_amdgcn_sched_barrier(0);
    double acc[GMAX][CPL];
#pragma unroll
    for (int u = 0; u < GMAX; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[u][cc] = 0.0;
#pragma unroll
    for (int k0 = 0; k0 < QD; k0 += KB) {
      double xv[KB][CPL];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (k0 + kk < QD) {
          const double *xr = x + (int64_t)jj[k0 + kk] * R + c0;
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) xv[kk][cc] = xr[cc];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (k0 + kk < QD) {
#pragma unroll
          for (int u = 0; u < GMAX; ++u)
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc) acc[u][cc] += vv[k0 + kk][u] * xv[kk][cc];
        }
      }
    }
    // rows longer than the window (rare). The start is made opaque so that the
    // compiler keeps its addresses in the loop: hoisted out of the group loop
    // they outlive the registers and spill at every thread's start, which at
    // one group pass per block writes more than the kernel's output.
    int64_t qs = slot + QD * SLOTS;
    asm volatile("" : "+v"(qs));
    for (int64_t q = qs; q < m; q += SLOTS) {
      const int32_t j = ci[base + q];
      const double *xr = x + (int64_t)j * R + c0;
      double xv[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) xv[cc] = xr[cc];
#pragma unroll
      for (int u = 0; u < GMAX; ++u) {
        const double vq = u < sz ? v[base + u * m + q] : 0.0;
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) acc[u][cc] += vq * xv[cc];
      }
    }
    // sum over the slots. Value i of a lane is column c0 + i / GMAX of row
    // i % GMAX; a lane ends with whole pairs of columns, stored 16 bytes a row.
    constexpr int LO = Log2<LPR>::v, HI = Log2<GROUP>::v, NV = GMAX * CPL;
    constexpr int CH = CPL >= 2 ? 2 : 1;  // columns a lane ends with
    using Plan = RsPlan<LO, HI, NV, CH * GMAX>;
    static_assert(Plan::held() == CH * GMAX, "a lane ends with CH columns of every row");
    double a[NV];
#pragma unroll
    for (int u = 0; u < GMAX; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) a[cc * GMAX + u] = acc[u][cc];
    // the lane's position is made opaque here so that the store offsets
    // derived from it are formed per group: hoisted out of the group loop they
    // outlive the registers and spill
    int lgv = lg;
    asm volatile("" : "+v"(lgv));
    const int first = xor_reduce_scatter<LO, HI - 1, NV, NV, CH * GMAX>(a, lgv, 0);
    if ((lgv & Plan::full_bits()) == 0) {
      double *yr = y + r0 * R + c0 + first / GMAX;
#pragma unroll
      for (int u = 0; u < GMAX; ++u) {
        if (u < sz) {
          if constexpr (CH == 2)
            *reinterpret_cast<double2 *>(yr + u * R) = make_double2(a[u], a[GMAX + u]);
          else
            yr[u * R] = a[u];
        }
      }
    }
  }
}

template <int R, int SLOTS, int CPL>
int launch_grp(const int32_t *ci, const double *v, int64_t ngroups, const SpGroup *grec, int64_t n, const double *x,
               double *y, hipStream_t s, double *partials, ColState *cols, const int *active) {
  constexpr int GPB = kBlock / (SLOTS * (R / CPL));
  // Short chunks keep the groups in flight on one XCD close together, so its
  // L2 serves more of the neighbouring x gathers (measured best per width).
  // At 16 columns: one pass per block with A's values nontemporal (100^3,
  // counters: 3.76 GB moved per launch against 7.29 GB with 16 passes and A
  // cached, 1.30 against 1.33 ms; one pass with A cached moves 3.58 GB but
  // takes 1.53 ms).
  static const int iters_env = std::getenv("ICPCG_SPMVG_ITERS") ? std::atoi(std::getenv("ICPCG_SPMVG_ITERS")) : 0;
  constexpr bool NT = R >= 16;
  const int ITERS = iters_env > 0 ? iters_env : (R >= 16 ? 1 : R >= 8 ? 8 : R >= 4 ? 2 : 1);
  int64_t nb = (ngroups + GPB * ITERS - 1) / (GPB * ITERS);
  if (nb < 1) nb = 1;
  const int64_t chunk = (ngroups + nb - 1) / nb;
  nb = (ngroups + chunk - 1) / chunk;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_spmv_grp<R, SLOTS, CPL, NT>), dim3((unsigned)nb), dim3(kBlock), 0, s, ci, v, ngroups, grec, x,
                     y, chunk, active);
  ICPCG_HIP_TRY(hipGetLastError());
  if (!partials) return ICPCG_OK;
  // p^T w for alpha: one deterministic pass over p = x and w = y
  return pcg_dot_pw(n, R, x, y, partials, cols, reinterpret_cast<const SolveFlags *>(active), s);
}

template <int R, int SLOTS>
int launch(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x, double *y,
           hipStream_t s, double *partials, ColState *cols, const int *active) {
  constexpr int CPL = R >= 4 ? 4 : R;
  constexpr int GPB = kBlock / (SLOTS * (R / CPL));
  // about 8 row passes per block, at most 4096 blocks (bounded partials)
  int64_t nb = (n + GPB * 8 - 1) / (GPB * 8);
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  const int64_t chunk = (n + nb - 1) / nb;
  nb = (n + chunk - 1) / chunk;
  if (nb < 1) nb = 1;
  if (partials) {
    hipLaunchKernelGGL((k_spmv<R, SLOTS, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, rp, ci, v, n, x, y, chunk,
                       partials, active);
    ICPCG_HIP_TRY(hipGetLastError());
    return pcg_pw_finalize(R, partials, (int)nb, cols, reinterpret_cast<const SolveFlags *>(active), s);
  }
  hipLaunchKernelGGL((k_spmv<R, SLOTS, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, rp, ci, v, n, x, y, chunk,
                     nullptr, nullptr);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace

// slots: entry slots per row (the lanes per row are slots * R / min(R, 4)).
int spmv(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x, double *y, int R,
         int slots, hipStream_t s, double *partials, ColState *cols, const int *active) {
  if (n <= 0) return ICPCG_OK;
#define ICPCG_SPMV_CASE(RR, SS) \
  if (R == RR && slots == SS) return launch<RR, SS>(rp, ci, v, n, x, y, s, partials, cols, active);
  ICPCG_SPMV_CASE(1, 8)
  ICPCG_SPMV_CASE(1, 16)
  ICPCG_SPMV_CASE(1, 32)
  ICPCG_SPMV_CASE(2, 8)
  ICPCG_SPMV_CASE(2, 16)
  ICPCG_SPMV_CASE(2, 32)
  ICPCG_SPMV_CASE(4, 8)
  ICPCG_SPMV_CASE(4, 16)
  ICPCG_SPMV_CASE(4, 32)
  ICPCG_SPMV_CASE(8, 8)
  ICPCG_SPMV_CASE(8, 16)
  ICPCG_SPMV_CASE(8, 32)
  ICPCG_SPMV_CASE(16, 4)
  ICPCG_SPMV_CASE(16, 8)
  ICPCG_SPMV_CASE(16, 16)
#undef ICPCG_SPMV_CASE
  set_error("spmv: unsupported (R, slots) = (" + std::to_string(R) + ", " + std::to_string(slots) + ")");
  return ICPCG_E_INVALID;
}

int spmv_grouped(const int32_t *ci, const double *v, int64_t ngroups, const SpGroup *grec, int64_t n,
                 const double *x, double *y, int R, int slots, hipStream_t s, double *partials, ColState *cols,
                 const int *active) {
  if (ngroups <= 0) return ICPCG_OK;
// a lane owns min(R, 8) columns: fewer lanes per row means fewer redundant
// index and value loads and a shorter butterfly, which outweighs the wider
// per-lane gathers
#define ICPCG_SPMVG_CASE(RR, SS) \
  if (R == RR && slots == SS) \
    return launch_grp<RR, SS, (RR < 8 ? RR : 8)>(ci, v, ngroups, grec, n, x, y, s, partials, cols, active);
  ICPCG_SPMVG_CASE(1, 16)
  ICPCG_SPMVG_CASE(1, 32)
  ICPCG_SPMVG_CASE(2, 16)
  ICPCG_SPMVG_CASE(2, 32)
  ICPCG_SPMVG_CASE(4, 16)
  ICPCG_SPMVG_CASE(4, 32)
  ICPCG_SPMVG_CASE(8, 16)
  ICPCG_SPMVG_CASE(8, 32)
  ICPCG_SPMVG_CASE(16, 16)
  ICPCG_SPMVG_CASE(16, 32)
#undef ICPCG_SPMVG_CASE
  set_error("grouped spmv: unsupported (R, slots) = (" + std::to_string(R) + ", " + std::to_string(slots) + ")");
  return ICPCG_E_INVALID;
}

int spmv_grouped_default_slots(int R) {
  if (const char *e = std::getenv("ICPCG_SPMVG_SLOTS")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  return R >= 8 ? 16 : 32;
}

int spmv_default_slots(int R) {
  if (const char *e = std::getenv("ICPCG_SPMV_SLOTS")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  (void)R;
  return 16;  // measured best at every width for rows of ~80 entries
}

}  // namespace icpcg
