// CSR sparse matrix times an R-column block, FP64 (w = A p of supplementary
// Algorithm 1), with an optional fused p^T w reduction (deterministic block
// partials; a one-block finalize kernel computes alpha = r^T z / p^T w). The
// fused dot takes p of each row from the x gathered for its diagonal column
// (passed through LDS), so it adds no load after the row's sum.
//
// Mapping (wave64): a group of SLOTS * R / CPL lanes owns one row (one row
// group in the grouped kernel); a lane owns CPL consecutive columns (min(R, 4)
// in the plain kernel, min(R, 8) in the grouped one) and strides over the
// row's entries slot, slot + SLOTS, ... Each lane first loads the indices and values of up
// to QD of its entries, then issues all their x gathers (each one contiguous
// piece of a row of the row-major block), so every wave keeps many loads in
// flight. Partial sums meet in a fixed butterfly. Each block owns a
// contiguous row range; block ids are remapped so that each XCD works on one
// contiguous part of the matrix and its L2 serves the neighbouring gathers.
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
    int jj[QD];
    double vv[QD];
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int64_t q = s + slot + k * SLOTS;
      jj[k] = q < e ? ci[q] : 0;
      vv[k] = q < e ? v[q] : 0.0;
    }
    double acc[CPL];
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) acc[cc] = 0.0;
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int64_t q = s + slot + k * SLOTS;
      if (q < e) {
        const double *xr = x + (int64_t)jj[k] * R + c0;
        double xv[CPL];
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) xv[cc] = xr[cc];
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) acc[cc] += vv[k] * xv[cc];
        if (DOT && jj[k] == row) {
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
// one iteration ahead, so a group costs two dependent trips (indices, then x).
template <int SLOTS> struct GrpDepth {
  static constexpr int v = (88 + SLOTS - 1) / SLOTS > 11 ? 11 : (88 + SLOTS - 1) / SLOTS;
};

// At least three waves per SIMD (at most 168 VGPRs): the 16-column variant
// with the fused dot would otherwise settle a few registers above it.
template <int R, int SLOTS, bool DOT, int CPL, int QD = GrpDepth<SLOTS>::v>
__global__ __launch_bounds__(kBlock, 3) void k_spmv_grp(const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                     int64_t ngroups, const SpGroup *__restrict__ grec,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     int64_t chunk, double *partials,
                                                     const int *__restrict__ active) {
  if (DOT && active && *active == 0) return;
  constexpr int GMAX = kSupernodeMax;
  constexpr int LPR = R / CPL;
  constexpr int GROUP = SLOTS * LPR;
  static_assert(GROUP <= 64 && 64 % GROUP == 0, "group must tile a wave");
  constexpr int GPB = kBlock / GROUP;
  const int t = threadIdx.x;
  const int g = t / GROUP, lg = t % GROUP, slot = lg / LPR, c0 = (lg % LPR) * CPL;
  __shared__ double pdiag[DOT ? GPB * GMAX * R : 1];  // per group: p of its rows, [u][column]
  double *pd = pdiag + (DOT ? g * GMAX * R : 0);
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t g0 = lb * chunk;
  const int64_t g1 = g0 + chunk < ngroups ? g0 + chunk : ngroups;
  double dot[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) dot[cc] = 0.0;
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
      jj[k] = q < m ? ci[base + q] : 0;
#pragma unroll
      for (int u = 0; u < GMAX; ++u)
        vv[k][u] = (q < m && u < sz) ? v[base + u * m + q] : 0.0;
    }
    double acc[GMAX][CPL];
#pragma unroll
    for (int u = 0; u < GMAX; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[u][cc] = 0.0;
    // for the fused p^T w: the group's rows are among its shared columns, so
    // p of row r0 + u is the x gathered for that column; the lane that
    // gathers it leaves it in the group's LDS table (read back after the
    // butterfly by the lanes that write w; one wave, so LDS order suffices)
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int64_t q = slot + k * SLOTS;
      if (q < m) {
        const double *xr = x + (int64_t)jj[k] * R + c0;
        double xv[CPL];
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) xv[cc] = xr[cc];
#pragma unroll
        for (int u = 0; u < GMAX; ++u)
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) acc[u][cc] += vv[k][u] * xv[cc];
        if (DOT && jj[k] >= r0 && jj[k] < r0 + sz) {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) pd[(jj[k] - r0) * R + c0 + cc] = xv[cc];
        }
      }
    }
    for (int64_t q = slot + QD * SLOTS; q < m; q += SLOTS) {
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
      if (DOT && j >= r0 && j < r0 + sz) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) pd[(j - r0) * R + c0 + cc] = xv[cc];
      }
    }
#pragma unroll
    for (int u = 0; u < GMAX; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[u][cc] = xor_sum_bits<Log2<LPR>::v, Log2<GROUP>::v>(acc[u][cc]);
    if (slot == 0) {
#pragma unroll
      for (int u = 0; u < GMAX; ++u) {
        if (u < sz) {
          const int64_t row = r0 + u;
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) {
            y[row * R + c0 + cc] = acc[u][cc];
            if (DOT) dot[cc] += pd[u * R + c0 + cc] * acc[u][cc];
          }
        }
      }
    }
  }
  if (DOT) {
    __shared__ double smem[CPL * kRedBlock];
    block_partials_cpl<R, CPL>(dot, partials, smem);
  }
}

template <int R, int SLOTS, int CPL>
int launch_grp(const int32_t *ci, const double *v, int64_t ngroups, const SpGroup *grec, const double *x, double *y,
               hipStream_t s, double *partials, ColState *cols, const int *active) {
  constexpr int GPB = kBlock / (SLOTS * (R / CPL));
  // Short chunks keep the groups in flight on one XCD close together, so its
  // L2 serves more of the neighbouring x gathers (measured best per width);
  // the fused p^T w partials bound the block count.
  static const int iters_env = std::getenv("ICPCG_SPMVG_ITERS") ? std::atoi(std::getenv("ICPCG_SPMVG_ITERS")) : 0;
  const int ITERS = iters_env > 0 ? iters_env : (R >= 16 ? 16 : R >= 8 ? 8 : R >= 4 ? 2 : 1);
  int64_t nb = (ngroups + GPB * ITERS - 1) / (GPB * ITERS);
  if (partials && nb > kMaxDotBlocks) nb = kMaxDotBlocks;
  if (nb < 1) nb = 1;
  const int64_t chunk = (ngroups + nb - 1) / nb;
  nb = (ngroups + chunk - 1) / chunk;
  if (nb < 1) nb = 1;
  if (partials) {
    hipLaunchKernelGGL((k_spmv_grp<R, SLOTS, true, CPL>), dim3((unsigned)nb), dim3(kBlock), 0, s, ci, v, ngroups, grec, x,
                       y, chunk, partials, active);
    ICPCG_HIP_TRY(hipGetLastError());
    return pcg_pw_finalize(R, partials, (int)nb, cols, reinterpret_cast<const SolveFlags *>(active), s);
  }
  hipLaunchKernelGGL((k_spmv_grp<R, SLOTS, false, CPL>), dim3((unsigned)nb), dim3(kBlock), 0, s, ci, v, ngroups, grec, x,
                     y, chunk, nullptr, nullptr);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
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

int spmv_grouped(const int32_t *ci, const double *v, int64_t ngroups, const SpGroup *grec, const double *x,
                 double *y, int R, int slots, hipStream_t s, double *partials, ColState *cols, const int *active) {
  if (ngroups <= 0) return ICPCG_OK;
// a lane owns min(R, 8) columns: fewer lanes per row means fewer redundant
// index and value loads and a shorter butterfly, which outweighs the wider
// per-lane gathers
#define ICPCG_SPMVG_CASE(RR, SS) \
  if (R == RR && slots == SS) \
    return launch_grp<RR, SS, (RR < 8 ? RR : 8)>(ci, v, ngroups, grec, x, y, s, partials, cols, active);
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
