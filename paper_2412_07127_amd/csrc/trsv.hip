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
//    reader spins on a device-scope load until the pattern is gone (the value
//    is its own flag, so no fences are needed). The smallest unfinished
//    position is always held by a running wave whose inputs are done, so the
//    co-resident grid always progresses; a wall-clock limit turns an
//    impossible wait into an error instead of a hang.
//  * Lanes of a wave are (slot, column): SLOTS = 64 / R lanes stride over the
//    off-block entries, R lanes cover the columns of one gathered row of the
//    row-major block (one contiguous load). Partial sums meet in a fixed
//    butterfly, so results are deterministic.
//  * Factor values may be FP64, FP32 or bfloat16 (widened to FP32); FP32 and
//    bfloat16 factors run FP32 arithmetic.
#include "internal.hpp"

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

template <typename TV, typename TA, typename TR, int R, bool UPPER>
__global__ __launch_bounds__(kBlock) void k_trsv(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const TV *__restrict__ val, const int32_t *__restrict__ sn_ptr,
                                                 const int32_t *__restrict__ sn_order, int64_t nsn,
                                                 const TR *__restrict__ rhs, TA *out, int *err,
                                                 long long limit) {
  constexpr int SLOTS = 64 / R;
  const int lane = threadIdx.x & 63, slot = lane / R, c = lane % R;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t t = w0; t < nsn; t += nw) {
    const int s = sn_order[t];
    const int a = sn_ptr[s];
    const int sz = sn_ptr[s + 1] - a;
    int64_t ro[kSmax + 1];
#pragma unroll
    for (int u = 0; u <= kSmax; ++u) ro[u] = u <= sz ? rp[a + u] : 0;
    // length of the shared off-block part and where its columns are listed
    const int m = UPPER ? (int)(ro[sz] - ro[sz - 1]) - 1 : (int)(ro[1] - ro[0]) - 1;
    const int64_t pcol = UPPER ? ro[sz - 1] + 1 : ro[0];
    TA acc[kSmax];
#pragma unroll
    for (int u = 0; u < kSmax; ++u) acc[u] = TA(0);
    for (int q = slot; q < m; q += SLOTS) {
      const int j = ci[pcol + q];
      const TA xj = wait_value<TA>(out + (int64_t)j * R + c, err, limit);
#pragma unroll
      for (int u = 0; u < kSmax; ++u) {
        if (u < sz) {
          const int64_t off = UPPER ? ro[u] + (sz - u) + q : ro[u] + q;
          acc[u] += widen<TA>(val[off]) * xj;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSmax; ++u) acc[u] = xor_sum_hi<Log2<R>::v>(acc[u]);
    if (slot == 0) {
      TA xs[kSmax];
      if (!UPPER) {
#pragma unroll
        for (int u = 0; u < kSmax; ++u) {
          if (u < sz) {
            const int64_t db = ro[u] + m;  // diagonal block of row a+u: columns a .. a+u
            TA sum = (TA)rhs[(int64_t)(a + u) * R + c] - acc[u];
#pragma unroll
            for (int w = 0; w < kSmax; ++w)
              if (w < u) sum -= widen<TA>(val[db + w]) * xs[w];
            xs[u] = sum / widen<TA>(val[db + u]);
          }
        }
      } else {
#pragma unroll
        for (int uu = kSmax - 1; uu >= 0; --uu) {
          if (uu < sz) {
            // row a+uu: diagonal first, then columns a+uu+1 .. a+sz-1
            TA sum = (TA)rhs[(int64_t)(a + uu) * R + c] - acc[uu];
#pragma unroll
            for (int w = 0; w < kSmax; ++w)
              if (w > uu && w < sz) sum -= widen<TA>(val[ro[uu] + (w - uu)]) * xs[w];
            xs[uu] = sum / widen<TA>(val[ro[uu]]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kSmax; ++u)
        if (u < sz) publish_value<TA>(out + (int64_t)(a + u) * R + c, xs[u]);
    }
  }
}

template <typename K>
int resident_blocks(K kernel, const Device &dev) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  return per_cu * dev.num_cu;
}

template <typename TV, typename TA, typename TR, int R, bool UPPER>
int launch(const TriSchedule &S, const int64_t *rp, const int32_t *ci, const TV *val, const TR *rhs, TA *out,
           hipStream_t s, const Device &dev, int *err) {
  if (S.nsn == 0) return ICPCG_OK;
  auto k = k_trsv<TV, TA, TR, R, UPPER>;
  int64_t grid = resident_blocks(k, dev);
  const int64_t need = (S.nsn + 3) / 4;
  if (need < grid) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kBlock), 0, s, rp, ci, val, S.sn_ptr.as<int32_t>(),
                     S.sn_order.as<int32_t>(), S.nsn, rhs, out, err, dev.wait_ticks);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

template <typename TV, typename TA, typename TR, bool UPPER>
int dispatch_r(int R, const TriSchedule &S, const int64_t *rp, const int32_t *ci, const TV *val, const TR *rhs,
               TA *out, hipStream_t s, const Device &dev, int *err) {
  switch (R) {
    case 1: return launch<TV, TA, TR, 1, UPPER>(S, rp, ci, val, rhs, out, s, dev, err);
    case 2: return launch<TV, TA, TR, 2, UPPER>(S, rp, ci, val, rhs, out, s, dev, err);
    case 4: return launch<TV, TA, TR, 4, UPPER>(S, rp, ci, val, rhs, out, s, dev, err);
    case 8: return launch<TV, TA, TR, 8, UPPER>(S, rp, ci, val, rhs, out, s, dev, err);
    case 16: return launch<TV, TA, TR, 16, UPPER>(S, rp, ci, val, rhs, out, s, dev, err);
    default:
      set_error("trsv: unsupported block width " + std::to_string(R));
      return ICPCG_E_INVALID;
  }
}

}  // namespace

// `out` must hold the pending pattern in every entry on entry.
int trsv(const icpcg_prec *P, bool upper, const void *rhs, bool rhs_f64, void *out, int R, int64_t, hipStream_t s,
         const Device &dev, int *err) {
  const int64_t *rp = upper ? P->urp.as<int64_t>() : P->lrp.as<int64_t>();
  const int32_t *ci = upper ? P->uci.as<int32_t>() : P->lci.as<int32_t>();
  const TriSchedule &S = upper ? P->su : P->sl;
  if (P->dtype == ICPCG_F64) {
    const double *v = upper ? P->uval.as<double>() : P->lval.as<double>();
    if (upper)
      return dispatch_r<double, double, double, true>(R, S, rp, ci, v, (const double *)rhs, (double *)out, s, dev, err);
    return dispatch_r<double, double, double, false>(R, S, rp, ci, v, (const double *)rhs, (double *)out, s, dev, err);
  }
  if (P->dtype == ICPCG_F32) {
    const float *v = upper ? P->uval_lo.as<float>() : P->lval_lo.as<float>();
    if (upper) {
      if (rhs_f64)
        return dispatch_r<float, float, double, true>(R, S, rp, ci, v, (const double *)rhs, (float *)out, s, dev, err);
      return dispatch_r<float, float, float, true>(R, S, rp, ci, v, (const float *)rhs, (float *)out, s, dev, err);
    }
    if (rhs_f64)
      return dispatch_r<float, float, double, false>(R, S, rp, ci, v, (const double *)rhs, (float *)out, s, dev, err);
    return dispatch_r<float, float, float, false>(R, S, rp, ci, v, (const float *)rhs, (float *)out, s, dev, err);
  }
  const unsigned short *v = upper ? P->uval_lo.as<unsigned short>() : P->lval_lo.as<unsigned short>();
  if (upper) {
    if (rhs_f64)
      return dispatch_r<unsigned short, float, double, true>(R, S, rp, ci, v, (const double *)rhs, (float *)out, s,
                                                             dev, err);
    return dispatch_r<unsigned short, float, float, true>(R, S, rp, ci, v, (const float *)rhs, (float *)out, s, dev,
                                                          err);
  }
  if (rhs_f64)
    return dispatch_r<unsigned short, float, double, false>(R, S, rp, ci, v, (const double *)rhs, (float *)out, s,
                                                            dev, err);
  return dispatch_r<unsigned short, float, float, false>(R, S, rp, ci, v, (const float *)rhs, (float *)out, s, dev,
                                                         err);
}

}  // namespace icpcg
