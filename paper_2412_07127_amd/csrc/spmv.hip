// CSR sparse matrix times an R-column block, FP64 (w = A p of supplementary
// Algorithm 1), with an optional fused, deterministic p^T w reduction that
// also computes alpha = r^T z / p^T w for the PCG columns.
//
// Mapping (wave64): a group of SLOTS * R / CPL lanes owns one row; a lane owns
// CPL = min(R, 4) consecutive columns and strides over the row's entries
// slot, slot + SLOTS, ... Each lane first loads the indices and values of up
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
                                                 int64_t chunk, double *partials, unsigned *counter,
                                                 ColState *cols) {
  constexpr int CPL = R >= 4 ? 4 : R;
  constexpr int LPR = R / CPL;
  constexpr int GROUP = SLOTS * LPR;
  static_assert(GROUP <= 64 && 64 % GROUP == 0, "group must tile a wave");
  constexpr int GPB = kBlock / GROUP;
  constexpr int QD = SpmvDepth<SLOTS>::v;
  const int t = threadIdx.x;
  const int g = t / GROUP, lg = t % GROUP, slot = lg / LPR, c0 = (lg % LPR) * CPL;
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
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) acc[cc] += vv[k] * xr[cc];
      }
    }
    for (int64_t q = s + slot + QD * SLOTS; q < e; q += SLOTS) {
      const double *xr = x + (int64_t)ci[q] * R + c0;
      const double vq = v[q];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[cc] += vq * xr[cc];
    }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) acc[cc] = xor_sum_bits<Log2<LPR>::v, Log2<GROUP>::v>(acc[cc]);
    if (slot == 0) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        y[row * R + c0 + cc] = acc[cc];
        if (DOT) dot[cc] += x[row * R + c0 + cc] * acc[cc];
      }
    }
  }
  if (DOT) {
    __shared__ double smem[CPL * kRedBlock];
    __shared__ double out[R];
    if (grid_reduce_cpl<R, CPL>(dot, partials, counter, smem, out)) {
      if (t < R) {
        ColState &cs = cols[t];
        if (cs.active) {
          const double pw = out[t];
          cs.pw = pw;
          if (!isfinite(pw)) { cs.status = ICPCG_E_NONFINITE; cs.active = 0; }
          else if (!(pw > 0.0)) { cs.status = ICPCG_E_BREAKDOWN; cs.active = 0; }
          else cs.alpha = cs.rz / pw;
        }
      }
    }
  }
}

template <int R, int SLOTS>
int launch(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x, double *y,
           hipStream_t s, double *partials, unsigned *counter, ColState *cols) {
  constexpr int CPL = R >= 4 ? 4 : R;
  constexpr int GPB = kBlock / (SLOTS * (R / CPL));
  // about 8 row passes per block, at most 4096 blocks (bounded partials)
  int64_t nb = (n + GPB * 8 - 1) / (GPB * 8);
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  const int64_t chunk = (n + nb - 1) / nb;
  nb = (n + chunk - 1) / chunk;
  if (nb < 1) nb = 1;
  if (partials)
    hipLaunchKernelGGL((k_spmv<R, SLOTS, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, rp, ci, v, n, x, y,
                       chunk, partials, counter, cols);
  else
    hipLaunchKernelGGL((k_spmv<R, SLOTS, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, rp, ci, v, n, x, y,
                       chunk, nullptr, nullptr, nullptr);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace

// slots: entry slots per row (the lanes per row are slots * R / min(R, 4)).
int spmv(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x, double *y, int R,
         int slots, hipStream_t s, double *partials, unsigned *counter, ColState *cols, int64_t, int) {
  if (n <= 0) return ICPCG_OK;
#define ICPCG_SPMV_CASE(RR, SS) \
  if (R == RR && slots == SS) return launch<RR, SS>(rp, ci, v, n, x, y, s, partials, counter, cols);
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

int spmv_default_slots(int R) {
  if (const char *e = std::getenv("ICPCG_SPMV_SLOTS")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  switch (R) {
    case 1: return 16;
    case 2: return 16;
    case 4: return 16;
    case 8: return 16;
    default: return 16;
  }
}

}  // namespace icpcg
