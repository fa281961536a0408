// Pattern pass of the reverse-mode derivative of Z = L^-T L^-1 R (not in the
// paper; derived from L Y = R and L^T Z = Y):
//   dL_ab = -sum_k (Z_ak Ybar_bk + Rbar_ak Y_bk)   for every stored (a, b) of L,
// with Ybar = L^-1 G and Rbar = L^-T Ybar computed by the triangular solves.
// One wave per row a; lanes are (entry slot, column), so the R columns of a
// gathered row b are one contiguous load, and the column sum is a fixed
// butterfly.
#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kBlock = 256;

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_dL(const int64_t *__restrict__ lrp, const int32_t *__restrict__ lci,
                                               int64_t n, const T *__restrict__ Z, const T *__restrict__ Yb,
                                               const T *__restrict__ Rb, const T *__restrict__ Y, T *__restrict__ dL) {
  constexpr int SLOTS = 64 / R;
  const int lane = threadIdx.x & 63, slot = lane / R, c = lane % R;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t a = w0; a < n; a += nw) {
    const T za = Z[a * R + c], ra = Rb[a * R + c];
    const int64_t s = lrp[a], e = lrp[a + 1];
    for (int64_t q0 = s; q0 < e; q0 += SLOTS) {
      const int64_t q = q0 + slot;
      T v = T(0);
      if (q < e) {
        const int64_t b = lci[q];
        v = za * Yb[b * R + c] + ra * Y[b * R + c];
      }
#pragma unroll
      for (int m = 1; m < R; m <<= 1) v += __shfl_xor(v, m, ICPCG_WAVE);
      if (c == 0 && q < e) dL[q] = -v;
    }
  }
}

template <typename T, int R>
int launch(const icpcg_prec *P, const T *Z, const T *Yb, const T *Rb, const T *Y, T *dL, hipStream_t s) {
  int64_t g = (P->n + 3) / 4;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL((k_dL<T, R>), dim3((unsigned)g), dim3(kBlock), 0, s, P->lrp.as<int64_t>(), P->lci.as<int32_t>(),
                     P->n, Z, Yb, Rb, Y, dL);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

template <typename T>
int dispatch(int R, const icpcg_prec *P, const T *Z, const T *Yb, const T *Rb, const T *Y, T *dL, hipStream_t s) {
  switch (R) {
    case 1: return launch<T, 1>(P, Z, Yb, Rb, Y, dL, s);
    case 2: return launch<T, 2>(P, Z, Yb, Rb, Y, dL, s);
    case 4: return launch<T, 4>(P, Z, Yb, Rb, Y, dL, s);
    case 8: return launch<T, 8>(P, Z, Yb, Rb, Y, dL, s);
    case 16: return launch<T, 16>(P, Z, Yb, Rb, Y, dL, s);
    default:
      set_error("apply_backward: unsupported block width " + std::to_string(R));
      return ICPCG_E_INVALID;
  }
}

}  // namespace

int prec_dL(const icpcg_prec *P, const void *Z, const void *Yb, const void *Rb, const void *Y, void *dL, int R,
            hipStream_t s) {
  if (P->dtype == ICPCG_F64)
    return dispatch<double>(R, P, (const double *)Z, (const double *)Yb, (const double *)Rb, (const double *)Y,
                            (double *)dL, s);
  return dispatch<float>(R, P, (const float *)Z, (const float *)Yb, (const float *)Rb, (const float *)Y, (float *)dL, s);
}

}  // namespace icpcg
