// Device-wide building blocks: scans, reductions, fills and a stable LSD radix
// sort (used for level sorting and the transpose of L).
#include <climits>
#include <cstdio>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

struct OpAdd {
  template <typename T> __device__ __host__ T operator()(T a, T b) const { return a + b; }
  template <typename T> static __device__ __host__ T identity() { return T(0); }
};
struct OpMax {
  template <typename T> __device__ __host__ T operator()(T a, T b) const { return a > b ? a : b; }
  template <typename T> static __device__ __host__ T identity() {
    return sizeof(T) == 8 ? (T)LLONG_MIN : (T)INT_MIN;
  }
};

// Inclusive scan of one value per thread over a 256-thread block.
template <typename T, typename Op>
__device__ T block_inclusive_scan(T v, Op op, T *lds_waves) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= d) v = op(o, v);
  }
  if (lane == 63) lds_waves[wid] = v;
  __syncthreads();
  T prefix = Op::template identity<T>();
  for (int w = 0; w < wid; ++w) prefix = op(prefix, lds_waves[w]);
  __syncthreads();
  return wid ? op(prefix, v) : v;
}

// Scan of one tile per block; writes the tile total to block_sums.
template <typename T, typename Op, bool EXCL>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const T *in, T *out, T *block_sums, int64_t n,
                                                       Op op) {
  __shared__ T waves[4];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  T loc[kItems];
  T acc = Op::template identity<T>();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    const T x = i < n ? in[i] : Op::template identity<T>();
    acc = op(acc, x);
    loc[k] = acc;  // inclusive within the thread
  }
  const T incl = block_inclusive_scan<T, Op>(acc, op, waves);
  // exclusive prefix of this thread: the previous lane's inclusive value, or
  // for a wave's first lane the combined totals of the earlier waves
  T excl_t = __shfl_up(incl, 1, 64);
  if ((threadIdx.x & 63) == 0) {
    const int wid = threadIdx.x >> 6;
    excl_t = Op::template identity<T>();
    for (int w = 0; w < wid; ++w) excl_t = op(excl_t, waves[w]);
  }
  T prev = Op::template identity<T>();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = EXCL ? op(excl_t, prev) : op(excl_t, loc[k]);
    prev = loc[k];
  }
  if (threadIdx.x == kBlock - 1 && block_sums) block_sums[blockIdx.x] = incl;
}

template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void k_add_offsets(T *__restrict__ out, const T *__restrict__ offs,
                                                        int64_t n, Op op) {
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (blockIdx.x == 0) return;
  const T o = offs[blockIdx.x];
  for (int k = threadIdx.x; k < kTile; k += kBlock) {
    const int64_t i = base + k;
    if (i < n) out[i] = op(o, out[i]);
  }
}

// out = scan(in). Exclusive scans start from the identity. Recursive on the
// tile totals. `in` and `out` may alias.
template <typename T, typename Op, bool EXCL>
int scan_impl(const T *in, T *out, int64_t n, hipStream_t s, Op op) {
  if (n <= 0) return ICPCG_OK;
  const int64_t nt = (n + kTile - 1) / kTile;
  DevBuf sums;
  if (nt > 1) {
    if (sums.reserve((size_t)nt * sizeof(T))) return ICPCG_E_NOMEM;
  }
  hipLaunchKernelGGL((k_scan_tiles<T, Op, EXCL>), dim3((unsigned)nt), dim3(kBlock), 0, s, in, out,
                     nt > 1 ? sums.as<T>() : nullptr, n, op);
  ICPCG_HIP_TRY(hipGetLastError());
  if (nt > 1) {
    // exclusive scan of tile totals gives each tile's offset
    int st = scan_impl<T, Op, true>(sums.as<T>(), sums.as<T>(), nt, s, op);
    if (st) return st;
    hipLaunchKernelGGL((k_add_offsets<T, Op>), dim3((unsigned)nt), dim3(kBlock), 0, s, out,
                       sums.as<T>(), n, op);
    ICPCG_HIP_TRY(hipGetLastError());
    ICPCG_HIP_TRY(hipStreamSynchronize(s));  // `sums` is freed on return
  }
  return ICPCG_OK;
}

// ---------------------------------------------------------------- reduce

template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void k_reduce(const T *__restrict__ in, int64_t n, T *__restrict__ out,
                                                   Op op) {
  __shared__ T sm[kBlock];
  T acc = Op::template identity<T>();
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    acc = op(acc, in[i]);
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sm[threadIdx.x] = op(sm[threadIdx.x], sm[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

struct OpMinD {
  __device__ __host__ double operator()(double a, double b) const { return a < b ? a : b; }
  template <typename T> static __device__ __host__ T identity() { return (T)INFINITY; }
};

template <typename T, typename Op>
int reduce_impl(const T *in, int64_t n, hipStream_t s, T *host_out, Op op) {
  const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
  DevBuf tmp;
  if (tmp.reserve(sizeof(T) * (nb + 1))) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL((k_reduce<T, Op>), dim3(nb), dim3(kBlock), 0, s, in, n, tmp.as<T>(), op);
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_reduce<T, Op>), dim3(1), dim3(kBlock), 0, s, tmp.as<T>(), (int64_t)nb,
                     tmp.as<T>() + nb, op);
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipMemcpyAsync(host_out, tmp.as<T>() + nb, sizeof(T), hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

// ------------------------------------------------------------------ fills

template <typename T>
__global__ void k_fill(T *out, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v;
}
__global__ void k_iota(uint32_t *out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)i;
}

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

// ------------------------------------------------------------- radix sort

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;

// Digit histogram of one tile: hist[d * ntiles + tile] (digit-major, so an
// exclusive scan gives every (digit, tile) its first output slot).
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                       int shift, uint32_t *__restrict__ hist,
                                                       int64_t ntiles) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = threadIdx.x; k < kSortTile; k += kBlock) {
    const int64_t i = base + k;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: elements are taken in order, 256 per round; the
// rank of an element among equal digits is (earlier rounds) + (earlier waves
// of this round) + (earlier lanes of its wave, found by matching the digit
// bit by bit with ballots).
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offs, int64_t ntiles) {
  __shared__ uint32_t base[kRadix];
  __shared__ uint32_t wcnt[4][kRadix];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  base[t] = offs[(int64_t)t * ntiles + blockIdx.x];
  for (int w = 0; w < 4; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int rnd = 0; rnd < kSortItems; ++rnd) {
    const int64_t i = tile0 + (int64_t)rnd * kBlock + t;
    const bool valid = i < n;
    uint32_t key = 0, val = 0;
    int d = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      d = (int)((key >> shift) & (kRadix - 1));
    }
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wid][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + (uint32_t)rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    wcnt[0][t] = wcnt[1][t] = wcnt[2][t] = wcnt[3][t] = 0;
    __syncthreads();
  }
}

}  // namespace

// ----------------------------------------------------------------- public

int host_error(hipError_t e, const char *expr, const char *file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), expr,
           file, line);
  set_error(buf);
  return e == hipErrorOutOfMemory ? ICPCG_E_NOMEM : ICPCG_E_DEVICE;
}

int DevBuf::reserve(size_t b) {
  if (b <= bytes && p) return ICPCG_OK;
  release();
  if (b == 0) b = 8;
  if (hipMalloc(&p, b) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    set_error("device allocation of " + std::to_string(b) + " bytes failed");
    return ICPCG_E_NOMEM;
  }
  bytes = b;
  return ICPCG_OK;
}

int scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, int64_t *total_host) {
  int64_t last_in = 0;
  if (total_host && n > 0)
    ICPCG_HIP_TRY(hipMemcpyAsync(&last_in, in + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  if (total_host) ICPCG_HIP_TRY(hipStreamSynchronize(s));
  int st = scan_impl<int64_t, OpAdd, true>(in, out, n, s, OpAdd());
  if (st) return st;
  if (total_host) {
    int64_t last_out = 0;
    if (n > 0) ICPCG_HIP_TRY(hipMemcpyAsync(&last_out, out + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    ICPCG_HIP_TRY(hipStreamSynchronize(s));
    *total_host = n > 0 ? last_out + last_in : 0;
  }
  return ICPCG_OK;
}

int scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, int32_t *total_host) {
  int32_t last_in = 0;
  if (total_host && n > 0) {
    ICPCG_HIP_TRY(hipMemcpyAsync(&last_in, in + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ICPCG_HIP_TRY(hipStreamSynchronize(s));
  }
  int st = scan_impl<int32_t, OpAdd, true>(in, out, n, s, OpAdd());
  if (st) return st;
  if (total_host) {
    int32_t last_out = 0;
    if (n > 0) ICPCG_HIP_TRY(hipMemcpyAsync(&last_out, out + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ICPCG_HIP_TRY(hipStreamSynchronize(s));
    *total_host = n > 0 ? last_out + last_in : 0;
  }
  return ICPCG_OK;
}

int scan_inclusive_max_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  return scan_impl<int32_t, OpMax, false>(in, out, n, s, OpMax());
}

int reduce_max_i32(const int32_t *in, int64_t n, hipStream_t s, int32_t *host_out) {
  return reduce_impl<int32_t, OpMax>(in, n, s, host_out, OpMax());
}

int reduce_min_f64(const double *in, int64_t n, hipStream_t s, double *host_out) {
  return reduce_impl<double, OpMinD>(in, n, s, host_out, OpMinD());
}

int fill_iota_u32(uint32_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return ICPCG_OK;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(kBlock), 0, s, out, n);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}
int fill_i32(int32_t *out, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return ICPCG_OK;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n)), dim3(kBlock), 0, s, out, v, n);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}
int fill_u64(uint64_t *out, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return ICPCG_OK;
  hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n)), dim3(kBlock), 0, s, out, v, n);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}
int fill_u32(uint32_t *out, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return ICPCG_OK;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n)), dim3(kBlock), 0, s, out, v, n);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                     uint32_t *vals_out, int64_t n, int bits, hipStream_t s) {
  if (n <= 0) return ICPCG_OK;
  if (n > (int64_t)UINT32_MAX) {
    set_error("radix sort: too many elements");
    return ICPCG_E_INVALID;
  }
  const int passes = bits <= 0 ? 1 : (bits + kRadixBits - 1) / kRadixBits;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  DevBuf hist, kb, vb;
  if (hist.reserve((size_t)ntiles * kRadix * sizeof(uint32_t))) return ICPCG_E_NOMEM;
  if (passes > 1) {
    if (kb.reserve((size_t)n * 4) || vb.reserve((size_t)n * 4)) return ICPCG_E_NOMEM;
  }
  // ping-pong so that the last pass writes keys_out / vals_out
  const uint32_t *ksrc = keys_in, *vsrc = vals_in;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    // passes alternate between (kb,vb) and (out); choose so the final lands in out
    uint32_t *kdst, *vdst;
    if (((passes - 1 - p) & 1) == 0) { kdst = keys_out; vdst = vals_out; }
    else { kdst = kb.as<uint32_t>(); vdst = vb.as<uint32_t>(); }
    (void)last;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kBlock), 0, s, ksrc, n,
                       p * kRadixBits, hist.as<uint32_t>(), ntiles);
    ICPCG_HIP_TRY(hipGetLastError());
    int st = scan_impl<int32_t, OpAdd, true>(hist.as<int32_t>(), hist.as<int32_t>(), ntiles * kRadix,
                                             s, OpAdd());
    if (st) return st;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kBlock), 0, s, ksrc, vsrc, kdst,
                       vdst, n, p * kRadixBits, hist.as<uint32_t>(), ntiles);
    ICPCG_HIP_TRY(hipGetLastError());
    ksrc = kdst;
    vsrc = vdst;
  }
  ICPCG_HIP_TRY(hipStreamSynchronize(s));  // temporaries are freed on return
  return ICPCG_OK;
}

}  // namespace icpcg
