// Internal helpers shared by the library's HIP translation units (gfx950,
// wave64). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <string>

#define ICPCG_WAVE 64

namespace icpcg {

// ------------------------------------------------------------ bit patterns

// A value that is still being produced holds a reserved NaN pattern
// ("value-as-flag"). A producer never stores that pattern: a computed NaN
// with the same payload is replaced by the canonical quiet NaN.
template <typename T> struct Flag;
template <> struct Flag<double> {
  using U = unsigned long long;
  static constexpr U kPending = 0xFFF80000DEADBEEFull;
  static constexpr U kCanonNaN = 0x7FF8000000000000ull;
};
template <> struct Flag<float> {
  using U = unsigned int;
  static constexpr U kPending = 0xFFF0DEADu;
  static constexpr U kCanonNaN = 0x7FC00000u;
};
template <> struct Flag<int> {
  using U = int;
  static constexpr U kPending = -1;
};

template <typename To, typename From>
__device__ __host__ __forceinline__ To bitcast(From f) {
  static_assert(sizeof(To) == sizeof(From), "size");
  To t;
  __builtin_memcpy(&t, &f, sizeof(To));
  return t;
}

// Device-scope (agent) relaxed atomics: on gfx950 these bypass the per-XCD L2
// coherence gap, so a value stored by one wave is observed by waves on every
// XCD without fences. Every access to a value-as-flag array inside the
// producing kernel goes through these two functions.
template <typename U>
__device__ __forceinline__ U ld_agent(const U *p) {
  return __hip_atomic_load(const_cast<U *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U>
__device__ __forceinline__ void st_agent(U *p, U v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait: spin until *p no longer holds the pending pattern. After
// `limit` wall-clock ticks the wait gives up, raises err and returns NaN so
// the kernel still terminates (the dependency order makes this unreachable
// for well-formed input; it guards against a broken schedule).
template <typename T>
__device__ __forceinline__ T wait_value(const T *p, int *err, long long limit) {
  using U = typename Flag<T>::U;
  const U *up = reinterpret_cast<const U *>(p);
  U v = ld_agent(up);
  if (v == Flag<T>::kPending) {
    const long long t0 = wall_clock64();
    do {
      __builtin_amdgcn_s_sleep(1);
      v = ld_agent(up);
      if (v != Flag<T>::kPending) break;
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = Flag<T>::kCanonNaN;
        break;
      }
    } while (true);
  }
  return bitcast<T>(v);
}

// Wait (one lane) until the value-as-flag FP64 entry *p no longer holds the
// pending pattern, with exponential backoff between polls so that many
// waiting waves do not flood the memory system. Returns false (and raises
// err) at the time limit, or when *abandon (nullable) becomes nonzero.
__device__ __forceinline__ bool poll_f64(const double *p, int *err, long long limit, const int *abandon) {
  const unsigned long long *u = reinterpret_cast<const unsigned long long *>(p);
  if (ld_agent(u) != Flag<double>::kPending) return true;
  const long long t0 = wall_clock64();
  int backoff = 1;
  while (true) {
    for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(2);
    if (backoff < 16) backoff <<= 1;
    if (ld_agent(u) != Flag<double>::kPending) return true;
    if (abandon && ld_agent(abandon)) return false;
    if (wall_clock64() - t0 > limit) {
      __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

// Next ticket of a one-wave work queue: lane 0 takes it with a (vector)
// atomic and the wave shares it. Tickets taken by one wave rise.
__device__ __forceinline__ unsigned take_ticket(unsigned *ticket) {
  unsigned t = 0;
  if (threadIdx.x == 0) t = atomicAdd(ticket, 1u);
  return __shfl(t, 0, ICPCG_WAVE);
}

template <typename T>
__device__ __forceinline__ void publish_value(T *p, T x) {
  using U = typename Flag<T>::U;
  U u = bitcast<U>(x);
  if (u == Flag<T>::kPending) u = Flag<T>::kCanonNaN;
  st_agent(reinterpret_cast<U *>(p), u);
}

__device__ __forceinline__ int wait_int(const int *p, int *err, long long limit) {
  int v = ld_agent(p);
  if (v < 0) {
    const long long t0 = wall_clock64();
    do {
      __builtin_amdgcn_s_sleep(1);
      v = ld_agent(p);
      if (v >= 0) break;
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = 0;
        break;
      }
    } while (true);
  }
  return v;
}

// ---------------------------------------------------------- bfloat16

// float -> bfloat16 bits, round to nearest even, NaN kept quiet.
__device__ __host__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  unsigned int u = bitcast<unsigned int>(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __host__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return bitcast<float>((unsigned int)h << 16);
}

// Load of one stored factor value widened to the arithmetic type.
template <typename TA, typename TV> __device__ __forceinline__ TA widen(TV v) { return (TA)v; }
template <> __device__ __forceinline__ float widen<float, unsigned short>(unsigned short v) {
  return bf16_to_f32(v);
}

// ------------------------------------------------------ wave reductions

// Butterfly sum over lanes whose index differs in bits [lo_bit, 6): lanes that
// share the low bits (the same column of a multi-column group) are combined.
// Fixed pattern, so the result is deterministic.
template <int LO_BIT, typename T>
__device__ __forceinline__ T xor_sum_from(T v) {
#pragma unroll
  for (int b = 32; b >= (1 << LO_BIT); b >>= 1) v += __shfl_xor(v, b, ICPCG_WAVE);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) { return xor_sum_from<0>(v); }

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int b = 32; b >= 1; b >>= 1) {
    int o = __shfl_xor(v, b, ICPCG_WAVE);
    v = o > v ? o : v;
  }
  return v;
}

template <int R> struct Log2;
template <> struct Log2<1> { static constexpr int v = 0; };
template <> struct Log2<2> { static constexpr int v = 1; };
template <> struct Log2<4> { static constexpr int v = 2; };
template <> struct Log2<8> { static constexpr int v = 3; };
template <> struct Log2<16> { static constexpr int v = 4; };
template <> struct Log2<32> { static constexpr int v = 5; };
template <> struct Log2<64> { static constexpr int v = 6; };

// Block index remapped so that consecutive logical blocks land on the same
// XCD: the dispatcher places workgroup b on XCD b % 8, so logical block
// (b % 8) * q + b / 8 gives each XCD one contiguous range (and its L2 the
// neighbouring rows' gathers). Blocks past 8 * floor(nb / 8) keep their id.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3;
  if (b < (q << 3)) return (b & 7) * q + (b >> 3);
  return b;
}

}  // namespace icpcg

// ------------------------------------------------------------- host side

#define ICPCG_HIP_TRY(expr)                                                         \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      return ::icpcg::host_error(_e, #expr, __FILE__, __LINE__);                    \
    }                                                                               \
  } while (0)

namespace icpcg {
int host_error(hipError_t e, const char *expr, const char *file, int line);
}
