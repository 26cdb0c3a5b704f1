// Device helpers shared by the kernels: wavefront scans and semiring traits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

template <class T>
__device__ inline T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Order-preserving map of fp32 to uint32: a < b (IEEE, with -0 < +0)
// iff key(a) < key(b).  A bijection, so equal keys mean equal bits.
__device__ inline uint32_t f32_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float f32_unkey(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// Semiring traits.  V: stored value type.  Acc: accumulator word held in the
// hash/dense accumulators.  order_free: the semiring addition is exactly
// associative and commutative, so contributions may be combined in any
// order with atomics; otherwise (fp64) contributions are added one k at a
// time in ascending k.
template <int SR>
struct Sem;

template <>
struct Sem<0> {  // (+, x) over int64, wrap-around
  using V = int64_t;
  using Acc = unsigned long long;
  static constexpr bool order_free = true;
  __device__ static Acc identity() { return 0ull; }
  __device__ static Acc mul(V a, V b) { return (Acc)a * (Acc)b; }
  __device__ static Acc to_acc(V v) { return (Acc)v; }
  __device__ static V from_acc(Acc a) { return (V)a; }
  __device__ static void atomic_combine(Acc* p, Acc x) { atomicAdd(p, x); }
  __device__ static V add(V a, V b) { return (V)((Acc)a + (Acc)b); }
};

template <>
struct Sem<1> {  // (min, +) over fp32
  using V = float;
  using Acc = uint32_t;
  static constexpr bool order_free = true;
  __device__ static Acc identity() { return 0xffffffffu; }
  __device__ static Acc mul(V a, V b) { return f32_key(__fadd_rn(a, b)); }
  __device__ static Acc to_acc(V v) { return f32_key(v); }
  __device__ static V from_acc(Acc a) { return f32_unkey(a); }
  __device__ static void atomic_combine(Acc* p, Acc x) { atomicMin(p, x); }
  __device__ static V add(V a, V b) { return f32_key(a) <= f32_key(b) ? a : b; }
};

template <>
struct Sem<2> {  // (+, x) over fp64, one rounding per operation
  using V = double;
  using Acc = double;
  static constexpr bool order_free = false;
  __device__ static Acc identity() { return 0.0; }
  __device__ static Acc mul(V a, V b) { return __dmul_rn(a, b); }
  __device__ static Acc to_acc(V v) { return v; }
  __device__ static V from_acc(Acc a) { return a; }
  __device__ static V add(V a, V b) { return __dadd_rn(a, b); }
};

template <>
struct Sem<3> {  // (or, and) on 32-bit words: each bit is one Boolean semiring
  using V = uint32_t;
  using Acc = uint32_t;
  static constexpr bool order_free = true;
  __device__ static Acc identity() { return 0u; }
  __device__ static Acc mul(V a, V b) { return a & b; }
  __device__ static Acc to_acc(V v) { return v; }
  __device__ static V from_acc(Acc a) { return a; }
  __device__ static void atomic_combine(Acc* p, Acc x) { atomicOr(p, x); }
  __device__ static V add(V a, V b) { return a | b; }
};

template <class T>
__device__ inline bool same_bits(T a, T b) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "value size");
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(uint64_t, a) == __builtin_bit_cast(uint64_t, b);
  } else {
    return __builtin_bit_cast(uint32_t, a) == __builtin_bit_cast(uint32_t, b);
  }
}

__device__ inline uint32_t hash_col(int32_t c) { return (uint32_t)c * 2654435761u; }

// Exclusive prefix of a flag over a workgroup of NT lanes, and its total.
// Every thread of the workgroup calls it (it holds two barriers); wsum holds
// NT/64 ints of LDS.
template <int NT>
__device__ inline int32_t block_flag_prefix(bool f, int32_t* wsum, int32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t b = __ballot(f);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  if (lane == 0) wsum[wv] = __popcll(b);
  __syncthreads();
  int32_t before = 0, tot = 0;
  for (int x = 0; x < NT / 64; ++x) {
    const int32_t c = wsum[x];
    if (x < wv) before += c;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return before + __popcll(b & lt);
}
