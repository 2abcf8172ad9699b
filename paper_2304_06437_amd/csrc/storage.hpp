// Population storage codecs and vector memory access.
//
// Populations are stored shifted, s_a = f_a - t_a*rho0 (their deviation from
// the rest state), so that 32- and 16-bit storage spend their precision on
// the dynamics and not on the constant t_a*rho0.  16-bit modes round to
// nearest even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbk {

struct bf16s {
  uint16_t bits;
};

template <typename S, typename C>
struct Codec;

template <>
struct Codec<double, double> {
  __device__ static inline double load(double s) { return s; }
  __device__ static inline double store(double c) { return c; }
};

template <>
struct Codec<float, float> {
  __device__ static inline float load(float s) { return s; }
  __device__ static inline float store(float c) { return c; }
};

template <>
struct Codec<_Float16, float> {
  __device__ static inline float load(_Float16 s) { return (float)s; }
  // v_cvt_f16_f32 under the default round-to-nearest-even mode
  __device__ static inline _Float16 store(float c) { return (_Float16)c; }
};

template <>
struct Codec<bf16s, float> {
  __device__ static inline float load(bf16s s) {
    return __uint_as_float(((uint32_t)s.bits) << 16);
  }
  // round to nearest, ties to even, on the upper 16 bits of the FP32 pattern
  __device__ static inline bf16s store(float c) {
    uint32_t u = __float_as_uint(c);
    bf16s r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
      r.bits = (uint16_t)((u >> 16) | 0x0040u);  // quiet NaN
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      r.bits = (uint16_t)(u >> 16);
    }
    return r;
  }
};

// V consecutive elements moved as one aligned block (global_load/store of
// up to 16 bytes per instruction).
template <typename T, int V>
struct alignas(V * sizeof(T) >= 16 ? 16 : V * sizeof(T)) Pack {
  T v[V];
};

template <typename S, typename C, int V>
__device__ inline void load_pack(const S* __restrict__ p, C (&out)[V]) {
  const Pack<S, V> pk = *reinterpret_cast<const Pack<S, V>*>(p);
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = Codec<S, C>::load(pk.v[e]);
}

template <typename S, typename C, int V>
__device__ inline void store_pack(S* __restrict__ p, const C (&in)[V]) {
  Pack<S, V> pk;
#pragma unroll
  for (int e = 0; e < V; ++e) pk.v[e] = Codec<S, C>::store(in[e]);
  *reinterpret_cast<Pack<S, V>*>(p) = pk;
}

template <typename T, int V>
__device__ inline void load_plain(const T* __restrict__ p, T (&out)[V]) {
  const Pack<T, V> pk = *reinterpret_cast<const Pack<T, V>*>(p);
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = pk.v[e];
}

template <typename T, int V>
__device__ inline void store_plain(T* __restrict__ p, const T (&in)[V]) {
  Pack<T, V> pk;
#pragma unroll
  for (int e = 0; e < V; ++e) pk.v[e] = in[e];
  *reinterpret_cast<Pack<T, V>*>(p) = pk;
}

}  // namespace lbk
