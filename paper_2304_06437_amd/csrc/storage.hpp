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

// The stored value is the round-to-nearest-even image of the FP32 value c.
// The empty asm pins c as an FP32 register value: without it the compiler
// may fold the conversion into the FMA that produced c (v_fma_mix*_f16, one
// rounding straight to 16 bits), whose result differs from rounding the
// FP32 value where that value sits next to a 16-bit tie.
__device__ __forceinline__ float fp32_value(float c) {
  asm("" : "+v"(c));
  return c;
}

template <>
struct Codec<_Float16, float> {
  __device__ static inline float load(_Float16 s) { return (float)s; }
  // v_cvt_f16_f32 under the default round-to-nearest-even mode
  __device__ static inline _Float16 store(float c) { return (_Float16)fp32_value(c); }
};

// fptrunc to bfloat: round to nearest, ties to even (v_cvt_pk_bf16_f32 on gfx950)
template <>
struct Codec<__bf16, float> {
  __device__ static inline float load(__bf16 s) { return (float)s; }
  __device__ static inline __bf16 store(float c) { return (__bf16)fp32_value(c); }
};

// Streaming hints: population and moment arrays are touched once per sweep,
// so loads and stores may bypass cache retention (nontemporal).
#ifndef LB_NT_LOAD
#define LB_NT_LOAD 1
#endif
#ifndef LB_NT_STORE
#define LB_NT_STORE 1
#endif

// Raw aligned move of NB bytes (2, 4, 8, or a multiple of 16).
template <int NB>
struct RawT;
template <>
struct RawT<2> { using T = unsigned short; };
template <>
struct RawT<4> { using T = unsigned int; };
template <>
struct RawT<8> { typedef unsigned int T __attribute__((ext_vector_type(2))); };
template <>
struct RawT<16> { typedef unsigned int T __attribute__((ext_vector_type(4))); };

template <int NB, bool NT>
__device__ __forceinline__ void raw_store(void* __restrict__ p, const void* src) {
  if constexpr (NB > 16) {
    static_assert(NB % 16 == 0, "raw_store size");
#pragma unroll
    for (int o = 0; o < NB; o += 16)
      raw_store<16, NT>((char*)p + o, (const char*)src + o);
  } else {
    using T = typename RawT<NB>::T;
    T v;
    __builtin_memcpy(&v, src, NB);
    if constexpr (NT) __builtin_nontemporal_store(v, (T*)p);
    else *(T*)p = v;
  }
}

template <int NB, bool NT>
__device__ __forceinline__ void raw_load(const void* __restrict__ p, void* dst) {
  if constexpr (NB > 16) {
    static_assert(NB % 16 == 0, "raw_load size");
#pragma unroll
    for (int o = 0; o < NB; o += 16)
      raw_load<16, NT>((const char*)p + o, (char*)dst + o);
  } else {
    using T = typename RawT<NB>::T;
    T v;
    if constexpr (NT) v = __builtin_nontemporal_load((const T*)p);
    else v = *(const T*)p;
    __builtin_memcpy(dst, &v, NB);
  }
}

template <typename T, int V>
struct Pack {
  T v[V];
};

// V consecutive elements moved as one aligned block (the address must be
// aligned to V * sizeof(T) bytes, up to 16).
template <typename S, typename C, int V, bool NT = (LB_NT_LOAD != 0)>
__device__ __forceinline__ void load_pack(const S* __restrict__ p, C (&out)[V]) {
  Pack<S, V> pk;
  raw_load<V * (int)sizeof(S), NT>(p, &pk);
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = Codec<S, C>::load(pk.v[e]);
}

template <typename S, typename C, int V, bool NT = (LB_NT_STORE != 0)>
__device__ __forceinline__ void store_pack(S* __restrict__ p, const C (&in)[V]) {
  Pack<S, V> pk;
#pragma unroll
  for (int e = 0; e < V; ++e) pk.v[e] = Codec<S, C>::store(in[e]);
  raw_store<V * (int)sizeof(S), NT>(p, &pk);
}

template <typename T, int V, bool NT = (LB_NT_LOAD != 0)>
__device__ __forceinline__ void load_plain(const T* __restrict__ p, T (&out)[V]) {
  Pack<T, V> pk;
  raw_load<V * (int)sizeof(T), NT>(p, &pk);
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = pk.v[e];
}

template <typename T, int V, bool NT = (LB_NT_STORE != 0)>
__device__ __forceinline__ void store_plain(T* __restrict__ p, const T (&in)[V]) {
  Pack<T, V> pk;
#pragma unroll
  for (int e = 0; e < V; ++e) pk.v[e] = in[e];
  raw_store<V * (int)sizeof(T), NT>(p, &pk);
}

}  // namespace lbk
