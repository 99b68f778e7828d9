// Device-side helpers shared by the HIP translation units of libssx.
#pragma once

#include "ssx_internal.h"

namespace ssx {

// storage type T -> compute type C (and trace/vector type V)
template <typename T> struct Tr;
template <> struct Tr<double> { using C = double; using V = double; };
template <> struct Tr<float> { using C = float; using V = float; };
template <> struct Tr<__half> { using C = float; using V = float; };
template <> struct Tr<__hip_bfloat16> { using C = float; using V = float; };

template <typename C> __device__ __forceinline__ C ldc(const double* p) { return C(*p); }
template <typename C> __device__ __forceinline__ C ldc(const float* p) { return C(*p); }
template <typename C> __device__ __forceinline__ C ldc(const __half* p) {
  return C(__half2float(*p));
}
template <typename C> __device__ __forceinline__ C ldc(const __hip_bfloat16* p) {
  return C(__bfloat162float(*p));
}
// The FP32 value is pinned in a register before a 16-bit store: otherwise the
// compiler may fold a preceding FMA into a mixed-precision FMA that rounds
// once, straight to 16 bits, in some kernels but not in others, and kernel
// variants would stop agreeing bitwise.
__device__ __forceinline__ float pin(float x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ void stc(double* p, double v) { *p = v; }
__device__ __forceinline__ void stc(float* p, float v) { *p = v; }
__device__ __forceinline__ void stc(__half* p, float v) { *p = __float2half(pin(v)); }
__device__ __forceinline__ void stc(__hip_bfloat16* p, float v) { *p = __float2bfloat16(pin(v)); }

// value as it reads back after a store to T
template <typename T, typename C> __device__ __forceinline__ C rnd(C v) {
  if constexpr (sizeof(T) == sizeof(C)) {
    return v;
  } else {
    T t;
    stc(&t, v);
    return ldc<C>(&t);
  }
}

// four consecutive elements, naturally aligned (one 128-bit access for
// float, two for double, one 64-bit access for 16-bit types)
template <typename T> struct alignas(4 * sizeof(T)) V4 { T e[4]; };

template <typename C, typename T>
__device__ __forceinline__ void ld4(C (&o)[4], const T* p) {
  const V4<T> v = *reinterpret_cast<const V4<T>*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = ldc<C>(&v.e[i]);
}
template <typename T, typename C>
__device__ __forceinline__ void st4(T* p, const C (&x)[4]) {
  V4<T> v;
#pragma unroll
  for (int i = 0; i < 4; ++i) stc(&v.e[i], x[i]);
  *reinterpret_cast<V4<T>*>(p) = v;
}

}  // namespace ssx
