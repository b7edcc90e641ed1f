// Small complex helpers on HIP vector types (double2 / float2).
#pragma once

#include <hip/hip_runtime.h>

namespace chebfi {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T> using C2 = typename Vec2<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) {
  return V{a.x * s, a.y * s};
}
// multiply by i*sgn (sgn = +1 or -1)
template <typename V> __device__ __forceinline__ V cmul_i(V a, int sgn) {
  return sgn > 0 ? V{-a.y, a.x} : V{a.y, -a.x};
}

template <typename T> __device__ __forceinline__ C2<T> to_c2(double2 v) {
  return C2<T>{(T)v.x, (T)v.y};
}

}  // namespace chebfi
