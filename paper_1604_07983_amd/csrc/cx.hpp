// cx.hpp -- minimal complex arithmetic shared by the device kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace nbs {

template <typename T> struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
using cd = cx<double>;
using cf = cx<float>;

template <typename T> __host__ __device__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cx<T>& operator+=(cx<T>& a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
// a += b * c
template <typename T> __host__ __device__ inline void cmac(cx<T>& a, cx<T> b, cx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// multiply by s * i (s = +-1)
template <typename T> __host__ __device__ inline cx<T> mul_si(cx<T> a, int s) {
  return s > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

template <typename To, typename Ti> __host__ __device__ inline cx<To> conv(cx<Ti> a) {
  return cx<To>{(To)a.re, (To)a.im};
}

}  // namespace nbs
