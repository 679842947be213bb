// Shared device/host helpers of the mpsl library: complex arithmetic on
// double2/float2 storage, status handling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mpsl.h"

namespace mpsl {

// Storage type of one complex number in precision T.
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cv_t = typename cvec<T>::type;

// Register-side complex number.
template <typename T> struct cx {
  T re, im;
};

template <typename T> __host__ __device__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __host__ __device__ inline cx<T> ld(const cv_t<T> &v) { return cx<T>{v.x, v.y}; }
template <typename T> __host__ __device__ inline cv_t<T> st(const cx<T> &v) {
  cv_t<T> o;
  o.x = v.re;
  o.y = v.im;
  return o;
}
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// acc += a * b
template <typename T> __host__ __device__ inline void cmac(cx<T> &acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

}  // namespace mpsl

#define MPSL_HIP_TRY(ctx, call)                                                              \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      (ctx)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_);      \
      return MPSL_EHIP;                                                                      \
    }                                                                                        \
  } while (0)
