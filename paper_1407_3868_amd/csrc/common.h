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

// One 16x16x4 matrix-core multiply-accumulate in precision T, D = A B + C.
// Operand layout (both precisions): lane i supplies A[i % 16][i / 16] and
// B[i / 16][i % 16]; result register j of lane i is D[row(i, j)][i % 16],
// row = 4 (i / 16) + j for f32 and i / 16 + 4 j for f64 (measured on gfx950
// with one-hot operands).
template <typename T> struct mfma4;
template <> struct mfma4<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mac(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};
template <> struct mfma4<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mac(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};

}  // namespace mpsl

#define MPSL_HIP_TRY(ctx, call)                                                              \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      (ctx)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_);      \
      return MPSL_EHIP;                                                                      \
    }                                                                                        \
  } while (0)
