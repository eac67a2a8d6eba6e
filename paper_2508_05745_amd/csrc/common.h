// Shared device/host helpers of the mpsb HIP library (complex arithmetic, launch checks).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpsb {

// ------------------------------------------------------------------ complex types
template <typename T> struct cplx { T re, im; };
using c32 = cplx<float>;
using c64d = cplx<double>;

template <typename T> __host__ __device__ inline cplx<T> mk(T r, T i) { return {r, i}; }
template <typename T> __host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ inline T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ inline cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> __host__ __device__ inline void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
template <typename T> __host__ __device__ inline void cfma_conj(cplx<T>& acc, cplx<T> a, cplx<T> b) {  // acc += a * conj(b)
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.im * b.re - a.re * b.im;
}

// ------------------------------------------------------------------ small structs passed by value
struct Mat4 { double v[32]; };      // 4x4 c128, row-major (re, im)
struct Kraus4 { double v[32]; };    // [4][2][2] c128
struct Mat2x2 { double v[8]; };     // 2x2 c128

}  // namespace mpsb
