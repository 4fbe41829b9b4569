// Complex arithmetic on HIP vector types (double2 = complex128, float2 = complex64).
#pragma once
#include <hip/hip_runtime.h>

namespace stf {

template <typename T> struct RealOf;
template <> struct RealOf<double2> { using type = double; };
template <> struct RealOf<float2> { using type = float; };

__host__ __device__ inline double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline float2 cmk(float r, float i) { return make_float2(r, i); }

template <typename T> __host__ __device__ inline T czero() { return T{0, 0}; }

template <typename T> __host__ __device__ inline T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ inline T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }

template <typename T> __host__ __device__ inline T cmul(T a, T b) {
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename T> __host__ __device__ inline T cmulc(T a, T b) {
  return T{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// acc + a*b
template <typename T> __host__ __device__ inline T cfma(T a, T b, T acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc - a*b
template <typename T> __host__ __device__ inline T cfms(T a, T b, T acc) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename T> __host__ __device__ inline typename RealOf<T>::type cabs2(T a) {
  return a.x * a.x + a.y * a.y;
}
// a / b (Smith's algorithm, avoids overflow in |b|^2)
template <typename T> __host__ __device__ inline T cdiv(T a, T b) {
  using R = typename RealOf<T>::type;
  if (fabs(b.x) >= fabs(b.y)) {
    R r = b.y / b.x, d = b.x + b.y * r;
    return T{(a.x + a.y * r) / d, (a.y - a.x * r) / d};
  } else {
    R r = b.x / b.y, d = b.x * r + b.y;
    return T{(a.x * r + a.y) / d, (a.y * r - a.x) / d};
  }
}

template <typename T> __host__ __device__ inline T from_d2(double2 v);
template <> __host__ __device__ inline double2 from_d2<double2>(double2 v) { return v; }
template <> __host__ __device__ inline float2 from_d2<float2>(double2 v) {
  return make_float2((float)v.x, (float)v.y);
}
__host__ __device__ inline double2 to_d2(double2 v) { return v; }
__host__ __device__ inline double2 to_d2(float2 v) { return make_double2(v.x, v.y); }

// Wavefront (64-lane) reductions.
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T> __device__ inline T wave_csum(T v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}
template <typename T> __device__ inline T shfl_xor_c(T v, int mask) {
  v.x = __shfl_xor(v.x, mask, 64);
  v.y = __shfl_xor(v.y, mask, 64);
  return v;
}
template <typename T> __device__ inline T shfl_c(T v, int lane) {
  v.x = __shfl(v.x, lane, 64);
  v.y = __shfl(v.y, lane, 64);
  return v;
}

}  // namespace stf
