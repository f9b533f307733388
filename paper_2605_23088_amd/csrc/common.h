// Shared device/host helpers of the gfx950 library (no paper arithmetic here).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define YDEV __device__ __forceinline__
// math shared by the kernels and the host-side checks of the device arithmetic
#define YHD __host__ __device__ __forceinline__

namespace yasps {

// Status bits raised by kernels into a device word and turned into a
// yasps_status by the host after the launch sequence.
enum : uint32_t {
  FLAG_DOMAIN = 1u,     // a contact stencil with d <= 0
  FLAG_NONFINITE = 2u,  // NaN / Inf met in an input position or a result
};

// Compile-time index of entry (i, j) of a packed upper-triangular N x N matrix.
template <int N>
YHD constexpr int tri(int i, int j) {
  return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
}

// Symmetric N x N matrix held in registers as its packed upper triangle.
// Every access must use indices that are compile-time constants after
// unrolling, otherwise the array would spill to scratch.
template <int N, class R = double>
struct Sym {
  static constexpr int SIZE = N * (N + 1) / 2;
  R v[SIZE];
  YHD R& operator()(int i, int j) { return v[tri<N>(i, j)]; }
  YHD R operator()(int i, int j) const { return v[tri<N>(i, j)]; }
};

YHD bool finite(double v) { return __builtin_isfinite(v); }

// Type-generic math for the float64 path and the float32 precision form.
YHD double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
YHD float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
YHD double sqrtR(double a) { return __builtin_sqrt(a); }
YHD float sqrtR(float a) { return __builtin_sqrtf(a); }
YHD double fabsR(double a) { return __builtin_fabs(a); }
YHD float fabsR(float a) { return __builtin_fabsf(a); }
YHD double fmaxR(double a, double b) { return __builtin_fmax(a, b); }
YHD float fmaxR(float a, float b) { return __builtin_fmaxf(a, b); }
YHD double logR(double a) { return log(a); }
YHD float logR(float a) { return logf(a); }

}  // namespace yasps
