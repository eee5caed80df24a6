// Internal helpers shared by the gfx950 kernels of liblofqmc.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 (CDNA4).  Operand/lane convention, checked on the
// device by the layout test of the test-suite:
//   lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]  (A: 16x4, B: 4x16)
//   accumulator element v of lane l is D[4 * v + l / 16][l % 16].
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4zero() { return d4{0.0, 0.0, 0.0, 0.0}; }

// Complex helpers on double2 (x = re, y = im).
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// 1/z by Smith's algorithm (avoids overflow of |z|^2).
__device__ __forceinline__ double2 crecip(double2 z) {
  if (fabs(z.x) >= fabs(z.y)) {
    double r = z.y / z.x, d = z.x + z.y * r;
    return make_double2(1.0 / d, -r / d);
  }
  double r = z.x / z.y, d = z.y + z.x * r;
  return make_double2(r / d, -1.0 / d);
}

// Deterministic wave64 sum: a fixed shuffle-down tree; the result is valid in
// lane 0 only (other lanes hold partial sums).
__device__ __forceinline__ double wave_sum_lane0(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
