// Internal helpers shared by the gfx950 kernels of liblofqmc.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 (CDNA4).  Operand/lane convention (any other layout
// would break every energy parity test on the device):
//   lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]  (A: 16x4, B: 4x16)
//   accumulator element v of lane l is D[4 * v + l / 16][l % 16].
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4zero() { return d4{0.0, 0.0, 0.0, 0.0}; }

// v_mfma_f64_4x4x4f64 (four independent 4x4x4 blocks per instruction).  Lane
// convention, read off one-hot inputs on the device:
//   lane l supplies A_b[l % 4][l / 16] and B_b[l / 16][l % 4] of block b = (l / 4) % 4,
//   and receives D_b[l / 16][l % 4].
// Four of them with A rows 4q + l % 4 (q = 0..3) and B = the 16x16x4 B
// fragment (B[l / 16][l % 16]) leave accumulator q of lane l holding
// D[4q + l / 16][l % 16]: the same element as element q of the 16x16x4
// accumulator.  On this chip the 4x4x4 form sustains close to the FP64 peak
// from one wave per SIMD, the 16x16x4 form about two thirds of it.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

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

// Wave64 maximum of a 64-bit unsigned key, returned in every lane.  Row-local
// butterflies use DPP (quad permutes and the row mirrors); the two cross-row
// steps use lane shuffles.  Max is associative and exact, so all lanes agree.
__device__ __forceinline__ unsigned long long dpp_max_u64(unsigned long long v, int ctrl) {
  const int lo = (int)(unsigned)(v & 0xffffffffull), hi = (int)(unsigned)(v >> 32);
  int olo, ohi;
  switch (ctrl) {
    case 0: olo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false); ohi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false); break;
    case 1: olo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false); ohi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false); break;
    case 2: olo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false); ohi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false); break;
    default: olo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false); ohi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false); break;
  }
  const unsigned long long o = ((unsigned long long)(unsigned)ohi << 32) | (unsigned)olo;
  return o > v ? o : v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  v = dpp_max_u64(v, 0);   // quad_perm [1,0,3,2]
  v = dpp_max_u64(v, 1);   // quad_perm [2,3,0,1]
  v = dpp_max_u64(v, 2);   // row_half_mirror
  v = dpp_max_u64(v, 3);   // row_mirror
  unsigned long long o = __shfl_xor(v, 16, 64);
  v = o > v ? o : v;
  o = __shfl_xor(v, 32, 64);
  return o > v ? o : v;
}

// Maximum of a 64-bit key over each row of 16 lanes (DPP only, no LDS-path
// shuffles); every lane of the row receives its row's maximum.
__device__ __forceinline__ unsigned long long row16_max_u64(unsigned long long v) {
  v = dpp_max_u64(v, 0);   // quad_perm [1,0,3,2]
  v = dpp_max_u64(v, 1);   // quad_perm [2,3,0,1]
  v = dpp_max_u64(v, 2);   // row_half_mirror
  v = dpp_max_u64(v, 3);   // row_mirror
  return v;
}
