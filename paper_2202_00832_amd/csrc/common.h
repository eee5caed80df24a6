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

// s_waitcnt vmcnt(0) through the builtin (not inline asm), so the compiler's
// own wait insertion sees it: the loads straight into LDS (buffer or global
// form) of the issuing lane are complete after it.  gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8 (expcnt and lgkmcnt at their
// maximum: no wait)
__device__ __forceinline__ void wait_vmcnt0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Complex product on double2 (x = re, y = im).
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Deterministic wave64 sum: a fixed shuffle-down tree; the result is valid in
// lane 0 only (other lanes hold partial sums).
__device__ __forceinline__ double wave_sum_lane0(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Wave64 maximum of a 32-bit unsigned key, returned as a wave-uniform
// (scalar) value.  Inside each row of 16 lanes: DPP quad permutes and the two
// row mirrors leave every lane with its row's maximum; across rows: the GFX9
// row broadcasts (lane 15 of each row into the next row, then lane 31 into
// rows 2 and 3) leave the maximum of all 64 lanes in lane 63, which is read
// into a scalar register.  Lanes outside a step's row mask keep their value.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_max_u32(unsigned v) {
  const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROWS, 0xF, false);
  return o > v ? o : v;
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = dpp_max_u32<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_max_u32<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_max_u32<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_max_u32<0x140, 0xF>(v);   // row_mirror
  v = dpp_max_u32<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_max_u32<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ unsigned long long u64_of(int lo, int hi) {
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Lane `lane` (wave-uniform) of a double, into scalar registers.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return __longlong_as_double((long long)u64_of(__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), lane),
                                                 __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane)));
}
