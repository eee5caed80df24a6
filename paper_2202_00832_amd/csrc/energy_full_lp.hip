// Two-body energy by the half-rotated Cholesky route (Eq. 16) with the
// exchange contraction T = Lbar_g^T theta in reduced precision:
//   FP32    : v_mfma_f32_16x16x4_f32 on FP32-rounded operands;
//   BF16X3  : split BF16, x = x_hi + x_lo with x_hi = bf16(x), x_lo = bf16(x - x_hi),
//             T = L_hi th_hi + L_hi th_lo + L_lo th_hi on v_mfma_f32_16x16x32_bf16
//             (the lo*lo product is dropped), FP32 accumulation.
// The exchange sum sum_ij T_ij T_ji and all sums over g and over chunks are
// FP64.  The Coulomb trace Tr T = sum_{r,i} Lbar_g[r][i] theta[r][i] is a
// plain contraction over (r, i) that costs 1/n of T; it stays FP64 (FP64
// MFMA), because the large traces would otherwise carry the rounding of the
// FP32 inputs straight into E_J = 2 sum_g (Tr T)^2.
//
// The operands are first rewritten once per call into padded layouts
// (M rounded up to a multiple of 32, n up to NP = 16 NB, zeros in the padding):
//   FP32   : lbar32 [X][Mp][NP] float,   theta32 [nw][Mp][NP] float2
//   BF16X3 : lbarbf [X][2][NP][Mp] (hi, lo planes, r fastest),
//            thetabf [nw][4][NP][Mp] (re_hi, re_lo, im_hi, im_lo planes)
// so that each MFMA operand fragment is one aligned load.
#include "common.h"
#include "kernels.h"
#include "lofqmc.h"

namespace lofqmc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// v_mfma_f32_16x16x4_f32: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16] for its eight values t.  For both, accumulator
// element v of lane l is D[4 (l / 16) + v][l % 16] (note: not the FP64
// layout; any other layout would break the reduced-precision parity tests).
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 f4zero() { return f4{0.0f, 0.0f, 0.0f, 0.0f}; }

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float xf = (float)x;
  hi = (__bf16)xf;
  lo = (__bf16)(xf - (float)hi);
}

constexpr int LP_SLAB = 32;   // rows of r per staged tile (and the padding unit of M)
constexpr int LP_MAXNP = 96;  // largest padded orbital count (n_occ <= 96)

int lp_padded_m(int M) { return (M + LP_SLAB - 1) / LP_SLAB * LP_SLAB; }

// ---------------------------------------------------------------------------
// operand rewrite: one workgroup per (matrix index, 32-row slab), through LDS
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void lp_convert_real_kernel(int M, int n, int Mp, int NP,
                                                              const double* __restrict__ src,
                                                              void* __restrict__ dst) {
  __shared__ double t[LP_SLAB][LP_MAXNP + 1];
  const int64_t g = blockIdx.y;
  const int r0 = LP_SLAB * blockIdx.x;
  const double* s = src + (size_t)g * M * n;
  for (int e = threadIdx.x; e < LP_SLAB * NP; e += 256) {
    const int rr = e / NP, i = e % NP, r = r0 + rr;
    t[rr][i] = (r < M && i < n) ? s[(size_t)r * n + i] : 0.0;
  }
  __syncthreads();
  if constexpr (MODE == LO_FP32) {
    float* d = (float*)dst + ((size_t)g * Mp + r0) * NP;
    for (int e = threadIdx.x; e < LP_SLAB * NP; e += 256) d[e] = (float)t[e / NP][e % NP];
  } else {
    __bf16* d = (__bf16*)dst + (size_t)g * 2 * NP * Mp;
    for (int e = threadIdx.x; e < LP_SLAB * NP; e += 256) {
      const int i = e / LP_SLAB, rr = e % LP_SLAB;
      __bf16 hi, lo;
      split_bf16(t[rr][i], hi, lo);
      d[(size_t)i * Mp + r0 + rr] = hi;
      d[((size_t)NP + i) * Mp + r0 + rr] = lo;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void lp_convert_complex_kernel(int M, int n, int Mp, int NP,
                                                                 const double2* __restrict__ src,
                                                                 void* __restrict__ dst) {
  __shared__ double2 t[LP_SLAB][LP_MAXNP + 1];
  const int64_t w = blockIdx.y;
  const int r0 = LP_SLAB * blockIdx.x;
  const double2* s = src + (size_t)w * M * n;
  for (int e = threadIdx.x; e < LP_SLAB * NP; e += 256) {
    const int rr = e / NP, i = e % NP, r = r0 + rr;
    t[rr][i] = (r < M && i < n) ? s[(size_t)r * n + i] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if constexpr (MODE == LO_FP32) {
    float2* d = (float2*)dst + ((size_t)w * Mp + r0) * NP;
    for (int e = threadIdx.x; e < LP_SLAB * NP; e += 256) {
      const double2 v = t[e / NP][e % NP];
      d[e] = make_float2((float)v.x, (float)v.y);
    }
  } else {
    __bf16* d = (__bf16*)dst + (size_t)w * 4 * NP * Mp;
    for (int e = threadIdx.x; e < LP_SLAB * NP; e += 256) {
      const int i = e / LP_SLAB, rr = e % LP_SLAB;
      const double2 v = t[rr][i];
      __bf16 rh, rl, ih, il;
      split_bf16(v.x, rh, rl);
      split_bf16(v.y, ih, il);
      const size_t o = (size_t)i * Mp + r0 + rr, pl = (size_t)NP * Mp;
      d[o] = rh;
      d[pl + o] = rl;
      d[2 * pl + o] = ih;
      d[3 * pl + o] = il;
    }
  }
}

// ---------------------------------------------------------------------------
// exchange: E_K partials per (chunk of Cholesky vectors, walker)
// ---------------------------------------------------------------------------
template <int NB>
struct LpCfg {
  static constexpr int NP = 16 * NB;
  static constexpr int NPAIR = NB * (NB - 1) / 2;
  static constexpr int NPH = (NPAIR + 1) / 2;   // off-diagonal pairs per half
  static constexpr int NDH = (NB + 1) / 2;      // diagonal blocks per half
  static constexpr int LDW = NP + 16;           // FP32 tile row stride (bank spread)
  static constexpr int TILE32 = LP_SLAB * LDW;  // floats per FP32 tile
  static constexpr int TILEBF = 2 * NP * LP_SLAB;   // bf16 per split tile (hi and lo)
};

// Same organisation as the FP64 kernel: 8 waves, walker slot ws = wave / 2
// (four walkers per workgroup share the staged Lbar tile) and half h =
// wave % 2 owning the off-diagonal block pairs q with q % 2 == h and the
// diagonal blocks I with I % 2 == h.  T[I,J] and (T^T)[I,J] are accumulated
// from shared fragments, so each element's exchange partner is lane-local.
template <int MODE, int NB>
struct LpLds {
  static constexpr int TILE_BYTES = MODE == LO_FP32 ? LpCfg<NB>::TILE32 * 4 : LpCfg<NB>::TILEBF * 2;
};

// One work item: walkers 4 grp .. 4 grp + 3 against Cholesky vectors
// [chunk * gchunk, (chunk + 1) * gchunk).  sTileBase: 2 * TILE_BYTES bytes of
// LDS (16-byte aligned), sDiagBase: 8 * NDH * 256 float2, sK: 8 double2.
template <int MODE, int NB>
__device__ __forceinline__ void exchange_item(int Mp, int64_t X, int64_t nw, int64_t gchunk, int64_t chunk,
                                              int64_t grp, const void* __restrict__ lbar_lp,
                                              const void* __restrict__ theta_lp, double* __restrict__ partial,
                                              unsigned char* sTileBase, float2* sDiagBase, double2* sK) {
  using C = LpCfg<NB>;
  constexpr int NP = C::NP;
  constexpr int TILE_BYTES = LpLds<MODE, NB>::TILE_BYTES;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int ws = wv >> 1, h = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t w = 4 * grp + ws;
  const bool wok = w < nw;
  const int64_t wc = wok ? w : 0;
  const int64_t g0 = chunk * gchunk;
  const int64_t g1 = (g0 + gchunk < X) ? g0 + gchunk : X;
  const int nslab = Mp / LP_SLAB;
  const int64_t ntiles = (g1 > g0) ? (g1 - g0) * nslab : 0;

  f4 dRe[C::NPH > 0 ? C::NPH : 1], dIm[C::NPH > 0 ? C::NPH : 1];
  f4 tRe[C::NPH > 0 ? C::NPH : 1], tIm[C::NPH > 0 ? C::NPH : 1];
  f4 gRe[C::NDH], gIm[C::NDH];
  auto zero_acc = [&]() {
#pragma unroll
    for (int q = 0; q < C::NPH; ++q) { dRe[q] = f4zero(); dIm[q] = f4zero(); tRe[q] = f4zero(); tIm[q] = f4zero(); }
#pragma unroll
    for (int q = 0; q < C::NDH; ++q) { gRe[q] = f4zero(); gIm[q] = f4zero(); }
  };
  zero_acc();
  double accKr = 0.0, accKi = 0.0;

  // ---- staging of one Lbar tile (32 rows of r for one g) through registers
  constexpr int PER32 = (LP_SLAB * NP + 511) / 512;           // floats per thread
  constexpr int CHBF = C::TILEBF / 8;                        // 16-byte chunks per split tile
  float pre32[MODE == LO_FP32 ? PER32 : 1];
  bf8 prebf;
  auto load_tile = [&](int64_t t) {
    const int64_t g = g0 + t / nslab;
    const int slab = (int)(t % nslab);
    if constexpr (MODE == LO_FP32) {
      const float* src = (const float*)lbar_lp + ((size_t)g * Mp + LP_SLAB * slab) * NP;
#pragma unroll
      for (int q = 0; q < PER32; ++q) {
        const int e = tid + 512 * q;
        pre32[q] = e < LP_SLAB * NP ? src[e] : 0.0f;
      }
    } else {
      if (tid < CHBF) {
        const int p = tid / (NP * 4), rem = tid % (NP * 4), i = rem / 4, qq = rem % 4;
        const __bf16* src = (const __bf16*)lbar_lp + (((size_t)g * 2 + p) * NP + i) * Mp + LP_SLAB * slab + 8 * qq;
        prebf = *(const bf8*)src;
      }
    }
  };
  auto store_tile = [&](int buf) {
    if constexpr (MODE == LO_FP32) {
      float* d = (float*)(sTileBase + buf * TILE_BYTES);
#pragma unroll
      for (int q = 0; q < PER32; ++q) {
        const int e = tid + 512 * q;
        if (e < LP_SLAB * NP) d[(e / NP) * C::LDW + e % NP] = pre32[q];
      }
    } else {
      if (tid < CHBF) ((bf8*)(sTileBase + buf * TILE_BYTES))[tid] = prebf;   // [p][i][r] with 4 chunks of 8 r per row
    }
  };

  if (ntiles > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();

  // FP32: theta fragments of K-step ks (4 rows) loaded one step ahead
  const float2* th32 = (const float2*)theta_lp + (size_t)wc * Mp * NP;
  auto load_theta32 = [&](int r, float2 (&tf)[NB]) {
#pragma unroll
    for (int I = 0; I < NB; ++I) tf[I] = wok ? th32[(size_t)r * NP + 16 * I + lr] : make_float2(0.0f, 0.0f);
  };
  // BF16X3: the four planes of each orbital block for one 32-row slab
  const __bf16* thbf = (const __bf16*)theta_lp + (size_t)wc * 4 * NP * Mp;
  auto load_thetabf = [&](int slab, bf8 (&tb)[NB][4]) {
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const bf8 z = {};
        tb[I][p] = wok ? *(const bf8*)(thbf + ((size_t)p * NP + 16 * I + lr) * Mp + LP_SLAB * slab + 8 * lk) : z;
      }
  };

  auto mma32 = [&](const float* Lt, int s, const float2 (&tf)[NB]) {
    float Lf[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) Lf[I] = Lt[(4 * s + lk) * C::LDW + 16 * I + lr];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      if ((I & 1) == h) {
        gRe[I >> 1] = mfma_f32(Lf[I], tf[I].x, gRe[I >> 1]);
        gIm[I >> 1] = mfma_f32(Lf[I], tf[I].y, gIm[I >> 1]);
      }
    }
    int q = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int J = I + 1; J < NB; ++J, ++q) {
        if ((q & 1) == h) {
          dRe[q >> 1] = mfma_f32(Lf[I], tf[J].x, dRe[q >> 1]);
          dIm[q >> 1] = mfma_f32(Lf[I], tf[J].y, dIm[q >> 1]);
          tRe[q >> 1] = mfma_f32(tf[I].x, Lf[J], tRe[q >> 1]);
          tIm[q >> 1] = mfma_f32(tf[I].y, Lf[J], tIm[q >> 1]);
        }
      }
    }
  };
  // product of two split operands: a_hi b_hi + a_hi b_lo + a_lo b_hi
  auto mm3 = [&](bf8 ah, bf8 al, bf8 bh, bf8 bl, f4 c) {
    c = mfma_bf16(al, bh, c);
    c = mfma_bf16(ah, bl, c);
    return mfma_bf16(ah, bh, c);
  };
  auto mmabf = [&](const bf8* Lt, const bf8 (&tb)[NB][4]) {
    bf8 Lh[NB], Ll[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      Lh[I] = Lt[(16 * I + lr) * 4 + lk];
      Ll[I] = Lt[(NP + 16 * I + lr) * 4 + lk];
    }
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      if ((I & 1) == h) {
        gRe[I >> 1] = mm3(Lh[I], Ll[I], tb[I][0], tb[I][1], gRe[I >> 1]);
        gIm[I >> 1] = mm3(Lh[I], Ll[I], tb[I][2], tb[I][3], gIm[I >> 1]);
      }
    }
    int q = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int J = I + 1; J < NB; ++J, ++q) {
        if ((q & 1) == h) {
          dRe[q >> 1] = mm3(Lh[I], Ll[I], tb[J][0], tb[J][1], dRe[q >> 1]);
          dIm[q >> 1] = mm3(Lh[I], Ll[I], tb[J][2], tb[J][3], dIm[q >> 1]);
          tRe[q >> 1] = mm3(tb[I][0], tb[I][1], Lh[J], Ll[J], tRe[q >> 1]);
          tIm[q >> 1] = mm3(tb[I][2], tb[I][3], Lh[J], Ll[J], tIm[q >> 1]);
        }
      }
    }
  };

  float2 tfa[NB], tfb[NB];
  // split BF16: theta of the next tile's slab, loaded once the products of the
  // current tile are issued (a second register set two slabs ahead was slower)
  bf8 tba[NB][4];
  if (ntiles > 0) {
    if constexpr (MODE == LO_FP32) load_theta32(lk, tfa);
    else load_thetabf(0, tba);
  }

  // the end of tile t: the exchange sum of a finished g, then the barrier
  auto finish_tile = [&](int kt) {
    if (kt == nslab - 1) {
      // exchange sum of this g in FP64: lane-local pairs, diagonal blocks via LDS
      double xr = 0.0, xi = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < C::NPH; ++q2) {
        if (2 * q2 + h < C::NPAIR) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double a = dRe[q2][v], b = dIm[q2][v], c = tRe[q2][v], d = tIm[q2][v];
            xr += 2.0 * (a * c - b * d);
            xi += 2.0 * (a * d + b * c);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < C::NDH; ++q) {
        if (2 * q + h < NB) {
#pragma unroll
          for (int v = 0; v < 4; ++v) sDiagBase[(wv * C::NDH + q) * 256 + (4 * lk + v) * 16 + lr] = make_float2(gRe[q][v], gIm[q][v]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < C::NDH; ++q) {
        if (2 * q + h < NB) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float2 pv = sDiagBase[(wv * C::NDH + q) * 256 + lr * 16 + 4 * lk + v];
            const double a = gRe[q][v], b = gIm[q][v];
            xr += a * (double)pv.x - b * (double)pv.y;
            xi += a * (double)pv.y + b * (double)pv.x;
          }
        }
      }
      accKr += xr;
      accKi += xi;
      zero_acc();
    }
    __syncthreads();
  };

  if constexpr (MODE == LO_FP32) {
    for (int64_t t = 0; t < ntiles; ++t) {
      const int buf = (int)(t & 1);
      if (t + 1 < ntiles) load_tile(t + 1);
      const int kt = (int)(t % nslab);
      const int ktn = (kt + 1 == nslab) ? 0 : kt + 1;   // next tile's slab (same or next g)
      const float* Lt = (const float*)(sTileBase + buf * TILE_BYTES);
      const int rb = LP_SLAB * kt + lk;
#pragma unroll
      for (int s = 0; s < LP_SLAB / 4; s += 2) {
        load_theta32(rb + 4 * (s + 1), tfb);
        mma32(Lt, s, tfa);
        const int rn = (s + 2 < LP_SLAB / 4) ? rb + 4 * (s + 2) : LP_SLAB * ktn + lk;
        load_theta32(rn, tfa);
        mma32(Lt, s + 1, tfb);
      }
      if (t + 1 < ntiles) store_tile(buf ^ 1);
      finish_tile(kt);
    }
  } else {
    for (int64_t t = 0; t < ntiles; ++t) {
      const int buf = (int)(t & 1);
      if (t + 1 < ntiles) load_tile(t + 1);
      const int kt = (int)(t % nslab);
      mmabf((const bf8*)(sTileBase + buf * TILE_BYTES), tba);
      load_thetabf((kt + 1 == nslab) ? 0 : kt + 1, tba);
      if (t + 1 < ntiles) store_tile(buf ^ 1);
      finish_tile(kt);
    }
  }

  accKr = wave_sum_lane0(accKr);
  accKi = wave_sum_lane0(accKi);
  if (lane == 0) sK[wv] = make_double2(accKr, accKi);
  __syncthreads();
  if (wok && h == 0 && lane == 0) {
    const double2 k0 = sK[wv], k1 = sK[wv + 1];
    double* out = partial + ((size_t)chunk * nw + w) * 4;
    out[0] = 0.0;
    out[1] = 0.0;
    out[2] = -(k0.x + k1.x);
    out[3] = -(k0.y + k1.y);
  }
}

template <int MODE, int NB>
__global__ __launch_bounds__(512, (MODE == LO_FP32 && NB <= 4) ? 2 : 1) void exchange_lp_kernel(
    int Mp, int64_t X, int64_t nw, int64_t gchunk, int nchunk, int64_t ngrp, const void* __restrict__ lbar_lp,
    const void* __restrict__ theta_lp, double* __restrict__ partial) {
  using C = LpCfg<NB>;
  __shared__ __attribute__((aligned(16))) unsigned char sTile[2 * LpLds<MODE, NB>::TILE_BYTES];
  __shared__ float2 sDiag[8 * C::NDH * 256];
  __shared__ double2 sK[8];
  int64_t chunk, grp;
  {
    const int64_t b = blockIdx.x;
    const int xcd = (int)(b & 7);
    const int64_t slot = b >> 3;
    const int64_t lin = slot * 8 + xcd;
    if (nchunk % 8 == 0 || 8 % nchunk == 0) {
      const int per_xcd_chunks = nchunk >= 8 ? nchunk / 8 : 1;
      const int xcds_per_chunk = nchunk >= 8 ? 1 : 8 / nchunk;
      chunk = (int64_t)(xcd / xcds_per_chunk) * per_xcd_chunks + (slot % per_xcd_chunks);
      grp = (slot / per_xcd_chunks) * xcds_per_chunk + (xcd % xcds_per_chunk);
    } else {
      chunk = lin % nchunk;
      grp = lin / nchunk;
    }
    if (grp >= ngrp || chunk >= nchunk) return;
  }
  exchange_item<MODE, NB>(Mp, X, nw, gchunk, chunk, grp, lbar_lp, theta_lp, partial, sTile, sDiag, sK);
}

// ---------------------------------------------------------------------------
// Several systems in one persistent launch (FP32): work items of all systems
// in one list, taken in order from an atomic counter by the resident
// workgroups until the list is exhausted; every item writes its own partial
// slot, so the result does not depend on which workgroup took it.
// ---------------------------------------------------------------------------
// Item of a system with NB orbital blocks, dispatched at compile time over
// NB = 1 .. NBMAX (the plan's largest), so the kernel holds the registers of
// the largest variant the plan uses and no more.
template <int NB, int NBMAX>
__device__ __forceinline__ void batched_item(const LpSys& d, int64_t chunk, int64_t grp, unsigned char* sTile,
                                             float2* sDiag, double2* sK) {
  static_assert(LpLds<LO_FP32, NB>::TILE_BYTES <= LpLds<LO_FP32, NBMAX>::TILE_BYTES &&
                LpCfg<NB>::NDH <= LpCfg<NBMAX>::NDH, "LDS sized for NBMAX");
  if constexpr (NB == NBMAX) {
    exchange_item<LO_FP32, NB>(d.Mp, d.X, d.nw, d.gchunk, chunk, grp, d.lb, d.tb, d.partial, sTile, sDiag, sK);
  } else {
    if (d.nb == NB)
      exchange_item<LO_FP32, NB>(d.Mp, d.X, d.nw, d.gchunk, chunk, grp, d.lb, d.tb, d.partial, sTile, sDiag, sK);
    else
      batched_item<NB + 1, NBMAX>(d, chunk, grp, sTile, sDiag, sK);
  }
}

template <int NBMAX>
__global__ __launch_bounds__(512, 1) void exchange_batched_kernel(int nsys, const LpSys* __restrict__ sys,
                                                                  int64_t nitems, unsigned* __restrict__ counter) {
  __shared__ __attribute__((aligned(16))) unsigned char sTile[2 * LpLds<LO_FP32, NBMAX>::TILE_BYTES];
  __shared__ float2 sDiag[8 * LpCfg<NBMAX>::NDH * 256];
  __shared__ double2 sK[8];
  __shared__ int64_t sItem;
  for (;;) {
    if (threadIdx.x == 0) sItem = (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t it = sItem;
    __syncthreads();
    if (it >= nitems) break;
    int s = 0;
    while (s + 1 < nsys && sys[s + 1].item0 <= it) ++s;
    const LpSys d = sys[s];
    const int64_t local = it - d.item0;
    batched_item<1, NBMAX>(d, local % d.nchunk, local / d.nchunk, sTile, sDiag, sK);
    __syncthreads();
  }
}

__global__ void batch_counter_reset_kernel(unsigned* counter) { *counter = 0u; }

// ---------------------------------------------------------------------------
// Coulomb traces in FP64: C[w][g] = sum_k theta_w[k] Lbar_g[k], k = (r, i)
// flattened (both operands are contiguous in k).  Workgroup tile: 16 walkers
// x 64 Cholesky vectors x one split of k; wave q owns vectors 16q .. 16q+15.
// ---------------------------------------------------------------------------
constexpr int CT_KS = 32;   // k per staged slab

__global__ __launch_bounds__(256) void coulomb_trace_kernel(int64_t K, int64_t X, int64_t nw, int64_t kper,
                                                            const double2* __restrict__ theta,
                                                            const double* __restrict__ lbar,
                                                            double2* __restrict__ cpart) {
  __shared__ double2 sT[2][16][CT_KS + 1];
  __shared__ double sL[2][64][CT_KS + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t w0 = 16 * (int64_t)blockIdx.x;
  const int64_t gb = 64 * (int64_t)blockIdx.y;
  const int64_t ks = blockIdx.z;
  const int64_t k0 = ks * kper;
  const int64_t k1 = (k0 + kper < K) ? k0 + kper : K;
  const int nsl = (int)((k1 - k0 + CT_KS - 1) / CT_KS);

  double2 pt[2];
  double pl[8];
  auto load = [&](int c) {
    const int64_t kb = k0 + (int64_t)CT_KS * c;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q, wl = e / CT_KS, kk = e % CT_KS;
      const int64_t w = w0 + wl, k = kb + kk;
      pt[q] = (w < nw && k < k1) ? theta[(size_t)w * K + k] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q, gl = e / CT_KS, kk = e % CT_KS;
      const int64_t g = gb + gl, k = kb + kk;
      pl[q] = (g < X && k < k1) ? lbar[(size_t)g * K + k] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      sT[buf][e / CT_KS][e % CT_KS] = pt[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      sL[buf][e / CT_KS][e % CT_KS] = pl[q];
    }
  };
  d4 accR = d4zero(), accI = d4zero();
  if (nsl > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int c = 0; c < nsl; ++c) {
    const int buf = c & 1;
    if (c + 1 < nsl) load(c + 1);
#pragma unroll
    for (int s = 0; s < CT_KS / 4; ++s) {
      const double2 a = sT[buf][lr][4 * s + lk];
      const double b = sL[buf][16 * wv + lr][4 * s + lk];
      accR = mfma16(a.x, b, accR);
      accI = mfma16(a.y, b, accI);
    }
    if (c + 1 < nsl) store(buf ^ 1);
    __syncthreads();
  }
  // D[row][col]: row = walker 4v + lk, col = vector 16 wv + lr
  const int64_t g = gb + 16 * wv + lr;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t w = w0 + 4 * v + lk;
    if (w < nw && g < X) cpart[((size_t)ks * nw + w) * X + g] = make_double2(accR[v], accI[v]);
  }
}

// E_J[w] = 2 sum_g (sum_s cpart[s][w][g])^2 in a fixed order; one wave per walker.
__global__ __launch_bounds__(256) void coulomb_finish_kernel(int64_t X, int64_t nw, int nsplit,
                                                             const double2* __restrict__ cpart,
                                                             double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nw) return;
  double jr = 0.0, ji = 0.0;
  for (int64_t g = lane; g < X; g += 64) {
    double cr = 0.0, ci = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      const double2 c = cpart[((size_t)s * nw + w) * X + g];
      cr += c.x;
      ci += c.y;
    }
    jr += cr * cr - ci * ci;
    ji += 2.0 * cr * ci;
  }
  jr = wave_sum_lane0(jr);
  ji = wave_sum_lane0(ji);
  if (lane == 0) {
    double* o = out + (size_t)w * 4;
    o[0] = 2.0 * jr;
    o[1] = 2.0 * ji;
    o[2] = 0.0;
    o[3] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int lp_nb(int n) { return (n + 15) / 16; }

size_t lp_theta_bytes(int precision, int M, int n, int64_t nw) {
  const size_t Mp = (size_t)lp_padded_m(M), NP = 16 * (size_t)lp_nb(n);
  return precision == LO_FP32 ? nw * Mp * NP * 8 : nw * 4 * NP * Mp * 2;
}

hipError_t launch_lp_convert_theta(hipStream_t s, int precision, int M, int n, int64_t nw, const double* theta,
                                   void* out) {
  if (nw <= 0) return hipSuccess;
  const int Mp = lp_padded_m(M), NP = 16 * lp_nb(n);
  const dim3 gt((unsigned)(Mp / LP_SLAB), (unsigned)nw);
  if (precision == LO_FP32)
    hipLaunchKernelGGL(lp_convert_complex_kernel<LO_FP32>, gt, dim3(256), 0, s, M, n, Mp, NP,
                       (const double2*)theta, out);
  else
    hipLaunchKernelGGL(lp_convert_complex_kernel<LO_BF16X3>, gt, dim3(256), 0, s, M, n, Mp, NP,
                       (const double2*)theta, out);
  return hipGetLastError();
}

static int ct_nsplit(int64_t K, int64_t X, int64_t nw) {
  const int64_t tiles = ((nw + 15) / 16) * ((X + 63) / 64);
  int s = 1;
  while (tiles * s < 1024 && K / (s * 2) >= 4 * CT_KS) s *= 2;
  return s;
}

size_t lp_lbar_bytes(int precision, int M, int n, int64_t X);
size_t coulomb_cpart_bytes(int M, int n, int64_t X, int64_t nw);

size_t full_lp_workspace(int precision, int M, int n, int64_t X, int64_t nw) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(lp_lbar_bytes(precision, M, n, X)) + al(lp_theta_bytes(precision, M, n, nw)) +
         al(coulomb_cpart_bytes(M, n, X, nw));
}

template <int MODE, int NB>
static hipError_t launch_exchange_lp(hipStream_t st, int Mp, int64_t X, int64_t nw, const void* lb, const void* tb,
                                     double* partial, int nchunk) {
  const int64_t ngrp = (nw + 3) / 4;
  const int64_t gchunk = (X + nchunk - 1) / nchunk;
  int64_t grid = ngrp * nchunk;
  if (nchunk % 8 == 0 || 8 % nchunk == 0) {
    const int per_xcd_chunks = nchunk >= 8 ? nchunk / 8 : 1;
    const int xcds_per_chunk = nchunk >= 8 ? 1 : 8 / nchunk;
    grid = 8 * (int64_t)per_xcd_chunks * ((ngrp + xcds_per_chunk - 1) / xcds_per_chunk);
  }
  hipLaunchKernelGGL((exchange_lp_kernel<MODE, NB>), dim3((unsigned)grid), dim3(512), 0, st, Mp, X, nw, gchunk,
                     nchunk, ngrp, lb, tb, partial);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_exchange_mode(hipStream_t st, int nb, int Mp, int64_t X, int64_t nw, const void* lb,
                                       const void* tb, double* partial, int nchunk) {
  switch (nb) {
    case 1: return launch_exchange_lp<MODE, 1>(st, Mp, X, nw, lb, tb, partial, nchunk);
    case 2: return launch_exchange_lp<MODE, 2>(st, Mp, X, nw, lb, tb, partial, nchunk);
    case 3: return launch_exchange_lp<MODE, 3>(st, Mp, X, nw, lb, tb, partial, nchunk);
    case 4: return launch_exchange_lp<MODE, 4>(st, Mp, X, nw, lb, tb, partial, nchunk);
    default:
      // the split-BF16 fragments of more than 64 orbitals do not fit the
      // register file; the host rejects that case
      if constexpr (MODE == LO_FP32) {
        if (nb == 5) return launch_exchange_lp<MODE, 5>(st, Mp, X, nw, lb, tb, partial, nchunk);
        return launch_exchange_lp<MODE, 6>(st, Mp, X, nw, lb, tb, partial, nchunk);
      }
      return hipErrorInvalidValue;
  }
}

int lp_orbital_blocks(int n) { return lp_nb(n); }

size_t lp_lbar_bytes(int precision, int M, int n, int64_t X) {
  const size_t Mp = (size_t)lp_padded_m(M), NP = 16 * (size_t)lp_nb(n);
  return precision == LO_FP32 ? X * Mp * NP * 4 : X * 2 * NP * Mp * 2;
}

size_t coulomb_cpart_bytes(int M, int n, int64_t X, int64_t nw) {
  return (size_t)ct_nsplit((int64_t)M * n, X, nw) * nw * X * 16;
}

hipError_t launch_lp_convert_operands(hipStream_t s, int precision, int M, int n, int64_t X, int64_t nw,
                                      const double* lbar, const double* theta, void* lb, void* tb) {
  const int Mp = lp_padded_m(M), NP = 16 * lp_nb(n);
  const dim3 gl((unsigned)(Mp / LP_SLAB), (unsigned)X), gt((unsigned)(Mp / LP_SLAB), (unsigned)nw);
  if (precision == LO_FP32) {
    hipLaunchKernelGGL(lp_convert_real_kernel<LO_FP32>, gl, dim3(256), 0, s, M, n, Mp, NP, lbar, lb);
    hipLaunchKernelGGL(lp_convert_complex_kernel<LO_FP32>, gt, dim3(256), 0, s, M, n, Mp, NP,
                       (const double2*)theta, tb);
  } else {
    hipLaunchKernelGGL(lp_convert_real_kernel<LO_BF16X3>, gl, dim3(256), 0, s, M, n, Mp, NP, lbar, lb);
    hipLaunchKernelGGL(lp_convert_complex_kernel<LO_BF16X3>, gt, dim3(256), 0, s, M, n, Mp, NP,
                       (const double2*)theta, tb);
  }
  return hipGetLastError();
}

hipError_t launch_coulomb_fp64(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* theta,
                               const double* lbar, void* cpart_ws, double* out_row, const ProfHook* prof) {
  const int64_t K = (int64_t)M * n;
  const int nsplit = ct_nsplit(K, X, nw);
  const int64_t kper = ((K + nsplit - 1) / nsplit + CT_KS - 1) / CT_KS * CT_KS;
  double2* cpart = (double2*)cpart_ws;
  prof_mark(prof, "coulomb_trace_kernel");
  hipLaunchKernelGGL(coulomb_trace_kernel, dim3((unsigned)((nw + 15) / 16), (unsigned)((X + 63) / 64), nsplit),
                     dim3(256), 0, s, K, X, nw, kper, (const double2*)theta, lbar, cpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_mark(prof, "coulomb_finish_kernel");
  hipLaunchKernelGGL(coulomb_finish_kernel, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, X, nw, nsplit, cpart,
                     out_row);
  return hipGetLastError();
}

hipError_t launch_energy_full_lp(hipStream_t s, int precision, int M, int n, int64_t X, int64_t nw,
                                 const double* lbar, const double* theta, void* work, double* partial, int nchunk,
                                 const ProfHook* prof) {
  if (nw <= 0 || X <= 0) return hipSuccess;
  const int Mp = lp_padded_m(M), nb = lp_nb(n);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t lbytes = lp_lbar_bytes(precision, M, n, X);
  const size_t tbytes = lp_theta_bytes(precision, M, n, nw);
  char* base = (char*)work;
  void* lb = base;
  void* tb = base + al(lbytes);
  void* cpart = base + al(lbytes) + al(tbytes);
  prof_mark(prof, "lp_convert_kernel");
  hipError_t e = launch_lp_convert_operands(s, precision, M, n, X, nw, lbar, theta, lb, tb);
  if (e != hipSuccess) return e;
  prof_mark(prof, "exchange_lp_kernel");
  e = precision == LO_FP32 ? launch_exchange_mode<LO_FP32>(s, nb, Mp, X, nw, lb, tb, partial, nchunk)
                           : launch_exchange_mode<LO_BF16X3>(s, nb, Mp, X, nw, lb, tb, partial, nchunk);
  if (e != hipSuccess) return e;
  return launch_coulomb_fp64(s, M, n, X, nw, theta, lbar, cpart, partial + (size_t)nchunk * nw * 4, prof);
}

hipError_t launch_exchange_batched(hipStream_t s, int nsys, const LpSys* d_sys, int64_t nitems, unsigned* counter,
                                   int grid, int nbmax) {
  if (nbmax < 1 || nbmax > 6) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_counter_reset_kernel, dim3(1), dim3(1), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nitems <= 0) return e;
  const dim3 g((unsigned)grid), b(512);
  switch (nbmax) {
    case 1: hipLaunchKernelGGL(exchange_batched_kernel<1>, g, b, 0, s, nsys, d_sys, nitems, counter); break;
    case 2: hipLaunchKernelGGL(exchange_batched_kernel<2>, g, b, 0, s, nsys, d_sys, nitems, counter); break;
    case 3: hipLaunchKernelGGL(exchange_batched_kernel<3>, g, b, 0, s, nsys, d_sys, nitems, counter); break;
    case 4: hipLaunchKernelGGL(exchange_batched_kernel<4>, g, b, 0, s, nsys, d_sys, nitems, counter); break;
    case 5: hipLaunchKernelGGL(exchange_batched_kernel<5>, g, b, 0, s, nsys, d_sys, nitems, counter); break;
    default: hipLaunchKernelGGL(exchange_batched_kernel<6>, g, b, 0, s, nsys, d_sys, nitems, counter); break;
  }
  return hipGetLastError();
}

}  // namespace lofqmc
