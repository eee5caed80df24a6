// LO route (Sec. 2.3.2, Eq. 22-23), pass 1 in reduced precision: the
// products (factor rows) x Q_o run on FP32 MFMA from FP32-rounded operands, or
// on BF16 MFMA from split operands x = x_hi + x_lo (products hi*hi + hi*lo +
// lo*hi), FP32 accumulation in both cases.  The projections are widened to
// FP64 when written, and pass 2 (the pair dot products and every sum) is the
// FP64 kernel.  Tiles, work units and the XCD order are those of the FP64
// pass 1: 64 output rows of one orbital x 64 walkers, eight waves, wave
// (q, h) owning row block q against walker half h.
//
// Operand layouts (written by the rewrite kernels, M padded to Mp, a multiple
// of 32, with zeros):
//   FP32   : factor rows [rows][Mp] float;     theta [nw][Mp][NP] float2
//   BF16X3 : factor rows [rows][2][Mp] (hi, lo); theta [nw][4][NP][Mp]
//            (re_hi, re_lo, im_hi, im_lo)
#include "common.h"
#include "kernels.h"
#include "lofqmc.h"

namespace lofqmc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Same operand conventions as the reduced-precision full route: lane l gives
// A[l % 16][k], B[k][l % 16] (k = l / 16 for FP32, 8 (l / 16) + t for BF16),
// accumulator element v of lane l is D[4 (l / 16) + v][l % 16].
__device__ __forceinline__ f4 lo_mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 lo_mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// factor rows FP64 [rows][M] -> FP32 [rows][Mp] and split BF16 [rows][2][Mp]
__global__ __launch_bounds__(256) void factor_rows_lp_kernel(int M, int Mp, const double* __restrict__ rows,
                                                             float* __restrict__ r32, __bf16* __restrict__ rbf) {
  const int64_t row = blockIdx.x;
  for (int r = threadIdx.x; r < Mp; r += 256) {
    const double x = r < M ? rows[(size_t)row * M + r] : 0.0;
    const float xf = (float)x;
    const __bf16 hi = (__bf16)xf;
    const __bf16 lo = (__bf16)(xf - (float)hi);
    r32[(size_t)row * Mp + r] = xf;
    rbf[((size_t)row * 2) * Mp + r] = hi;
    rbf[((size_t)row * 2 + 1) * Mp + r] = lo;
  }
}

hipError_t launch_factor_rows_lp(hipStream_t s, int M, int64_t nrows, const double* rows, float* r32,
                                 __bf16* rbf) {
  if (nrows <= 0) return hipSuccess;
  const int Mp = lp_padded_m(M);
  hipLaunchKernelGGL(factor_rows_lp_kernel, dim3((unsigned)nrows), dim3(256), 0, s, M, Mp, rows, r32, rbf);
  return hipGetLastError();
}

constexpr int LP1_ROWS = 64;
constexpr int LP1_WT = 64;

template <int MODE>
__global__ __launch_bounds__(512, 2) void lo_pass1_lp_kernel(int Mp, int NP, int64_t nw, const void* __restrict__ rows_lp,
                                                             const int* __restrict__ rowidx,
                                                             const int* __restrict__ tile_orb,
                                                             const int* __restrict__ tile_row0,
                                                             const int* __restrict__ tile_nrows,
                                                             const int* __restrict__ blk, int nblk, int tmax,
                                                             const void* __restrict__ theta_lp,
                                                             double2* __restrict__ qbar, int nwt) {
  // FP32: A [64][16 + 1] float, B [16][64] float2 per buffer (16-row slabs)
  // BF16: A [2][64][32] bf16, B [4][64][32] bf16 per buffer (32-row slabs)
  constexpr int A_BYTES = MODE == LO_FP32 ? LP1_ROWS * 17 * 4 : 2 * LP1_ROWS * 32 * 2;
  constexpr int B_BYTES = MODE == LO_FP32 ? 16 * LP1_WT * 8 : 4 * LP1_WT * 32 * 2;
  __shared__ __attribute__((aligned(16))) unsigned char sA[2][A_BYTES];
  __shared__ __attribute__((aligned(16))) unsigned char sB[2][B_BYTES];
  int t;
  int64_t w0;
  {
    const int xcd = blockIdx.x & 7;
    const int slot = blockIdx.x >> 3;
    const int64_t u = 8 * (int64_t)(slot / tmax) + xcd;
    if (u >= (int64_t)nblk * nwt) return;
    const int b = (int)(u / nwt);
    t = blk[b] + slot % tmax;
    if (t >= blk[b + 1]) return;
    w0 = (u % nwt) * LP1_WT;
  }
  const int o = tile_orb[t];
  const int row0 = tile_row0[t];
  const int nrows = tile_nrows[t];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int q = wv & 3, hw = wv >> 2;
  const int lr = lane & 15, lk = lane >> 4;
  const bool active = 16 * q < nrows;
  constexpr int SLAB = MODE == LO_FP32 ? 16 : 32;
  const int nslab = Mp / SLAB;

  // this thread's staged factor row(s), resolved once
  const int arow_i = MODE == LO_FP32 ? (tid >> 3) : (tid & 255) >> 2;   // row within the tile
  const int64_t arow = arow_i < nrows ? rowidx[row0 + arow_i] : -1;

  f4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  // FP32 staging: A 64 rows x 16 r = 1024 floats (2 per thread), B 16 r x 64 w
  // float2 (2 per thread).  BF16 staging: A 64 rows x 2 planes x 4 chunks of 8
  // r (1 chunk per thread), B 64 w x 4 planes x 4 chunks (2 per thread).
  float pa32[2];
  float2 pb32[2];
  bf8 pabf;
  bf8 pbbf[2];
  auto load = [&](int c) {
    if constexpr (MODE == LO_FP32) {
      const float* R = (const float*)rows_lp;
      const float2* T = (const float2*)theta_lp;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int r = 16 * c + 2 * (tid & 7) + p;
        pa32[p] = arow >= 0 ? R[(size_t)arow * Mp + r] : 0.0f;
      }
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int e = tid + 512 * p, rr = e / LP1_WT, ww = e % LP1_WT;
        const int64_t w = w0 + ww;
        pb32[p] = w < nw ? T[((size_t)w * Mp + 16 * c + rr) * NP + o] : make_float2(0.0f, 0.0f);
      }
    } else {
      const __bf16* R = (const __bf16*)rows_lp;
      const __bf16* T = (const __bf16*)theta_lp;
      const int pl = tid >> 8, ch = tid & 3;
      const bf8 z = {};
      pabf = arow >= 0 ? *(const bf8*)(R + ((size_t)arow * 2 + pl) * Mp + 32 * c + 8 * ch) : z;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int e = tid + 512 * p;             // (w, plane, chunk) = (e / 16, (e / 4) % 4, e % 4)
        const int ww = e >> 4, pq = (e >> 2) & 3, cq = e & 3;
        const int64_t w = w0 + ww;
        pbbf[p] = w < nw ? *(const bf8*)(T + (((size_t)w * 4 + pq) * NP + o) * Mp + 32 * c + 8 * cq) : z;
      }
    }
  };
  auto store = [&](int buf) {
    if constexpr (MODE == LO_FP32) {
      float* A = (float*)sA[buf];
      float2* B = (float2*)sB[buf];
#pragma unroll
      for (int p = 0; p < 2; ++p) A[arow_i * 17 + 2 * (tid & 7) + p] = pa32[p];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int e = tid + 512 * p;
        B[(e / LP1_WT) * LP1_WT + e % LP1_WT] = pb32[p];
      }
    } else {
      bf8* A = (bf8*)sA[buf];   // [plane][row][chunk]
      bf8* B = (bf8*)sB[buf];   // [plane][w][chunk]
      const int pl = tid >> 8, ch = tid & 3;
      A[(pl * LP1_ROWS + arow_i) * 4 + ch] = pabf;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int e = tid + 512 * p;
        const int ww = e >> 4, pq = (e >> 2) & 3, cq = e & 3;
        B[(pq * LP1_WT + ww) * 4 + cq] = pbbf[p];
      }
    }
  };

  load(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nslab; ++c) {
    const int buf = c & 1;
    if (c + 1 < nslab) load(c + 1);
    if (active) {
      if constexpr (MODE == LO_FP32) {
        const float* A = (const float*)sA[buf];
        const float2* B = (const float2*)sB[buf];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int rr = 4 * s4 + lk;
          const float a = A[(16 * q + lr) * 17 + rr];
          const float2 b0 = B[rr * LP1_WT + 32 * hw + lr];
          const float2 b1 = B[rr * LP1_WT + 32 * hw + 16 + lr];
          acc[0] = lo_mfma_f32(a, b0.x, acc[0]);
          acc[1] = lo_mfma_f32(a, b0.y, acc[1]);
          acc[2] = lo_mfma_f32(a, b1.x, acc[2]);
          acc[3] = lo_mfma_f32(a, b1.y, acc[3]);
        }
      } else {
        const bf8* A = (const bf8*)sA[buf];
        const bf8* B = (const bf8*)sB[buf];
        const bf8 ah = A[(0 * LP1_ROWS + 16 * q + lr) * 4 + lk];
        const bf8 al = A[(1 * LP1_ROWS + 16 * q + lr) * 4 + lk];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ww = 32 * hw + 16 * h + lr;
#pragma unroll
          for (int part = 0; part < 2; ++part) {
            const bf8 bh = B[((2 * part) * LP1_WT + ww) * 4 + lk];
            const bf8 bl = B[((2 * part + 1) * LP1_WT + ww) * 4 + lk];
            f4 a4 = acc[2 * h + part];
            a4 = lo_mfma_bf16(al, bh, a4);
            a4 = lo_mfma_bf16(ah, bl, a4);
            acc[2 * h + part] = lo_mfma_bf16(ah, bh, a4);
          }
        }
      }
    }
    if (c + 1 < nslab) store(buf ^ 1);
    __syncthreads();
  }
  // D[row][walker]: lane holds rows 4 lk + v of the block, walker 16 half + lr
  if (active) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t w = w0 + 32 * hw + 16 * h + lr;
      if (w < nw) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int lrow = 16 * q + 4 * lk + v;
          if (lrow < nrows)
            qbar[(size_t)(row0 + lrow) * nw + w] =
                make_double2((double)acc[2 * h][v], (double)acc[2 * h + 1][v]);
        }
      }
    }
  }
}

int lo_lp_tile_rows() { return LP1_ROWS; }

hipError_t launch_lo_pass1_lp(hipStream_t s, int precision, int M, int n, int64_t nw, int ntiles,
                              const void* rows_lp, const int* rowidx, const int* tiles, const int* blk, int nblk,
                              int tmax, const void* theta_lp, double* qbar) {
  if (nw <= 0 || ntiles <= 0) return hipSuccess;
  const int Mp = lp_padded_m(M);
  const int NP = 16 * ((n + 15) / 16);
  const int nwt = (int)((nw + LP1_WT - 1) / LP1_WT);
  const int64_t units = (int64_t)nblk * nwt;
  const int64_t grid = (int64_t)8 * ((units + 7) / 8) * tmax;
  if (precision == LO_FP32)
    hipLaunchKernelGGL(lo_pass1_lp_kernel<LO_FP32>, dim3((unsigned)grid), dim3(512), 0, s, Mp, NP, nw, rows_lp,
                       rowidx, tiles, tiles + ntiles, tiles + 2 * ntiles, blk, nblk, tmax, theta_lp,
                       (double2*)qbar, nwt);
  else
    hipLaunchKernelGGL(lo_pass1_lp_kernel<LO_BF16X3>, dim3((unsigned)grid), dim3(512), 0, s, Mp, NP, nw, rows_lp,
                       rowidx, tiles, tiles + ntiles, tiles + 2 * ntiles, blk, nblk, tmax, theta_lp,
                       (double2*)qbar, nwt);
  return hipGetLastError();
}

}  // namespace lofqmc
