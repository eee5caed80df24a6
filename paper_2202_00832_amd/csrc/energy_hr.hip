// Two-body energy by the half-rotated ERI route (Sec. 2.2, Eq. 17), FP64.
//
// Y^[ij]_rs = sum_g Lbar^g_ri Lbar^g_sj is stored for the pairs i <= j
// (Y^[ji] is its transpose), row-major [pair][r][s].  Per walker
//   J_ij = theta_i . (Y^[ij] theta_j),   X_ij = theta_j . (Y^[ij] theta_i)
// (complex, bilinear), E_J = 2 sum w_ij J_ij, E_K = -sum w_ij X_ij with weight 1
// for i = j and 2 for i < j.
//
// One workgroup per (pair, 32-walker tile), pairs fastest in the grid, eight
// waves: wave (g, h) forms rows 16 g .. 16 g + 15 of a 64-row chunk of
// Y^[ij] theta_j (h = 0) or
// Y^[ij] theta_i (h = 1) on the FP64 4x4x4 MFMA (16 accumulators per lane),
// with 16-column slabs of Y and the two theta columns staged in LDS
// (double-buffered).  The product never leaves registers: each chunk is dotted
// with theta_i (h = 0) or theta_j (h = 1) at once, the lanes and waves are
// summed in a fixed order, and the pair's weighted (E_J, E_K) for each walker
// is written to its own partial slot; the slots are summed over pairs in a
// fixed order by the partial reduction of the full route.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

constexpr int HR_ROWS = 64;
constexpr int HR_WT = 32;

__global__ __launch_bounds__(512, 2) void hr_energy_kernel(int M, int64_t nw, int npairs, const double* __restrict__ Y,
                                                           const int* __restrict__ pairs,
                                                           const double2* __restrict__ theta, int64_t so, int64_t sr,
                                                           int64_t sw, double* __restrict__ partial) {
  __shared__ double sA[2][HR_ROWS][17];          // [row][s], padded against bank conflicts
  __shared__ double2 sB[2][2][16][HR_WT];        // [vector h][s][walker]
  __shared__ double2 sRed[2][4][HR_WT];          // [h][row group][walker]
  // pairs vary fastest: the workgroups in flight share one walker tile, whose
  // theta columns then stay in the caches while the pair blocks stream
  const int p = (int)(blockIdx.x % npairs);
  const int64_t w0 = (int64_t)(blockIdx.x / npairs) * HR_WT;
  const int i = pairs[2 * p], j = pairs[2 * p + 1];
  const double* Yp = Y + (size_t)p * M * M;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int g = wv & 3, h = wv >> 2;
  const int lr = lane & 15, lk = lane >> 4;
  const int od = h == 0 ? i : j;   // orbital the product is dotted with

  // staging of slab c of chunk r0: A = 64 rows x 16 s, B = 2 x 16 s x 32 walkers
  double pa[2];
  double2 pb[2];
  auto load = [&](int r0, int c) {
    const int s0 = 16 * c;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 512 * q;
      const int row = r0 + (e >> 4), s = s0 + (e & 15);
      pa[q] = (row < M && s < M) ? Yp[(size_t)row * M + s] : 0.0;
      const int hv = e >> 9, rem = e & 511;
      const int sb = s0 + (rem >> 5);
      const int64_t w = w0 + (rem & 31);
      const int o = hv == 0 ? j : i;
      pb[q] = (sb < M && w < nw) ? theta[o * so + sb * sr + w * sw] : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 512 * q;
      sA[buf][e >> 4][e & 15] = pa[q];
      const int hv = e >> 9, rem = e & 511;
      sB[buf][hv][rem >> 5][rem & 31] = pb[q];
    }
  };

  double2 dot[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};   // walkers lr, 16 + lr
  const int nslab = (M + 15) / 16;
  for (int r0 = 0; r0 < M; r0 += HR_ROWS) {
    // acc[q][c]: rows r0 + 16 g + 4 q + lk, walker block c / 2, part c % 2
    double acc[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[q][c] = 0.0;
    load(r0, 0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nslab; ++c) {
      const int buf = c & 1;
      if (c + 1 < nslab) load(r0, c + 1);
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int ss = 4 * s4 + lk;
        const double2 b0 = sB[buf][h][ss][lr];
        const double2 b1 = sB[buf][h][ss][16 + lr];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double a = sA[buf][16 * g + 4 * q + (lane & 3)][ss];
          acc[q][0] = mfma4(a, b0.x, acc[q][0]);
          acc[q][1] = mfma4(a, b0.y, acc[q][1]);
          acc[q][2] = mfma4(a, b1.x, acc[q][2]);
          acc[q][3] = mfma4(a, b1.y, acc[q][3]);
        }
      }
      if (c + 1 < nslab) store(buf ^ 1);
      __syncthreads();
    }
    // dot the chunk with the other orbital's theta
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int64_t w = w0 + 16 * hh + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + 16 * g + 4 * q + lk;
        if (r < M && w < nw) {
          const double2 t = theta[od * so + r * sr + w * sw];
          const double2 d = make_double2(acc[q][2 * hh], acc[q][2 * hh + 1]);
          dot[hh] = make_double2(dot[hh].x + d.x * t.x - d.y * t.y, dot[hh].y + d.x * t.y + d.y * t.x);
        }
      }
    }
  }
  // sum over the four row offsets lk of each walker (fixed shuffle order), then
  // over the four row groups
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      dot[hh].x += __shfl_xor(dot[hh].x, off, 64);
      dot[hh].y += __shfl_xor(dot[hh].y, off, 64);
    }
  }
  if (lk == 0) {
    sRed[h][g][lr] = dot[0];
    sRed[h][g][16 + lr] = dot[1];
  }
  __syncthreads();
  if (tid < HR_WT) {
    const int64_t w = w0 + tid;
    if (w < nw) {
      double2 J = make_double2(0.0, 0.0), X = make_double2(0.0, 0.0);
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        J.x += sRed[0][gg][tid].x;
        J.y += sRed[0][gg][tid].y;
        X.x += sRed[1][gg][tid].x;
        X.y += sRed[1][gg][tid].y;
      }
      const double wt = i == j ? 1.0 : 2.0;
      reinterpret_cast<double4*>(partial)[(size_t)p * nw + w] =
          make_double4(2.0 * wt * J.x, 2.0 * wt * J.y, -wt * X.x, -wt * X.y);
    }
  }
}

hipError_t launch_hr_energy(hipStream_t s, int M, int n, int64_t nw, int npairs, const double* Y, const int* pairs,
                            const double* theta, int orbital_major, double* partial) {
  if (nw <= 0 || npairs <= 0) return hipSuccess;
  const int nwt = (int)((nw + HR_WT - 1) / HR_WT);
  const int64_t so = orbital_major ? (int64_t)M * nw : 1;
  const int64_t sr = orbital_major ? nw : n;
  const int64_t sw = orbital_major ? 1 : (int64_t)M * n;
  hipLaunchKernelGGL(hr_energy_kernel, dim3((unsigned)((int64_t)npairs * nwt)), dim3(512), 0, s, M, nw, npairs, Y,
                     pairs, (const double2*)theta, so, sr, sw, partial);
  return hipGetLastError();
}

}  // namespace lofqmc
