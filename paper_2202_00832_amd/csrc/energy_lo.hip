// Two-body energy by the LO route (Sec. 2.3.2, Eq. 22-23), FP64.
//
// Stored factors: for every pair i <= j the rows [Ubar^T ; Vbar] (2 K_ij x M).
// Each stored row multiplies the walker column of both orbitals of its pair:
//   orbital i:  [Ubar^T Q_i ; Vbar Q_i] = [QL_i ; QR_i]
//   orbital j:  [Ubar^T Q_j ; Vbar Q_j] = [QL_j ; QR_j]
// so, grouping the rows by orbital, the four vectors of Eq. 23 for all pairs
// come from one dense product per orbital o: (rows touching o) x Q_o, with the
// walkers as the wide dimension (pass 1, FP64 MFMA).  Pass 2 forms the dot
// products of Eq. 22 per pair and walker,
//   J_ij = QL_i . QR_j,   X_ij = QL_j . QR_i   (complex, bilinear),
// with weight 1 for i = j and 2 for i < j (Y^[ji] = (Y^[ij])^T), and sums
// E_J = 2 sum J, E_K = -sum X in a fixed order per pair chunk.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

// Pass 1: tile = up to LO_TILE_ROWS (192) output rows of one orbital o x 32
// walkers.  The rows touching one orbital number about 2 x (sum of its pair
// ranks), nearly the same for every orbital of a localized basis, so one tile
// usually covers an orbital and each theta element is fetched once per
// orbital.  Eight waves; wave v owns rows 24v .. 24v + 23 (six groups of 4)
// against all 32 walkers (two 16-walker blocks, real and imaginary part) on
// the FP64 4x4x4 MFMA: 24 accumulators, 24 MFMA per K-step from 6 + 2 LDS
// reads.  Per 16-row slab of r the factor rows (gathered through rowidx) and
// Q_o of the 32 walkers are staged in LDS (double-buffered).
//
// theta element (o, r, w) is read at theta[o * so + r * sr + w * sw], which
// serves both layouts: walker-major [w][r][o] and orbital-major [o][r][w].
// Work units (block of LO_OBLK orbitals, walker tile) go round-robin over the
// 8 XCDs (workgroups are dispatched round-robin over XCDs) and the tiles of
// one unit run side by side on one XCD: with walker-major theta the orbitals
// of a block share cache lines, which that XCD's L2 then fetches once.
constexpr int LO_TILE_ROWS = 192;
constexpr int LO_WT = 32;
constexpr int LO_OBLK = 8;
constexpr int LO_WROWS = LO_TILE_ROWS / 8;   // rows per wave (24)
constexpr int LO_QG = LO_WROWS / 4;          // 4-row groups per wave (6)

__global__ __launch_bounds__(512, 2) void lo_pass1_kernel(int M, int64_t nw, const double* __restrict__ rows,
                                                          const int* __restrict__ rowidx,
                                                          const int* __restrict__ tile_orb,
                                                          const int* __restrict__ tile_row0,
                                                          const int* __restrict__ tile_nrows,
                                                          const int* __restrict__ blk, int nblk, int tmax,
                                                          const double2* __restrict__ theta, int64_t so,
                                                          int64_t sr, int64_t sw, double2* __restrict__ qbar,
                                                          int64_t orow, int64_t ow, int nwt) {
  __shared__ double sA[2][LO_TILE_ROWS][17];   // [row][r], padded against bank conflicts
  __shared__ double2 sB[2][16][LO_WT];         // [r][walker]
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
    w0 = (u % nwt) * LO_WT;
  }
  const int o = tile_orb[t];
  const int row0 = tile_row0[t];
  const int nrows = tile_nrows[t];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int rw = LO_WROWS * wv;                // first row of this wave
  const bool active = rw < nrows;
  const double2* tho = theta + o * so;

  // staging: A = nrows x 16 doubles (each row 128 contiguous bytes), B = 16 x 32 complex
  constexpr int A_PER = LO_TILE_ROWS * 16 / 512;   // 6
  double pa[A_PER];
  double2 pb;
  // the gathered factor rows of this thread, resolved once (a row index read
  // inside the slab loop would put a dependent global load on every slab)
  int arow[A_PER];
#pragma unroll
  for (int p = 0; p < A_PER; ++p) {
    const int row = (tid + 512 * p) >> 4;
    arow[p] = row < nrows ? rowidx[row0 + row] : -1;
  }
  const int brr = tid / LO_WT, bww = tid % LO_WT;
  const int64_t bw = w0 + bww;
  // theta (HBM) is fetched one slab ahead, across the products; the factor
  // rows (small, reused by every walker tile, so mostly cache hits) after them,
  // which keeps two workgroups per CU
  auto load_a = [&](int c) {
    const int rbase = 16 * c;
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int r = rbase + ((tid + 512 * p) & 15);
      pa[p] = (arow[p] >= 0 && r < M) ? rows[(size_t)arow[p] * M + r] : 0.0;
    }
  };
  auto load_b = [&](int c) {
    const int r = 16 * c + brr;
    pb = (r < M && bw < nw) ? tho[r * sr + bw * sw] : make_double2(0.0, 0.0);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int e = tid + 512 * p;
      sA[buf][e >> 4][e & 15] = pa[p];
    }
    sB[buf][brr][bww] = pb;
  };

  // acc[q][c]: rows rw + 4q + lk, walker column c (block h = c / 2, part = c % 2)
  // -- one FP64 4x4x4 accumulator each (see mfma4)
  double acc[LO_QG][4];
#pragma unroll
  for (int q = 0; q < LO_QG; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = 0.0;
  const int nchunk = (M + 15) / 16;
  load_a(0);
  load_b(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) load_b(c + 1);
    if (active) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int rr = 4 * s4 + lk;
        const double2 b0 = sB[buf][rr][lr];
        const double2 b1 = sB[buf][rr][16 + lr];
#pragma unroll
        for (int q = 0; q < LO_QG; ++q) {
          const double a = sA[buf][rw + 4 * q + (lane & 3)][rr];
          acc[q][0] = mfma4(a, b0.x, acc[q][0]);
          acc[q][1] = mfma4(a, b0.y, acc[q][1]);
          acc[q][2] = mfma4(a, b1.x, acc[q][2]);
          acc[q][3] = mfma4(a, b1.y, acc[q][3]);
        }
      }
    }
    if (c + 1 < nchunk) {
      load_a(c + 1);
      store(buf ^ 1);
    }
    __syncthreads();
  }
  // lane holds rows rw + 4q + lk, walker 16h + lr
  if (active) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t w = w0 + 16 * h + lr;
      if (w < nw) {
#pragma unroll
        for (int q = 0; q < LO_QG; ++q) {
          const int lrow = rw + 4 * q + lk;
          if (lrow < nrows)
            qbar[(size_t)(row0 + lrow) * orow + w * ow] = make_double2(acc[q][2 * h], acc[q][2 * h + 1]);
        }
      }
    }
  }
}

int lo_tile_rows() { return LO_TILE_ROWS; }
int lo_orbital_block() { return LO_OBLK; }

hipError_t launch_lo_pass1(hipStream_t s, int M, int n, int64_t nw, int ntiles, const double* rows,
                           const int* rowidx, const int* tiles, const int* blk, int nblk, int tmax,
                           const double* theta, int orbital_major, double* qbar, int64_t out_walker_stride) {
  if (nw <= 0 || ntiles <= 0) return hipSuccess;
  const int nwt = (int)((nw + LO_WT - 1) / LO_WT);
  const int64_t units = (int64_t)nblk * nwt;
  const int64_t grid = (int64_t)8 * ((units + 7) / 8) * tmax;
  const int64_t so = orbital_major ? (int64_t)M * nw : 1;
  const int64_t sr = orbital_major ? nw : n;
  const int64_t sw = orbital_major ? 1 : (int64_t)M * n;
  hipLaunchKernelGGL(lo_pass1_kernel, dim3((unsigned)grid), dim3(512), 0, s, M, nw, rows, rowidx, tiles,
                     tiles + ntiles, tiles + 2 * ntiles, blk, nblk, tmax, (const double2*)theta, so, sr, sw,
                     (double2*)qbar, out_walker_stride ? (int64_t)1 : nw,
                     out_walker_stride ? out_walker_stride : (int64_t)1, nwt);
  return hipGetLastError();
}
// Pass 2: one thread per walker, a contiguous chunk of pairs per grid row.
__global__ __launch_bounds__(64) void lo_pass2_kernel(int64_t nw, int npairs, int per_chunk,
                                                      const int* __restrict__ pK, const int64_t* __restrict__ offI,
                                                      const int64_t* __restrict__ offJ,
                                                      const double* __restrict__ pw,
                                                      const double2* __restrict__ qbar,
                                                      double* __restrict__ partial) {
  const int64_t w = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int chunk = blockIdx.y;
  if (w >= nw) return;
  const int p0 = chunk * per_chunk;
  const int p1 = (p0 + per_chunk < npairs) ? p0 + per_chunk : npairs;
  double jr = 0.0, ji = 0.0, xr = 0.0, xi = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int K = pK[p];
    const double wt = pw[p];
    const double2* gi = qbar + (size_t)offI[p] * nw + w;   // [QL_i ; QR_i]
    const double2* gj = qbar + (size_t)offJ[p] * nw + w;   // [QL_j ; QR_j]
    double sjr = 0.0, sji = 0.0, sxr = 0.0, sxi = 0.0;
    for (int k = 0; k < K; ++k) {
      const double2 qli = gi[(size_t)k * nw];
      const double2 qri = gi[(size_t)(K + k) * nw];
      const double2 qlj = gj[(size_t)k * nw];
      const double2 qrj = gj[(size_t)(K + k) * nw];
      sjr += qli.x * qrj.x - qli.y * qrj.y;
      sji += qli.x * qrj.y + qli.y * qrj.x;
      sxr += qlj.x * qri.x - qlj.y * qri.y;
      sxi += qlj.x * qri.y + qlj.y * qri.x;
    }
    jr += wt * sjr;
    ji += wt * sji;
    xr += wt * sxr;
    xi += wt * sxi;
  }
  double* out = partial + ((size_t)chunk * nw + w) * 4;
  out[0] = 2.0 * jr;
  out[1] = 2.0 * ji;
  out[2] = -xr;
  out[3] = -xi;
}

int lo_pass2_chunks(int npairs) {
  int c = (npairs + 3) / 4;
  if (c > 512) c = 512;
  if (c < 1) c = 1;
  return c;
}

hipError_t launch_lo_pass2(hipStream_t s, int64_t nw, int npairs, int nchunk, const int* pK, const int64_t* offI,
                           const int64_t* offJ, const double* pw, const double* qbar, double* partial) {
  if (nw <= 0) return hipSuccess;
  const int per = (npairs + nchunk - 1) / nchunk;
  dim3 grid((unsigned)((nw + 63) / 64), nchunk);
  hipLaunchKernelGGL(lo_pass2_kernel, grid, dim3(64), 0, s, nw, npairs, per > 0 ? per : 1, pK, offI, offJ, pw,
                     (const double2*)qbar, partial);
  return hipGetLastError();
}

}  // namespace lofqmc
