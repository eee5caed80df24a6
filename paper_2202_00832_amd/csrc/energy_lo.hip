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

// theta[w][r][j] -> thetaT[j][r][w] (complex); tile of 32 walkers x 32 orbitals.
__global__ __launch_bounds__(256) void theta_transpose_kernel(int M, int n, int64_t nw,
                                                              const double2* __restrict__ theta,
                                                              double2* __restrict__ thetaT) {
  __shared__ double2 t[32][33];
  const int j0 = blockIdx.x * 32;
  const int64_t w0 = (int64_t)blockIdx.y * 32;
  const int r = blockIdx.z;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t w = w0 + yy;
    const int j = j0 + tx;
    t[yy][tx] = (w < nw && j < n) ? theta[((size_t)w * M + r) * n + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int j = j0 + yy;
    const int64_t w = w0 + tx;
    if (w < nw && j < n) thetaT[((size_t)j * M + r) * nw + w] = t[tx][yy];
  }
}

hipError_t launch_theta_transpose(hipStream_t s, int M, int n, int64_t nw, const double* theta, double* thetaT) {
  if (nw <= 0) return hipSuccess;
  dim3 grid((n + 31) / 32, (unsigned)((nw + 31) / 32), M);
  hipLaunchKernelGGL(theta_transpose_kernel, grid, dim3(256), 0, s, M, n, nw, (const double2*)theta,
                     (double2*)thetaT);
  return hipGetLastError();
}

// Pass 1: tile = up to 64 output rows of one orbital o (wave q: 16 rows) x 64
// walkers (four 16-walker column blocks, real and imaginary part each).
__global__ __launch_bounds__(256) void lo_pass1_kernel(int M, int64_t nw, const double* __restrict__ rows,
                                                       const int* __restrict__ rowidx,
                                                       const int* __restrict__ tile_orb,
                                                       const int* __restrict__ tile_row0,
                                                       const int* __restrict__ tile_nrows,
                                                       const double2* __restrict__ thetaT,
                                                       double2* __restrict__ qbar) {
  const int t = blockIdx.x;
  const int o = tile_orb[t];
  const int row0 = tile_row0[t];
  const int nrows = tile_nrows[t];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t w0 = (int64_t)blockIdx.y * 64;
  const int myrow = 16 * wv + lr;
  const bool rok = myrow < nrows;
  const double* frow = rows + (size_t)(rok ? rowidx[row0 + myrow] : 0) * M;
  const double2* tho = thetaT + (size_t)o * M * nw;

  d4 aR[4], aI[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) { aR[b] = d4zero(); aI[b] = d4zero(); }
  for (int r0 = 0; r0 < M; r0 += 4) {
    const int r = r0 + lk;
    const double a = (rok && r < M) ? frow[r] : 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t w = w0 + 16 * b + lr;
      const double2 bv = (r < M && w < nw) ? tho[(size_t)r * nw + w] : make_double2(0.0, 0.0);
      aR[b] = mfma16(a, bv.x, aR[b]);
      aI[b] = mfma16(a, bv.y, aI[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t w = w0 + 16 * b + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int lrow = 16 * wv + 4 * v + lk;
      if (lrow < nrows && w < nw) qbar[(size_t)(row0 + lrow) * nw + w] = make_double2(aR[b][v], aI[b][v]);
    }
  }
}

hipError_t launch_lo_pass1(hipStream_t s, int M, int64_t nw, int ntiles, const double* rows, const int* rowidx,
                           const int* tile_orb, const int* tile_row0, const int* tile_nrows, const double* thetaT,
                           double* qbar) {
  if (nw <= 0 || ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles, (unsigned)((nw + 63) / 64));
  hipLaunchKernelGGL(lo_pass1_kernel, grid, dim3(256), 0, s, M, nw, rows, rowidx, tile_orb, tile_row0, tile_nrows,
                     (const double2*)thetaT, (double2*)qbar);
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
  int c = (npairs + 15) / 16;
  if (c > 128) c = 128;
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
