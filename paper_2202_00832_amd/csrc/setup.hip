// Set-up kernels (run once per system, not on the per-walker path):
// half-rotation of the Cholesky vectors, pair blocks Y^[ij] of the
// half-rotated ERI (Sec. 2.2-2.3.1) and packing of truncated SVD factors.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

// Strided batched FP64 GEMM, 64x64 output tile, 4x4 per thread.
__global__ __launch_bounds__(256) void gemm_setup_kernel(int Mr, int Nc, int K, const double* __restrict__ A,
                                                         int64_t a_m, int64_t a_k, const double* __restrict__ B,
                                                         int64_t b_k, int64_t b_n, double* __restrict__ C,
                                                         int64_t c_m, int64_t c_n,
                                                         const int64_t* __restrict__ bases) {
  __shared__ double sA[16][65];
  __shared__ double sB[16][65];
  const int bt = blockIdx.z;
  const int64_t ab = bases[3 * bt], bb = bases[3 * bt + 1], cb = bases[3 * bt + 2];
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const bool a_kfast = (a_k == 1);
  const bool b_kfast = (b_k == 1);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      int kk, mm;
      if (a_kfast) { kk = e & 15; mm = e >> 4; } else { kk = e >> 6; mm = e & 63; }
      const int m = m0 + mm, k = k0 + kk;
      sA[kk][mm] = (m < Mr && k < K) ? A[ab + m * a_m + k * a_k] : 0.0;
      int kb, nn;
      if (b_kfast) { kb = e & 15; nn = e >> 4; } else { kb = e >> 6; nn = e & 63; }
      const int c = n0 + nn, k2 = k0 + kb;
      sB[kb][nn] = (c < Nc && k2 < K) ? B[bb + k2 * b_k + c * b_n] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= Mr) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + tx + 16 * j;
      if (c < Nc) C[cb + m * c_m + c * c_n] = acc[i][j];
    }
  }
}

hipError_t launch_gemm_setup(hipStream_t s, int Mr, int Nc, int K, const double* A, int64_t a_m, int64_t a_k,
                             const double* B, int64_t b_k, int64_t b_n, double* C, int64_t c_m, int64_t c_n,
                             const int64_t* bases, int batch) {
  if (batch <= 0 || Mr <= 0 || Nc <= 0) return hipSuccess;
  dim3 grid((Mr + 63) / 64, (Nc + 63) / 64, batch);
  hipLaunchKernelGGL(gemm_setup_kernel, grid, dim3(256), 0, s, Mr, Nc, K, A, a_m, a_k, B, b_k, b_n, C, c_m, c_n,
                     bases);
  return hipGetLastError();
}

// lbar[g][r][i] -> lbarT[i][g][r]; one block per (g, 64-row slab of r).
__global__ __launch_bounds__(256) void lbar_transpose_kernel(int M, int n, int64_t X, const double* __restrict__ lbar,
                                                             double* __restrict__ lbarT) {
  __shared__ double t[64][65];
  const int64_t g = blockIdx.y;
  const int r0 = blockIdx.x * 64;
  for (int i0 = 0; i0 < n; i0 += 64) {
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int rr = e >> 6, ii = e & 63;
      const int r = r0 + rr, i = i0 + ii;
      t[rr][ii] = (r < M && i < n) ? lbar[((size_t)g * M + r) * n + i] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int ii = e >> 6, rr = e & 63;
      const int r = r0 + rr, i = i0 + ii;
      if (r < M && i < n) lbarT[((size_t)i * X + g) * M + r] = t[rr][ii];
    }
    __syncthreads();
  }
}

hipError_t launch_lbar_transpose(hipStream_t s, int M, int n, int64_t X, const double* lbar, double* lbarT) {
  if (X <= 0) return hipSuccess;
  dim3 grid((M + 63) / 64, (unsigned)X);
  hipLaunchKernelGGL(lbar_transpose_kernel, grid, dim3(256), 0, s, M, n, X, lbar, lbarT);
  return hipGetLastError();
}

// Factor rows of batch entry b (rank K, first row row_off): rows K of
// Ubar^T = (U Sigma^(1/2))^T, then K rows of Vbar = Sigma^(1/2) V.
// U and VT are column-major M x M (LAPACK convention of the SVD routine).
__global__ __launch_bounds__(256) void pack_factors_kernel(int M, const double* __restrict__ U,
                                                           const double* __restrict__ VT,
                                                           const double* __restrict__ S, const int* __restrict__ Kb,
                                                           const int64_t* __restrict__ row_off,
                                                           double* __restrict__ rows) {
  const int b = blockIdx.y;
  const int k = blockIdx.x;
  const int K = Kb[b];
  if (k >= 2 * K) return;
  const size_t mm = (size_t)M * M;
  const int kk = (k < K) ? k : k - K;
  const double sq = sqrt(S[(size_t)b * M + kk]);
  double* dst = rows + (size_t)(row_off[b] + k) * M;
  for (int r = threadIdx.x; r < M; r += blockDim.x) {
    const double v = (k < K) ? U[b * mm + (size_t)kk * M + r] : VT[b * mm + (size_t)r * M + kk];
    dst[r] = v * sq;
  }
}

hipError_t launch_pack_factors(hipStream_t s, int M, int nb, const double* U, const double* VT, const double* S,
                               const int* K, const int64_t* row_off, double* rows) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(2 * M, nb);
  hipLaunchKernelGGL(pack_factors_kernel, grid, dim3(256), 0, s, M, U, VT, S, K, row_off, rows);
  return hipGetLastError();
}

}  // namespace lofqmc
