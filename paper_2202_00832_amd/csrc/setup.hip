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
// Row k of the packed block of problem b: k < K is column k of U scaled by
// sqrt(S_k), K <= k < 2K is row k - K of VT scaled the same way.  U is
// column-major with leading dimension M (problem stride u_stride), VT has
// leading dimension vt_ld (problem stride vt_stride), S problem stride s_stride.
__global__ __launch_bounds__(256) void pack_factors_kernel(int M, const double* __restrict__ U, int64_t u_stride,
                                                           const double* __restrict__ VT, int vt_ld,
                                                           int64_t vt_stride, const double* __restrict__ S,
                                                           int64_t s_stride, const int* __restrict__ Kb,
                                                           const int64_t* __restrict__ row_off,
                                                           double* __restrict__ rows) {
  const int b = blockIdx.y;
  const int k = blockIdx.x;
  const int K = Kb[b];
  if (k >= 2 * K) return;
  const int kk = (k < K) ? k : k - K;
  const double sq = sqrt(S[(size_t)b * s_stride + kk]);
  double* dst = rows + (size_t)(row_off[b] + k) * M;
  for (int r = threadIdx.x; r < M; r += blockDim.x) {
    const double v = (k < K) ? U[b * u_stride + (size_t)kk * M + r] : VT[b * vt_stride + (size_t)r * vt_ld + kk];
    dst[r] = v * sq;
  }
}

hipError_t launch_pack_factors(hipStream_t s, int M, int nb, int kmax, const double* U, int64_t u_stride,
                               const double* VT, int vt_ld, int64_t vt_stride, const double* S, int64_t s_stride,
                               const int* K, const int64_t* row_off, double* rows) {
  if (nb <= 0 || kmax <= 0) return hipSuccess;
  dim3 grid(2 * kmax, nb);
  hipLaunchKernelGGL(pack_factors_kernel, grid, dim3(256), 0, s, M, U, u_stride, VT, vt_ld, vt_stride, S, s_stride,
                     K, row_off, rows);
  return hipGetLastError();
}

// Columns of each M x L block (column-major, ld M) replaced by an orthonormal
// basis of their span, column by column: classical Gram-Schmidt passes, each
// followed by a normalisation, repeated until a pass keeps at least half of
// the norm (at least two passes; the usual reorthogonalisation test).  A
// column that is lost in the span of the earlier ones (its projection falls
// below 1e-12 of its norm, as happens where the sketch is wider than the
// block's numerical rank) is replaced by a unit vector and orthogonalised in
// turn, so Q stays orthonormal also for rank-deficient blocks.  One workgroup
// per block; every projection coefficient and norm is a wave reduction in a
// fixed order, so every decision is uniform over the workgroup.
__global__ __launch_bounds__(256) void orth_kernel(int M, int L, double* __restrict__ A, int64_t stride) {
  __shared__ double sDot[64];
  __shared__ double sNorm;
  double* Z = A + blockIdx.x * stride;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  auto norm2 = [&](const double* z) {
    if (wv == 0) {
      double d = 0.0;
      for (int r = lane; r < M; r += 64) d += z[r] * z[r];
      d = wave_sum_lane0(d);
      if (lane == 0) sNorm = d;
    }
    __syncthreads();
    const double v = sqrt(sNorm);
    __syncthreads();
    return v;
  };
  for (int k = 0; k < L; ++k) {
    double* zk = Z + (size_t)k * M;
    double before = norm2(zk);
    int fresh = 0;
    for (int pass = 0; pass < 8; ++pass) {
      // coefficients q_j . z_k, j < k: wave wv takes j = wv, wv + 4, ...
      for (int j = wv; j < k; j += 4) {
        const double* qj = Z + (size_t)j * M;
        double d = 0.0;
        for (int r = lane; r < M; r += 64) d += qj[r] * zk[r];
        d = wave_sum_lane0(d);
        if (lane == 0) sDot[j] = d;
      }
      __syncthreads();
      for (int r = tid; r < M; r += 256) {
        double v = zk[r];
        for (int j = 0; j < k; ++j) v -= sDot[j] * Z[(size_t)j * M + r];
        zk[r] = v;
      }
      __syncthreads();
      const double after = norm2(zk);
      if (!(after > 1e-12 * before)) {
        // lost in the span: restart from unit vector e_m
        const int m = (k + fresh++) % M;
        for (int r = tid; r < M; r += 256) zk[r] = r == m ? 1.0 : 0.0;
        __syncthreads();
        before = 1.0;
        continue;
      }
      const double inv = 1.0 / after;
      for (int r = tid; r < M; r += 256) zk[r] *= inv;
      __syncthreads();
      if (pass > 0 && after >= 0.5 * before) break;
      before = 1.0;
    }
  }
}

hipError_t launch_orth(hipStream_t s, int M, int L, int nb, double* A, int64_t stride) {
  if (nb <= 0 || L <= 0) return hipSuccess;
  hipLaunchKernelGGL(orth_kernel, dim3(nb), dim3(256), 0, s, M, L, A, stride);
  return hipGetLastError();
}

}  // namespace lofqmc
