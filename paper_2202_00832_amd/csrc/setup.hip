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

// ---------------------------------------------------------------------------
// Foster-Boys localization of the occupied orbitals (set-up, Sec. 3): Jacobi
// sweeps maximising B = sum_i sum_d (X_d[i][i])^2, X_d = C^T diag(x_d) C.
// For the pair i < j (row order) with h_d = (X_d[i][i] - X_d[j][j]) / 2 and
// c_d = X_d[i][j], the rotation i' = cs i + sn j, j' = -sn i + cs j by
// 4t = atan2(2 sum_d c_d h_d, sum_d (h_d^2 - c_d^2)) maximises the pair's part
// of B; every rotation is applied, columns of X_d first, then rows.  X lives in
// LDS, the accumulated rotation (transposed, Ut[i][k] = U[k][i]) in global
// memory.  One workgroup; every thread computes the angle from LDS.
// ---------------------------------------------------------------------------
constexpr int BOYS_LDS_DOUBLES = 15360;   // 120 KB: D n^2 <= 15360

// X[d][i][j] = sum_r C[r][i] x_d[r] C[r][j]; one thread per (d, i, j)
__global__ __launch_bounds__(256) void boys_project_kernel(int M, int n, int D, const double* __restrict__ C,
                                                           const double* __restrict__ pos,
                                                           double* __restrict__ X) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= D * n * n) return;
  const int d = e / (n * n), i = (e / n) % n, j = e % n;
  double s = 0.0;
  for (int r = 0; r < M; ++r) s += C[(size_t)r * n + i] * pos[(size_t)d * M + r] * C[(size_t)r * n + j];
  X[e] = s;
}

__global__ __launch_bounds__(256) void boys_jacobi_kernel(int n, int D, int max_sweeps, double tol,
                                                          const double* __restrict__ Xg, double* __restrict__ Ut,
                                                          double* __restrict__ stats) {
  __shared__ double sX[BOYS_LDS_DOUBLES];
  const int tid = threadIdx.x;
  const int nn = n * n;
  for (int e = tid; e < D * nn; e += 256) sX[e] = Xg[e];
  for (int e = tid; e < nn; e += 256) Ut[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  auto functional = [&]() {
    double b = 0.0;
    for (int d = 0; d < D; ++d)
      for (int i = 0; i < n; ++i) {
        const double v = sX[d * nn + i * n + i];
        b += v * v;
      }
    return b;
  };
  double prev = functional();
  const double first = prev;
  int sweeps = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int i = 0; i < n; ++i) {
      for (int j = i + 1; j < n; ++j) {
        double ch = 0.0, hc = 0.0;
        for (int d = 0; d < D; ++d) {
          const double h = 0.5 * (sX[d * nn + i * n + i] - sX[d * nn + j * n + j]);
          const double c = sX[d * nn + i * n + j];
          ch += c * h;
          hc += h * h - c * c;
        }
        const double t = 0.25 * atan2(2.0 * ch, hc);
        const double cs = cos(t), sn = sin(t);
        __syncthreads();   // every thread has read the pair's entries
        // columns i and j of every X_d
        for (int e = tid; e < D * n; e += 256) {
          const int d = e / n, k = e % n;
          double* row = sX + d * nn + k * n;
          const double xi = row[i], xj = row[j];
          row[i] = xi * cs + xj * sn;
          row[j] = -xi * sn + xj * cs;
        }
        // rows i and j of Ut (columns of U)
        for (int k = tid; k < n; k += 256) {
          const double ui = Ut[(size_t)i * n + k], uj = Ut[(size_t)j * n + k];
          Ut[(size_t)i * n + k] = cs * ui + sn * uj;
          Ut[(size_t)j * n + k] = -sn * ui + cs * uj;
        }
        __syncthreads();
        // rows i and j of every X_d
        for (int e = tid; e < D * n; e += 256) {
          const int d = e / n, k = e % n;
          double* Xd = sX + d * nn;
          const double xi = Xd[i * n + k], xj = Xd[j * n + k];
          Xd[i * n + k] = cs * xi + sn * xj;
          Xd[j * n + k] = -sn * xi + cs * xj;
        }
        __syncthreads();
      }
    }
    ++sweeps;
    const double b = functional();
    const bool done = b - prev <= tol * fabs(b);
    prev = b;
    if (done) break;
  }
  if (tid == 0) {
    stats[0] = first;
    stats[1] = prev;
    stats[2] = (double)sweeps;
  }
}

// out[r][i] = sum_k C[r][k] Ut[i][k]; one thread per (r, i)
__global__ __launch_bounds__(256) void boys_apply_kernel(int M, int n, const double* __restrict__ C,
                                                         const double* __restrict__ Ut, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * n) return;
  const int r = (int)(e / n), i = (int)(e % n);
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += C[(size_t)r * n + k] * Ut[(size_t)i * n + k];
  out[e] = s;
}

int boys_max_lds_doubles() { return BOYS_LDS_DOUBLES; }

size_t boys_workspace(int M, int n, int D) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(sizeof(double) * (size_t)D * n * n) + al(sizeof(double) * (size_t)n * n) +
         al(sizeof(double) * (size_t)M * n) + al(sizeof(double) * 4);
}

hipError_t launch_boys(hipStream_t s, int M, int n, int D, const double* pos, double* C, int max_sweeps, double tol,
                       void* work, double* stats_dev) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* base = (char*)work;
  double* X = (double*)base;
  double* Ut = (double*)(base + al(sizeof(double) * (size_t)D * n * n));
  double* C0 = (double*)((char*)Ut + al(sizeof(double) * (size_t)n * n));
  hipError_t e = hipMemcpyAsync(C0, C, sizeof(double) * (size_t)M * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(boys_project_kernel, dim3((unsigned)((D * n * n + 255) / 256)), dim3(256), 0, s, M, n, D, C0, pos,
                     X);
  hipLaunchKernelGGL(boys_jacobi_kernel, dim3(1), dim3(256), 0, s, n, D, max_sweeps, tol, X, Ut, stats_dev);
  hipLaunchKernelGGL(boys_apply_kernel, dim3((unsigned)(((int64_t)M * n + 255) / 256)), dim3(256), 0, s, M, n, C0, Ut,
                     C);
  return hipGetLastError();
}

}  // namespace lofqmc
