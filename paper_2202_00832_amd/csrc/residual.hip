// Learned correction of the LO energy (not part of the paper's method).
//
// A 3-layer perceptron f: R^3 -> R (3 -> 128 -> 128 -> 1, tanh, standardised
// inputs) maps per-orbital features of a walker to a share of the energy that
// the LO truncation drops; the walker's prediction is sum_i f(x_i).  Features
// of orbital i: x0 = sum_j K_ij (retained ranks), x1 = sum_j m_ij (discarded
// singular-value mass), x2 = ||theta[:, i]||_2.
//
// Parameters: one float vector, W1[128][3], b1[128], W2[128][128], b2[128],
// w3[128], b3, shift[3], scale[3] (shift and scale are not trained).
//
// Kernels: features; FP32 forward that keeps the activations; per-walker sum
// and loss; backward through the rows; weight gradients as fixed-order sums
// over row splits; Adam; and a BF16 inference kernel (BF16 MFMA for the
// 128 x 128 layer, FP32 accumulation).  Every reduction has a fixed order, so
// results are bitwise reproducible.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int RW = 128;   // width
constexpr int RF = 3;     // features
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + RW * RF, OFF_W2 = OFF_B1 + RW, OFF_B2 = OFF_W2 + RW * RW,
              OFF_W3 = OFF_B2 + RW, OFF_B3 = OFF_W3 + RW, OFF_SHIFT = OFF_B3 + 1, OFF_SCALE = OFF_SHIFT + RF,
              NPAR = OFF_SCALE + RF;

int residual_nparam() { return NPAR; }

// x[w][i] = (Ksum_i, mass_i, ||theta_w[:, i]||); one thread per (walker, orbital)
__global__ __launch_bounds__(256) void residual_features_kernel(int M, int n, int64_t nw,
                                                                const double2* __restrict__ theta,
                                                                const float* __restrict__ orb,
                                                                float* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nw * n) return;
  const int64_t w = e / n;
  const int i = (int)(e % n);
  const double2* t = theta + (size_t)w * M * n + i;
  double s = 0.0;
  for (int r = 0; r < M; ++r) {
    const double2 v = t[(size_t)r * n];
    s += v.x * v.x + v.y * v.y;
  }
  x[e * RF + 0] = orb[2 * i];
  x[e * RF + 1] = orb[2 * i + 1];
  x[e * RF + 2] = (float)sqrt(s);
}

// ---------------------------------------------------------------------------
// FP32 forward over 64-row tiles: h1 = tanh(W1 z + b1), h2 = tanh(W2 h1 + b2),
// y = w3 . h2 + b3.  Thread (tr, tc) computes rows 4 tr .. 4 tr + 3 against
// columns tc + 16 j, j < 8.
// ---------------------------------------------------------------------------
constexpr int RT = 64;   // rows per tile

__global__ __launch_bounds__(256) void residual_forward_kernel(int64_t N, const float* __restrict__ p,
                                                               const float* __restrict__ x,
                                                               float* __restrict__ h1g, float* __restrict__ h2g,
                                                               float* __restrict__ y) {
  __shared__ float sW2[RW][RW + 1];
  __shared__ float sH1[RT][RW + 1];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * RT;
  for (int e = tid; e < RW * RW; e += 256) sW2[e / RW][e % RW] = p[OFF_W2 + e];
  for (int e = tid; e < RT * RW; e += 256) {
    const int rr = e / RW, k = e % RW;
    const int64_t row = row0 + rr;
    float v = 0.0f;
    if (row < N) {
      float a = p[OFF_B1 + k];
#pragma unroll
      for (int f = 0; f < RF; ++f)
        a += p[OFF_W1 + k * RF + f] * ((x[row * RF + f] - p[OFF_SHIFT + f]) * p[OFF_SCALE + f]);
      v = tanhf(a);
      h1g[row * RW + k] = v;
    }
    sH1[rr][k] = v;
  }
  __syncthreads();
  const int tr = tid >> 4, tc = tid & 15;
  float acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0f;
  for (int k = 0; k < RW; ++k) {
    float a[4], b[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = sH1[4 * tr + i][k];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = sW2[tc + 16 * j][k];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + 4 * tr + i;
    float part = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = tc + 16 * j;
      const float h = tanhf(acc[i][j] + p[OFF_B2 + c]);
      if (row < N) h2g[row * RW + c] = h;
      part = fmaf(p[OFF_W3 + c], h, part);
    }
    // fixed-order sum over the 16 threads tc of this row group
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) part += __shfl_xor(part, off, 16);
    if (tc == 0 && row < N) y[row] = part + p[OFF_B3];
  }
}

// pred[w] = sum_i y[w n + i] (FP64, fixed order); with a target also
// g[w] = 2 (pred - t) / nw and loss = mean (pred - t)^2 (one workgroup).
__global__ __launch_bounds__(1024) void residual_walker_kernel(int64_t nw, int n, const float* __restrict__ y,
                                                               const double* __restrict__ target,
                                                               double* __restrict__ pred, float* __restrict__ g,
                                                               double* __restrict__ loss) {
  __shared__ double sL[1024];
  double l = 0.0;
  for (int64_t w = threadIdx.x; w < nw; w += 1024) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += y[w * n + i];
    if (pred) pred[w] = s;
    if (target) {
      const double r = s - target[w];
      g[w] = (float)(2.0 * r / (double)nw);
      l += r * r;
    }
  }
  sL[threadIdx.x] = l;
  __syncthreads();
  for (int off = 512; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sL[threadIdx.x] += sL[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss && target) *loss = sL[0] / (double)nw;
}

// backward through the rows: dz2 = g_row w3 (1 - h2^2), dz1 = (W2^T dz2) (1 - h1^2)
__global__ __launch_bounds__(256) void residual_backward_rows_kernel(int64_t N, int n, const float* __restrict__ p,
                                                                     const float* __restrict__ g,
                                                                     const float* __restrict__ h1g,
                                                                     const float* __restrict__ h2g,
                                                                     float* __restrict__ dz1g,
                                                                     float* __restrict__ dz2g) {
  __shared__ float sW2[RW][RW + 1];
  __shared__ float sD2[RT][RW + 1];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * RT;
  for (int e = tid; e < RW * RW; e += 256) sW2[e / RW][e % RW] = p[OFF_W2 + e];
  for (int e = tid; e < RT * RW; e += 256) {
    const int rr = e / RW, c = e % RW;
    const int64_t row = row0 + rr;
    float v = 0.0f;
    if (row < N) {
      const float h = h2g[row * RW + c];
      v = g[row / n] * p[OFF_W3 + c] * (1.0f - h * h);
      dz2g[row * RW + c] = v;
    }
    sD2[rr][c] = v;
  }
  __syncthreads();
  // dh1[row][k] = sum_c dz2[row][c] W2[c][k]; thread: rows 4 tr + i, k = tc + 16 j
  const int tr = tid >> 4, tc = tid & 15;
  float acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0f;
  for (int c = 0; c < RW; ++c) {
    float a[4], b[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = sD2[4 * tr + i][c];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = sW2[c][tc + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + 4 * tr + i;
    if (row >= N) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = tc + 16 * j;
      const float h = h1g[row * RW + k];
      dz1g[row * RW + k] = acc[i][j] * (1.0f - h * h);
    }
  }
}

// Weight gradients summed over the rows [s * per, (s + 1) * per) of split s:
//   dW2[c][k] = sum dz2[row][c] h1[row][k]   (thread: c = 8 (tid / 16) + a, k = (tid % 16) + 16 b)
//   dW1[k][f] = sum dz1[row][k] z[row][f],  db1 = sum dz1,  db2 = sum dz2,
//   dw3[c] = sum g_row h2[row][c],  db3 = sum g_row.
__global__ __launch_bounds__(256) void residual_weight_grad_kernel(int64_t N, int n, int64_t per,
                                                                   const float* __restrict__ p,
                                                                   const float* __restrict__ x,
                                                                   const float* __restrict__ g,
                                                                   const float* __restrict__ h1g,
                                                                   const float* __restrict__ h2g,
                                                                   const float* __restrict__ dz1g,
                                                                   const float* __restrict__ dz2g,
                                                                   float* __restrict__ part) {
  __shared__ float sA[RT][RW + 1];   // dz2 rows
  __shared__ float sB[RT][RW + 1];   // h1 rows
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = (r0 + per < N) ? r0 + per : N;
  const int ta = tid >> 4, tb = tid & 15;
  float acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = 0.0f;
  // small gradients: thread tid < 128 owns column tid of db1, db2, dw3, dW1
  float s_db1 = 0.0f, s_db2 = 0.0f, s_dw3 = 0.0f, s_dw1[RF] = {0.0f, 0.0f, 0.0f}, s_db3 = 0.0f;
  for (int64_t c0 = r0; c0 < r1; c0 += RT) {
    __syncthreads();
    for (int e = tid; e < RT * RW; e += 256) {
      const int rr = e / RW, k = e % RW;
      const int64_t row = c0 + rr;
      const bool ok = row < r1;
      sA[rr][k] = ok ? dz2g[row * RW + k] : 0.0f;
      sB[rr][k] = ok ? h1g[row * RW + k] : 0.0f;
    }
    __syncthreads();
    for (int rr = 0; rr < RT; ++rr) {
      float a[8], b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = sA[rr][8 * ta + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) b[q] = sB[rr][tb + 16 * q];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
    }
    if (tid < RW) {
      const int k = tid;
      const int64_t end = (c0 + RT < r1) ? c0 + RT : r1;
      for (int64_t row = c0; row < end; ++row) {
        const float d1 = dz1g[row * RW + k];
        s_db1 += d1;
        s_db2 += sA[row - c0][k];
        const float gr = g[row / n];
        s_dw3 = fmaf(gr, h2g[row * RW + k], s_dw3);
#pragma unroll
        for (int f = 0; f < RF; ++f)
          s_dw1[f] = fmaf(d1, (x[row * RF + f] - p[OFF_SHIFT + f]) * p[OFF_SCALE + f], s_dw1[f]);
        if (k == 0) s_db3 += gr;
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * NPAR;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) out[OFF_W2 + (8 * ta + a) * RW + tb + 16 * b] = acc[a][b];
  if (tid < RW) {
    out[OFF_B1 + tid] = s_db1;
    out[OFF_B2 + tid] = s_db2;
    out[OFF_W3 + tid] = s_dw3;
#pragma unroll
    for (int f = 0; f < RF; ++f) out[OFF_W1 + tid * RF + f] = s_dw1[f];
    if (tid == 0) out[OFF_B3] = s_db3;
  }
  if (tid < 2 * RF) out[OFF_SHIFT + tid] = 0.0f;
}

// grad[e] = sum_s part[s][e] in order of s (FP64 accumulation)
__global__ __launch_bounds__(256) void residual_grad_reduce_kernel(int nsplit, const float* __restrict__ part,
                                                                   float* __restrict__ grad) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= NPAR) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * NPAR + e];
  grad[e] = (float)s;
}

// Adam (Kingma & Ba) on the trained parameters; shift and scale are left alone.
// The coefficients (1 - beta) and the bias corrections are formed in FP64.
__global__ __launch_bounds__(256) void residual_adam_kernel(float* __restrict__ p, const float* __restrict__ grad,
                                                            float* __restrict__ m, float* __restrict__ v, double c1,
                                                            double c2, float lr, double beta1, double beta2,
                                                            float eps) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= OFF_SHIFT) return;
  const float b1 = (float)beta1, b2 = (float)beta2;
  const float a1 = (float)(1.0 - beta1), a2 = (float)(1.0 - beta2);
  const float gg = grad[e];
  const float mm = b1 * m[e] + a1 * gg;
  const float vv = b2 * v[e] + a2 * gg * gg;
  m[e] = mm;
  v[e] = vv;
  const float mh = (float)(mm / c1), vh = (float)(vv / c2);
  p[e] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// BF16 inference: one wave per 16 rows.  h1 (FP32, rounded to BF16) is the A
// operand and W2 (BF16, staged in LDS as [c][k]) the B operand of
// v_mfma_f32_16x16x32_bf16 (lane l gives A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16]; accumulator v of lane l is D[4 (l / 16) + v][l % 16]);
// the first and last layers stay FP32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void residual_infer_bf16_kernel(int64_t N, const float* __restrict__ p,
                                                                  const float* __restrict__ x,
                                                                  float* __restrict__ y) {
  constexpr int LD = RW + 8;   // row stride (bf16): spreads the 16 rows of a fragment over the banks
  __shared__ __attribute__((aligned(16))) __bf16 sW2[RW * LD];
  const int tid = threadIdx.x;
  for (int e = tid; e < RW * RW; e += 256) sW2[(e / RW) * LD + e % RW] = (__bf16)p[OFF_W2 + e];
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t rbase = ((int64_t)blockIdx.x * 4 + wv) * 16;
  const int64_t row = rbase + lr;
  float z[RF];
#pragma unroll
  for (int f = 0; f < RF; ++f)
    z[f] = row < N ? (x[row * RF + f] - p[OFF_SHIFT + f]) * p[OFF_SCALE + f] : 0.0f;
  f4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int s = 0; s < RW / 32; ++s) {
    bf8 a;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = 32 * s + 8 * lk + t;
      float h = p[OFF_B1 + k];
#pragma unroll
      for (int f = 0; f < RF; ++f) h += p[OFF_W1 + k * RF + f] * z[f];
      a[t] = (__bf16)tanhf(h);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf8 b = *(const bf8*)&sW2[(16 * c + lr) * LD + 32 * s + 8 * lk];
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
  }
  // rows 4 lk + v, column 16 c + lr
  float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int col = 16 * c + lr;
    const float w3 = p[OFF_W3 + col], b2 = p[OFF_B2 + col];
#pragma unroll
    for (int v = 0; v < 4; ++v) part[v] = fmaf(w3, tanhf(acc[c][v] + b2), part[v]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float s = part[v];
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 16);
    const int64_t r = rbase + 4 * lk + v;
    if (lr == 0 && r < N) y[r] = s + p[OFF_B3];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int64_t rw_splits(int64_t N) {
  int64_t s = (N + 4095) / 4096;   // about 4096 rows per split
  return s < 1 ? 1 : (s > 1024 ? 1024 : s);
}

size_t residual_train_workspace(int64_t nw, int n) {
  const size_t N = (size_t)nw * n;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return 4 * al(N * RW * 4) + al(N * 4) + al((size_t)nw * 4) + al((size_t)rw_splits((int64_t)N) * NPAR * 4) +
         al(NPAR * 4);
}

hipError_t launch_residual_features(hipStream_t s, int M, int n, int64_t nw, const double* theta, const float* orb,
                                    float* x) {
  if (nw <= 0) return hipSuccess;
  const int64_t tot = nw * n;
  hipLaunchKernelGGL(residual_features_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, n, nw,
                     (const double2*)theta, orb, x);
  return hipGetLastError();
}

hipError_t launch_residual_predict(hipStream_t s, int bf16, int64_t nw, int n, const float* params, const float* x,
                                   void* work, double* pred) {
  if (nw <= 0) return hipSuccess;
  const int64_t N = nw * n;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* base = (char*)work;
  float* y = (float*)base;
  if (bf16) {
    hipLaunchKernelGGL(residual_infer_bf16_kernel, dim3((unsigned)((N + 63) / 64)), dim3(256), 0, s, N, params, x,
                       y);
  } else {
    float* h1 = (float*)(base + al(N * 4));
    float* h2 = (float*)(base + al(N * 4) + al((size_t)N * RW * 4));
    hipLaunchKernelGGL(residual_forward_kernel, dim3((unsigned)((N + RT - 1) / RT)), dim3(256), 0, s, N, params, x,
                       h1, h2, y);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(residual_walker_kernel, dim3(1), dim3(1024), 0, s, nw, n, y, (const double*)nullptr, pred,
                     (float*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

size_t residual_predict_workspace(int bf16, int64_t nw, int n) {
  const size_t N = (size_t)nw * n;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return bf16 ? al(N * 4) : al(N * 4) + 2 * al(N * RW * 4);
}

hipError_t launch_residual_train_step(hipStream_t s, int64_t nw, int n, float* params, float* m, float* v,
                                      int64_t step, float lr, const float* x, const double* target, void* work,
                                      float* grad_out, double* loss, double* pred) {
  if (nw <= 0) return hipSuccess;
  const int64_t N = nw * n;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* base = (char*)work;
  float* h1 = (float*)base;
  float* h2 = (float*)(base + al(N * RW * 4));
  float* dz1 = (float*)(base + 2 * al(N * RW * 4));
  float* dz2 = (float*)(base + 3 * al(N * RW * 4));
  float* y = (float*)(base + 4 * al(N * RW * 4));
  float* g = (float*)(base + 4 * al(N * RW * 4) + al(N * 4));
  const int64_t ns = rw_splits(N);
  float* part = (float*)(base + 4 * al(N * RW * 4) + al(N * 4) + al((size_t)nw * 4));
  float* grad = grad_out ? grad_out : (float*)((char*)part + al((size_t)ns * NPAR * 4));
  const unsigned tiles = (unsigned)((N + RT - 1) / RT);
  hipLaunchKernelGGL(residual_forward_kernel, dim3(tiles), dim3(256), 0, s, N, params, x, h1, h2, y);
  hipLaunchKernelGGL(residual_walker_kernel, dim3(1), dim3(1024), 0, s, nw, n, y, target, pred, g, loss);
  hipLaunchKernelGGL(residual_backward_rows_kernel, dim3(tiles), dim3(256), 0, s, N, n, params, g, h1, h2, dz1,
                     dz2);
  const int64_t per = (N + ns - 1) / ns;
  hipLaunchKernelGGL(residual_weight_grad_kernel, dim3((unsigned)ns), dim3(256), 0, s, N, n, per, params, x, g, h1,
                     h2, dz1, dz2, part);
  hipLaunchKernelGGL(residual_grad_reduce_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, s, (int)ns, part, grad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || step <= 0) return e;
  const double c1 = 1.0 - pow(0.9, (double)step), c2 = 1.0 - pow(0.999, (double)step);
  hipLaunchKernelGGL(residual_adam_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, s, params, grad, m, v, c1, c2, lr,
                     0.9, 0.999, 1e-8f);
  return hipGetLastError();
}

}  // namespace lofqmc
