// Learned correction of the LO energy (not part of the paper's method).
//
// A 3-layer perceptron f: R^4 -> R (4 -> 128 -> 128 -> 1, tanh, standardised
// inputs) maps per-orbital features of a walker to a share of the energy that
// the LO truncation drops; the walker's prediction is sum_i f(x_i).  Features
// of orbital i: x0 = sum_j K_ij (retained ranks), x1 = sum_j m_ij (discarded
// singular-value mass), x2 = ||theta[:, i]||_2, x3 = Re(g_i . theta[:, i]) with
// g_i the gradient of the dropped energy E_HR - E_LO with respect to column i
// of theta at the trial (theta = Psi), formed once per set of factors.
//
// Parameters: one float vector, W1[128][4], b1[128], W2[128][128], b2[128],
// w3[128], b3, shift[4], scale[4] (shift and scale are not trained).
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
constexpr int RF = 4;     // features
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + RW * RF, OFF_W2 = OFF_B1 + RW, OFF_B2 = OFF_W2 + RW * RW,
              OFF_W3 = OFF_B2 + RW, OFF_B3 = OFF_W3 + RW, OFF_SHIFT = OFF_B3 + 1, OFF_SCALE = OFF_SHIFT + RF,
              NPAR = OFF_SCALE + RF;

int residual_nparam() { return NPAR; }

// x[w][i] = (Ksum_i, mass_i, ||theta_w[:, i]||, Re(g_i . theta_w[:, i]));
// one thread per (walker, orbital); grad is [M][n] like theta
__global__ __launch_bounds__(256) void residual_features_kernel(int M, int n, int64_t nw,
                                                                const double2* __restrict__ theta,
                                                                const float* __restrict__ orb,
                                                                const double* __restrict__ grad,
                                                                float* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nw * n) return;
  const int64_t w = e / n;
  const int i = (int)(e % n);
  const double2* t = theta + (size_t)w * M * n + i;
  double s = 0.0, d = 0.0;
  for (int r = 0; r < M; ++r) {
    const double2 v = t[(size_t)r * n];
    s += v.x * v.x + v.y * v.y;
    d += grad[(size_t)r * n + i] * v.x;
  }
  x[e * RF + 0] = orb[2 * i];
  x[e * RF + 1] = orb[2 * i + 1];
  x[e * RF + 2] = (float)sqrt(s);
  x[e * RF + 3] = (float)d;
}

// ---------------------------------------------------------------------------
// Gradient of the dropped energy at the trial (set-up, FP64).  Both E_HR
// (Eq. 17) and E_LO (Eq. 22) are E(Q) = sum_ij 2 Q_i^T A^[ij] Q_j -
// Q_j^T A^[ij] Q_i with A^[ji] = A^[ij]^T, so with Q = Psi
//   grad_i = sum_j 4 A^[ij] psi_j - 2 A^[ji] psi_j.
// Exact part, A^[ij] = sum_g Lbar_g[:, i] Lbar_g[:, j]^T and
// T0_g[i][j] = Lbar_g[:, i] . psi_j, C_g = sum_i T0_g[i][i]:
//   G_i = 4 sum_g C_g Lbar_g[:, i] - 2 sum_g sum_j Lbar_g[:, j] T0_g[i][j].
// LO part from the stored rows u_k (of Ubar^T) and v_k (of Vbar) of pair
// (a, b), a <= b, summed over k (both orderings of a < b counted):
//   i = a < b: 4 u (v . psi_b) - 2 v (u . psi_b)
//   i = b > a: 4 v (u . psi_a) - 2 u (v . psi_a)
//   i = a = b: u (v . psi_a) + v (u . psi_a)
// ---------------------------------------------------------------------------

// T0[g][i][j]; one thread per (g, i, j)
__global__ __launch_bounds__(256) void residual_t0_kernel(int M, int n, int64_t X, const double* __restrict__ lbar,
                                                          const double* __restrict__ trial,
                                                          double* __restrict__ t0) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (e >= X * nn) return;
  const int64_t g = e / nn;
  const int i = (int)((e % nn) / n), j = (int)(e % n);
  const double* L = lbar + (size_t)g * M * n;
  double s = 0.0;
  for (int r = 0; r < M; ++r) s += L[(size_t)r * n + i] * trial[(size_t)r * n + j];
  t0[e] = s;
}

// C[g] = sum_i T0[g][i][i]; one thread per g
__global__ __launch_bounds__(256) void residual_trace_kernel(int n, int64_t X, const double* __restrict__ t0,
                                                             double* __restrict__ c) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= X) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += t0[(size_t)g * n * n + (size_t)i * n + i];
  c[g] = s;
}

// grad[r][i] = G_i[r] (exact part); one thread per (r, i)
__global__ __launch_bounds__(256) void residual_grad_exact_kernel(int M, int n, int64_t X,
                                                                  const double* __restrict__ lbar,
                                                                  const double* __restrict__ t0,
                                                                  const double* __restrict__ c,
                                                                  double* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * n) return;
  const int r = (int)(e / n), i = (int)(e % n);
  double acc = 0.0;
  for (int64_t g = 0; g < X; ++g) {
    const double* Lr = lbar + ((size_t)g * M + r) * n;
    const double* T = t0 + (size_t)g * n * n + (size_t)i * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += Lr[j] * T[j];
    acc += 4.0 * c[g] * Lr[i] - 2.0 * s;
  }
  grad[e] = acc;
}

// d[rho] = (row_rho . psi_a, row_rho . psi_b) for stored row rho of pair
// (a, b) = pair_of_row[rho]; one wave per row, lanes over r, fixed-order sum
__global__ __launch_bounds__(256) void residual_row_dots_kernel(int M, int n, int64_t total_rows,
                                                                const double* __restrict__ rows,
                                                                const int* __restrict__ pair_of_row,
                                                                const double* __restrict__ trial,
                                                                double* __restrict__ d) {
  const int64_t rho = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (rho >= total_rows) return;
  const int a = pair_of_row[2 * rho], b = pair_of_row[2 * rho + 1];
  const double* row = rows + (size_t)rho * M;
  double sa = 0.0, sb = 0.0;
  for (int r = lane; r < M; r += 64) {
    const double v = row[r];
    sa += v * trial[(size_t)r * n + a];
    sb += v * trial[(size_t)r * n + b];
  }
  for (int off = 32; off >= 1; off >>= 1) {
    sa += __shfl_xor(sa, off, 64);
    sb += __shfl_xor(sb, off, 64);
  }
  if (lane == 0) {
    d[2 * rho] = sa;
    d[2 * rho + 1] = sb;
  }
}

// grad[r][i] -= LO part; one thread per (r, i).  pair_off / pair_k: [n][n]
// first row and rank of the stored pair (a, b), a <= b.
__global__ __launch_bounds__(256) void residual_grad_lo_kernel(int M, int n, const double* __restrict__ rows,
                                                               const int64_t* __restrict__ pair_off,
                                                               const int* __restrict__ pair_k,
                                                               const double* __restrict__ d,
                                                               double* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * n) return;
  const int r = (int)(e / n), i = (int)(e % n);
  double acc = 0.0;
  for (int j = 0; j < n; ++j) {
    const int a = i < j ? i : j, b = i < j ? j : i;
    const int64_t off = pair_off[a * n + b];
    const int K = pair_k[a * n + b];
    for (int k = 0; k < K; ++k) {
      const int64_t ru = off + k, rv = off + K + k;
      const double u = rows[(size_t)ru * M + r], v = rows[(size_t)rv * M + r];
      const double du_a = d[2 * ru], du_b = d[2 * ru + 1], dv_a = d[2 * rv], dv_b = d[2 * rv + 1];
      if (a == b)
        acc += u * dv_a + v * du_a;
      else if (i == a)
        acc += 4.0 * u * dv_b - 2.0 * v * du_b;
      else
        acc += 4.0 * v * du_a - 2.0 * u * dv_a;
    }
  }
  grad[e] -= acc;
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
  float s_db1 = 0.0f, s_db2 = 0.0f, s_dw3 = 0.0f, s_dw1[RF] = {}, s_db3 = 0.0f;
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
                                    const double* grad, float* x) {
  if (nw <= 0) return hipSuccess;
  const int64_t tot = nw * n;
  hipLaunchKernelGGL(residual_features_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, n, nw,
                     (const double2*)theta, orb, grad, x);
  return hipGetLastError();
}

// t[w] = (1000 Re(sum_c e_exact[w][c] - sum_c e_lo[w][c]) - shift) / scale
__global__ __launch_bounds__(256) void residual_target_kernel(int64_t nw, const double2* __restrict__ e_exact,
                                                              const double2* __restrict__ e_lo, double shift,
                                                              double scale, double* __restrict__ t) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= nw) return;
  const double d = (e_exact[2 * w].x + e_exact[2 * w + 1].x) - (e_lo[2 * w].x + e_lo[2 * w + 1].x);
  t[w] = (1000.0 * d - shift) / scale;
}

// out[w] = E_J + E_K (+ (pred[w] scale + shift) / 1000 on the real part)
__global__ __launch_bounds__(256) void residual_apply_kernel(int64_t nw, const double2* __restrict__ e,
                                                             const double* __restrict__ pred, double scale,
                                                             double shift, double2* __restrict__ out) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= nw) return;
  double2 v;
  v.x = e[2 * w].x + e[2 * w + 1].x;
  v.y = e[2 * w].y + e[2 * w + 1].y;
  if (pred) v.x += (pred[w] * scale + shift) / 1000.0;
  out[w] = v;
}

hipError_t launch_residual_target(hipStream_t s, int64_t nw, const double* e_exact, const double* e_lo, double shift,
                                  double scale, double* t) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(residual_target_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, nw,
                     (const double2*)e_exact, (const double2*)e_lo, shift, scale, t);
  return hipGetLastError();
}

hipError_t launch_residual_apply(hipStream_t s, int64_t nw, const double* energy, const double* pred, double scale,
                                 double shift, double* out) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(residual_apply_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, nw,
                     (const double2*)energy, pred, scale, shift, (double2*)out);
  return hipGetLastError();
}

size_t residual_gradient_workspace(int n, int64_t X, int64_t total_rows) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(sizeof(double) * (size_t)X * n * n) + al(sizeof(double) * (size_t)X) +
         al(sizeof(double) * 2 * (size_t)total_rows);
}

hipError_t launch_residual_gradient(hipStream_t s, int M, int n, int64_t X, const double* lbar, const double* trial,
                                    int64_t total_rows, const double* rows, const int* pair_of_row,
                                    const int64_t* pair_off, const int* pair_k, void* work, double* grad) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* base = (char*)work;
  double* t0 = (double*)base;
  double* c = (double*)(base + al(sizeof(double) * (size_t)X * n * n));
  double* d = (double*)((char*)c + al(sizeof(double) * (size_t)X));
  const int64_t mn = (int64_t)M * n;
  if (X > 0) {
    const int64_t tot = X * n * n;
    hipLaunchKernelGGL(residual_t0_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, n, X, lbar, trial,
                       t0);
    hipLaunchKernelGGL(residual_trace_kernel, dim3((unsigned)((X + 255) / 256)), dim3(256), 0, s, n, X, t0, c);
  }
  hipLaunchKernelGGL(residual_grad_exact_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, M, n, X, lbar,
                     t0, c, grad);
  if (total_rows > 0) {
    hipLaunchKernelGGL(residual_row_dots_kernel, dim3((unsigned)((total_rows + 3) / 4)), dim3(256), 0, s, M, n,
                       total_rows, rows, pair_of_row, trial, d);
    hipLaunchKernelGGL(residual_grad_lo_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, M, n, rows,
                       pair_off, pair_k, d, grad);
  }
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
