// Green's-function intermediate Q = theta = phi (Psi_T^T phi)^{-1} (Eq. 15)
// for a batch of walkers, FP64.  One workgroup (4 waves) per walker:
//   1. O = Psi_T^T phi on MFMA (real trial x complex walker -> two real
//      16x16 blocks per block pair), written to LDS;
//   2. in-place Gauss-Jordan exchange with partial pivoting (largest
//      |re|+|im| among the rows not yet used as pivots), 4x4 register blocks
//      per thread; gives O^{-1}, log det O and the zero-pivot index;
//   3. theta = phi O^{-1} on MFMA (complex x complex as four real products)
//      with O^{-1} read from LDS.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

template <int NB>
__global__ __launch_bounds__(256) void green_theta_kernel(int M, int n, const double* __restrict__ trial,
                                                          const double2* __restrict__ phi,
                                                          double2* __restrict__ theta,
                                                          double2* __restrict__ logov, int* __restrict__ info) {
  constexpr int NP = 16 * NB;
  extern __shared__ double2 smem[];
  double2* sO = smem;               // [NP][NP]: O, then O^{-1}
  double2* sColBuf = sO + NP * NP;  // column k before the exchange (two buffers)
  double2* sRow = sColBuf + 2 * NP; // pivot row scaled by 1/pivot
  __shared__ int sUsed[NP];
  __shared__ int sPiv[NP];
  __shared__ int sPinv[NP];
  __shared__ int sZero;
  __shared__ double2 sInv;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int lr = lane & 15;   // row of A / column of B and D within a 16-block
  const int lk = lane >> 4;   // k index of A and B, row group of D
  const size_t w = blockIdx.x;
  const double2* ph = phi + w * (size_t)M * n;

  // ---------------------------------------------------------------- phase 1
  constexpr int NPAIR = NB * NB;
  constexpr int PPW = (NPAIR + 3) / 4;
  d4 accR[PPW], accI[PPW];
#pragma unroll
  for (int p = 0; p < PPW; ++p) { accR[p] = d4zero(); accI[p] = d4zero(); }

  for (int r0 = 0; r0 < M; r0 += 4) {
    const int r = r0 + lk;
#pragma unroll
    for (int p = 0; p < PPW; ++p) {
      const int bp = wv + 4 * p;
      if (bp < NPAIR) {
        const int I = bp / NB, J = bp % NB;
        const int i = 16 * I + lr, j = 16 * J + lr;
        const double a = (r < M && i < n) ? trial[(size_t)r * n + i] : 0.0;
        const double2 b = (r < M && j < n) ? ph[(size_t)r * n + j] : make_double2(0.0, 0.0);
        accR[p] = mfma16(a, b.x, accR[p]);
        accI[p] = mfma16(a, b.y, accI[p]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int bp = wv + 4 * p;
    if (bp < NPAIR) {
      const int I = bp / NB, J = bp % NB;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * I + 4 * v + lk, col = 16 * J + lr;
        sO[row * NP + col] = make_double2(accR[p][v], accI[p][v]);
      }
    }
  }
  if (tid < NP) sUsed[tid] = (tid < n) ? 0 : 1;
  if (tid == 0) sZero = 0;
  __syncthreads();

  // ---------------------------------------------------------------- phase 2
  const int ty = tid >> 4, tx = tid & 15;   // owns rows ty+16a, cols tx+16b
  double2 e[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) e[a][b] = sO[(ty + 16 * a) * NP + tx + 16 * b];

  double logabs = 0.0, arg = 0.0;  // lane 0 of wave 0 only
  for (int k = 0; k < n; ++k) {
    // column k goes to alternating buffers: a thread may still read the
    // previous step's column while another publishes this one
    double2* sCol = sColBuf + (k & 1) * NP;
    // publish column k
    if (tx == (k & 15)) {
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b == (k >> 4)) sCol[ty + 16 * a] = e[a][b];
      }
    }
    __syncthreads();
    if (wv == 0) {
      double mag = -1.0;
      if (lane < NP && !sUsed[lane]) mag = fabs(sCol[lane].x) + fabs(sCol[lane].y);
      int idx = lane;
      // max with lowest index on ties (fixed shuffle tree)
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double om = __shfl_down(mag, off, 64);
        const int oi = __shfl_down(idx, off, 64);
        if (om > mag || (om == mag && oi < idx)) { mag = om; idx = oi; }
      }
      if (lane == 0) {
        const int p = idx;
        sPiv[k] = p;
        sUsed[p] = 1;
        const double2 piv = sCol[p];
        if (!(mag > 0.0)) {
          sZero = k + 1;
        } else {
          sInv = crecip(piv);
          logabs += log(hypot(piv.x, piv.y));
          arg += atan2(piv.y, piv.x);
        }
      }
    }
    __syncthreads();
    if (sZero) break;
    const int p = sPiv[k];
    const double2 inv = sInv;
    // publish the pivot row scaled by 1/pivot
    if (ty == (p & 15)) {
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        if (a == (p >> 4)) {
#pragma unroll
          for (int b = 0; b < NB; ++b) sRow[tx + 16 * b] = cmul(e[a][b], inv);
        }
      }
    }
    __syncthreads();
    // exchange step on pivot (p, k)
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = ty + 16 * a;
      const double2 cik = sCol[i];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = tx + 16 * b;
        const double2 rpj = sRow[j];
        double2 v = e[a][b];
        if (i == p) {
          v = (j == k) ? inv : make_double2(-rpj.x, -rpj.y);
        } else if (j == k) {
          v = cmul(cik, inv);
        } else {
          v = csub(v, cmul(cik, rpj));
        }
        e[a][b] = v;
      }
    }
    // sCol / sRow are rewritten only after the next barrier
  }
  const int zero = sZero;

  // un-permute: O^{-1}[k][p_m] = R[p_k][m]
  if (!zero && tid < n) sPinv[sPiv[tid]] = tid;
  __syncthreads();
  if (!zero) {
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = ty + 16 * a;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int m = tx + 16 * b;
        if (i < n && m < n) sO[sPinv[i] * NP + sPiv[m]] = e[a][b];
      }
    }
  }
  // padded rows/columns of O^{-1} are zero
  for (int idx = tid; idx < NP * NP; idx += 256) {
    const int row = idx / NP, col = idx % NP;
    if (row >= n || col >= n) sO[idx] = make_double2(0.0, 0.0);
  }
  if (tid == 0) {
    info[w] = zero;
    if (logov) {
      double2 ld;
      if (zero) {
        ld = make_double2(__builtin_nan(""), __builtin_nan(""));
      } else {
        // sign of the permutation k -> p_k from its cycle count
        int cycles = 0;
        unsigned long long seen = 0ull;
        for (int s = 0; s < n; ++s) {
          if (seen >> s & 1ull) continue;
          ++cycles;
          int c = s;
          while (!(seen >> c & 1ull)) { seen |= 1ull << c; c = sPiv[c]; }
        }
        double im = arg + ((n - cycles) & 1 ? M_PI : 0.0);
        im = remainder(im, 2.0 * M_PI);  // (-pi, pi]
        if (im <= -M_PI) im += 2.0 * M_PI;
        ld = make_double2(logabs, im);
      }
      logov[w] = ld;
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- phase 3
  double2* th = theta + w * (size_t)M * n;
  const int nrb = (M + 15) / 16;
  const int ksteps = (n + 3) / 4;
  for (int rb = wv; rb < nrb; rb += 4) {
    d4 aR[NB], aI[NB];
#pragma unroll
    for (int J = 0; J < NB; ++J) { aR[J] = d4zero(); aI[J] = d4zero(); }
    const int r = 16 * rb + lr;
    for (int ks = 0; ks < ksteps; ++ks) {
      const int kk = 4 * ks + lk;
      const double2 av = (r < M && kk < n) ? ph[(size_t)r * n + kk] : make_double2(0.0, 0.0);
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        const double2 bv = sO[kk * NP + 16 * J + lr];
        aR[J] = mfma16(av.x, bv.x, aR[J]);
        aR[J] = mfma16(-av.y, bv.y, aR[J]);
        aI[J] = mfma16(av.x, bv.y, aI[J]);
        aI[J] = mfma16(av.y, bv.x, aI[J]);
      }
    }
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      const int j = 16 * J + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + 4 * v + lk;
        if (row < M && j < n) {
          th[(size_t)row * n + j] = zero ? make_double2(__builtin_nan(""), __builtin_nan(""))
                                         : make_double2(aR[J][v], aI[J][v]);
        }
      }
    }
  }
}

template <int NB>
static hipError_t launch_gt(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                            double* theta, double* logov, int* info) {
  constexpr int NP = 16 * NB;
  const size_t lds = sizeof(double2) * (NP * NP + 3 * NP);
  hipError_t e = hipFuncSetAttribute((const void*)green_theta_kernel<NB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(green_theta_kernel<NB>, dim3((unsigned)nw), dim3(256), lds, s, M, n, trial,
                     (const double2*)phi, (double2*)theta, (double2*)logov, info);
  return hipGetLastError();
}

hipError_t launch_green_theta(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                              double* theta, double* logov, int* info) {
  if (nw <= 0) return hipSuccess;
  if (n <= 16) return launch_gt<1>(s, M, n, nw, trial, phi, theta, logov, info);
  if (n <= 32) return launch_gt<2>(s, M, n, nw, trial, phi, theta, logov, info);
  if (n <= 48) return launch_gt<3>(s, M, n, nw, trial, phi, theta, logov, info);
  return launch_gt<4>(s, M, n, nw, trial, phi, theta, logov, info);
}

}  // namespace lofqmc
