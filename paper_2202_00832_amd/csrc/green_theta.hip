// Green's-function intermediate Q = theta = phi (Psi_T^T phi)^{-1} (Eq. 15)
// for a batch of walkers, FP64, as three kernels so that the latency-bound
// elimination does not hold the MFMA work back:
//   1. overlap_kernel: O_w = Psi_T^T phi_w on v_mfma_f64_16x16x4_f64 (real
//      trial x complex walker -> two real 16x16 blocks per block pair);
//      16-row slabs of phi_w and Psi_T are staged in LDS with coalesced loads,
//      prefetched two slabs ahead.  One workgroup per walker.
//   2. invert_kernel: in-place Gauss-Jordan exchange with partial pivoting
//      (largest |re|+|im| among the rows not yet used as pivots, compared to
//      45 bits, lowest row on ties); one wave per 16-column panel with a row
//      per lane, one barrier per elimination step.  Gives O^{-1}, log det O
//      and the zero-pivot index.
//   3. apply_kernel: theta = phi O^{-1} on MFMA with three real products per
//      complex block (re = P1 - P2, im = P3 - P1 - P2 with P1 = a_re b_re,
//      P2 = a_im b_im, P3 = (a_re + a_im)(b_re + b_im)); one workgroup per
//      walker with O^{-1} in LDS, one wave per 16-row block.  theta is written
//      walker-major [w][r][j] or, with the orbital-major flag, as [j][r][w];
//      walkers 8g .. 8g+7 then run on the same XCD so that their interleaved
//      16-byte stores meet in one L2.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

template <int NB>
struct GtCfg {
  static constexpr int NP = 16 * NB;
  static constexpr int KC = 16;                // rows of r per overlap slab
  static constexpr int SLOTS = KC * NP;        // complex slots of a phi slab
  static constexpr int PER = (SLOTS + 255) / 256;
  static constexpr int NKS = NP / 4;           // K-steps of theta = phi O^{-1}
};

// ---------------------------------------------------------------------------
// 1. O_w = Psi_T^T phi_w, written as a padded NP x NP complex block per walker
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256) void overlap_kernel(int M, int n, const double* __restrict__ trial,
                                                      const double2* __restrict__ phi,
                                                      double2* __restrict__ O) {
  using C = GtCfg<NB>;
  constexpr int NP = C::NP;
  __shared__ double2 sPh[2][C::SLOTS];
  __shared__ double sPs[2][C::SLOTS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const size_t w = blockIdx.x;
  const double2* ph = phi + w * (size_t)M * n;

  constexpr int NPAIR = NB * NB;
  constexpr int PPW = (NPAIR + 3) / 4;
  d4 accR[PPW], accI[PPW];
#pragma unroll
  for (int p = 0; p < PPW; ++p) { accR[p] = d4zero(); accI[p] = d4zero(); }

  double2 pP0[C::PER], pP1[C::PER], pP2[C::PER];
  double pS0[C::PER], pS1[C::PER], pS2[C::PER];
  auto load_slab = [&](int c, double2 (&dP)[C::PER], double (&dS)[C::PER]) {
#pragma unroll
    for (int q = 0; q < C::PER; ++q) {
      const int s = tid + 256 * q;
      const int rr = s / NP, j = s % NP;
      const int r = C::KC * c + rr;
      const bool ok = s < C::SLOTS && r < M && j < n;
      dP[q] = ok ? ph[(size_t)r * n + j] : make_double2(0.0, 0.0);
      dS[q] = ok ? trial[(size_t)r * n + j] : 0.0;
    }
  };
  auto store_slab = [&](int buf, const double2 (&sP)[C::PER], const double (&sS)[C::PER]) {
#pragma unroll
    for (int q = 0; q < C::PER; ++q) {
      const int s = tid + 256 * q;
      if (s < C::SLOTS) {
        sPh[buf][s] = sP[q];
        sPs[buf][s] = sS[q];
      }
    }
  };
  auto mma_slab = [&](int buf) {
#pragma unroll
    for (int s4 = 0; s4 < C::KC / 4; ++s4) {
      const int row = (4 * s4 + lk) * NP;
      if constexpr (NB == 4) {
        // wave q owns the pairs (I, q): one B fragment per K-step
        const double2 b = sPh[buf][row + 16 * wv + lr];
#pragma unroll
        for (int p = 0; p < PPW; ++p) {
          const double a = sPs[buf][row + 16 * p + lr];
          accR[p] = mfma16(a, b.x, accR[p]);
          accI[p] = mfma16(a, b.y, accI[p]);
        }
      } else {
#pragma unroll
        for (int p = 0; p < PPW; ++p) {
          const int bp = wv + 4 * p;
          if (bp < NPAIR) {
            const int I = bp / NB, J = bp % NB;
            const double a = sPs[buf][row + 16 * I + lr];
            const double2 b = sPh[buf][row + 16 * J + lr];
            accR[p] = mfma16(a, b.x, accR[p]);
            accI[p] = mfma16(a, b.y, accI[p]);
          }
        }
      }
    }
  };
  const int nslab = (M + C::KC - 1) / C::KC;
  // iteration c: issue slab c+2, multiply slab c, store slab c+1
  auto iter = [&](int c, double2 (&nP)[C::PER], double (&nS)[C::PER], const double2 (&sP)[C::PER],
                  const double (&sS)[C::PER]) {
    if (c + 2 < nslab) load_slab(c + 2, nP, nS);
    mma_slab(c & 1);
    if (c + 1 < nslab) store_slab((c + 1) & 1, sP, sS);
    __syncthreads();
  };
  load_slab(0, pP0, pS0);
  if (nslab > 1) load_slab(1, pP1, pS1);
  store_slab(0, pP0, pS0);
  __syncthreads();
  for (int c = 0; c < nslab; c += 3) {
    iter(c, pP2, pS2, pP1, pS1);
    if (c + 1 < nslab) iter(c + 1, pP0, pS0, pP2, pS2);
    if (c + 2 < nslab) iter(c + 2, pP1, pS1, pP0, pS0);
  }
  double2* Ow = O + w * (size_t)NP * NP;
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int bp = wv + 4 * p;
    if (bp < NPAIR) {
      const int I = bp / NB, J = bp % NB;
#pragma unroll
      for (int v = 0; v < 4; ++v) Ow[(16 * I + 4 * v + lk) * NP + 16 * J + lr] = make_double2(accR[p][v], accI[p][v]);
    }
  }
}

// ---------------------------------------------------------------------------
// 2. O_w -> O_w^{-1} in place (padded rows/columns zero), log det, info.
//    Wave q owns the 16 columns 16q .. 16q+15 of every row; lane l holds rows
//    l and l + 64.  Step k: the wave owning column k picks the pivot row (its
//    column is already updated), publishes the column through LDS, and after
//    one barrier every wave reads the multipliers of its rows and the pivot
//    row of its own columns (written by its lane p) from LDS, and updates.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(64 * NB) void invert_kernel(int n, double2* __restrict__ O,
                                                          double2* __restrict__ logov, int* __restrict__ info) {
  constexpr int NP = 16 * NB;
  constexpr int RPL = (NP + 63) / 64;        // rows per lane
  __shared__ double2 sCol[2][NP];
  __shared__ int sPiv[NP];
  __shared__ int sPinv[NP];
  __shared__ double2 sPivV[NP];
  __shared__ double2 sRowW[NB][16];
  __shared__ int sZero;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const size_t w = blockIdx.x;
  double2* Ow = O + w * (size_t)NP * NP;

  double2 e[RPL][16];
  bool used[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int row = lane + 64 * t;
    used[t] = row >= n;   // padding rows are never pivots
#pragma unroll
    for (int j = 0; j < 16; ++j) e[t][j] = row < NP ? Ow[(size_t)row * NP + 16 * wv + j] : make_double2(0.0, 0.0);
  }
  if (tid == 0) sZero = 0;
  __syncthreads();

  int zero = 0;
  for (int kb = 0; kb < NB; ++kb) {
    // fixed trip count (fully unrolled, so e[][c] stays in registers); the
    // step conditions are uniform, so the barrier inside is reached by all
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int k = 16 * kb + c;
      if (k >= n || zero) continue;
      if (wv == kb) {
        // pivot: largest |re|+|im| (45 leading bits) among unused rows, lowest row on ties
        unsigned long long key = 0ull;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int row = lane + 64 * t;
          const double2 v = e[t][c];
          const unsigned long long mb = (unsigned long long)__double_as_longlong(fabs(v.x) + fabs(v.y));
          const unsigned long long kt = used[t] ? 0ull : ((mb & ~127ull) | (unsigned long long)(127 - row));
          key = kt > key ? kt : key;
          if (row < NP) sCol[k & 1][row] = v;
        }
        key = wave_max_u64(key);
        if (lane == 0) {
          if ((key >> 7) == 0ull) {
            sZero = k + 1;
          } else {
            sPiv[k] = 127 - (int)(key & 127ull);
          }
        }
      }
      __syncthreads();
      zero = sZero;
      if (zero) continue;
      const int p = sPiv[k];
      const double2 piv = sCol[k & 1][p];
      const double rn = 1.0 / (piv.x * piv.x + piv.y * piv.y);
      const double2 inv = make_double2(piv.x * rn, -piv.y * rn);
      if (wv == 0 && lane == 0) sPivV[k] = piv;
      // pivot row (own 16 columns): lane p % 64 writes it to this wave's LDS
      // slot and every lane of the wave reads it back; a wavefront-scope
      // release/acquire pair around a wave barrier orders the two (without
      // it the compiler may let the other lanes read before the write)
      const int pl = p & 63, pt = p >> 6;
      if (lane == pl) {
#pragma unroll
        for (int j = 0; j < 16; ++j) sRowW[wv][j] = (RPL > 1 && pt == 1) ? e[RPL - 1][j] : e[0][j];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double2 apj[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) apj[j] = sRowW[wv][j];
      // uniform exchange update A[i][j] -= m_i A[p][j] with m_i = (A[i][k] + [i == p]) / pivot,
      // which leaves -A[p][j] / pivot on the pivot row; the owner of column k then
      // writes A[i][k] / pivot (1 / pivot on row p)
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = lane + 64 * t;
        double2 ci = row < NP ? sCol[k & 1][row] : make_double2(0.0, 0.0);
        const double2 cc = row == p ? make_double2(1.0, 0.0) : ci;
        ci.x += row == p ? 1.0 : 0.0;
        const double2 mi = cmul(ci, inv);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          double2 v = e[t][j];
          v.x = fma(-mi.x, apj[j].x, fma(mi.y, apj[j].y, v.x));
          v.y = fma(-mi.x, apj[j].y, fma(-mi.y, apj[j].x, v.y));
          e[t][j] = v;
        }
        if (wv == kb) e[t][c] = cmul(cc, inv);
        if (row == p) used[t] = true;
      }
    }
  }
  __syncthreads();

  // un-permute: O^{-1}[k][p_m] = R[p_k][m]; padded rows/columns stay zero
  if (!zero && tid < n) sPinv[sPiv[tid]] = tid;
  __syncthreads();
  if (!zero) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = lane + 64 * t;
      if (i < n) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int m = 16 * wv + j;
          if (m < n) Ow[(size_t)sPinv[i] * NP + sPiv[m]] = e[t][j];
        }
      }
    }
  }
  if (wv == 0) {
    // log det O = sum_k log(pivot_k) + i pi * parity of the permutation k -> p_k;
    // the parity is that of its number of inversions, counted by all lanes
    double la = 0.0, ar = 0.0;
    int inv_count = 0;
    if (!zero) {
      for (int k = lane; k < n; k += 64) {
        const double2 pv = sPivV[k];
        la += log(hypot(pv.x, pv.y));
        ar += atan2(pv.y, pv.x);
        const int pk = sPiv[k];
        for (int j = k + 1; j < n; ++j) inv_count += sPiv[j] < pk ? 1 : 0;
      }
    }
    la = wave_sum_lane0(la);
    ar = wave_sum_lane0(ar);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) inv_count += __shfl_down(inv_count, off, 64);
    if (lane == 0) {
      info[w] = zero;
      if (logov) {
        double2 ld;
        if (zero) {
          ld = make_double2(__builtin_nan(""), __builtin_nan(""));
        } else {
          double im = ar + ((inv_count & 1) ? M_PI : 0.0);
          im = remainder(im, 2.0 * M_PI);  // (-pi, pi]
          if (im <= -M_PI) im += 2.0 * M_PI;
          ld = make_double2(la, im);
        }
        logov[w] = ld;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3. theta_w = phi_w O_w^{-1}; one 512-thread workgroup per walker, O_w^{-1}
//    staged once in LDS, wave (q, h) takes the 16-row blocks q, q+4, ...
//    against half h of the column blocks
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(512) void apply_kernel(int M, int n, int64_t nw, const double2* __restrict__ phi,
                                                    const double2* __restrict__ Oinv, const int* __restrict__ info,
                                                    double2* __restrict__ theta, int orbital_major) {
  using C = GtCfg<NB>;
  constexpr int NP = C::NP;
  __shared__ double2 sB[NP * NP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // workgroups go round-robin over the 8 XCDs; walkers 8g .. 8g+7 share an
  // XCD so that their interleaved orbital-major 16-byte stores meet in one L2
  int64_t w;
  {
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, slot = b >> 3;
    w = 8 * (xcd + 8 * (slot >> 3)) + (slot & 7);
    if (w >= nw) return;
  }
  const double2* Bw = Oinv + w * (size_t)NP * NP;
  for (int e = tid; e < NP * NP; e += 512) sB[e] = Bw[e];
  __syncthreads();
  const int ksteps = (n + 3) / 4;
  const double2* ph = phi + w * (size_t)M * n;
  const bool bad = info[w] != 0;
  const double nan = __builtin_nan("");
  // wave (q, h): 16-row blocks q, q+4, ... against the column blocks of half
  // h (JH blocks each), which keeps the accumulators to 3 * JH 16x16 blocks
  constexpr int JH = (NB + 1) / 2;
  const int q = wv >> 1, hf = wv & 1;
  const int nrb = (M + 15) / 16;
  for (int rb = q; rb < nrb; rb += 4) {
    const int r = 16 * rb + lr;
    d4 P1[JH], P2[JH], P3[JH];
#pragma unroll
    for (int J = 0; J < JH; ++J) { P1[J] = d4zero(); P2[J] = d4zero(); P3[J] = d4zero(); }
    // K-steps in groups of four (bounded prefetch of phi)
    for (int kg = 0; kg < (ksteps + 3) / 4; ++kg) {
      double2 av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = 16 * kg + 4 * u + lk;
        av[u] = (r < M && kk < n) ? ph[(size_t)r * n + kk] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = 16 * kg + 4 * u + lk;
        const double as = av[u].x + av[u].y;
#pragma unroll
        for (int J = 0; J < JH; ++J) {
          const int JJ = hf * JH + J;
          if (JJ < NB) {
            const double2 bv = kk < NP ? sB[kk * NP + 16 * JJ + lr] : make_double2(0.0, 0.0);
            P1[J] = mfma16(av[u].x, bv.x, P1[J]);
            P2[J] = mfma16(av[u].y, bv.y, P2[J]);
            P3[J] = mfma16(as, bv.x + bv.y, P3[J]);
          }
        }
      }
    }
#pragma unroll
    for (int J = 0; J < JH; ++J) {
      const int j = 16 * (hf * JH + J) + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + 4 * v + lk;
        if (hf * JH + J < NB && row < M && j < n) {
          const double re = P1[J][v] - P2[J][v];
          const double im = P3[J][v] - P1[J][v] - P2[J][v];
          const double2 val = bad ? make_double2(nan, nan) : make_double2(re, im);
          if (orbital_major)
            theta[((size_t)j * M + row) * nw + w] = val;
          else
            theta[(w * (size_t)M + row) * n + j] = val;
        }
      }
    }
  }
}

size_t green_theta_workspace(int n, int64_t nw) {
  const size_t NP = 16 * (size_t)((n + 15) / 16);
  return sizeof(double2) * NP * NP * (size_t)nw;
}

template <int NB>
static hipError_t launch_gt(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                            double* theta, double* logov, int* info, int orbital_major, double* work,
                            const ProfHook* prof) {
  double2* O = reinterpret_cast<double2*>(work);
  prof_mark(prof, "overlap_kernel");
  hipLaunchKernelGGL(overlap_kernel<NB>, dim3((unsigned)nw), dim3(256), 0, s, M, n, trial, (const double2*)phi, O);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_mark(prof, "invert_kernel");
  hipLaunchKernelGGL(invert_kernel<NB>, dim3((unsigned)nw), dim3(64 * NB), 0, s, n, O, (double2*)logov, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = 64 * ((nw + 63) / 64);
  prof_mark(prof, "apply_kernel");
  hipLaunchKernelGGL(apply_kernel<NB>, dim3((unsigned)grid), dim3(512), 0, s, M, n, nw, (const double2*)phi,
                     (const double2*)O, info, (double2*)theta, orbital_major);
  return hipGetLastError();
}

hipError_t launch_green_theta(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                              double* theta, double* logov, int* info, int orbital_major, double* work,
                              const ProfHook* prof) {
  if (nw <= 0) return hipSuccess;
  if (n <= 16) return launch_gt<1>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major, work, prof);
  if (n <= 32) return launch_gt<2>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major, work, prof);
  if (n <= 48) return launch_gt<3>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major, work, prof);
  if (n <= 64) return launch_gt<4>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major, work, prof);
  if (n <= 80) return launch_gt<5>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major, work, prof);
  return launch_gt<6>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major, work, prof);
}

}  // namespace lofqmc
