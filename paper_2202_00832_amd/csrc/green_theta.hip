// Green's-function intermediate Q = theta = phi (Psi_T^T phi)^{-1} (Eq. 15)
// for a batch of walkers, FP64.  One workgroup (4 waves) per walker:
//   1. O = Psi_T^T phi on MFMA (real trial x complex walker -> two real
//      16x16 blocks per block pair).  16-row slabs of phi and Psi_T are
//      staged in LDS with coalesced loads, double-buffered.
//   2. In-place Gauss-Jordan exchange with partial pivoting (largest
//      |re|+|im| among the rows not yet used as pivots, compared to 46 bits,
//      lowest row on ties), 4x4 register blocks per thread.  Every wave
//      repeats the pivot search (a DPP max over a 64-bit key) on the published
//      column, so a step needs two barriers.  Gives O^{-1}, the pivots (for
//      log det O, summed afterwards in parallel) and the zero-pivot index.
//   3. theta = phi O^{-1} on MFMA with three real products per complex block
//      (re = P1 - P2, im = P3 - P1 - P2 with P1 = a_re b_re, P2 = a_im b_im,
//      P3 = (a_re + a_im)(b_re + b_im)), O^{-1} from LDS, the next half slab
//      of phi prefetched into registers while the current one is multiplied.
//      theta is written walker-major [w][r][j] or, with the orbital-major
//      flag, as [j][r][w]; then consecutive walkers are placed on the same XCD
//      so that the interleaved 16-byte stores meet in one L2.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

template <int NB>
struct GtCfg {
  static constexpr int NP = 16 * NB;
  static constexpr int KC = 16;                                    // rows of r per phase-1 slab
  static constexpr int PH_SLOTS = KC * NP;                         // complex slots of a phi slab
  static constexpr int PER = (PH_SLOTS + 255) / 256;
  static constexpr size_t P1_BYTES = 2 * PH_SLOTS * sizeof(double2) + 2 * PH_SLOTS * sizeof(double);
  static constexpr size_t P2_BYTES = (size_t)(NP * NP + 3 * NP) * sizeof(double2);
  static constexpr size_t LDS = P1_BYTES > P2_BYTES ? P1_BYTES : P2_BYTES;
  static constexpr int NKS = NP / 4;                               // max K-steps of phase 3
  static constexpr int NKH = NKS / 2;                              // K-steps per prefetched half slab
};

template <int NB>
__global__ __launch_bounds__(256, 2) void green_theta_kernel(int M, int n, const double* __restrict__ trial,
                                                             const double2* __restrict__ phi,
                                                             double2* __restrict__ theta,
                                                             double2* __restrict__ logov, int* __restrict__ info,
                                                             int orbital_major, int64_t nw) {
  using C = GtCfg<NB>;
  constexpr int NP = C::NP;
  extern __shared__ double4 smem_raw[];
  char* smem = reinterpret_cast<char*>(smem_raw);
  __shared__ int sPiv[NP];
  __shared__ int sPinv[NP];
  __shared__ double2 sPivV[NP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int lr = lane & 15;   // row of A / column of B and D within a 16-block
  const int lk = lane >> 4;   // k index of A and B, row group of D
  // orbital-major output: walkers w..w+7 share 128-byte lines of theta, so
  // keep consecutive walkers on one XCD (workgroups go round-robin over 8 XCDs)
  size_t w = blockIdx.x;
  if (orbital_major) {
    const size_t per = (nw + 7) / 8;
    w = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (w >= (size_t)nw) return;
  }
  const double2* ph = phi + w * (size_t)M * n;

  // ---------------------------------------------------------------- phase 1
  double2* sPh = reinterpret_cast<double2*>(smem);                          // [2][KC][NP]
  double* sPs = reinterpret_cast<double*>(smem + 2 * C::PH_SLOTS * sizeof(double2));  // [2][KC][NP]
  constexpr int NPAIR = NB * NB;
  constexpr int PPW = (NPAIR + 3) / 4;
  d4 accR[PPW], accI[PPW];
#pragma unroll
  for (int p = 0; p < PPW; ++p) { accR[p] = d4zero(); accI[p] = d4zero(); }

  // slab c is loaded into registers two iterations before it is consumed
  // (three register sets), stored to LDS one iteration before, double-buffered
  double2 pP0[C::PER], pP1[C::PER], pP2[C::PER];
  double pS0[C::PER], pS1[C::PER], pS2[C::PER];
  auto load_slab = [&](int c, double2 (&dP)[C::PER], double (&dS)[C::PER]) {
#pragma unroll
    for (int q = 0; q < C::PER; ++q) {
      const int s = tid + 256 * q;
      const int rr = s / NP, j = s % NP;
      const int r = C::KC * c + rr;
      const bool ok = s < C::PH_SLOTS && r < M && j < n;
      dP[q] = ok ? ph[(size_t)r * n + j] : make_double2(0.0, 0.0);
      dS[q] = ok ? trial[(size_t)r * n + j] : 0.0;
    }
  };
  auto store_slab = [&](int buf, const double2 (&sP)[C::PER], const double (&sS)[C::PER]) {
#pragma unroll
    for (int q = 0; q < C::PER; ++q) {
      const int s = tid + 256 * q;
      if (s < C::PH_SLOTS) {
        sPh[buf * C::PH_SLOTS + s] = sP[q];
        sPs[buf * C::PH_SLOTS + s] = sS[q];
      }
    }
  };
  auto mma_slab = [&](int buf) {
    const double2* P = sPh + buf * C::PH_SLOTS;
    const double* S = sPs + buf * C::PH_SLOTS;
#pragma unroll
    for (int s4 = 0; s4 < C::KC / 4; ++s4) {
      const int row = (4 * s4 + lk) * NP;
      if constexpr (NB == 4) {
        // wave q owns the pairs (I, q): one B fragment per K-step
        const double2 b = P[row + 16 * wv + lr];
#pragma unroll
        for (int p = 0; p < PPW; ++p) {
          const double a = S[row + 16 * p + lr];
          accR[p] = mfma16(a, b.x, accR[p]);
          accI[p] = mfma16(a, b.y, accI[p]);
        }
      } else {
#pragma unroll
        for (int p = 0; p < PPW; ++p) {
          const int bp = wv + 4 * p;
          if (bp < NPAIR) {
            const int I = bp / NB, J = bp % NB;
            const double a = S[row + 16 * I + lr];
            const double2 b = P[row + 16 * J + lr];
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

  // phase-1 staging is dead; the same LDS now holds O, then O^{-1}
  double2* sO = reinterpret_cast<double2*>(smem);   // [NP][NP]
  double2* sColBuf = sO + NP * NP;                 // two column buffers
  double2* sRow = sColBuf + 2 * NP;                // pivot row scaled by 1/pivot
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int bp = wv + 4 * p;
    if (bp < NPAIR) {
      const int I = bp / NB, J = bp % NB;
#pragma unroll
      for (int v = 0; v < 4; ++v) sO[(16 * I + 4 * v + lk) * NP + 16 * J + lr] = make_double2(accR[p][v], accI[p][v]);
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- phase 2
  const int ty = tid >> 4, tx = tid & 15;   // owns rows ty+16a, cols tx+16b
  double2 e[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) e[a][b] = sO[(ty + 16 * a) * NP + tx + 16 * b];
  // publish column 0
  if (tx == 0) {
#pragma unroll
    for (int a = 0; a < NB; ++a) sColBuf[ty + 16 * a] = e[a][0];
  }
  __syncthreads();

  // pivot bookkeeping, replicated in every lane: lane l tracks rows
  // (l & 15) + 16 m, m < NB, as bit m of `used`
  unsigned used = 0u;
#pragma unroll
  for (int m = 0; m < NB; ++m)
    if ((lr + 16 * m) >= n) used |= 1u << m;
  int zero = 0;
  for (int k = 0; k < n; ++k) {
    const double2* col = sColBuf + (k & 1) * NP;
    // pivot search, identical in every 16-lane row of every wave: key =
    // |re|+|im| (46 leading bits, monotone as an integer) with 63 - row in the
    // low 6 bits; max over the lane's NB rows, then over the 16 lanes (DPP)
    unsigned long long key = 0ull;
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      const double2 cv = col[lr + 16 * m];
      const unsigned long long mb = (unsigned long long)__double_as_longlong(fabs(cv.x) + fabs(cv.y));
      const unsigned long long km = (used >> m & 1u) ? 0ull : ((mb & ~63ull) | (unsigned long long)(63 - (lr + 16 * m)));
      key = km > key ? km : key;
    }
    key = row16_max_u64(key);
    const int p = __builtin_amdgcn_readfirstlane(63 - (int)(key & 63ull));
    if ((key >> 6) == 0ull) { zero = k + 1; break; }
    if ((p & 15) == lr) used |= 1u << (p >> 4);
    const double2 piv = col[p];                 // uniform LDS address: broadcast read
    // 1/piv = conj(piv) / |piv|^2 (O is an overlap of normalised orbitals, far
    // from the over/underflow range of |piv|^2)
    const double rn = 1.0 / (piv.x * piv.x + piv.y * piv.y);
    const double2 inv = make_double2(piv.x * rn, -piv.y * rn);
    if (tid == 0) {
      sPiv[k] = p;
      sPivV[k] = piv;
    }
    if (ty == (p & 15)) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
        if (a == (p >> 4)) {
#pragma unroll
          for (int b = 0; b < NB; ++b) sRow[tx + 16 * b] = cmul(e[a][b], inv);
        }
    }
    __syncthreads();
    // exchange step on pivot (p, k); all LDS reads issued first.  With
    // c'_i = A[i][k] + [i == p] every element takes the same update
    //   A[i][j] -= c'_i R[j],  R[j] = A[p][j] / pivot,
    // which gives A[i][j] - A[i][k] R[j] off the pivot row and -R[j] on it
    // (the exchange operator); column k is then overwritten by its owners
    // with A[i][k] / pivot (1 / pivot on the pivot row).
    double2 cik[NB], rpj[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) cik[a] = col[ty + 16 * a];
#pragma unroll
    for (int b = 0; b < NB; ++b) rpj[b] = sRow[tx + 16 * b];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      double2 c = cik[a];
      c.x += ((ty + 16 * a) == p) ? 1.0 : 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double2 r = rpj[b];
        double2 v = e[a][b];
        v.x = fma(-c.x, r.x, fma(c.y, r.y, v.x));
        v.y = fma(-c.x, r.y, fma(-c.y, r.x, v.y));
        e[a][b] = v;
      }
    }
    if (tx == (k & 15)) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b == (k >> 4)) {
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            const double2 cc = ((ty + 16 * a) == p) ? make_double2(1.0, 0.0) : cik[a];
            e[a][b] = cmul(cc, inv);
          }
        }
    }
    // the owners of column k+1 publish it for the next step
    if (k + 1 < n && tx == ((k + 1) & 15)) {
      double2* ncol = sColBuf + ((k + 1) & 1) * NP;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b == ((k + 1) >> 4)) {
#pragma unroll
          for (int a = 0; a < NB; ++a) ncol[ty + 16 * a] = e[a][b];
        }
    }
    __syncthreads();
  }

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
  for (int idx = tid; idx < NP * NP; idx += 256) {
    const int row = idx / NP, col = idx % NP;
    if (row >= n || col >= n) sO[idx] = make_double2(0.0, 0.0);
  }
  if (wv == 0) {
    // log det O = sum_k log(pivot_k) + i pi (parity of k -> p_k)
    double la = 0.0, ar = 0.0;
    if (!zero && lane < n) {
      const double2 pv = sPivV[lane];
      la = log(hypot(pv.x, pv.y));
      ar = atan2(pv.y, pv.x);
    }
    la = wave_sum_lane0(la);
    ar = wave_sum_lane0(ar);
    if (lane == 0) {
      info[w] = zero;
      if (logov) {
        double2 ld;
        if (zero) {
          ld = make_double2(__builtin_nan(""), __builtin_nan(""));
        } else {
          int cycles = 0;
          unsigned long long seen = 0ull;
          for (int s2 = 0; s2 < n; ++s2) {
            if (seen >> s2 & 1ull) continue;
            ++cycles;
            int c = s2;
            while (!(seen >> c & 1ull)) { seen |= 1ull << c; c = sPiv[c]; }
          }
          double im = ar + ((n - cycles) & 1 ? M_PI : 0.0);
          im = remainder(im, 2.0 * M_PI);  // (-pi, pi]
          if (im <= -M_PI) im += 2.0 * M_PI;
          ld = make_double2(la, im);
        }
        logov[w] = ld;
      }
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- phase 3
  const int nrb = (M + 15) / 16;
  const int ksteps = (n + 3) / 4;
  double2 fa[C::NKH], fb[C::NKH];
  auto load_half = [&](int rb, int h, double2* f) {
    const int r = 16 * rb + lr;
#pragma unroll
    for (int q = 0; q < C::NKH; ++q) {
      const int kk = 4 * (C::NKH * h + q) + lk;
      f[q] = (rb < nrb && r < M && kk < n) ? ph[(size_t)r * n + kk] : make_double2(0.0, 0.0);
    }
  };
  d4 P1[NB], P2[NB], P3[NB];
  auto mult_half = [&](int h, const double2* f) {
#pragma unroll
    for (int q = 0; q < C::NKH; ++q) {
      const int ks = C::NKH * h + q;
      if (ks < ksteps) {
        const double2 av = f[q];
        const double as = av.x + av.y;
        const int kk = 4 * ks + lk;
#pragma unroll
        for (int J = 0; J < NB; ++J) {
          const double2 bv = sO[kk * NP + 16 * J + lr];
          P1[J] = mfma16(av.x, bv.x, P1[J]);
          P2[J] = mfma16(av.y, bv.y, P2[J]);
          P3[J] = mfma16(as, bv.x + bv.y, P3[J]);
        }
      }
    }
  };
  const double nan = __builtin_nan("");
  auto store_rows = [&](int rb) {
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      const int j = 16 * J + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + 4 * v + lk;
        if (row < M && j < n) {
          const double re = P1[J][v] - P2[J][v];
          const double im = P3[J][v] - P1[J][v] - P2[J][v];
          const double2 val = zero ? make_double2(nan, nan) : make_double2(re, im);
          if (orbital_major)
            theta[((size_t)j * M + row) * nw + w] = val;
          else
            theta[(w * (size_t)M + row) * n + j] = val;
        }
      }
    }
  };
  if (wv < nrb) load_half(wv, 0, fa);
  for (int rb = wv; rb < nrb; rb += 4) {
    load_half(rb, 1, fb);
#pragma unroll
    for (int J = 0; J < NB; ++J) { P1[J] = d4zero(); P2[J] = d4zero(); P3[J] = d4zero(); }
    mult_half(0, fa);
    load_half(rb + 4, 0, fa);
    mult_half(1, fb);
    store_rows(rb);
  }
}

template <int NB>
static hipError_t launch_gt(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                            double* theta, double* logov, int* info, int orbital_major) {
  const size_t lds = GtCfg<NB>::LDS;
  hipError_t e = hipFuncSetAttribute((const void*)green_theta_kernel<NB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t grid = orbital_major ? 8 * ((nw + 7) / 8) : nw;
  hipLaunchKernelGGL(green_theta_kernel<NB>, dim3((unsigned)grid), dim3(256), lds, s, M, n, trial,
                     (const double2*)phi, (double2*)theta, (double2*)logov, info, orbital_major, nw);
  return hipGetLastError();
}

hipError_t launch_green_theta(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                              double* theta, double* logov, int* info, int orbital_major) {
  if (nw <= 0) return hipSuccess;
  if (n <= 16) return launch_gt<1>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major);
  if (n <= 32) return launch_gt<2>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major);
  if (n <= 48) return launch_gt<3>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major);
  return launch_gt<4>(s, M, n, nw, trial, phi, theta, logov, info, orbital_major);
}

}  // namespace lofqmc
