// Two-body energy by the half-rotated Cholesky route (Eq. 16), FP64 MFMA.
//
// For walker w and Cholesky vector g:  T = Lbar_g^T theta_w  (n x n complex),
//   Coulomb  c_{wg} = Tr T,          E_J[w] = 2 sum_g c_{wg}^2
//   exchange x_{wg} = Tr(T T),       E_K[w] = -sum_g x_{wg}.
// T is never written to memory.  Each wave owns one walker and holds the
// whole T of the current g in MFMA accumulators, as 16x16 blocks.  For an
// off-diagonal block pair (I < J) the wave accumulates T[I,J] = Lbar^T theta
// and the transposed block (T^T)[I,J] = theta^T Lbar: with the same operand
// fragments both land with every element's exchange partner T_ji in the same
// lane and register as T_ij, so sum_ij T_ij T_ji is a lane-local product.
// Diagonal blocks are transposed through LDS.  The Lbar tile of each K-step
// is staged once in LDS (double-buffered) and shared by the four walkers of
// the workgroup.  Per-chunk partial sums are reduced in a fixed order by a
// second kernel, so results are deterministic.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

template <int NB>
struct FullCfg {
  static constexpr int NP = 16 * NB;
  static constexpr int NPAIR = NB * (NB - 1) / 2;
  static constexpr int TILE = 16 * NP;                 // 16 rows of r, NP orbitals
  static constexpr int PER_THREAD = (TILE + 255) / 256;
};

template <int NB>
__global__ __launch_bounds__(256, 1) void energy_full_kernel(int M, int n, int64_t X, int64_t nw, int64_t gchunk,
                                                             int nchunk, const double* __restrict__ lbar,
                                                             const double2* __restrict__ theta,
                                                             double* __restrict__ partial) {
  using C = FullCfg<NB>;
  constexpr int NP = C::NP;
  __shared__ double sL[2][C::TILE];
  __shared__ double2 sDiag[4][NB][256];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t grp = blockIdx.x / nchunk;
  const int64_t chunk = blockIdx.x % nchunk;
  const int64_t w = 4 * grp + wv;
  const bool wok = w < nw;
  const double2* th = theta + (wok ? w : 0) * (size_t)M * n;
  const int64_t g0 = chunk * gchunk;
  const int64_t g1 = (g0 + gchunk < X) ? g0 + gchunk : X;
  const int nkt = (M + 15) / 16;
  const int64_t ntiles = (g1 > g0) ? (g1 - g0) * nkt : 0;

  // cooperative load of Lbar tile t (g = g0 + t / nkt, rows 16 * (t % nkt) ...)
  double pre[C::PER_THREAD];
  auto load_tile = [&](int64_t t) {
    const int64_t g = g0 + t / nkt;
    const int rbase = 16 * (int)(t % nkt);
    const double* Lg = lbar + (size_t)g * M * n;
#pragma unroll
    for (int q = 0; q < C::PER_THREAD; ++q) {
      const int e = tid + 256 * q;
      const int rr = e / NP, i = e % NP;
      const int r = rbase + rr;
      pre[q] = (e < C::TILE && r < M && i < n) ? Lg[(size_t)r * n + i] : 0.0;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < C::PER_THREAD; ++q) {
      const int e = tid + 256 * q;
      if (e < C::TILE) sL[buf][e] = pre[q];
    }
  };

  d4 dRe[C::NPAIR > 0 ? C::NPAIR : 1], dIm[C::NPAIR > 0 ? C::NPAIR : 1];
  d4 tRe[C::NPAIR > 0 ? C::NPAIR : 1], tIm[C::NPAIR > 0 ? C::NPAIR : 1];
  d4 gRe[NB], gIm[NB];
  double accJr = 0.0, accJi = 0.0, accKr = 0.0, accKi = 0.0;

  auto zero_acc = [&]() {
#pragma unroll
    for (int q = 0; q < C::NPAIR; ++q) { dRe[q] = d4zero(); dIm[q] = d4zero(); tRe[q] = d4zero(); tIm[q] = d4zero(); }
#pragma unroll
    for (int I = 0; I < NB; ++I) { gRe[I] = d4zero(); gIm[I] = d4zero(); }
  };
  zero_acc();

  if (ntiles > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int buf = (int)(t & 1);
    if (t + 1 < ntiles) load_tile(t + 1);
    const int kt = (int)(t % nkt);
    const double* Lt = sL[buf];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = 16 * kt + 4 * s + lk;
      double Lf[NB];
      double2 tf[NB];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        Lf[I] = Lt[(4 * s + lk) * NP + 16 * I + lr];
        const int j = 16 * I + lr;
        tf[I] = (wok && r < M && j < n) ? th[(size_t)r * n + j] : make_double2(0.0, 0.0);
      }
      int q = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        gRe[I] = mfma16(Lf[I], tf[I].x, gRe[I]);
        gIm[I] = mfma16(Lf[I], tf[I].y, gIm[I]);
#pragma unroll
        for (int J = I + 1; J < NB; ++J, ++q) {
          dRe[q] = mfma16(Lf[I], tf[J].x, dRe[q]);
          dIm[q] = mfma16(Lf[I], tf[J].y, dIm[q]);
          tRe[q] = mfma16(tf[I].x, Lf[J], tRe[q]);
          tIm[q] = mfma16(tf[I].y, Lf[J], tIm[q]);
        }
      }
    }
    if (t + 1 < ntiles) store_tile(buf ^ 1);

    if (kt == nkt - 1) {
      // ---- epilogue for this g: Coulomb trace and exchange sum
      double xr = 0.0, xi = 0.0, cr = 0.0, ci = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < C::NPAIR; ++q2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          xr += 2.0 * (dRe[q2][v] * tRe[q2][v] - dIm[q2][v] * tIm[q2][v]);
          xi += 2.0 * (dRe[q2][v] * tIm[q2][v] + dIm[q2][v] * tRe[q2][v]);
        }
      }
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          sDiag[wv][I][(4 * v + lk) * 16 + lr] = make_double2(gRe[I][v], gIm[I][v]);
          if (4 * v + lk == lr) { cr += gRe[I][v]; ci += gIm[I][v]; }
        }
      }
      __syncthreads();
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double2 pv = sDiag[wv][I][lr * 16 + 4 * v + lk];
          xr += gRe[I][v] * pv.x - gIm[I][v] * pv.y;
          xi += gRe[I][v] * pv.y + gIm[I][v] * pv.x;
        }
      }
      cr = wave_sum_lane0(cr);
      ci = wave_sum_lane0(ci);
      if (lane == 0) {
        accJr += cr * cr - ci * ci;
        accJi += 2.0 * cr * ci;
      }
      accKr += xr;
      accKi += xi;
      zero_acc();
    }
    __syncthreads();
  }

  accKr = wave_sum_lane0(accKr);
  accKi = wave_sum_lane0(accKi);
  if (wok && lane == 0) {
    double* out = partial + ((size_t)chunk * nw + w) * 4;
    out[0] = 2.0 * accJr;
    out[1] = 2.0 * accJi;
    out[2] = -accKr;
    out[3] = -accKi;
  }
}

// energy[w] = sum_c partial[c][w] in a fixed order: lane l adds chunks
// l, l+64, ... and a fixed shuffle tree combines the lanes (one wave per walker).
__global__ __launch_bounds__(256) void reduce_partials_kernel(int64_t nw, int nchunk,
                                                              const double* __restrict__ partial,
                                                              const int* __restrict__ info,
                                                              double* __restrict__ energy) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nw) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int c = lane; c < nchunk; c += 64) {
    const double4 p = reinterpret_cast<const double4*>(partial)[(size_t)c * nw + w];
    s0 += p.x;
    s1 += p.y;
    s2 += p.z;
    s3 += p.w;
  }
  s0 = wave_sum_lane0(s0);
  s1 = wave_sum_lane0(s1);
  s2 = wave_sum_lane0(s2);
  s3 = wave_sum_lane0(s3);
  if (lane == 0) {
    if (info && info[w] != 0) s0 = s1 = s2 = s3 = __builtin_nan("");
    reinterpret_cast<double4*>(energy)[w] = make_double4(s0, s1, s2, s3);
  }
}

template <int NB>
static hipError_t launch_full_nb(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* lbar,
                                 const double* theta, double* partial, int nchunk) {
  const int64_t ngrp = (nw + 3) / 4;
  const int64_t gchunk = (X + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(energy_full_kernel<NB>, dim3((unsigned)(ngrp * nchunk)), dim3(256), 0, s, M, n, X, nw,
                     gchunk, nchunk, lbar, (const double2*)theta, partial);
  return hipGetLastError();
}

int full_num_chunks(int64_t X, int64_t nw) {
  // about two workgroups per compute unit (256 CUs) when there are few walkers
  const int64_t ngrp = (nw + 3) / 4;
  int64_t c = (512 + ngrp - 1) / ngrp;
  if (c < 1) c = 1;
  if (c > X) c = X > 0 ? X : 1;
  if (c > 4096) c = 4096;
  return (int)c;
}

hipError_t launch_energy_full(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* lbar,
                              const double* theta, double* partial, int nchunk) {
  if (nw <= 0) return hipSuccess;
  if (n <= 16) return launch_full_nb<1>(s, M, n, X, nw, lbar, theta, partial, nchunk);
  if (n <= 32) return launch_full_nb<2>(s, M, n, X, nw, lbar, theta, partial, nchunk);
  if (n <= 48) return launch_full_nb<3>(s, M, n, X, nw, lbar, theta, partial, nchunk);
  return launch_full_nb<4>(s, M, n, X, nw, lbar, theta, partial, nchunk);
}

hipError_t launch_reduce_partials(hipStream_t s, int64_t nw, int nchunk, const double* partial, const int* info,
                                  double* energy) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, nw, nchunk,
                     partial, info, energy);
  return hipGetLastError();
}

}  // namespace lofqmc
