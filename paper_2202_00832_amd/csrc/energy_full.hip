// Two-body energy by the half-rotated Cholesky route (Eq. 16), FP64 MFMA.
//
// For walker w and Cholesky vector g:  T = Lbar_g^T theta_w  (n x n complex),
//   Coulomb  c_{wg} = Tr T,          E_J[w] = 2 sum_g c_{wg}^2
//   exchange x_{wg} = Tr(T T),       E_K[w] = -sum_g x_{wg}.
// T is never written to memory.  T is cut into 16x16 blocks; the block pairs
// (I < J) and the diagonal blocks are dealt out over S = 2 P wave slices: the
// two waves of a walker in a workgroup, times P passes (a second grid
// dimension, P = 1 up to 64 orbitals).  For an off-diagonal block pair a wave
// accumulates T[I,J] = Lbar^T theta and the transposed block
// (T^T)[I,J] = theta^T Lbar: with the same operand fragments both land with
// every element's exchange partner T_ji in the same lane and register as
// T_ij, so sum_ij T_ij T_ji is a lane-local product.  Diagonal blocks are
// transposed through LDS.  With one pass the Coulomb trace comes from the
// diagonal blocks (the two halves combined through LDS); with several, where
// no workgroup holds every diagonal block, one wave per walker sums it
// straight from its operand fragments (each lane holds Lbar[r][i] and
// theta[r][i] of the same r and i).  The Lbar tile of each K-step is staged
// once in LDS (double-buffered) and shared by the four walkers of the
// workgroup.  Per-(pass, chunk) partial sums are reduced in a fixed order by
// a second kernel, so results are deterministic.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

template <int NB, int P>
struct FullCfg {
  static constexpr int NP = 16 * NB;
  static constexpr int S = 2 * P;                       // wave slices per walker
  static constexpr int NPAIR = NB * (NB - 1) / 2;
  static constexpr int NPS = (NPAIR + S - 1) / S;       // off-diagonal pairs per slice
  static constexpr int NDS = (NB + S - 1) / S;          // diagonal blocks per slice
  static constexpr int TILE = 16 * NP;                  // 16 rows of r, NP orbitals
  static constexpr int PER_THREAD = (TILE + 511) / 512;
};

// Passes per orbital-block count: the accumulators of one slice stay within
// about 112 registers (3 block pairs and one diagonal block from 65 orbitals up).
constexpr int full_passes(int NB) { return NB <= 4 ? 1 : (NB == 5 ? 2 : (NB == 6 ? 3 : 4)); }

// 8 waves: walker slot ws = wave / 2 (four walkers per workgroup) and half
// h = wave % 2; with pass p = blockIdx.y, slice sl = 2 p + h owns the
// off-diagonal pairs q with q % S == sl and the diagonal blocks I with
// I % S == sl.
template <int NB, int P>
__global__ __launch_bounds__(512, 1) void energy_full_kernel(int M, int n, int64_t X, int64_t nw, int64_t gchunk,
                                                             int nchunk, int64_t ngrp,
                                                             const double* __restrict__ lbar,
                                                             const double2* __restrict__ theta,
                                                             double* __restrict__ partial) {
  using C = FullCfg<NB, P>;
  constexpr int NP = C::NP;
  constexpr int S = C::S;
  __shared__ double sL[2][C::TILE];
  __shared__ double2 sDiag[8][C::NDS][256];
  __shared__ double2 sK[8];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int ws = wv >> 1, h = wv & 1;
  const int pass = (int)blockIdx.y;
  const int sl = 2 * pass + h;
  const bool coulomb = (sl == 0);
  const int lr = lane & 15, lk = lane >> 4;
  // XCD-aware order (workgroups go round-robin over 8 XCDs): the workgroups
  // of one XCD share a chunk of Cholesky vectors, so each Lbar tile is read
  // into that XCD's L2 once.
  int64_t chunk, grp;
  {
    const int64_t b = blockIdx.x;
    const int xcd = (int)(b & 7);
    const int64_t slot = b >> 3;
    const int64_t lin = slot * 8 + xcd;           // default linear order
    if (nchunk % 8 == 0 || 8 % nchunk == 0) {
      // chunk-major within an XCD
      const int per_xcd_chunks = nchunk >= 8 ? nchunk / 8 : 1;
      const int xcds_per_chunk = nchunk >= 8 ? 1 : 8 / nchunk;
      chunk = (int64_t)(xcd / xcds_per_chunk) * per_xcd_chunks + (slot % per_xcd_chunks);
      grp = (slot / per_xcd_chunks) * xcds_per_chunk + (xcd % xcds_per_chunk);
    } else {
      chunk = lin % nchunk;
      grp = lin / nchunk;
    }
    if (grp >= ngrp || chunk >= nchunk) return;
  }
  const int64_t w = 4 * grp + ws;
  const bool wok = w < nw;
  const double2* th = theta + (wok ? w : 0) * (size_t)M * n;
  const int64_t g0 = chunk * gchunk;
  const int64_t g1 = (g0 + gchunk < X) ? g0 + gchunk : X;
  const int nkt = (M + 15) / 16;
  const int64_t ntiles = (g1 > g0) ? (g1 - g0) * nkt : 0;

  double pre[C::PER_THREAD];
  auto load_tile = [&](int64_t t) {
    const int64_t g = g0 + t / nkt;
    const int rbase = 16 * (int)(t % nkt);
    const double* Lg = lbar + (size_t)g * M * n;
#pragma unroll
    for (int q = 0; q < C::PER_THREAD; ++q) {
      const int e = tid + 512 * q;
      const int rr = e / NP, i = e % NP;
      const int r = rbase + rr;
      pre[q] = (e < C::TILE && r < M && i < n) ? Lg[(size_t)r * n + i] : 0.0;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < C::PER_THREAD; ++q) {
      const int e = tid + 512 * q;
      if (e < C::TILE) sL[buf][e] = pre[q];
    }
  };
  // theta fragments of K-step u (r = 4 u' + lk within the current g)
  auto load_theta = [&](int kstep, double2 (&tf)[NB]) {
    const int r = 4 * kstep + lk;
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      const int j = 16 * I + lr;
      tf[I] = (wok && r < M && j < n) ? th[(size_t)r * n + j] : make_double2(0.0, 0.0);
    }
  };

  d4 dRe[C::NPS > 0 ? C::NPS : 1], dIm[C::NPS > 0 ? C::NPS : 1];
  d4 tRe[C::NPS > 0 ? C::NPS : 1], tIm[C::NPS > 0 ? C::NPS : 1];
  d4 gRe[C::NDS], gIm[C::NDS];
  double cr = 0.0, ci = 0.0;                       // Coulomb trace of the current g (this lane's share)
  double accJr = 0.0, accJi = 0.0, accKr = 0.0, accKi = 0.0;
  auto zero_acc = [&]() {
#pragma unroll
    for (int q = 0; q < C::NPS; ++q) { dRe[q] = d4zero(); dIm[q] = d4zero(); tRe[q] = d4zero(); tIm[q] = d4zero(); }
#pragma unroll
    for (int q = 0; q < C::NDS; ++q) { gRe[q] = d4zero(); gIm[q] = d4zero(); }
  };
  zero_acc();

  auto mma_step = [&](const double* Lt, int s, const double2 (&tf)[NB]) {
    double Lf[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) Lf[I] = Lt[(4 * s + lk) * NP + 16 * I + lr];
    if (P > 1 && coulomb) {
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        cr = fma(Lf[I], tf[I].x, cr);
        ci = fma(Lf[I], tf[I].y, ci);
      }
    }
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      if (I % S == sl) {
        gRe[I / S] = mfma16(Lf[I], tf[I].x, gRe[I / S]);
        gIm[I / S] = mfma16(Lf[I], tf[I].y, gIm[I / S]);
      }
    }
    int q = 0;   // flattened pair index (static after unrolling)
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int J = I + 1; J < NB; ++J, ++q) {
        if (q % S == sl) {
          dRe[q / S] = mfma16(Lf[I], tf[J].x, dRe[q / S]);
          dIm[q / S] = mfma16(Lf[I], tf[J].y, dIm[q / S]);
          tRe[q / S] = mfma16(tf[I].x, Lf[J], tRe[q / S]);
          tIm[q / S] = mfma16(tf[I].y, Lf[J], tIm[q / S]);
        }
      }
    }
  };

  double2 tfa[NB], tfb[NB];
  if (ntiles > 0) {
    load_tile(0);
    store_tile(0);
    load_theta(0, tfa);
  }
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int buf = (int)(t & 1);
    if (t + 1 < ntiles) load_tile(t + 1);
    const int kt = (int)(t % nkt);
    const int ktn = (kt + 1 == nkt) ? 0 : kt + 1;   // next tile's row block (same or next g)
    const double* Lt = sL[buf];
    // K-steps 4 kt .. 4 kt + 3; theta of the next K-step is loaded one step ahead
    load_theta(4 * kt + 1, tfb);
    mma_step(Lt, 0, tfa);
    load_theta(4 * kt + 2, tfa);
    mma_step(Lt, 1, tfb);
    load_theta(4 * kt + 3, tfb);
    mma_step(Lt, 2, tfa);
    load_theta(4 * ktn, tfa);
    mma_step(Lt, 3, tfb);
    if (t + 1 < ntiles) store_tile(buf ^ 1);

    if (kt == nkt - 1) {
      // ---- epilogue for this g: Coulomb trace and exchange sum
      double xr = 0.0, xi = 0.0;
#pragma unroll
      for (int q = 0; q < C::NPAIR; ++q) {
        if (q % S == sl) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            xr += 2.0 * (dRe[q / S][v] * tRe[q / S][v] - dIm[q / S][v] * tIm[q / S][v]);
            xi += 2.0 * (dRe[q / S][v] * tIm[q / S][v] + dIm[q / S][v] * tRe[q / S][v]);
          }
        }
      }
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        if (I % S == sl) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            sDiag[wv][I / S][(4 * v + lk) * 16 + lr] = make_double2(gRe[I / S][v], gIm[I / S][v]);
            // one pass: the trace from this slice's diagonal blocks
            if (P == 1 && 4 * v + lk == lr) {
              cr += gRe[I / S][v];
              ci += gIm[I / S][v];
            }
          }
        }
      }
      if (P == 1) {
        // the two halves' diagonal traces, combined through LDS by half 0
        const double tr = wave_sum_lane0(cr), ti = wave_sum_lane0(ci);
        if (lane == 0) sK[wv] = make_double2(tr, ti);
      } else if (coulomb) {
        const double tr = wave_sum_lane0(cr), ti = wave_sum_lane0(ci);
        if (lane == 0) {
          accJr += tr * tr - ti * ti;
          accJi += 2.0 * tr * ti;
        }
      }
      cr = 0.0;
      ci = 0.0;
      __syncthreads();
      if (P == 1 && h == 0 && lane == 0) {
        const double tr = sK[wv].x + sK[wv + 1].x, ti = sK[wv].y + sK[wv + 1].y;
        accJr += tr * tr - ti * ti;
        accJi += 2.0 * tr * ti;
      }
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        if (I % S == sl) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double2 pv = sDiag[wv][I / S][lr * 16 + 4 * v + lk];
            xr += gRe[I / S][v] * pv.x - gIm[I / S][v] * pv.y;
            xi += gRe[I / S][v] * pv.y + gIm[I / S][v] * pv.x;
          }
        }
      }
      accKr += xr;
      accKi += xi;
      zero_acc();
    }
    __syncthreads();
  }

  // per-walker partial of this (pass, chunk): the two halves are combined
  // through LDS in a fixed order; E_J comes from slice 0 only
  accKr = wave_sum_lane0(accKr);
  accKi = wave_sum_lane0(accKi);
  if (lane == 0) sK[wv] = make_double2(accKr, accKi);
  __syncthreads();
  if (wok && h == 0 && lane == 0) {
    const double2 k0 = sK[wv], k1 = sK[wv + 1];
    double* out = partial + (((size_t)pass * nchunk + chunk) * nw + w) * 4;
    out[0] = 2.0 * accJr;
    out[1] = 2.0 * accJi;
    out[2] = -(k0.x + k1.x);
    out[3] = -(k0.y + k1.y);
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
    if (info && info[w] > 0) s0 = s1 = s2 = s3 = __builtin_nan("");   // exact zero pivot
    reinterpret_cast<double4*>(energy)[w] = make_double4(s0, s1, s2, s3);
  }
}

template <int NB>
static hipError_t launch_full_nb(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* lbar,
                                 const double* theta, double* partial, int nchunk) {
  constexpr int P = full_passes(NB);
  const int64_t ngrp = (nw + 3) / 4;
  const int64_t gchunk = (X + nchunk - 1) / nchunk;
  // grid covers every (group, chunk); the XCD-aware order may leave a few
  // slots without work, which return at once
  int64_t grid = ngrp * nchunk;
  if (nchunk % 8 == 0 || 8 % nchunk == 0) {
    const int per_xcd_chunks = nchunk >= 8 ? nchunk / 8 : 1;
    const int xcds_per_chunk = nchunk >= 8 ? 1 : 8 / nchunk;
    const int64_t slots = per_xcd_chunks * ((ngrp + xcds_per_chunk - 1) / xcds_per_chunk);
    grid = 8 * slots;
  }
  hipLaunchKernelGGL((energy_full_kernel<NB, P>), dim3((unsigned)grid, P), dim3(512), 0, s, M, n, X, nw, gchunk,
                     nchunk, ngrp, lbar, (const double2*)theta, partial);
  return hipGetLastError();
}

int full_num_passes(int n) { return full_passes((n + 15) / 16); }

int full_num_chunks(int64_t X, int64_t nw) {
  // one workgroup (8 waves) per compute unit (256 CUs): chunks of Cholesky
  // vectors so that groups x chunks covers the machine about once
  const int64_t ngrp = (nw + 3) / 4;
  int64_t c = 1;
  while (c < 4096 && ngrp * c < 256 && c < X) c *= 2;
  return (int)c;
}

hipError_t launch_energy_full(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* lbar,
                              const double* theta, double* partial, int nchunk) {
  if (nw <= 0) return hipSuccess;
  switch ((n + 15) / 16) {
    case 1: return launch_full_nb<1>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    case 2: return launch_full_nb<2>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    case 3: return launch_full_nb<3>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    case 4: return launch_full_nb<4>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    case 5: return launch_full_nb<5>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    case 6: return launch_full_nb<6>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    case 7: return launch_full_nb<7>(s, M, n, X, nw, lbar, theta, partial, nchunk);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_partials(hipStream_t s, int64_t nw, int nchunk, const double* partial, const int* info,
                                  double* energy) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, nw, nchunk,
                     partial, info, energy);
  return hipGetLastError();
}

}  // namespace lofqmc
