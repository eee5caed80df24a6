// Multi-determinant LO energy (Sec. 2.1.1 Eq. 12; Sec. 2.3.2 Eq. 19-23), FP64.
//
// Trial orbitals C (M x n_cas): the reference determinant holds columns
// 0 .. n-1, the last nao of them active; the active virtual orbitals are
// columns n .. n + nav - 1.  Determinant d replaces hole h_m (an active
// occupied column) by particle p_m.  With A = Psi_0^T phi, theta = phi A^{-1}
// and T = C_av^T theta (nav x n), the SMW update of Eq. 20-21 reads, for every
// determinant,
//   R_d = T[p_d, h_d]              (the matrix I + V^dT A^{-1} U^d),
//   det A_d = det A det R_d,
//   Q^d column of orbital o = s_o theta_o - sum_a theta_a (B_d tau_o)_a,
//   B_d = E_h R_d^{-1} E_p^T       (nao x nav),
// with s_o = 1, tau_o = T[:, o] for o < n and s_o = 0, tau_o = -e_{o-n} for an
// active virtual o.  The column of a hole cancels exactly (B_d tau_h = e_h),
// and a virtual orbital that d leaves empty gets B_d e = 0, which is the zero
// padding of Sec. 2.3.2.  The closed-shell weights w_d = c_d det(R_d)^2 / sum
// (both spins share the spatial determinant) enter the weighted pair sums of
// Eq. 22 only through two moments per walker,
//   Bbar = sum_d w_d B_d,   Omega[a,p,b,q] = sum_d w_d B_d[a,p] B_d[b,q],
// so with mu_o = Bbar tau_o, the projections QL_x = Ubar^T theta_x,
// QR_x = Vbar theta_x of Eq. 23 (x: the pair's own columns and the active
// columns a), G_ab = QL_a . QR_b and H[p,q] = sum_ab G_ab Omega[a,p,b,q]:
//   J_ij = s_i s_j QL_i.QR_j - s_i QL_i.QR(mu_j) - s_j QL(mu_i).QR_j + tau_i^T H tau_j
//   X_ij = s_i s_j QL_j.QR_i - s_j QL_j.QR(mu_i) - s_i QL(mu_j).QR_i + tau_j^T H tau_i
// (QL(v) = sum_a v_a QL_a).  The sum over determinants is done once per
// walker; the per-pair work does not grow with the number of determinants.
//
// Pass 1 forms T next to every orbital's own projections (the active virtual
// orbitals are extra rows of its tile).
// md_prep_kernel: one workgroup per walker: the pivoted Gauss-Jordan
// inverse and determinant of every padded R_d (eps <= 6, identity-padded to
// NA x NA, so every determinant runs the same branch-free code), the
// unnormalised moments summed over determinants in a fixed order, then scaled
// by 1 / sum_d c_d det(R_d)^2.
// It also contracts Omega with each orbital's tau once per walker:
//   Y_o[a][b][q] = sum_p Omega[a,p,b,q] tau_o[p].
// md_energy_kernel: one workgroup per (walker, chunk of pairs), a thread per
// pair; tau and mu of the walker in LDS.  Omega is symmetric under
// (a,p) <-> (b,q) (a sum of w_d B_d[a,p] B_d[b,q]), so with
// M[a][b] = sum_q Y_i[a][b][q] tau_j[q] the two determinant-averaged terms are
//   tau_i^T H tau_j = sum_ab G_ab M[a][b],   tau_j^T H tau_i = sum_ab G_ab M[b][a]:
// NA^3 + 2 NA^2 complex products per pair instead of the NA^4 of forming H.
#include "common.h"
#include "kernels.h"

namespace lofqmc {

constexpr int MD_MAXN = 128;   // largest n_occ and n_cas (LDS tables)

__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}

template <int NA>
__global__ __launch_bounds__(256) void md_prep_kernel(int n, int nao, int nav, int ndet, int hstride,
                                                      const int* __restrict__ tpos,
                                                      const double2* __restrict__ qbar, int64_t n_out,
                                                      const int* __restrict__ exc,
                                                      const int* __restrict__ holes, const int* __restrict__ parts,
                                                      const double* __restrict__ coef, double2* __restrict__ tau,
                                                      double2* __restrict__ bbar, double2* __restrict__ omega,
                                                      double2* __restrict__ ycon, int ncas,
                                                      double2* __restrict__ ovr) {
  constexpr int NA2 = NA * NA;
  constexpr int NA3 = NA2 * NA;
  constexpr int NA4 = NA2 * NA2;
  constexpr int NE = (NA4 + 255) / 256;        // Omega entries per thread
  constexpr int CH = NA <= 5 ? 128 : 64;       // determinants per round (LDS: CH x NA^2 complex)
  __shared__ double2 sT[NA][MD_MAXN];
  __shared__ double2 sB[CH][NA2];
  __shared__ double2 sW[CH];
  __shared__ double2 sS;
  const int64_t w = blockIdx.x;
  const int tid = threadIdx.x;

  // T[v][c] = C_av[:, v] . theta_c, formed by pass 1 next to orbital c's own rows
  const double2* qw = qbar + w * n_out;
  for (int e = tid; e < NA * n; e += 256) {
    const int v = e / n, c = e % n;
    const double2 t = v < nav ? qw[tpos[c] + v] : make_double2(0.0, 0.0);
    sT[v][c] = t;
    tau[(w * NA + v) * n + c] = t;
  }
  __syncthreads();

  double2 bacc = make_double2(0.0, 0.0);
  double2 oacc[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) oacc[k] = make_double2(0.0, 0.0);
  double2 sacc = make_double2(0.0, 0.0);
  const int act0 = n - nao;

  for (int d0 = 0; d0 < ndet; d0 += CH) {
    if (tid < CH) {
      const int d = d0 + tid;
#pragma unroll
      for (int e = 0; e < NA2; ++e) sB[tid][e] = make_double2(0.0, 0.0);
      double2 wgt = make_double2(0.0, 0.0);
      if (d < ndet) {
        const int eps = exc[d];
        // rows of hstride >= NA entries: every index read below stays in the row
        const int* hd = holes + (size_t)d * hstride;
        const int* pd = parts + (size_t)d * hstride;
        // R_d padded with the identity to NA x NA
        double2 a[NA][NA];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
          for (int k = 0; k < NA; ++k) {
            double2 v = make_double2(m == k ? 1.0 : 0.0, 0.0);
            if (m < eps && k < eps) v = sT[pd[m]][act0 + hd[k]];
            a[m][k] = v;
          }
        // in-place Gauss-Jordan inverse with partial pivoting (largest |re|+|im|)
        double2 det = make_double2(1.0, 0.0);
        bool sing = false;
        int piv[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          int p = k;
          double best = fabs(a[k][k].x) + fabs(a[k][k].y);
#pragma unroll
          for (int r = k + 1; r < NA; ++r) {
            const double v = fabs(a[r][k].x) + fabs(a[r][k].y);
            if (v > best) {
              best = v;
              p = r;
            }
          }
          piv[k] = p;
#pragma unroll
          for (int r = k + 1; r < NA; ++r) {
            const bool s = r == p;
#pragma unroll
            for (int c = 0; c < NA; ++c) {
              const double2 x = a[k][c], y = a[r][c];
              a[k][c] = csel(s, y, x);
              a[r][c] = csel(s, x, y);
            }
          }
          if (p != k) det = make_double2(-det.x, -det.y);
          const double2 pv = a[k][k];
          det = cmul(det, pv);
          const double nrm = pv.x * pv.x + pv.y * pv.y;
          if (nrm == 0.0) sing = true;
          const double2 rp = nrm == 0.0 ? make_double2(0.0, 0.0) : make_double2(pv.x / nrm, -pv.y / nrm);
          a[k][k] = make_double2(1.0, 0.0);
#pragma unroll
          for (int c = 0; c < NA; ++c) a[k][c] = cmul(a[k][c], rp);
#pragma unroll
          for (int r = 0; r < NA; ++r) {
            if (r == k) continue;
            const double2 f = a[r][k];
            a[r][k] = make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < NA; ++c) {
              const double2 t = cmul(f, a[k][c]);
              a[r][c] = make_double2(a[r][c].x - t.x, a[r][c].y - t.y);
            }
          }
        }
        // the row interchanges come back as column interchanges, last first
#pragma unroll
        for (int k = NA - 1; k >= 0; --k) {
#pragma unroll
          for (int c = k + 1; c < NA; ++c) {
            const bool s = piv[k] == c;
#pragma unroll
            for (int r = 0; r < NA; ++r) {
              const double2 x = a[r][k], y = a[r][c];
              a[r][k] = csel(s, y, x);
              a[r][c] = csel(s, x, y);
            }
          }
        }
        if (!sing) {
          wgt = cmul(make_double2(coef[d], 0.0), cmul(det, det));
#pragma unroll
          for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int k = 0; k < NA; ++k)
              if (m < eps && k < eps) sB[tid][hd[m] * NA + pd[k]] = a[m][k];
        }
      }
      sW[tid] = wgt;
    }
    __syncthreads();
    const int nd = ndet - d0 < CH ? ndet - d0 : CH;
    for (int dd = 0; dd < nd; ++dd) {
      const double2 wg = sW[dd];
      if (tid < NA2) bacc = cfma(wg, sB[dd][tid], bacc);
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int e = tid + 256 * k;
        if (e < NA4) oacc[k] = cfma(wg, cmul(sB[dd][e / NA2], sB[dd][e % NA2]), oacc[k]);
      }
      if (tid == 0) sacc = cadd(sacc, wg);
    }
    __syncthreads();
  }
  if (tid == 0) sS = sacc;
  __syncthreads();
  const double2 S = sS;
  const double nrm = S.x * S.x + S.y * S.y;
  const double2 rs = make_double2(S.x / nrm, -S.y / nrm);   // NaN moments when S = 0
  if (tid < NA2) bbar[w * NA2 + tid] = cmul(bacc, rs);
  // Omega in LDS (over the determinant blocks, no longer needed) for Y
  double2* sOmg = &sB[0][0];
  static_assert(CH * NA2 >= NA4, "Omega fits the determinant blocks");
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + 256 * k;
    if (e < NA4) {
      const double2 v = cmul(oacc[k], rs);
      omega[w * NA4 + e] = v;
      sOmg[e] = v;
    }
  }
  if (tid == 0 && ovr) ovr[w] = S;
  __syncthreads();
  // Y_o[a][b][q] = sum_p Omega[a,p,b,q] tau_o[p]: tau_o = T[:, o] for an
  // occupied o, -e_{o-n} for an active virtual one (Omega[a,p,b,q] at
  // (a NA + p) NA^2 + b NA + q)
  double2* yw = ycon + (size_t)w * ncas * NA3;
  for (int e = tid; e < ncas * NA3; e += 256) {
    const int o = e / NA3, r = e % NA3;
    const int a = r / NA2, b = (r / NA) % NA, q = r % NA;
    double2 y = make_double2(0.0, 0.0);
    if (o < n) {
#pragma unroll
      for (int pp = 0; pp < NA; ++pp) y = cfma(sOmg[(a * NA + pp) * NA2 + b * NA + q], sT[pp][o], y);
    } else if (o - n < NA) {
      const double2 v = sOmg[(a * NA + (o - n)) * NA2 + b * NA + q];
      y = make_double2(-v.x, -v.y);
    }
    yw[e] = y;
  }
}

template <int NA>
__global__ __launch_bounds__(256) void md_energy_kernel(int n, int ncas, int nao, int64_t nw, int npairs,
                                                        int per_chunk, const int* __restrict__ pi,
                                                        const int* __restrict__ pj, const int* __restrict__ pK,
                                                        const int64_t* __restrict__ offI,
                                                        const int64_t* __restrict__ offJ,
                                                        const int64_t* __restrict__ offA, int64_t act_stride,
                                                        int64_t n_out,
                                                        const double2* __restrict__ qbar,
                                                        const double2* __restrict__ tau,
                                                        const double2* __restrict__ bbar,
                                                        const double2* __restrict__ ycon,
                                                        double* __restrict__ partial) {
  constexpr int NA2 = NA * NA;
  constexpr int NA3 = NA2 * NA;
  __shared__ double2 sTau[MD_MAXN][NA];
  __shared__ double2 sBb[NA2];
  __shared__ double2 sMu[MD_MAXN][NA];     // mu_o = Bbar tau_o
  __shared__ double4 sRed[4];
  // consecutive walkers on one XCD (workgroups go round-robin over the 8
  // XCDs), so the cache lines of qbar that neighbouring walkers share are
  // fetched into one L2
  const int64_t nw8 = (nw + 7) / 8;
  const int64_t w = (int64_t)(blockIdx.x & 7) * nw8 + (blockIdx.x >> 3);
  if (w >= nw) return;
  const int chunk = blockIdx.y;
  const int tid = threadIdx.x;
  if (tid < NA2) sBb[tid] = bbar[w * NA2 + tid];
  for (int e = tid; e < ncas * NA; e += 256) {
    const int o = e / NA, p = e % NA;
    sTau[o][p] = o < n ? tau[(w * NA + p) * n + o] : make_double2(o - n == p ? -1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < ncas * NA; e += 256) {
    const int o = e / NA, a = e % NA;
    double2 m = make_double2(0.0, 0.0);
    for (int q = 0; q < NA; ++q) m = cfma(sBb[a * NA + q], sTau[o][q], m);
    sMu[o][a] = m;
  }
  __syncthreads();

  const double2* __restrict__ qw = qbar + w * n_out;
  const int as32 = (int)act_stride;
  const int p0 = chunk * per_chunk;
  const int p1 = p0 + per_chunk < npairs ? p0 + per_chunk : npairs;
  double2 accJ = make_double2(0.0, 0.0), accX = make_double2(0.0, 0.0);
  for (int p = p0 + tid; p < p1; p += 256) {
    const int i = pi[p], j = pj[p], K = pK[p];
    const double wt = i == j ? 1.0 : 2.0;
    // keeps the compiler from hoisting the walker's LDS tables into registers
    // across pairs
    asm volatile("" ::: "memory");
    double2 mi[NA], mj[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      mi[a] = sMu[i][a];
      mj[a] = sMu[j][a];
    }
    const bool own_i = i < n, own_j = j < n;
    // the walker's projections are contiguous rows (qbar is [nw][n_out], so
    // the 64 pairs of a wave read nearby rows); an active virtual orbital has
    // no own column: its loads read the pair's first active-column rows and
    // are then replaced by zero
    const int rA = (int)offA[p];
    const int rI = own_i ? (int)offI[p] : rA;
    const int rJ = own_j ? (int)offJ[p] : rA;
    double2 J = make_double2(0.0, 0.0), X = make_double2(0.0, 0.0);
    double2 G[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NA; ++b) G[a][b] = make_double2(0.0, 0.0);
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      const double2 z = make_double2(0.0, 0.0);
      const double2 pli = csel(own_i, qw[rI + k], z);
      const double2 pri = csel(own_i, qw[rI + K + k], z);
      const double2 plj = csel(own_j, qw[rJ + k], z);
      const double2 prj = csel(own_j, qw[rJ + K + k], z);
      double2 la[NA], ra[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        // padded active columns (a >= nao) read column 0 and are zeroed
        const int ra0 = rA + (a < nao ? a : 0) * as32;
        la[a] = csel(a < nao, qw[ra0 + k], z);
        ra[a] = csel(a < nao, qw[ra0 + K + k], z);
      }
      double2 sLi = z, sRi = z, sLj = z, sRj = z;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        sLi = cfma(la[a], mi[a], sLi);
        sRi = cfma(ra[a], mi[a], sRi);
        sLj = cfma(la[a], mj[a], sLj);
        sRj = cfma(ra[a], mj[a], sRj);
      }
      // s_i, s_j are folded into the zeroed own projections
      J = cfma(pli, make_double2(prj.x - sRj.x, prj.y - sRj.y), J);
      J = cfma(make_double2(-sLi.x, -sLi.y), prj, J);
      X = cfma(plj, make_double2(pri.x - sRi.x, pri.y - sRi.y), X);
      X = cfma(make_double2(-sLj.x, -sLj.y), pri, X);
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NA; ++b) G[a][b] = cfma(la[a], ra[b], G[a][b]);
    }
    // determinant-averaged terms through Y_i of this pair's orbital i:
    // M[a][b] = sum_q Y_i[a][b][q] tau_j[q], J += sum G_ab M[a][b],
    // X += sum G_ab M[b][a] (Y_i read through the cache: the pairs of a wave
    // mostly share i, so their loads share addresses)
    {
      const double2* yi = ycon + ((size_t)w * ncas + i) * NA3;
      double2 tj[NA];
#pragma unroll
      for (int q = 0; q < NA; ++q) tj[q] = sTau[j][q];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
#pragma unroll
        for (int b = 0; b < NA; ++b) {
          double2 yv[NA];
#pragma unroll
          for (int q = 0; q < NA; ++q) yv[q] = yi[(a * NA + b) * NA + q];
          double2 m = make_double2(0.0, 0.0);
#pragma unroll
          for (int q = 0; q < NA; ++q) m = cfma(yv[q], tj[q], m);
          J = cfma(G[a][b], m, J);
          X = cfma(G[b][a], m, X);
        }
      }
    }
    accJ = make_double2(accJ.x + wt * J.x, accJ.y + wt * J.y);
    accX = make_double2(accX.x + wt * X.x, accX.y + wt * X.y);
  }
  // fixed-order reduction over the workgroup
  double v0 = wave_sum_lane0(accJ.x), v1 = wave_sum_lane0(accJ.y);
  double v2 = wave_sum_lane0(accX.x), v3 = wave_sum_lane0(accX.y);
  if ((tid & 63) == 0) sRed[tid >> 6] = make_double4(v0, v1, v2, v3);
  __syncthreads();
  if (tid == 0) {
    double4 s = sRed[0];
    for (int q = 1; q < 4; ++q) {
      s.x += sRed[q].x;
      s.y += sRed[q].y;
      s.z += sRed[q].z;
      s.w += sRed[q].w;
    }
    reinterpret_cast<double4*>(partial)[(size_t)chunk * nw + w] = make_double4(2.0 * s.x, 2.0 * s.y, -s.z, -s.w);
  }
}

int md_max_orbitals() { return MD_MAXN; }
int md_max_active() { return 6; }

size_t md_walker_bytes(int na, int n, int ncas) {
  const size_t na2 = (size_t)na * na;
  return sizeof(double2) * ((size_t)na * n + na2 + na2 * na2 + (size_t)ncas * na2 * na);
}

int md_pair_chunks(int npairs) {
  int c = npairs / 512;
  if (c < 1) c = 1;
  if (c > 16) c = 16;
  return c;
}

struct MdWork {
  double2 *tau, *bbar, *omega, *ycon;
};
static MdWork md_work(const MdArgs& g, void* work) {
  const int na = g.nao > g.nav ? g.nao : g.nav;
  const size_t na2 = (size_t)na * na;
  MdWork m;
  m.tau = (double2*)work;
  m.bbar = m.tau + (size_t)g.nw * na * g.n;
  m.omega = m.bbar + (size_t)g.nw * na2;
  m.ycon = m.omega + (size_t)g.nw * na2 * na2;
  return m;
}

template <int NA>
static hipError_t launch_prep_na(hipStream_t s, const MdArgs& g, const MdWork& m, double2* ovr) {
  hipLaunchKernelGGL((md_prep_kernel<NA>), dim3((unsigned)g.nw), dim3(256), 0, s, g.n, g.nao, g.nav, g.ndet,
                     g.hstride, g.tpos, (const double2*)g.qbar, g.n_out, g.exc, g.holes, g.parts, g.coef, m.tau,
                     m.bbar, m.omega, m.ycon, g.ncas, ovr);
  return hipGetLastError();
}

template <int NA>
static hipError_t launch_pairs_na(hipStream_t s, const MdArgs& g, const MdWork& m, int nchunk, double* partial) {
  const int per = (g.npairs + nchunk - 1) / nchunk;
  const int64_t nw8 = (g.nw + 7) / 8;
  hipLaunchKernelGGL((md_energy_kernel<NA>), dim3((unsigned)(8 * nw8), nchunk), dim3(256), 0, s, g.n, g.ncas, g.nao,
                     g.nw, g.npairs, per, g.pi, g.pj, g.pK, g.offI, g.offJ, g.offA, g.act_stride, g.n_out,
                     (const double2*)g.qbar, m.tau, m.bbar, m.ycon, partial);
  return hipGetLastError();
}

hipError_t launch_md_prep(hipStream_t s, const MdArgs& g, void* work, double* ovr) {
  if (g.nw <= 0) return hipSuccess;
  const MdWork m = md_work(g, work);
  double2* o = (double2*)ovr;
#define PREP_CALL(NA) launch_prep_na<NA>(s, g, m, o)
  switch (g.nao > g.nav ? g.nao : g.nav) {
    case 1: return PREP_CALL(1);
    case 2: return PREP_CALL(2);
    case 3: return PREP_CALL(3);
    case 4: return PREP_CALL(4);
    case 5: return PREP_CALL(5);
    case 6: return PREP_CALL(6);
    default: return hipErrorInvalidValue;
  }
#undef PREP_CALL
}

hipError_t launch_md_pairs(hipStream_t s, const MdArgs& g, void* work, int nchunk, double* partial) {
  if (g.nw <= 0 || g.npairs <= 0) return hipSuccess;
  const MdWork m = md_work(g, work);
#define PAIRS_CALL(NA) launch_pairs_na<NA>(s, g, m, nchunk, partial)
  switch (g.nao > g.nav ? g.nao : g.nav) {
    case 1: return PAIRS_CALL(1);
    case 2: return PAIRS_CALL(2);
    case 3: return PAIRS_CALL(3);
    case 4: return PAIRS_CALL(4);
    case 5: return PAIRS_CALL(5);
    case 6: return PAIRS_CALL(6);
    default: return hipErrorInvalidValue;
  }
#undef PAIRS_CALL
}

}  // namespace lofqmc
