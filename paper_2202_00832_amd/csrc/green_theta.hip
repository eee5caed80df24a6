// Green's-function intermediate Q = theta = phi (Psi_T^T phi)^{-1} (Eq. 15)
// for a batch of walkers, FP64, as three kernels so that the latency-bound
// elimination does not hold the MFMA work back:
//   1. overlap_kernel: O_w = Psi_T^T phi_w on v_mfma_f64_16x16x4_f64 (real
//      trial x complex walker -> two real 16x16 blocks per block pair);
//      16-row slabs of phi_w and Psi_T are staged in LDS with coalesced loads,
//      prefetched two slabs ahead.  One workgroup per walker.
//   2. invert_kernel: exchange (Gauss-Jordan) elimination with partial
//      pivoting, blocked by 8-column half-panels: each is swept inside one
//      wave (no workgroup barrier per step), the other waves then apply its
//      rank-8 update to their columns.  Gives O^{-1} in pivot order with the
//      pivot rows, log det O and the zero-pivot index.
//   3. apply_kernel: theta = phi O^{-1} on MFMA with three real products per
//      complex block (re = P1 - P2, im = P3 - P1 - P2 with P1 = a_re b_re,
//      P2 = a_im b_im, P3 = (a_re + a_im)(b_re + b_im)); one workgroup per
//      walker with O^{-1} in LDS (put back in natural order while it is staged),
//      one wave per 16-row block.  theta is written
//      walker-major [w][r][j], as [w][j][r] (theta_w^T, with the MFMA operands
//      swapped so that the stores stay 256-byte runs), or orbital-major as
//      [j][r][w]; walkers 8g .. 8g+7 then run on the same XCD so that their
//      interleaved 16-byte stores meet in one L2.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace lofqmc {

template <int NB>
struct GtCfg {
  static constexpr int NP = 16 * NB;
  static constexpr int KC = 16;                // rows of r per overlap slab
  static constexpr int SLOTS = KC * NP;        // complex slots of a phi slab
  static constexpr int OW = NB <= 3 ? 4 : 8;    // waves of the overlap kernel
  static constexpr int OT = 64 * OW;            // its threads
  static constexpr int PER = (SLOTS + OT - 1) / OT;
  static constexpr int NKS = NP / 4;           // K-steps of theta = phi O^{-1}
};

// ---------------------------------------------------------------------------
// 1. O_w = Psi_T^T phi_w, written as a padded NP x NP complex block per walker
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(GtCfg<NB>::OT) void overlap_kernel(int M, int n, int64_t w0, const double* __restrict__ trial,
                                                      const double2* __restrict__ phi,
                                                      double2* __restrict__ O) {
  using C = GtCfg<NB>;
  constexpr int NP = C::NP;
  __shared__ double2 sPh[2][C::SLOTS];
  __shared__ double sPs[2][C::SLOTS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const size_t w = w0 + blockIdx.x;
  const double2* ph = phi + w * (size_t)M * n;

  constexpr int NPAIR = NB * NB;
  constexpr int PPW = (NPAIR + C::OW - 1) / C::OW;
  d4 accR[PPW], accI[PPW];
#pragma unroll
  for (int p = 0; p < PPW; ++p) { accR[p] = d4zero(); accI[p] = d4zero(); }

  double2 pP0[C::PER], pP1[C::PER], pP2[C::PER];
  double pS0[C::PER], pS1[C::PER], pS2[C::PER];
  auto load_slab = [&](int c, double2 (&dP)[C::PER], double (&dS)[C::PER]) {
#pragma unroll
    for (int q = 0; q < C::PER; ++q) {
      const int s = tid + C::OT * q;
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
      const int s = tid + C::OT * q;
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
      if constexpr (NB == 4 && C::OW == 4) {
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
          const int bp = wv + C::OW * p;
          if (bp < NPAIR) {
            const int I = bp / NB, J = bp % NB;
            const double a = sPs[buf][row + 16 * I + lr];
            const double2 b = sPh[buf][row + 16 * J + lr];
            accR[p] = mfma16(a, b.x, accR[p]);
            accI[p] = mfma16(a, b.y, accI[p]);
          }
        }
      }
      // beyond 96 orbitals: operands of one K-step at a time (register file)
      if constexpr (NB > 6) __builtin_amdgcn_sched_barrier(0);
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
    const int bp = wv + C::OW * p;
    if (bp < NPAIR) {
      const int I = bp / NB, J = bp % NB;
#pragma unroll
      for (int v = 0; v < 4; ++v) Ow[(16 * I + 4 * v + lk) * NP + 16 * J + lr] = make_double2(accR[p][v], accI[p][v]);
    }
  }
}

// ---------------------------------------------------------------------------
// 1'. The same product on the FP64 4x4x4 MFMA form, for NB <= 4, M a multiple
//    of 16 and n even (so that every 16-byte chunk of a trial or walker row
//    is whole and aligned).  CS workgroups of four waves per walker, each
//    taking NP / CS columns of O (so a CU holds four workgroups and their
//    slab barriers overlap); wave v owns the 4-row groups g = v + 4q (rows
//    i = 4g .. 4g + 3) against the workgroup's columns.
//    The trial fragment (4 rows x 4 r) is the operand the four blocks of an
//    MFMA share; each block takes 4 walker columns, so one MFMA gives a
//    4 x 16 tile, and per K-step a wave issues 2 NB^2 / CS MFMAs (real and
//    imaginary part) from NB + NB / CS LDS reads.  16-row slabs of Psi_T and phi_w
//    are loaded straight into LDS through buffer descriptors one slab ahead
//    (as in LO pass 1).  Psi_T sits in LDS as [r][i] with the 16-byte column
//    pairs of row r XOR-swizzled by 2 (r & 3), so a fragment read (4 rows r x
//    4 consecutive i) falls in 8 distinct bank groups; phi_w as [r][j].
//    Columns i, j >= n load a valid neighbour and their outputs are written
//    as the zeros of the padded block.
// ---------------------------------------------------------------------------
template <int NB, int CS>
__global__ __launch_bounds__(256) void overlap4_kernel(int M, int n, int64_t w0, const double* __restrict__ trial,
                                                       const double2* __restrict__ phi, double2* __restrict__ O) {
  static_assert(NB % CS == 0, "column parts of whole blocks");
  constexpr int NP = 16 * NB;
  constexpr int NJ = NP / CS;               // columns of this workgroup
  constexpr int CB = NB / CS;               // their 16-column blocks
  constexpr int NWV = 4;
  constexpr int A_CH = 8 * NP;              // 16-byte chunks of a trial slab (16 rows x NP doubles)
  constexpr int B_CH = 16 * NJ;             // of a walker slab (16 rows x NJ complex)
  constexpr int A_LD = (A_CH + 255) / 256;  // wave-instructions per thread for A (ceil)
  constexpr int B_LD = B_CH / 256;          // for B (exactly CB)
  __shared__ __attribute__((aligned(16))) double sA0[16 * NP];
  __shared__ __attribute__((aligned(16))) double sA1[16 * NP];
  __shared__ __attribute__((aligned(16))) double2 sB0[16 * NJ];
  __shared__ __attribute__((aligned(16))) double2 sB1[16 * NJ];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t w = w0 + blockIdx.x / CS;
  const int j0 = NJ * (int)(blockIdx.x % CS);

  // chunk offsets (bytes from the slab's first row) of this thread's loads
  uint32_t aoff[A_LD], boff[B_LD];
#pragma unroll
  for (int k = 0; k < A_LD; ++k) {
    const int S = 256 * k + tid;                      // chunk slot in LDS
    const int r = (S / (NP / 2)) & 15;
    const int cp = (S % (NP / 2)) ^ (2 * (r & 3));    // logical column pair
    const int i = min(2 * cp, n - 2);
    aoff[k] = (uint32_t)(((size_t)r * n + i) * sizeof(double));
  }
#pragma unroll
  for (int k = 0; k < B_LD; ++k) {
    const int S = 256 * k + tid;
    const int r = S / NJ, j = min(j0 + S % NJ, n - 1);
    boff[k] = (uint32_t)(((size_t)r * n + j) * sizeof(double2));
  }
  const __amdgpu_buffer_rsrc_t ares =
      __builtin_amdgcn_make_buffer_rsrc((void*)trial, 0, (int)((size_t)M * n * sizeof(double)), 0x00020000);
  const __amdgpu_buffer_rsrc_t bres = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(phi + w * (size_t)M * n), 0, (int)((size_t)M * n * sizeof(double2)), 0x00020000);
  auto issue = [&](int c, double* sa, double2* sb) __attribute__((always_inline)) {
    const int srow = 16 * c * n;   // first element of the slab's rows
#pragma unroll
    for (int k = 0; k < A_LD; ++k) {
      if (A_CH % 256 == 0 || 256 * k + 64 * wv < A_CH) {
        auto* dst = (__attribute__((address_space(3))) void*)(sa + 2 * (256 * k + 64 * wv));
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ares, dst, 16, (int)aoff[k], srow * (int)sizeof(double), 0, 0);
      }
    }
#pragma unroll
    for (int k = 0; k < B_LD; ++k) {
      auto* dst = (__attribute__((address_space(3))) void*)(sb + 256 * k + 64 * wv);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(bres, dst, 16, (int)boff[k], srow * (int)sizeof(double2), 0, 0);
    }
  };

  // acc[q][c][p]: rows 4 (wv + 4 q) + lk, columns j0 + 16 c + lr, part p (re, im)
  double acc[NB][CB][2];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[q][c][0] = acc[q][c][1] = 0.0;
  // A operand of this lane: row i = 4 (wv + 4 q) + (lane & 3), r = 4 s4 + lk:
  // column pair 2 (wv + 4 q) + ((lane & 3) >> 1) of row r, element lane & 1
  const int e2 = 2 * (lk & 3);   // swizzle of row r = 4 s4 + lk (r & 3 = lk)
  auto compute = [&](const double* sa, const double2* sb) __attribute__((always_inline)) {
    double a[2][NB];
    double2 b[2][CB];
    auto read = [&](int s4, int slot) __attribute__((always_inline)) {
      const int r = 4 * s4 + lk;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int cp = (2 * (wv + NWV * q) + ((lane & 3) >> 1)) ^ e2;
        a[slot][q] = sa[r * NP + 2 * cp + (lane & 1)];
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) b[slot][c] = sb[r * NJ + 16 * c + lr];
    };
    read(0, 0);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int u = s4 & 1;
      if (s4 < 3) read(s4 + 1, u ^ 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          acc[q][c][0] = mfma4(a[u][q], b[u][c].x, acc[q][c][0]);
          acc[q][c][1] = mfma4(a[u][q], b[u][c].y, acc[q][c][1]);
        }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  const int nslab = M / 16;
  issue(0, sA0, sB0);
  wait_vmcnt0();
  __syncthreads();
  for (int c = 0; c < nslab; c += 2) {
    if (c + 1 < nslab) issue(c + 1, sA1, sB1);
    compute(sA0, sB0);
    wait_vmcnt0();
    __syncthreads();
    if (c + 1 < nslab) {
      if (c + 2 < nslab) issue(c + 2, sA0, sB0);
      compute(sA1, sB1);
      wait_vmcnt0();
      __syncthreads();
    }
  }
  double2* Ow = O + w * (size_t)NP * NP;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int i = 4 * (wv + NWV * q) + lk;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int j = j0 + 16 * c + lr;
      const bool in = i < n && j < n;
      Ow[(size_t)i * NP + j] = in ? make_double2(acc[q][c][0], acc[q][c][1]) : make_double2(0.0, 0.0);
    }
  }
}

// ---------------------------------------------------------------------------
// 2. O_w -> R_w, the exchange (Gauss-Jordan) inverse in pivot order:
//    O_w^{-1}[k][p_m] = R_w[p_k][m], with the pivot rows p_k written to perm;
//    log det O_w and the zero-pivot index.  Wave q owns the 16 columns
//    16q .. 16q+15 of every row (lane l holds rows l and l + 64).
//
//    Blocked by half-panels of 8 columns: half h of wave b's columns is
//    swept by wave b alone: for each of its columns k, the pivot row p (the
//    largest |re|+|im| among rows not yet used, compared on its exponent and
//    leading 14 mantissa bits, lowest row on ties), then A[i][j] -= m_i A[p][j] on the half's columns with
//    m_i = (A[i][k] + [i == p]) / A[p][k], and column k set to A[i][k] / A[p][k]
//    (1 / A[p][k] on row p).  The eight sweeps act on any other column as
//    one rank-8 update: with P the half's pivot rows, Z = A[P, J] taken
//    before the half and F the swept columns,
//        A[:, J] <- (rows not in P ? A[:, J] : 0) - F Z,
//    which every other wave applies to its own columns after one barrier and
//    wave b to its other half straight from its registers, so it sweeps its
//    second half without waiting for the others.  (Sixteen-column panels
//    broadcast sixteen pivot-row entries per step through v_readlane, which
//    made the serial sweep issue-bound.)
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(64 * NB) void invert_kernel(int n, int64_t w0, double2* __restrict__ O, int* __restrict__ perm,
                                                          double2* __restrict__ logov, int* __restrict__ info,
                                                          int flag_small) {
  constexpr int NP = 16 * NB;
  constexpr int RPL = (NP + 63) / 64;        // rows per lane
  constexpr int FS = 9;                      // padded row stride of the half-panel copy
  __shared__ double2 sF[2][NP * FS];         // swept half-panel columns, by half
  __shared__ double2 sZ[NB][8][16];          // per wave: its columns of the half-panel's pivot rows
  __shared__ int sPiv[NP];
  __shared__ double2 sPivV[NP];
  __shared__ int sZero[2];
  __shared__ int sInvW[2 * NB];              // per half-panel: inversions of the pivot order
  __shared__ int sSmall[2 * NB];             // per half-panel: first step with a small pivot (flag_small)
  __shared__ double sOmax[NB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const size_t w = w0 + blockIdx.x;
  double2* Ow = O + w * (size_t)NP * NP;

  // the padded block is block-diag(O, I): the padding steps pivot on their own
  // diagonal and leave O's block alone, so every panel runs 16 full steps
  double2 e[RPL][16];
  bool used[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int row = lane + 64 * t;
    used[t] = row >= NP;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int col = 16 * wv + j;
      e[t][j] = row < NP ? Ow[(size_t)row * NP + col] : make_double2(0.0, 0.0);
      if (row >= n && row < NP && row == col) e[t][j] = make_double2(1.0, 0.0);
    }
  }

  // with flag_small: the largest |re| + |im| of O's entries, and pivots below
  // 2^-40 of it mark the overlap as nearly singular (reported as info = -k)
  double thr = -1.0;
  if (flag_small) {
    double m = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = lane + 64 * t;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (row < n && 16 * wv + j < n) m = fmax(m, fabs(e[t][j].x) + fabs(e[t][j].y));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (lane == 0) sOmax[wv] = m;
    __syncthreads();
    double om = 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) om = fmax(om, sOmax[q]);
    thr = om * 0x1p-40;
  }
  int small = 0;

  int zero = 0;
  // sweep of half H of wave b's columns (8 H .. 8 H + 7), then its publication
  auto sweep_half = [&](auto hc, int b) __attribute__((always_inline)) {
    constexpr int H = decltype(hc)::value;
    // inversions of k -> p_k: the rows still unused at step k are the later
    // pivots, so the step adds the number of unused rows below p_k.  Lane c
    // keeps the pivot row and value of step c (no branches inside the sweep,
    // so its eight steps form one block the scheduler can overlap).
    int inversions = 0;
    int myp = 0;
    double mypr = 1.0, mypi = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int jc = 8 * H + c;               // this wave's column
      const int k = 16 * b + jc;
      // key: exponent and leading 14 mantissa bits of |re|+|im| above the
      // complement of the row index (largest magnitude, lowest row on ties)
      unsigned key = 0u;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = lane + 64 * t;
        const double2 v = e[t][jc];
        const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(fabs(v.x) + fabs(v.y)) >> 32);
        const unsigned kt = used[t] ? 0u : (((hi >> 6) << 7) | (unsigned)(127 - row));
        key = kt > key ? kt : key;
      }
      key = wave_max_u32(key);
      // no pivot left (singular): record the first such step; the sweeps go
      // on with zero multipliers and the result is discarded
      const bool ok = (key >> 7) != 0u && zero == 0;
      zero = (zero == 0 && !ok) ? k + 1 : zero;
      const int p = 127 - (int)(key & 127u);
      const int pl = p & 63, pt = p >> 6;
#pragma unroll
      for (int t = 0; t < RPL; ++t) inversions += __popcll(__ballot(!used[t] && lane + 64 * t < p));
      // pivot value and, inside the update, the pivot row (the half's 8
      // columns) from lane pl, read into scalar registers one entry at a time
      const double2 piv = make_double2(readlane_f64(RPL > 1 && pt == 1 ? e[RPL - 1][jc].x : e[0][jc].x, pl),
                                       readlane_f64(RPL > 1 && pt == 1 ? e[RPL - 1][jc].y : e[0][jc].y, pl));
      small = (small == 0 && ok && k < n && fabs(piv.x) + fabs(piv.y) < thr) ? k + 1 : small;
      // 1 / |pivot|^2: hardware reciprocal refined by two Newton steps
      const double d = fma(piv.x, piv.x, piv.y * piv.y);
      double r = __builtin_amdgcn_rcp(d);
      r = fma(r, fma(-d, r, 1.0), r);
      r = fma(r, fma(-d, r, 1.0), r);
      const double rn = ok ? r : 0.0;
      const double2 inv = make_double2(piv.x * rn, -piv.y * rn);
      // (selects on scalars: a select of two double2 values goes through scratch)
      myp = lane == c ? p : myp;
      mypr = lane == c ? piv.x : mypr;
      mypi = lane == c ? piv.y : mypi;
      double2 mi[RPL], cc[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = lane + 64 * t;
        double2 ci = e[t][jc];
        cc[t].x = row == p ? 1.0 : ci.x;
        cc[t].y = row == p ? 0.0 : ci.y;
        ci.x += row == p ? 1.0 : 0.0;
        const double2 m = cmul(ci, inv);
        mi[t].x = ok ? m.x : 0.0;
        mi[t].y = ok ? m.y : 0.0;
      }
#pragma unroll
      for (int j = 8 * H; j < 8 * H + 8; ++j) {
        const double2 src = (RPL > 1 && pt == 1) ? e[RPL - 1][j] : e[0][j];
        const double2 a = make_double2(readlane_f64(src.x, pl), readlane_f64(src.y, pl));
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          double2 v = e[t][j];
          v.x = fma(-mi[t].x, a.x, fma(mi[t].y, a.y, v.x));
          v.y = fma(-mi[t].x, a.y, fma(-mi[t].y, a.x, v.y));
          e[t][j] = v;
        }
      }
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const double2 v = cmul(cc[t], inv);
        e[t][jc].x = ok ? v.x : e[t][jc].x;
        e[t][jc].y = ok ? v.y : e[t][jc].y;
        if (lane + 64 * t == p) used[t] = true;
      }
    }
    // publish the swept columns (every row) and the outcome
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = lane + 64 * t;
      if (row < NP) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sF[H][row * FS + j] = e[t][8 * H + j];
      }
    }
    if (lane < 8) {
      sPiv[16 * b + 8 * H + lane] = myp;
      sPivV[16 * b + 8 * H + lane] = make_double2(mypr, mypi);
    }
    if (lane == 0) {
      sZero[H] = zero;
      sInvW[2 * b + H] = inversions;
      sSmall[2 * b + H] = small;
    }
  };
  // Z = this wave's columns J0 .. J0 + NJ - 1 at the pivot rows of half-panel
  // hp (first column k0 = 8 hp), through wave-local LDS (a wavefront-scope
  // release/acquire pair around a wave barrier orders the writes before the
  // reads of the other lanes); then the pivot rows of those columns zeroed
  auto take_z = [&](auto j0c, auto njc, int hp, bool (&inp)[RPL]) __attribute__((always_inline)) {
    constexpr int J0 = decltype(j0c)::value, NJ = decltype(njc)::value;
    int pos[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) pos[t] = -1;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int pc = sPiv[8 * hp + c];
#pragma unroll
      for (int t = 0; t < RPL; ++t)
        if (lane + 64 * t == pc) pos[t] = c;
    }
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      inp[t] = pos[t] >= 0;
      if (pos[t] >= 0) {
        used[t] = true;
#pragma unroll
        for (int j = 0; j < NJ; ++j) sZ[wv][pos[t]][j] = e[t][J0 + j];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      if (inp[t]) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) e[t][J0 + j] = make_double2(0.0, 0.0);
      }
    }
  };
  // rank-8 update of all sixteen columns of a wave that did not sweep
  // half-panel hp, with F from LDS (buffer H)
  auto update_other = [&](int hp, int H) __attribute__((always_inline)) {
    bool inp[RPL];
    take_z(std::integral_constant<int, 0>{}, std::integral_constant<int, 16>{}, hp, inp);
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = lane + 64 * t;
      if (row < NP) {
        // per swept column: the Z row's loads are all issued before the
        // products (a scheduling barrier keeps them apart), so each product
        // waits only for its own operand; c is not unrolled (only j must be static)
#pragma unroll 1
        for (int c = 0; c < 8; ++c) {
          double2 z[16];
          const double2 f = sF[H][row * FS + c];
#pragma unroll
          for (int j = 0; j < 16; ++j) z[j] = sZ[wv][c][j];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            e[t][j].x = fma(-f.x, z[j].x, fma(f.y, z[j].y, e[t][j].x));
            e[t][j].y = fma(-f.x, z[j].y, fma(-f.y, z[j].x, e[t][j].y));
          }
        }
      }
    }
  };
  // rank-8 update of the sweeping wave's other half by its half H, with F
  // from its own registers
  auto update_self = [&](auto hc, int hp) __attribute__((always_inline)) {
    constexpr int H = decltype(hc)::value;
    constexpr int JO = 8 * (1 - H), FO = 8 * H;
    bool inp[RPL];
    take_z(std::integral_constant<int, JO>{}, std::integral_constant<int, 8>{}, hp, inp);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      double2 z[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) z[j] = sZ[wv][c][j];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const double2 f = e[t][FO + c];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          e[t][JO + j].x = fma(-f.x, z[j].x, fma(f.y, z[j].y, e[t][JO + j].x));
          e[t][JO + j].y = fma(-f.x, z[j].y, fma(-f.y, z[j].x, e[t][JO + j].y));
        }
      }
    }
  };
  // the sweeping wave runs at raised issue priority from its first half
  // through its second, so that on a SIMD shared with other waves (the rank-8
  // updates, the other walker's workgroup) the serial chain issues first
  // (225 against 235 us for green_theta at 512 walkers; raising the next
  // sweeper's update as well gave nothing)
  for (int b = 0; b < NB; ++b) {
    if (wv == b) {
      __builtin_amdgcn_s_setprio(3);
      sweep_half(std::integral_constant<int, 0>{}, b);
    }
    __syncthreads();
    zero = sZero[0];
    if (zero) break;
    if (wv == b)
      update_self(std::integral_constant<int, 0>{}, 2 * b);
    else
      update_other(2 * b, 0);
    if (wv == b) {
      sweep_half(std::integral_constant<int, 1>{}, b);
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    zero = sZero[1];
    if (zero) break;
    if (wv == b)
      update_self(std::integral_constant<int, 1>{}, 2 * b + 1);
    else
      update_other(2 * b + 1, 1);
  }
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();

  // R in pivot order, row-contiguous (identity on the padding)
  if (!zero) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = lane + 64 * t;
      if (row < NP) {
#pragma unroll
        for (int j = 0; j < 16; ++j) Ow[(size_t)row * NP + 16 * wv + j] = e[t][j];
      }
    }
  }
  if (wv == 0) {
    // pivot rows: a permutation of 0..NP-1, the identity on the padding
    for (int i = lane; i < NP; i += 64) perm[w * NP + i] = zero ? i : sPiv[i];
    // log det O = sum_k log(pivot_k) + i pi * parity of the permutation k -> p_k
    double la = 0.0, ar = 0.0;
    int inv_count = 0;
    if (!zero) {
      for (int k = lane; k < n; k += 64) {
        const double2 pv = sPivV[k];
        la += log(hypot(pv.x, pv.y));
        ar += atan2(pv.y, pv.x);
      }
#pragma unroll
      for (int b = 0; b < 2 * NB; ++b) inv_count += sInvW[b];
    }
    la = wave_sum_lane0(la);
    ar = wave_sum_lane0(ar);
    if (lane == 0) {
      // the first small pivot: the panels are swept in order, so the first
      // panel that recorded one
      int first_small = 0;
      if (flag_small && !zero) {
        for (int b = 2 * NB - 1; b >= 0; --b) first_small = sSmall[b] ? sSmall[b] : first_small;
      }
      info[w] = zero ? zero : -first_small;
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
// 3. theta_w = phi_w O_w^{-1}; one 512-thread workgroup per walker and part of
//    CB column blocks (all NB of them up to 96 orbitals; beyond that the
//    columns of O_w^{-1} no longer fit the LDS and blockIdx.y picks the part),
//    the part of O_w^{-1} staged once in LDS, wave (q, h) takes the 16-row
//    blocks q, q+4, ... against half h of the part's column blocks.
//    TRANS (theta written as theta_w^T, [nw][n][M]): the two MFMA operands
//    swap places, so the products give the blocks of theta_w^T = O_w^{-T}
//    phi_w^T from the same fragments (same loads, same sums) and each lane's
//    outputs run along r, the contiguous index of that layout.
// ---------------------------------------------------------------------------
template <int NB, int CB, bool TRANS>
__global__ __launch_bounds__(512) void apply_kernel(int M, int n, int64_t nw, int64_t w0, int64_t nwc,
                                                    const double2* __restrict__ phi,
                                                    const double2* __restrict__ Oinv, const int* __restrict__ perm,
                                                    const int* __restrict__ info,
                                                    double2* __restrict__ theta, int orbital_major) {
  using C = GtCfg<NB>;
  constexpr int NP = C::NP;
  constexpr int CW = 16 * CB;                  // columns of one part
  __shared__ double2 sB[NP * CW];
  __shared__ int sP[NP], sPi[NP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // first column of the part (a compile-time 0 with a single part, which
  // keeps the indexing and the bounds below static)
  const int c0 = CB == NB ? 0 : CW * (int)blockIdx.y;
  // workgroups go round-robin over the 8 XCDs; walkers 8g .. 8g+7 share an
  // XCD so that their interleaved orbital-major 16-byte stores meet in one L2
  int64_t w;
  {
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, slot = b >> 3;
    w = 8 * (xcd + 8 * (slot >> 3)) + (slot & 7);
    if (w >= nwc) return;
    w += w0;
  }
  // O_w^{-1} into LDS from R_w in pivot order: O^{-1}[pinv[i]][piv[m]] = R[i][m]
  const double2* Bw = Oinv + w * (size_t)NP * NP;
  const bool bad = info[w] > 0;   // an exact zero pivot (a negative info only warns)
  if (!bad) {
    for (int i = tid; i < NP; i += 512) {
      const int p = perm[w * NP + i];
      sP[i] = p;
      if ((unsigned)p < (unsigned)NP) sPi[p] = i;
    }
  }
  __syncthreads();
  if (CB == NB) {
    for (int e = tid; e < NP * NP; e += 512) {
      if (bad) {
        sB[e] = make_double2(0.0, 0.0);
      } else {
        const int i = e / NP, m = e % NP;
        sB[sPi[i] * NP + sP[m]] = Bw[e];
      }
    }
  } else {
    // the part's columns only: entries of R whose column lands in [c0, c0 + CW)
    for (int e = tid; e < NP * NP; e += 512) {
      const int i = e / NP, m = e % NP;
      if (bad) {
        if (m < CW) sB[i * CW + m] = make_double2(0.0, 0.0);
      } else {
        const int c = sP[m] - c0;
        if (c >= 0 && c < CW) sB[sPi[i] * CW + c] = Bw[e];
      }
    }
  }
  __syncthreads();
  const int ksteps = (n + 3) / 4;
  const double2* ph = phi + w * (size_t)M * n;
  const double nan = __builtin_nan("");
  // wave (q, h): 16-row blocks q, q+4, ... against the column blocks of half
  // h (JH blocks each), which keeps the accumulators to 3 * JH 16x16 blocks
  constexpr int JH = (CB + 1) / 2;
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
          const int JJ = hf * JH + J;   // block within the part
          if (JJ < CB && c0 + 16 * JJ < NP) {
            const double2 bv = kk < NP ? sB[kk * CW + 16 * JJ + lr] : make_double2(0.0, 0.0);
            if constexpr (TRANS) {
              P1[J] = mfma16(bv.x, av[u].x, P1[J]);
              P2[J] = mfma16(bv.y, av[u].y, P2[J]);
              P3[J] = mfma16(bv.x + bv.y, as, P3[J]);
            } else {
              P1[J] = mfma16(av[u].x, bv.x, P1[J]);
              P2[J] = mfma16(av[u].y, bv.y, P2[J]);
              P3[J] = mfma16(as, bv.x + bv.y, P3[J]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int J = 0; J < JH; ++J) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // element v of the accumulator: (row 4 v + lk, column lr) of the
        // 16 x 16 block, (r, j) or, with TRANS, (j, r)
        const int j = c0 + 16 * (hf * JH + J) + (TRANS ? 4 * v + lk : lr);
        const int row = 16 * rb + (TRANS ? lr : 4 * v + lk);
        if (hf * JH + J < CB && row < M && j < n) {
          const double re = P1[J][v] - P2[J][v];
          const double im = P3[J][v] - P1[J][v] - P2[J][v];
          const double2 val = bad ? make_double2(nan, nan) : make_double2(re, im);
          if (TRANS)
            theta[(w * (size_t)n + j) * M + row] = val;
          else if (orbital_major)
            theta[((size_t)j * M + row) * nw + w] = val;
          else
            theta[(w * (size_t)M + row) * n + j] = val;
        }
      }
    }
  }
}

// workspace: the overlap matrices (then R), [nw][NP][NP] complex, followed at
// a 256-byte boundary by the pivot rows [nw][NP] int32
static size_t gt_perm_offset(int n, int64_t nw) {
  const size_t NP = 16 * (size_t)((n + 15) / 16);
  return (sizeof(double2) * NP * NP * (size_t)nw + 255) / 256 * 256;
}

size_t green_theta_workspace(int n, int64_t nw) {
  const size_t NP = 16 * (size_t)((n + 15) / 16);
  return gt_perm_offset(n, nw) + sizeof(int) * NP * (size_t)nw;
}

template <int NB>
static hipError_t launch_gt(hipStream_t s, int M, int n, int64_t nw, int64_t w0, int64_t nwc, const double* trial,
                            const double* phi, double* theta, double* logov, int* info, int theta_layout,
                            double* work, const ProfHook* prof, int flag_small) {
  double2* O = reinterpret_cast<double2*>(work);
  int* perm = reinterpret_cast<int*>(reinterpret_cast<char*>(work) + gt_perm_offset(n, nw));
  // the 4x4x4 form where its loads are whole 16-byte chunks of full slabs
  // and the buffer offsets of one walker fit 32 bits
  bool four = false;
  if constexpr (NB <= 4) four = M % 16 == 0 && n % 2 == 0 && (int64_t)M * n * 16 <= (int64_t)INT32_MAX;
  if (four) {
    prof_mark(prof, "overlap4_kernel");
    // one workgroup per walker (two column parts measured slower at 60 orbitals)
    if constexpr (NB <= 4) {
      constexpr int CS = 1;
      hipLaunchKernelGGL((overlap4_kernel<NB, CS>), dim3((unsigned)(nwc * CS)), dim3(256), 0, s, M, n, w0, trial,
                         (const double2*)phi, O);
    }
  } else {
    prof_mark(prof, "overlap_kernel");
    hipLaunchKernelGGL(overlap_kernel<NB>, dim3((unsigned)nwc), dim3(GtCfg<NB>::OT), 0, s, M, n, w0, trial,
                       (const double2*)phi, O);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_mark(prof, "invert_kernel");
  hipLaunchKernelGGL(invert_kernel<NB>, dim3((unsigned)nwc), dim3(64 * NB), 0, s, n, w0, O, perm, (double2*)logov,
                     info, flag_small);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = 64 * ((nwc + 63) / 64);
  // up to 96 orbitals O^{-1} fits the LDS whole; beyond, two column parts
  constexpr int CB = NB <= 6 ? NB : (NB + 1) / 2;
  constexpr int parts = (NB + CB - 1) / CB;
  prof_mark(prof, "apply_kernel");
  if (theta_layout == THETA_TRANSPOSED)
    hipLaunchKernelGGL((apply_kernel<NB, CB, true>), dim3((unsigned)grid, parts), dim3(512), 0, s, M, n, nw, w0, nwc,
                       (const double2*)phi, (const double2*)O, perm, info, (double2*)theta, 0);
  else
    hipLaunchKernelGGL((apply_kernel<NB, CB, false>), dim3((unsigned)grid, parts), dim3(512), 0, s, M, n, nw, w0,
                       nwc, (const double2*)phi, (const double2*)O, perm, info, (double2*)theta,
                       theta_layout == THETA_ORBITAL ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_green_theta(hipStream_t s, int M, int n, int64_t nw, int64_t w0, int64_t nwc, const double* trial,
                              const double* phi, double* theta, double* logov, int* info, int theta_layout,
                              double* work, const ProfHook* prof, int flag_small) {
  if (nwc <= 0) return hipSuccess;
  if (n <= 16) return launch_gt<1>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
  if (n <= 32) return launch_gt<2>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
  if (n <= 48) return launch_gt<3>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
  if (n <= 64) return launch_gt<4>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
  if (n <= 80) return launch_gt<5>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
  if (n <= 96) return launch_gt<6>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
  return launch_gt<7>(s, M, n, nw, w0, nwc, trial, phi, theta, logov, info, theta_layout, work, prof, flag_small);
}

}  // namespace lofqmc
