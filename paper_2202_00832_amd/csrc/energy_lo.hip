// Two-body energy by the LO route (Sec. 2.3.2, Eq. 22-23), FP64.
//
// Stored factors: for every pair i <= j the rows [Ubar^T ; Vbar] (2 K_ij x M).
// Each stored row multiplies the walker column of both orbitals of its pair:
//   orbital i:  [Ubar^T Q_i ; Vbar Q_i] = [QL_i ; QR_i]
//   orbital j:  [Ubar^T Q_j ; Vbar Q_j] = [QL_j ; QR_j]
// so, grouping the rows by orbital, the four vectors of Eq. 23 for all pairs
// come from one dense product per orbital o: (rows touching o) x Q_o, with the
// walkers as the wide dimension (pass 1, FP64 MFMA).  Pass 2 forms the dot
// products of Eq. 22 per pair and walker,
//   J_ij = QL_i . QR_j,   X_ij = QL_j . QR_i   (complex, bilinear),
// with weight 1 for i = j and 2 for i < j (Y^[ji] = (Y^[ij])^T), and sums
// E_J = 2 sum J, E_K = -sum X in a fixed order per chunk of rank rows.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace lofqmc {

// Pass 1: tile = up to LO_TILE_ROWS (192) output rows of one orbital o x 32
// walkers.  The rows touching one orbital number about 2 x (sum of its pair
// ranks), nearly the same for every orbital of a localized basis, so one tile
// usually covers an orbital and each theta element is fetched once per
// orbital.  Eight waves; wave v owns rows 24v .. 24v + 23 (six groups of 4)
// against all 32 walkers (two 16-walker blocks, real and imaginary part) on
// the FP64 4x4x4 MFMA: 24 accumulators, 24 MFMA per K-step from 6 + 2 LDS
// reads.  Per 16-row slab of r the factor rows (gathered through rowidx) and
// Q_o of the 32 walkers are staged in LDS (double-buffered): lo_pass1_kernel
// loads both straight into LDS one slab ahead (M a multiple of 16);
// lo_pass1_reg_kernel, for any M, stages them through registers (theta one
// slab ahead, the factor rows after the products, to stay at two workgroups
// per CU) and zero-fills a partial last slab.
//
// theta element (o, r, w) is read at theta[o * so + r * sr + w * sw], which
// serves the three layouts: walker-major [w][r][o], orbital-major [o][r][w]
// and transposed walker-major [w][o][r].
// Work units (block of LO_OBLK orbitals, walker tile) go round-robin over the
// 8 XCDs (workgroups are dispatched round-robin over XCDs) and the tiles of
// one unit run side by side on one XCD: with walker-major theta the orbitals
// of a block share cache lines, which that XCD's L2 then fetches once.
constexpr int LO_TILE_ROWS = 192;
constexpr int LO_WT = 32;
constexpr int LO_OBLK = 8;
constexpr int LO_WROWS = LO_TILE_ROWS / 8;   // rows per wave (24)
constexpr int LO_QG = LO_WROWS / 4;          // 4-row groups per wave (6)

__global__ __launch_bounds__(512, 2) void lo_pass1_reg_kernel(int M, int64_t nw, const double* __restrict__ rows,
                                                          const int* __restrict__ rowidx,
                                                          const int* __restrict__ tile_orb,
                                                          const int* __restrict__ tile_row0,
                                                          const int* __restrict__ tile_nrows,
                                                          const int* __restrict__ blk, int nblk, int tmax,
                                                          const double2* __restrict__ theta, int64_t so,
                                                          int64_t sr, int64_t sw, double2* __restrict__ qbar,
                                                          int64_t orow, int64_t ow, int nwt) {
  __shared__ double sA[2][LO_TILE_ROWS][17];   // [row][r], padded against bank conflicts
  __shared__ double2 sB[2][16][LO_WT];         // [r][walker]
  int t;
  int64_t w0;
  {
    const int xcd = blockIdx.x & 7;
    const int slot = blockIdx.x >> 3;
    const int64_t u = 8 * (int64_t)(slot / tmax) + xcd;
    if (u >= (int64_t)nblk * nwt) return;
    const int b = (int)(u / nwt);
    t = blk[b] + slot % tmax;
    if (t >= blk[b + 1]) return;
    w0 = (u % nwt) * LO_WT;
  }
  const int o = tile_orb[t];
  const int row0 = tile_row0[t];
  const int nrows = tile_nrows[t];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int rw = LO_WROWS * wv;                // first row of this wave
  const bool active = rw < nrows;
  const double2* tho = theta + o * so;

  // staging: A = nrows x 16 doubles (each row 128 contiguous bytes), B = 16 x 32 complex
  constexpr int A_PER = LO_TILE_ROWS * 16 / 512;   // 6
  double pa[A_PER];
  double2 pb;
  // the gathered factor rows of this thread, resolved once (a row index read
  // inside the slab loop would put a dependent global load on every slab)
  int arow[A_PER];
#pragma unroll
  for (int p = 0; p < A_PER; ++p) {
    const int row = (tid + 512 * p) >> 4;
    arow[p] = row < nrows ? rowidx[row0 + row] : -1;
  }
  const int brr = tid / LO_WT, bww = tid % LO_WT;
  const int64_t bw = w0 + bww;
  // theta (HBM) is fetched one slab ahead, across the products; the factor
  // rows (small, reused by every walker tile, so mostly cache hits) after them,
  // which keeps two workgroups per CU
  auto load_a = [&](int c) {
    const int rbase = 16 * c;
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int r = rbase + ((tid + 512 * p) & 15);
      pa[p] = (arow[p] >= 0 && r < M) ? rows[(size_t)arow[p] * M + r] : 0.0;
    }
  };
  auto load_b = [&](int c) {
    const int r = 16 * c + brr;
    pb = (r < M && bw < nw) ? tho[r * sr + bw * sw] : make_double2(0.0, 0.0);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int e = tid + 512 * p;
      sA[buf][e >> 4][e & 15] = pa[p];
    }
    sB[buf][brr][bww] = pb;
  };

  // acc[q][c]: rows rw + 4q + lk, walker column c (block h = c / 2, part = c % 2)
  // -- one FP64 4x4x4 accumulator each (see mfma4)
  double acc[LO_QG][4];
#pragma unroll
  for (int q = 0; q < LO_QG; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = 0.0;
  const int nchunk = (M + 15) / 16;
  load_a(0);
  load_b(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) load_b(c + 1);
    if (active) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int rr = 4 * s4 + lk;
        const double2 b0 = sB[buf][rr][lr];
        const double2 b1 = sB[buf][rr][16 + lr];
#pragma unroll
        for (int q = 0; q < LO_QG; ++q) {
          const double a = sA[buf][rw + 4 * q + (lane & 3)][rr];
          acc[q][0] = mfma4(a, b0.x, acc[q][0]);
          acc[q][1] = mfma4(a, b0.y, acc[q][1]);
          acc[q][2] = mfma4(a, b1.x, acc[q][2]);
          acc[q][3] = mfma4(a, b1.y, acc[q][3]);
        }
      }
    }
    if (c + 1 < nchunk) {
      load_a(c + 1);
      store(buf ^ 1);
    }
    __syncthreads();
  }
  // lane holds rows rw + 4q + lk, walker 16h + lr
  if (active) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t w = w0 + 16 * h + lr;
      if (w < nw) {
#pragma unroll
        for (int q = 0; q < LO_QG; ++q) {
          const int lrow = rw + 4 * q + lk;
          if (lrow < nrows)
            qbar[(size_t)(row0 + lrow) * orow + w * ow] = make_double2(acc[q][2 * h], acc[q][2 * h + 1]);
        }
      }
    }
  }
}

// The same product with both operand tiles loaded straight into LDS
// (global_load_lds_dwordx4: lane L of a wave writes 16 bytes at the wave's
// LDS base + 16 L), one slab ahead, so their latency overlaps the products of
// the current slab without holding them in registers.  Used when M is a
// multiple of 16 (every slab full: a lane cannot zero-fill what it loads).
// The A tile is stored unpadded with the column pairs of row r XOR-swizzled
// by 2 (r & 3): the 4 rows x 2 column pairs of one MFMA operand read fall in 8
// distinct 16-byte bank groups.  Rows past the tile and walkers past nw load
// a valid address and their outputs are discarded.
// Eight waves, 192-row tiles, two workgroups per CU (an orbital touching more
// rows is cut into near-equal tiles, each gathering its theta column again;
// with the operand reads pipelined as below this measured faster than one
// 384-row tile in a sixteen-wave workgroup, whose slab barriers no second
// workgroup on the CU covers).
// The tile's 4-row groups are dealt to the waves in turn (group g to wave
// g % 8), so a tile that is not full leaves every SIMD (waves v and v + 4)
// the same number of groups to within one, instead of idling the SIMDs whose
// waves hold the end of the tile.
// BUF: the slab loads go through buffer descriptors (buffer_load_dwordx4 ...
// lds, 32-bit byte offsets from the factor rows and from the tile's theta
// slice).  The global-address form (global_load_lds) is a FLAT-encoded
// instruction that writes LDS; while one is in flight the compiler orders
// every LDS read by lgkmcnt(0), so the operand reads of the next K-step could
// not overlap the products of the current one.  The buffer form is counted by
// vmcnt alone and keeps the graded waits; the global form is kept for byte
// offsets beyond 2^31 (factor rows or one orbital's theta slice).
// TR (theta as [w][o][r], r contiguous): the 16 x 32 theta slab is loaded as
// 32 runs of 16 consecutive r (256 bytes, two cache lines per walker) instead
// of 512 elements from as many lines; it sits in LDS as [walker][r] with r
// XOR-swizzled by the walker's low four bits, so the operand reads (16
// walkers x 4 r per read) spread over all bank groups.

// calls f(integral_constant<q>) for the wave-uniform group count q in 1 .. N
template <int N, typename F>
__device__ __forceinline__ void with_group_count(int q, F&& f) {
  if constexpr (N > 0) {
    if (q == N)
      f(std::integral_constant<int, N>{});
    else
      with_group_count<N - 1>(q, f);
  }
}

template <bool BUF, bool TR>
__global__ __launch_bounds__(512) void lo_pass1_kernel(int M, int64_t nw, const double* __restrict__ rows,
                                                       const int* __restrict__ rowidx,
                                                       const int* __restrict__ tile_orb,
                                                       const int* __restrict__ tile_row0,
                                                       const int* __restrict__ tile_nrows,
                                                       const int* __restrict__ blk, int nblk, int tmax,
                                                       const double2* __restrict__ theta, int64_t so,
                                                       int64_t sr, int64_t sw, double2* __restrict__ qbar,
                                                       int64_t orow, int64_t ow, int nwt, uint32_t rows_bytes,
                                                       uint32_t theta_bytes) {
  // two buffers as distinct objects (and the slab loop unrolled by two), so
  // the compiler sees that the reads of one buffer and the loads in flight
  // into the other cannot alias and does not wait for the loads before reading
  constexpr int NWV = 8;
  constexpr int QG = LO_QG;
  constexpr int TILE = LO_TILE_ROWS;
  constexpr int NT = 64 * NWV;
  __shared__ __attribute__((aligned(16))) double sA0[TILE * 16];   // swizzled [row][r]
  __shared__ __attribute__((aligned(16))) double sA1[TILE * 16];
  __shared__ __attribute__((aligned(16))) double2 sB0[16 * LO_WT];         // [r][walker]
  __shared__ __attribute__((aligned(16))) double2 sB1[16 * LO_WT];
  int t;
  int64_t w0;
  {
    const int xcd = blockIdx.x & 7;
    const int slot = blockIdx.x >> 3;
    const int64_t u = 8 * (int64_t)(slot / tmax) + xcd;
    if (u >= (int64_t)nblk * nwt) return;
    const int b = (int)(u / nwt);
    t = blk[b] + slot % tmax;
    if (t >= blk[b + 1]) return;
    w0 = (u % nwt) * LO_WT;
  }
  const int o = tile_orb[t];
  const int row0 = tile_row0[t];
  const int nrows = tile_nrows[t];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // this wave's groups: rows 4 (wv + NWV q) .. + 3 for q < qv
  const int ngroups = (nrows + 3) / 4;
  const int qv = ngroups > wv ? min(QG, (ngroups - wv + NWV - 1) / NWV) : 0;
  const double2* tho = theta + o * so;

  // A: TILE rows x 8 column pairs of 16-byte slots, three per thread: slot
  // S = NT k + tid holds row S / 8, column pair (S % 8) ^ (2 (row & 3))
  constexpr int A_LD = TILE * 8 / NT;   // 3
  const double* asrc[A_LD];
  uint32_t aoffs[A_LD];
#pragma unroll
  for (int k = 0; k < A_LD; ++k) {
    const int S = NT * k + tid;
    const int row = S >> 3;
    const int cp = (S & 7) ^ (2 * (row & 3));
    const int ar = rowidx[row0 + (row < nrows ? row : 0)];
    asrc[k] = rows + (size_t)ar * M + 2 * cp;
    aoffs[k] = (uint32_t)(((size_t)ar * M + 2 * cp) * sizeof(double));
  }
  // B: 16 x 32 slots, slot tid holds r = tid / 32, walker tid % 32, or with
  // TR walker tid / 16, r = (tid % 16) ^ (walker % 16) (walkers clamped to a
  // valid one)
  const int bwl = TR ? tid / 16 : tid % LO_WT;
  const int brl = TR ? (tid % 16) ^ (bwl & 15) : tid / LO_WT;
  const int64_t bw = w0 + bwl < nw ? w0 + bwl : nw - 1;
  const double2* bsrc = tho + brl * sr + bw * sw;
  const uint32_t boff = (uint32_t)((brl * sr + bw * sw) * sizeof(double2));
  // raw descriptors (stride 0, byte ranges rows_bytes and theta_bytes; the
  // third word is the gfx9 default data format); only used when BUF
  const __amdgpu_buffer_rsrc_t ares = __builtin_amdgcn_make_buffer_rsrc((void*)rows, 0, (int)rows_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t bres = __builtin_amdgcn_make_buffer_rsrc((void*)tho, 0, (int)theta_bytes, 0x00020000);
  auto issue = [&](int c, double* sa, double2* sb) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < A_LD; ++k) {
      auto* dst = (__attribute__((address_space(3))) void*)(sa + (NT * k + 64 * wv) * 2);
      if constexpr (BUF)
        // the slab offset goes in soffset (the instruction offset would also
        // move the LDS destination)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ares, dst, 16, (int)aoffs[k], 16 * c * (int)sizeof(double), 0, 0);
      else
        __builtin_amdgcn_global_load_lds((const void*)(asrc[k] + 16 * c), dst, 16, 0, 0);
    }
    auto* dst = (__attribute__((address_space(3))) void*)(sb + 64 * wv);
    if constexpr (BUF)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(bres, dst, 16, (int)boff, (int)(16 * c * sr * (int64_t)sizeof(double2)), 0,
                                               0);
    else
      __builtin_amdgcn_global_load_lds((const void*)(bsrc + 16 * c * sr), dst, 16, 0, 0);
  };

  // acc[q][c]: rows 4 (wv + NWV q) + lk, walker column c (block h = c / 2, part = c % 2)
  double acc[QG][4];
#pragma unroll
  for (int q = 0; q < QG; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = 0.0;
  // A operand of this lane: row 4 (wv + NWV q) + (lane & 3) (so row & 3 =
  // lane & 3), column 4 s4 + lk, i.e. column pair 2 s4 + (lk >> 1), element lk & 1
  const int e2 = 2 * (lane & 3);
  const int abase = (4 * wv + (lane & 3)) * 16 + (lk & 1);
  const int nchunk = M / 16;
  // NQ = qv, the wave-uniform group count, as a constant: one straight run
  // of MFMAs per count, no tests inside the slab.  The operands of K-step
  // s4 + 1 are read from LDS into a second register set before the products
  // of K-step s4 (scheduling barriers keep that order), so a product waits
  // only for reads issued a whole K-step earlier.
  auto compute = [&](const double* sa, const double2* sb, auto nqc) __attribute__((always_inline)) {
    constexpr int NQ = decltype(nqc)::value;
    double a[2][NQ];
    double2 b0[2], b1[2];
    auto read = [&](int s4, int slot) __attribute__((always_inline)) {
      const int rr = 4 * s4 + lk;
      if constexpr (TR) {
        b0[slot] = sb[lr * 16 + (rr ^ lr)];
        b1[slot] = sb[(16 + lr) * 16 + (rr ^ lr)];
      } else {
        b0[slot] = sb[rr * LO_WT + lr];
        b1[slot] = sb[rr * LO_WT + 16 + lr];
      }
      const int aoff = abase + 2 * (((2 * s4) ^ e2) | (lk >> 1));
#pragma unroll
      for (int q = 0; q < NQ; ++q) a[slot][q] = sa[aoff + 64 * NWV * q];
    };
    read(0, 0);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int u = s4 & 1;
      if (s4 < 3) read(s4 + 1, u ^ 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        acc[q][0] = mfma4(a[u][q], b0[u].x, acc[q][0]);
        acc[q][1] = mfma4(a[u][q], b0[u].y, acc[q][1]);
        acc[q][2] = mfma4(a[u][q], b1[u].x, acc[q][2]);
        acc[q][3] = mfma4(a[u][q], b1[u].y, acc[q][3]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto compute_wave = [&](const double* sa, const double2* sb) __attribute__((always_inline)) {
    with_group_count<QG>(qv, [&](auto nqc) __attribute__((always_inline)) { compute(sa, sb, nqc); });
  };
  issue(0, sA0, sB0);
  wait_vmcnt0();
  __syncthreads();
  for (int c = 0; c < nchunk; c += 2) {
    if (c + 1 < nchunk) issue(c + 1, sA1, sB1);
    compute_wave(sA0, sB0);
    wait_vmcnt0();
    __syncthreads();
    if (c + 1 < nchunk) {
      if (c + 2 < nchunk) issue(c + 2, sA0, sB0);
      compute_wave(sA1, sB1);
      wait_vmcnt0();
      __syncthreads();
    }
  }
  // lane holds rows 4 (wv + NWV q) + lk, walker 16h + lr
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t w = w0 + 16 * h + lr;
    if (w < nw) {
#pragma unroll
      for (int q = 0; q < QG; ++q) {
        const int lrow = 4 * (wv + NWV * q) + lk;
        if (q < qv && lrow < nrows)
          qbar[(size_t)(row0 + lrow) * orow + w * ow] = make_double2(acc[q][2 * h], acc[q][2 * h + 1]);
      }
    }
  }
}

const char* lo_pass1_name(int M) { return M % 16 == 0 ? "lo_pass1_kernel" : "lo_pass1_reg_kernel"; }
int lo_tile_rows() { return LO_TILE_ROWS; }
int lo_orbital_block() { return LO_OBLK; }


hipError_t launch_lo_pass1(hipStream_t s, int M, int n, int64_t nw, int ntiles, const double* rows,
                           int64_t rows_count, const int* rowidx, const int* tiles, const int* blk, int nblk,
                           int tmax, const double* theta, int theta_layout, double* qbar,
                           int64_t out_walker_stride) {
  if (nw <= 0 || ntiles <= 0) return hipSuccess;
  const int nwt = (int)((nw + LO_WT - 1) / LO_WT);
  const int64_t units = (int64_t)nblk * nwt;
  const int64_t grid = (int64_t)8 * ((units + 7) / 8) * tmax;
  const bool om = theta_layout == THETA_ORBITAL, tr = theta_layout == THETA_TRANSPOSED;
  const int64_t so = om ? (int64_t)M * nw : tr ? (int64_t)M : 1;
  const int64_t sr = om ? nw : tr ? 1 : n;
  const int64_t sw = om ? 1 : (int64_t)M * n;
  const int64_t orow_ = out_walker_stride ? (int64_t)1 : nw;
  const int64_t ow_ = out_walker_stride ? out_walker_stride : (int64_t)1;
  if (M % 16 != 0) {
    hipLaunchKernelGGL(lo_pass1_reg_kernel, dim3((unsigned)grid), dim3(512), 0, s, M, nw, rows, rowidx, tiles,
                       tiles + ntiles, tiles + 2 * ntiles, blk, nblk, tmax, (const double2*)theta, so, sr, sw,
                       (double2*)qbar, orow_, ow_, nwt);
    return hipGetLastError();
  }
  // byte ranges the buffer form addresses: all factor rows, and one orbital's
  // theta elements from its first (r = 0, w = 0) to its last
  const int64_t abytes = rows_count * M * (int64_t)sizeof(double);
  const int64_t bbytes = ((int64_t)(M - 1) * sr + (nw - 1) * sw + 1) * (int64_t)sizeof(double2);
  const int64_t lim = INT32_MAX;   // descriptor range and offsets are 32-bit (kept signed)
  const bool buf = abytes <= lim && bbytes <= lim;
  auto kern = tr ? (buf ? lo_pass1_kernel<true, true> : lo_pass1_kernel<false, true>)
                 : (buf ? lo_pass1_kernel<true, false> : lo_pass1_kernel<false, false>);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(512), 0, s, M, nw, rows, rowidx, tiles, tiles + ntiles, tiles + 2 * ntiles, blk, nblk, tmax,
                     (const double2*)theta, so, sr, sw, (double2*)qbar, orow_, ow_, nwt, (uint32_t)(buf ? abytes : 0),
                     (uint32_t)(buf ? bbytes : 0));
  return hipGetLastError();
}
// Pass 2: one thread per walker; the four waves of a workgroup take four
// consecutive chunks of LO_P2_CHUNK entries for the same 64 walkers and their
// sums are added in LDS in wave order, so each grid row writes one partial
// slot per walker for 4 LO_P2_CHUNK entries.  An entry is one rank row K of a
// stored pair with the output rows of QL_i, QR_j, QL_j, QR_i and the pair
// weight, so every chunk has the same fixed trip count and a wave issues the
// loads of all its entries at once (a loop over pairs of varying rank put one
// memory round trip per pair on the path).  The entry tables are read at
// wave-uniform indices (scalar loads).
constexpr int LO_P2_CHUNK = 8;
constexpr int LO_P2_WAVES = 4;

__global__ __launch_bounds__(256) void lo_pass2_kernel(int64_t nw, const int* __restrict__ ent, int64_t nent,
                                                       const double* __restrict__ entw,
                                                       const double2* __restrict__ qbar,
                                                       double* __restrict__ partial, int with_j) {
  __shared__ double4 sRed[LO_P2_WAVES][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t w = (int64_t)blockIdx.x * 64 + lane;
  const int64_t wl = w < nw ? w : nw - 1;     // every wave reaches the barrier
  const int64_t e0 = ((int64_t)blockIdx.y * LO_P2_WAVES + q) * LO_P2_CHUNK;
  double2 ql_i[LO_P2_CHUNK], qr_j[LO_P2_CHUNK], ql_j[LO_P2_CHUNK], qr_i[LO_P2_CHUNK];
#pragma unroll
  for (int e = 0; e < LO_P2_CHUNK; ++e) {
    ql_i[e] = qbar[(size_t)ent[e0 + e] * nw + wl];
    qr_j[e] = qbar[(size_t)ent[nent + e0 + e] * nw + wl];
    ql_j[e] = qbar[(size_t)ent[2 * nent + e0 + e] * nw + wl];
    qr_i[e] = qbar[(size_t)ent[3 * nent + e0 + e] * nw + wl];
  }
  double jr = 0.0, ji = 0.0, xr = 0.0, xi = 0.0;
#pragma unroll
  for (int e = 0; e < LO_P2_CHUNK; ++e) {
    const double wt = entw[e0 + e];
    jr += wt * (ql_i[e].x * qr_j[e].x - ql_i[e].y * qr_j[e].y);
    ji += wt * (ql_i[e].x * qr_j[e].y + ql_i[e].y * qr_j[e].x);
    xr += wt * (ql_j[e].x * qr_i[e].x - ql_j[e].y * qr_i[e].y);
    xi += wt * (ql_j[e].x * qr_i[e].y + ql_j[e].y * qr_i[e].x);
  }
  sRed[q][lane] = with_j ? make_double4(2.0 * jr, 2.0 * ji, -xr, -xi) : make_double4(0.0, 0.0, -xr, -xi);
  __syncthreads();
  if (q == 0 && w < nw) {
    double4 t = sRed[0][lane];
#pragma unroll
    for (int k = 1; k < LO_P2_WAVES; ++k) {
      const double4 u = sRed[k][lane];
      t.x += u.x;
      t.y += u.y;
      t.z += u.z;
      t.w += u.w;
    }
    reinterpret_cast<double4*>(partial)[(size_t)blockIdx.y * nw + w] = t;
  }
}

int lo_pass2_chunk() { return LO_P2_CHUNK * LO_P2_WAVES; }

hipError_t launch_lo_pass2(hipStream_t s, int64_t nw, int64_t nent, const int* ent, const double* entw,
                           const double* qbar, double* partial, int with_j) {
  if (nw <= 0 || nent <= 0) return hipSuccess;
  dim3 grid((unsigned)((nw + 63) / 64), (unsigned)(nent / (LO_P2_CHUNK * LO_P2_WAVES)));
  hipLaunchKernelGGL(lo_pass2_kernel, grid, dim3(64 * LO_P2_WAVES), 0, s, nw, ent, nent, entw,
                     (const double2*)qbar, partial, with_j);
  return hipGetLastError();
}

}  // namespace lofqmc
