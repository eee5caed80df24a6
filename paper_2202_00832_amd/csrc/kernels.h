// Host-callable launchers of the gfx950 kernels (internal to liblofqmc).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lofqmc {

// Optional per-kernel timing: when set, mark(ctx, name) is called on the host
// right before each kernel launch named `name` (it records a HIP event on the
// launch stream); mark(ctx, nullptr) closes the last interval.
struct ProfHook {
  void* ctx;
  void (*mark)(void* ctx, const char* name);
};
inline void prof_mark(const ProfHook* h, const char* name) {
  if (h && h->mark) h->mark(h->ctx, name);
}

// ---- per-walker path
// work: device workspace of green_theta_workspace(n, nw) bytes (the overlap
// matrices and their inverses in pivot order, then the pivot rows)
// The launch covers walkers w0 .. w0 + nwc - 1 of the nw addressed by the
// arrays (and by the workspace), so disjoint walker ranges can run on
// different streams.
size_t green_theta_workspace(int n, int64_t nw);
// Layouts of theta (complex, element (w, r, o): walker, basis index, orbital)
enum ThetaLayout {
  THETA_WALKER = 0,       // [nw][M][n]: theta_w row-major
  THETA_ORBITAL = 1,      // [n][M][nw]: walkers contiguous
  THETA_TRANSPOSED = 2    // [nw][n][M]: theta_w^T, the basis index contiguous
};
// flag_small: info = -k for the first pivot k below 2^-40 of the largest |re| + |im| of O
hipError_t launch_green_theta(hipStream_t s, int M, int n, int64_t nw, int64_t w0, int64_t nwc, const double* trial,
                              const double* phi, double* theta, double* logov, int* info, int theta_layout,
                              double* work, const ProfHook* prof, int flag_small);

int full_num_chunks(int64_t X, int64_t nw);
// passes of the FP64 full route at n orbitals (partial rows = passes x chunks)
int full_num_passes(int n);
hipError_t launch_energy_full(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* lbar,
                              const double* theta, double* partial, int nchunk);
// reduced-precision variant (precision LO_FP32 or LO_BF16X3): work is a device
// buffer of full_lp_workspace(...) bytes; partial holds nchunk + 1 chunk rows
// (the exchange chunks, then the Coulomb row)
size_t full_lp_workspace(int precision, int M, int n, int64_t X, int64_t nw);
hipError_t launch_energy_full_lp(hipStream_t s, int precision, int M, int n, int64_t X, int64_t nw,
                                 const double* lbar, const double* theta, void* work, double* partial, int nchunk,
                                 const ProfHook* prof);
hipError_t launch_reduce_partials(hipStream_t s, int64_t nw, int nchunk, const double* partial, const int* info,
                                  double* energy);

// tiles: device int [3][ntiles] (orbital, first output row, row count), tiles
// sorted by orbital; blk: device int [nblk + 1], first tile of each block of
// lo_orbital_block() orbitals; tmax: most tiles in one block.
// qbar: output row r of walker w at r * nw + w (walkers fastest), or, with a
// nonzero out_walker_stride, at w * out_walker_stride + r (rows fastest)
// tiles of at most lo_tile_rows() rows; rows_count: rows in `rows` (every
// rowidx entry is below it)
hipError_t launch_lo_pass1(hipStream_t s, int M, int n, int64_t nw, int ntiles, const double* rows,
                           int64_t rows_count, const int* rowidx, const int* tiles, const int* blk, int nblk,
                           int tmax, const double* theta, int theta_layout, double* qbar,
                           int64_t out_walker_stride);
// name of the pass-1 kernel launch_lo_pass1 runs for this M (direct-to-LDS
// staging when M is a multiple of 16, register staging otherwise)
const char* lo_pass1_name(int M);
int lo_tile_rows();
int lo_lp_tile_rows();
int lo_orbital_block();
// pass 2 over entries (one per rank row of a stored pair): ent [4][nent]
// output rows of QL_i, QR_j, QL_j, QR_i, entw [nent] the pair weights; nent a
// multiple of lo_pass2_chunk() (entries per partial slot),
// partial [nent / lo_pass2_chunk()][nw][4]
int lo_pass2_chunk();
// with_j = 0 leaves the Coulomb part of every partial at zero (exchange only)
hipError_t launch_lo_pass2(hipStream_t s, int64_t nw, int64_t nent, const int* ent, const double* entw,
                           const double* qbar, double* partial, int with_j);

// ---- reduced precision helpers (M padded to a multiple of 32, n to 16 NB)
int lp_padded_m(int M);
int lp_orbital_blocks(int n);   // NB = ceil(n / 16)
size_t lp_lbar_bytes(int precision, int M, int n, int64_t X);
size_t coulomb_cpart_bytes(int M, int n, int64_t X, int64_t nw);
// lbar and theta -> the padded reduced-precision copies lb, tb
hipError_t launch_lp_convert_operands(hipStream_t s, int precision, int M, int n, int64_t X, int64_t nw,
                                      const double* lbar, const double* theta, void* lb, void* tb);
// FP64 Coulomb sums: out_row[w] = (2 sum_g (Tr T_wg)^2, 0) as one partial row [nw][4]
hipError_t launch_coulomb_fp64(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* theta,
                               const double* lbar, void* cpart_ws, double* out_row, const ProfHook* prof);
// one system of a batched FP32 exchange launch; items [item0, item0 + ngrp * nchunk)
struct LpSys {
  int Mp, nb;
  int64_t X, nw, gchunk, nchunk, item0;
  const void* lb;
  const void* tb;
  double* partial;
};
// resets the item counter (a kernel, so the sequence can be captured in a
// graph) and runs the persistent kernel over all items with `grid` workgroups;
// nbmax (1..6): the largest nb of the systems, which selects the kernel
hipError_t launch_exchange_batched(hipStream_t s, int nsys, const LpSys* d_sys, int64_t nitems, unsigned* counter,
                                   int grid, int nbmax);
// theta [nw][M][n] complex -> FP32 [nw][Mp][NP] float2, or split BF16
// [nw][4][NP][Mp] (re_hi, re_lo, im_hi, im_lo); lp_theta_bytes gives the size
size_t lp_theta_bytes(int precision, int M, int n, int64_t nw);
hipError_t launch_lp_convert_theta(hipStream_t s, int precision, int M, int n, int64_t nw, const double* theta,
                                   void* out);
// factor rows [rows][M] -> FP32 [rows][Mp] and split BF16 [rows][2][Mp]
hipError_t launch_factor_rows_lp(hipStream_t s, int M, int64_t nrows, const double* rows, float* r32,
                                 __bf16* rbf);
// pass 1 of the LO route from the reduced-precision copies (tables as launch_lo_pass1)
hipError_t launch_lo_pass1_lp(hipStream_t s, int precision, int M, int n, int64_t nw, int ntiles,
                              const void* rows_lp, const int* rowidx, const int* tiles, const int* blk, int nblk,
                              int tmax, const void* theta_lp, double* qbar);

// ---- learned residual of the LO energy
int residual_nparam();
size_t residual_train_workspace(int64_t nw, int n);
size_t residual_predict_workspace(int bf16, int64_t nw, int n);
// orb: device float [n][2] (sum_j K_ij, sum_j discarded mass); grad: device
// double [M][n] (gradient of the dropped energy at the trial); x: [nw][n][4]
hipError_t launch_residual_features(hipStream_t s, int M, int n, int64_t nw, const double* theta, const float* orb,
                                    const double* grad, float* x);
// grad [M][n] = d(E_HR - E_LO)/d theta at theta = trial, from lbar [X][M][n],
// trial [M][n] and the stored factor rows (pair_of_row [total_rows][2],
// pair_off int64 [n][n], pair_k int [n][n] for a <= b); work of
// residual_gradient_workspace bytes
size_t residual_gradient_workspace(int n, int64_t X, int64_t total_rows);
// energies are complex [nw][2] (E_J, E_K); t, pred: double [nw]; out: complex [nw]
hipError_t launch_residual_target(hipStream_t s, int64_t nw, const double* e_exact, const double* e_lo, double shift,
                                  double scale, double* t);
hipError_t launch_residual_apply(hipStream_t s, int64_t nw, const double* energy, const double* pred, double scale,
                                 double shift, double* out);
hipError_t launch_residual_gradient(hipStream_t s, int M, int n, int64_t X, const double* lbar, const double* trial,
                                    int64_t total_rows, const double* rows, const int* pair_of_row,
                                    const int64_t* pair_off, const int* pair_k, void* work, double* grad);
hipError_t launch_residual_predict(hipStream_t s, int bf16, int64_t nw, int n, const float* params, const float* x,
                                   void* work, double* pred);
// step <= 0: gradient (and loss, predictions) only, no update
hipError_t launch_residual_train_step(hipStream_t s, int64_t nw, int n, float* params, float* m, float* v,
                                      int64_t step, float lr, const float* x, const double* target, void* work,
                                      float* grad_out, double* loss, double* pred);

// ---- half-rotated ERI route
// Y: device [npairs][M][M] (row-major pair blocks, i <= j); pairs: device int
// [npairs][2]; partial: device [npairs][nw][4] doubles, reduced by
// launch_reduce_partials with nchunk = npairs.
hipError_t launch_hr_energy(hipStream_t s, int M, int n, int64_t nw, int npairs, const double* Y, const int* pairs,
                            const double* theta, int orbital_major, double* partial);

// ---- multi-determinant LO energy
// Arguments of one evaluation: the pass-1 output qbar, rows fastest
// ([nw][n_out]), with T[v][o] = C_av[:, v] . theta_o at row tpos[o] + v; the
// determinant tables [ndet][hstride] (hstride >= NA = max(nao, nav); hole and
// particle indices relative to the active sets); the pair tables (own output
// rows of orbitals i, j or -1, first output row of the pair's rows in the
// active-column region, act_stride rows per active column).
struct MdArgs {
  int M, n, ncas, nao, nav, ndet, hstride, npairs;
  int64_t nw, act_stride, n_out;
  const int* tpos;
  const int* exc;
  const int* holes;
  const int* parts;
  const double* coef;
  const int* pi;
  const int* pj;
  const int* pK;
  const int64_t* offI;
  const int64_t* offJ;
  const int64_t* offA;
  const double* qbar;
};
int md_max_orbitals();
int md_max_active();
// per-walker device bytes of T, the moments and the contractions Y_o (work of
// launch_md_prep / launch_md_pairs is nw times this)
size_t md_walker_bytes(int na, int n, int ncas);
int md_pair_chunks(int npairs);
// prep: T, the determinant moments (into work) and ovr, device complex [nw]
// (sum_d c_d det(R_d)^2) or null; pairs: the weighted pair sums into partial
// [nchunk][nw][4], reduced by launch_reduce_partials
hipError_t launch_md_prep(hipStream_t s, const MdArgs& g, void* work, double* ovr);
hipError_t launch_md_pairs(hipStream_t s, const MdArgs& g, void* work, int nchunk, double* partial);

// ---- set-up
// C_b(m, c) = sum_k A_b(m, k) B_b(k, c), element (m, k) of A at a_base[b] + m * a_m + k * a_k, etc.
// bases: device int64 [batch][3] = (a_base, b_base, c_base).
hipError_t launch_gemm_setup(hipStream_t s, int Mr, int Nc, int K, const double* A, int64_t a_m, int64_t a_k,
                             const double* B, int64_t b_k, int64_t b_n, double* C, int64_t c_m, int64_t c_n,
                             const int64_t* bases, int batch);
// Foster-Boys localization of C [M][n] in place (D diagonal position
// operators pos [D][M], D n^2 <= boys_max_lds_doubles()); stats_dev [3]:
// functional before, after, sweeps run
int boys_max_lds_doubles();
size_t boys_workspace(int M, int n, int D);
hipError_t launch_boys(hipStream_t s, int M, int n, int D, const double* pos, double* C, int max_sweeps, double tol,
                       void* work, double* stats_dev);
// orthonormal basis of the columns of each M x L block (L <= 64), in place
hipError_t launch_orth(hipStream_t s, int M, int L, int nb, double* A, int64_t stride);
// lbar[g][r][i] -> lbarT[i][g][r]
hipError_t launch_lbar_transpose(hipStream_t s, int M, int n, int64_t X, const double* lbar, double* lbarT);
// pack truncated SVD factors of a batch of problems (K[b] <= kmax): U column-major
// M x kmax (ld M), VT kmax x M with leading dimension vt_ld, S per problem
hipError_t launch_pack_factors(hipStream_t s, int M, int nb, int kmax, const double* U, int64_t u_stride,
                               const double* VT, int vt_ld, int64_t vt_stride, const double* S, int64_t s_stride,
                               const int* K, const int64_t* row_off, double* rows);

}  // namespace lofqmc
