/*
 * lofqmc.h - C ABI of the MI355X (gfx950) library for the ph-AFQMC walker
 * two-body local energy with the localized-orbital (LO) compression of
 * Weber et al., "A Localized-Orbital Energy Evaluation for Auxiliary-Field
 * Quantum Monte Carlo" (arXiv 2202.00832).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Restricted closed shell: one spatial determinant per walker is used for
 *    both spins, so E2 carries the factors 4 (Coulomb) and 2 (exchange)
 *    inside the 1/2 of Eq. 19.  E_local here is the two-body energy
 *    E2 = E_J + E_K (the workloads define no one-body term).
 *  - All sizes are int64_t.  Arrays are row-major.  Complex numbers are
 *    complex128 stored interleaved as (re, im) pairs of double; a "complex
 *    [a][b]" array is therefore a double array of 2*a*b elements.
 *  - Unless a call says "host", array pointers are DEVICE pointers owned by the
 *    caller, and every call is asynchronous on the context's HIP stream.
 *  - Return value: LO_OK (0) or a negative LO_E* code; lo_last_error() then
 *    describes the failure.  Argument validation happens before any device
 *    work is queued, so a failed call has no side effects.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef LOFQMC_H
#define LOFQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lo_ctx lo_ctx;
typedef struct lo_factors lo_factors;
typedef struct lo_hr lo_hr;

enum lo_status {
  LO_OK = 0,
  LO_EINVAL = -1,        /* bad argument (NULL, negative or inconsistent size, eps < 0 or NaN) */
  LO_ENOMEM = -2,        /* device or host allocation failed */
  LO_EHIP = -3,          /* a HIP runtime call failed */
  LO_EUNSUPPORTED = -4,  /* valid request outside what this library implements */
  LO_ESOLVER = -5        /* the dense SVD used while building LO factors failed */
};

/* Layout of theta (the Q matrices) produced by green_theta and read by the
 * energy calls.  Default: walker-major complex [nw][M][n_occ].  With
 * LO_THETA_ORBITAL_MAJOR: orbital-major complex [n_occ][M][nw] (walkers
 * contiguous).  With LO_THETA_TRANSPOSED: each walker's theta transposed,
 * complex [nw][n_occ][M] (the basis index contiguous), the layout whose
 * orbital columns the LO energy's pass 1 loads in whole cache lines.  At
 * most one of the two layout flags. */
enum lo_flags {
  LO_THETA_ORBITAL_MAJOR = 1u,
  /* local_energy_lo: E_J from the FP64 Cholesky traces Tr(Lbar_g^T theta)
   * (Eq. 16, exact) instead of the LO pair sums; E_K stays LO.  Needs the
   * lbar argument and walker-major theta. */
  LO_EXACT_COULOMB = 2u,
  /* green_theta: report nearly singular overlaps as info < 0 (see there) */
  LO_FLAG_SMALL_PIVOT = 4u,
  LO_THETA_TRANSPOSED = 8u
};

/* Arithmetic of the energy contractions.  Reduced precision applies to the
 * exchange contraction T = Lbar_g^T theta of local_energy_full (the Coulomb
 * traces, the exchange sums and every sum over g stay FP64) and to the
 * projections QL = Ubar^T Q, QR = Vbar Q of local_energy_lo (the pair dot
 * products and all sums stay FP64).  green_theta is always FP64. */
enum lo_precision {
  LO_FP64 = 0,   /* FP64 everywhere */
  LO_FP32 = 1,   /* T from FP32-rounded operands on FP32 MFMA (FP32 accumulation) */
  LO_BF16X3 = 2, /* T from split BF16 operands x = x_hi + x_lo, products
                    hi*hi + hi*lo + lo*hi on BF16 MFMA (FP32 accumulation) */
  LO_BF16 = 3    /* plain BF16 operands, FP32 accumulation: only for
                    lo_residual_predict */
};

/* ---------------------------------------------------------------- context */

/* Creates a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream).  The context owns only small metadata and a device workspace that
 * grows on first use of a size and is reused afterwards.  No device work; on
 * a host with a GPU it also looks up, once per device, the address of the
 * fixed scratch of local_energy_lo_noalloc on the current device (LO_EHIP if
 * that fails). */
int lo_create(lo_ctx** ctx, void* hip_stream);

/* Re-binds the context to another stream (no synchronisation). */
int lo_set_stream(lo_ctx* ctx, void* hip_stream);

/* Blocks until all work queued on the context's stream has finished. */
int lo_synchronize(lo_ctx* ctx);

/* Frees the context and its workspace.  NULL is accepted. */
int lo_destroy(lo_ctx* ctx);

/* Last error message of this context (never NULL; "" after success). */
const char* lo_last_error(const lo_ctx* ctx);

/* Kernel timing (diagnostics, not part of the method).  While enabled, every
 * kernel that the per-walker calls launch is preceded by a HIP event recorded
 * on the context's stream, and each call ends with one more, so each kernel's
 * duration is measured on the stream it runs on (a few microseconds of
 * overhead per launch).  lo_profile_enable(ctx, 0 or 1) discards earlier
 * records and switches recording off or on.  Records accumulate until
 * lo_profile_summary, so call it every few thousand launches. */
int lo_profile_enable(lo_ctx* ctx, int enable);

/* Synchronises the context's stream and reports, per kernel name (sorted by
 * name), the number of launches and their summed duration in milliseconds
 * since the last enable or summary; then clears the sums.
 *   names    : host char[max_kernels][64], NUL-terminated kernel names
 *   launches : host int64[max_kernels]
 *   total_ms : host double[max_kernels]
 *   count    : receives the number of distinct kernels (entries beyond
 *              max_kernels are not written). */
int lo_profile_summary(lo_ctx* ctx, int max_kernels, char* names, int64_t* launches, double* total_ms,
                       int* count);

/* ------------------------------------------------------------- set-up calls */

/* Half-rotated Cholesky vectors (Sec. 2.2, the definition below Eq. 15):
 *   lbar[g][r][i] = sum_p chol[g][r][p] * trial[p][i]
 * i.e. Lbar^g_{ri} with the trial contracted into the second index of the
 * (symmetric) Cholesky matrix L^g, where V_pqrs = (pr|qs) =
 * sum_g L^g_pr L^g_qs.  The trial is real, so conjugation is immaterial.
 *   chol  : [n_chol][M][M] double
 *   trial : [M][n_occ]     double, orthonormal columns (already localized
 *                          if the LO route will be used)
 *   lbar  : [n_chol][M][n_occ] double (output)
 * Cost n_chol*M^2*n_occ; run once per system. */
int build_half_rotated_chol(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol,
                            const double* chol, const double* trial, double* lbar);

/* LO factors (Sec. 2.3.1, Eq. 18).  For every occupied pair i <= j the block
 *   Y^[ij]_{rs} = sum_g Lbar^g_{ri} Lbar^g_{sj}            (M x M)
 * is decomposed Y = U Sigma V; singular values sigma_K >= epsilon are kept
 * (epsilon == 0 keeps all M), and Ubar = U Sigma^(1/2), Vbar = Sigma^(1/2) V.
 * Pairs j < i are never stored: Y^[ji] = (Y^[ij])^T, whose factors are
 * (Vbar^T, Ubar^T), so the energy calls use the stored block for both orders.
 * epsilon is an absolute threshold in Hartree on singular values.
 *   lbar    : [n_chol][M][n_occ] double (device, from build_half_rotated_chol)
 *   out     : receives a library-owned handle (device storage), released by
 *             lo_factors_destroy.
 * Synchronous: returns after the factors are on the device.  The SVD is
 * computed with rocSOLVER (a set-up step; not on the per-walker path). */
int build_lo_factors(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol,
                     const double* lbar, double epsilon, lo_factors** out);

/* LO factors from a randomized SVD of every pair block (the approximate
 * decomposition Sec. 2.3.1 mentions as a cheaper set-up): randomized subspace
 * iteration (Halko, Martinsson and Tropp, SIAM Rev. 53 (2011), Alg. 4.4),
 *   Z = Y Omega, then power_iters times Q = orth(Z), Q' = orth(Y^T Q),
 *   Z = Y Q'; Q = orth(Z); B = Q^T Y = U_B Sigma V; U = Q U_B,
 * with orth a classical Gram-Schmidt repeated on each column until a pass
 * keeps at least half of its norm (two to eight passes); a column that falls
 * to 1e-12 of its norm (a rank-deficient sketch) is replaced by a unit vector
 * (e_k, then e_k+1, ... while they too fall in the span) and orthogonalised.
 * Singular values of B with sigma >= epsilon are kept as in build_lo_factors;
 * the set-up costs O(M^2 sketch) per pair instead of O(M^3).
 *   sketch      : columns of the test matrix, 1 <= sketch <= min(M, 64); if every one of
 *                 the sketch singular values of some pair reaches epsilon the
 *                 call fails with LO_EUNSUPPORTED (a larger sketch is needed)
 *   power_iters : 0..16
 *   omega       : [M][sketch] double (device, row-major), the random test
 *                 matrix (the caller draws it, e.g. standard normal)
 *   epsilon     : > 0
 * The discarded mass reported for a pair sums only the discarded singular
 * values the sketch resolves.  Other arguments and the handle as for
 * build_lo_factors. */
int build_lo_factors_randomized(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar,
                                double epsilon, int64_t sketch, int power_iters, const double* omega,
                                lo_factors** out);

int lo_factors_destroy(lo_factors* f);

/* Host-side description of a handle.  Any output pointer may be NULL.
 *   ranks        : host int32 [n_occ][n_occ], M_SVD^[ij] (symmetric)
 *   first_dropped: host double [n_occ][n_occ], largest discarded singular
 *                  value of Y^[ij] (0 if none was discarded)
 *   total_rows   : number of stored factor rows (sum over i<=j of 2 K_ij)
 *   bytes        : device bytes held by the factor rows */
int lo_factors_info(const lo_factors* f, int64_t* M, int64_t* n_occ, int32_t* ranks,
                    double* first_dropped, int64_t* total_rows, int64_t* bytes);

/* Copies the stored factors to host memory for inspection:
 *   rows      : host double [total_rows][M]; for pair (i <= j) with rank K
 *               the block starting at row_offset[i*n_occ+j] holds K rows of
 *               Ubar^T followed by K rows of Vbar.
 *   row_offset: host int64 [n_occ][n_occ] (-1 for i > j).
 * Synchronous. */
int lo_factors_export(const lo_factors* f, double* rows, int64_t* row_offset);

/* Kind of a factor set, for lo_factors_import: flags = 0 for factors of the
 * exact SVD (build_lo_factors), LO_FACTORS_RANDOMIZED for the randomized
 * set-up (its diagonal-pair Vbar rows are kept apart from Ubar^T). */
#define LO_FACTORS_RANDOMIZED 1u
int lo_factors_flags(const lo_factors* f, unsigned* flags);

/* Rebuilds a factor handle from what lo_factors_info, lo_factors_discarded,
 * lo_factors_export and lo_factors_flags return (a checkpoint of the set-up,
 * Sec. 2.3.1: the SVDs need not be repeated).
 *   M, n_occ, n_chol : shapes of the set the factors were built from
 *   ranks            : host int32 [n_occ][n_occ], symmetric, 0..M
 *   row_offset       : host int64 [n_occ][n_occ]; the pairs i <= j with K > 0
 *                      must tile rows 0 .. sum 2 K - 1 (entries i > j ignored)
 *   first_dropped, discarded : host double [n_occ][n_occ] or NULL (zeros)
 *   rows             : host double [total_rows][M] as lo_factors_export
 *   flags            : lo_factors_flags of the exported handle
 * The handle computes the same energies, bit for bit, as the exported one.
 * Synchronous; library-owned like build_lo_factors' handles. */
int lo_factors_import(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const int32_t* ranks,
                      const int64_t* row_offset, const double* first_dropped, const double* discarded,
                      const double* rows, unsigned flags, lo_factors** out);

/* -------------------------------------------------------- per-walker calls */

/* Green's-function intermediate Q of Eq. 15 ("theta"):
 *   O_w = trial^T phi_w (n_occ x n_occ), inverted by Gauss-Jordan elimination
 *   with partial pivoting, theta_w = phi_w O_w^{-1},
 *   log_ovlp[w] = log det O_w (one spin; imaginary part in (-pi, pi]).
 *   trial    : [M][n_occ] double (real)
 *   phi      : complex [nw][M][n_occ] walker determinants
 *   theta    : complex [nw][M][n_occ] (output), or [n_occ][M][nw] when flags
 *              holds LO_THETA_ORBITAL_MAJOR, or [nw][n_occ][M] with
 *              LO_THETA_TRANSPOSED (the same values in each layout)
 *   log_ovlp : complex [nw] (output; may be NULL)
 *   info     : int32 [nw] (output): 0, or k > 0 if the k-th pivot (1-based)
 *              of O_w is exactly zero; theta_w is then undefined and the
 *              energy calls return NaN for that walker.  With flags holding
 *              LO_FLAG_SMALL_PIVOT also -k < 0 if, with no zero pivot, the
 *              k-th pivot is the first whose |re| + |im| lies below 2^-40 of
 *              the largest |re| + |im| of O_w's entries (a nearly singular
 *              overlap): a warning only, theta_w and the energies are still
 *              computed (and large).
 * Always FP64.  Supports n_occ <= 112.  flags: LO_THETA_ORBITAL_MAJOR or
 * LO_THETA_TRANSPOSED, LO_FLAG_SMALL_PIVOT. */
int green_theta(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t nw, const double* trial,
                const double* phi, double* theta, double* log_ovlp, int32_t* info, unsigned flags);

/* Two-body energy by the half-rotated Cholesky route (Sec. 2.2, Eq. 16):
 *   T_{wg} = Lbar_g^T theta_w (n_occ x n_occ, complex)
 *   E_J[w] = 2 sum_g (Tr T_{wg})^2,   E_K[w] = -sum_g Tr(T_{wg} T_{wg}).
 * The per-(w, g) matrix T is never written to memory.
 *   lbar      : [n_chol][M][n_occ] double
 *   theta     : complex [nw][M][n_occ] (walker-major)
 *   info      : int32 [nw] from green_theta, or NULL (all valid)
 *   precision : LO_FP64, LO_FP32 or LO_BF16X3 (enum lo_precision); the
 *               reduced ones first rewrite lbar and theta into a padded
 *               FP32 or split-BF16 copy in the context workspace and support
 *               nw <= 65535 and n_chol <= 65535
 *   energy    : complex [nw][2] (output) = (E_J, E_K) per walker
 * flags must be 0 (a theta layout flag gives LO_EUNSUPPORTED, any other bit
 * LO_EINVAL).  Supports n_occ <= 112 (LO_FP64), <= 96 (LO_FP32) or <= 64
 * (LO_BF16X3). */
int local_energy_full(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, int64_t nw,
                      const double* lbar, const double* theta, const int32_t* info,
                      int precision, unsigned flags, double* energy);

/* Two-body energy by the LO route (Sec. 2.3.2, Eq. 22 with Eq. 23):
 *   for each ordered pair [ij]:  QL_i = Ubar^T Q_i, QR_j = Vbar Q_j,
 *   QL_j = Ubar^T Q_j, QR_i = Vbar Q_i (complex K_ij-vectors, bilinear),
 *   E_J = 2 sum_ij QL_i . QR_j,   E_K = -sum_ij QL_j . QR_i.
 *   factors : handle from build_lo_factors (shapes M, n_occ taken from it)
 *   theta   : complex [nw][M][n_occ], or [n_occ][M][nw] with flags
 *             LO_THETA_ORBITAL_MAJOR, or [nw][n_occ][M] with
 *             LO_THETA_TRANSPOSED (all are read in place; the transposed one
 *             is the fastest to read at M a multiple of 16)
 *   info    : int32 [nw] or NULL
 *   lbar    : NULL, or with LO_EXACT_COULOMB the [n_chol][M][n_occ] vectors
 *             the factors were built from (E_J then comes from their traces)
 *   energy  : complex [nw][2] (output) = (E_J, E_K)
 * precision: LO_FP64, LO_FP32 or LO_BF16X3 (enum lo_precision); the reduced
 * ones need [nw][M][n_occ] theta (LO_EUNSUPPORTED otherwise), nw <= 65535 and
 * n_occ <= 96 (LO_FP32) or <= 64 (LO_BF16X3),
 * and rewrite theta into a padded FP32 or split-BF16 copy in the context
 * workspace first.  flags may hold one of LO_THETA_ORBITAL_MAJOR,
 * LO_THETA_TRANSPOSED and LO_EXACT_COULOMB. */
int local_energy_lo(lo_ctx* ctx, const lo_factors* factors, int64_t nw, const double* theta,
                    const int32_t* info, int precision, unsigned flags, const double* lbar, double* energy);

/* local_energy_lo without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results as local_energy_lo;
 * the intermediates live in a fixed scratch array of LO_NOALLOC_SCRATCH_BYTES
 * (128 MiB) that every GPU the library runs on holds until the process ends,
 * instead of the context workspace.  A call needs
 *   16 nw n_out_rows + 32 nw n_chunks (+ the reduced-precision theta copy,
 *   + the Cholesky-trace partials of LO_EXACT_COULOMB)
 * bytes, each part rounded up to 256 (n_out_rows is the orbital-grouped row
 * count of the factors, about 11 k at M = 400, n_occ = 60, eps = 1e-5, so
 * about 700 walkers fit per call); a larger call returns LO_EUNSUPPORTED
 * before any device work.  All calls on one GPU share that GPU's array:
 * calls that overlap on one GPU (several streams or contexts, or several
 * host threads) race, so serialise them.  The kernels write every scratch
 * byte they read within the call, so no clearing is needed. */
#define LO_NOALLOC_SCRATCH_BYTES (128ull << 20)
int local_energy_lo_noalloc(lo_ctx* ctx, const lo_factors* factors, int64_t nw, const double* theta,
                            const int32_t* info, int precision, unsigned flags, const double* lbar, double* energy);

/* ------------------------------------------------ localization (set-up)
 *
 * Foster-Boys localization of the occupied trial orbitals (Sec. 3: the
 * orbitals are localized before the pair blocks are compressed, so that each
 * pair block has low numerical rank).  Maximises
 *   B = sum_i sum_d (C[:, i]^T diag(x_d) C[:, i])^2
 * over orthogonal rotations of the columns by Jacobi sweeps: pairs i < j in
 * row order, each rotated by the angle that maximises its part of B
 * (4t = atan2(2 sum_d c_d h_d, sum_d (h_d^2 - c_d^2)), h_d half the difference
 * of the two centroids, c_d the cross term), until a sweep raises B by at
 * most tol * B or max_sweeps sweeps have run.
 *   positions : device double [n_pos][M], the diagonal of each position
 *               operator in the basis (n_pos <= 3; the chain: x = p)
 *   orbitals  : device double [M][n_occ], orthonormal columns; replaced by
 *               the localized orbitals (same span)
 *   stats     : host double [3] or NULL: B before, B after, sweeps run
 * Requires n_pos * n_occ^2 <= 15360 (the rotated matrices stay in LDS: up to
 * 112 orbitals with one position operator, 71 with three).  Synchronous. */
int lo_localize_boys(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_pos, const double* positions, double* orbitals,
                     int max_sweeps, double tol, double* stats);

/* ------------------------------------------------ half-rotated ERI route
 *
 * The route the LO compression approximates (Sec. 2.2, Eq. 17): the pair
 * blocks
 *   Y^[ij]_{rs} = sum_g Lbar^g_{ri} Lbar^g_{sj}       (M x M, i <= j)
 * are stored whole (n_occ (n_occ + 1) / 2 * M^2 doubles: 2.3 GB at M = 400,
 * n_occ = 60), and per walker
 *   E_J = 2 sum_ij Q_i^T Y^[ij] Q_j,   E_K = -sum_ij Q_j^T Y^[ij] Q_i
 * (complex, bilinear); Y^[ji] = (Y^[ij])^T, so the pairs i < j count twice. */

/* Builds the pair blocks on the device (library-owned handle, released by
 * lo_hr_destroy; LO_ENOMEM when they do not fit).  lbar as for
 * build_lo_factors.  Synchronous. */
int build_hr_eri(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar, lo_hr** out);

int lo_hr_destroy(lo_hr* h);

/* Any output pointer may be NULL; bytes = device bytes of the pair blocks. */
int lo_hr_info(const lo_hr* h, int64_t* M, int64_t* n_occ, int64_t* bytes);

/* Energy by Eq. 17, FP64.
 *   h      : handle from build_hr_eri (shapes M, n_occ taken from it)
 *   theta  : complex [nw][M][n_occ], or [n_occ][M][nw] with flags
 *            LO_THETA_ORBITAL_MAJOR
 *   info   : int32 [nw] or NULL (walkers with info > 0 get NaN)
 *   energy : complex [nw][2] (output) = (E_J, E_K)
 * flags may hold LO_THETA_ORBITAL_MAJOR only.  The kernel reads theta columns
 * of 32 walkers, contiguous in the orbital-major layout, which is about twice
 * as fast here as walker-major.  Partial sums of npairs x nw x 32 bytes live in
 * the context workspace. */
int local_energy_hr(lo_ctx* ctx, const lo_hr* h, int64_t nw, const double* theta, const int32_t* info,
                    unsigned flags, double* energy);

/* ---------------------------------------- multi-determinant (CAS) trials
 *
 * Trial psi_T = sum_d c_d |Phi_d> (Sec. 2.1.1, Eq. 12) over the orbitals
 * C (M x n_cas) of an LO factor handle built from lbar of all n_cas orbitals:
 * the reference determinant Phi_0 holds columns 0 .. n_occ-1, of which the
 * last n_act_occ are active; columns n_occ .. n_cas-1 are the active virtual
 * orbitals.  Determinant d replaces the reference columns holes[d][m] by the
 * orbitals particles[d][m] (m < n_exc[d]), in place, hole m by particle m.
 * Every determinant is doubly occupied with the same spatial orbitals for
 * both spins (closed shell), so <Phi_d|phi> = det(Phi_d^T phi)^2.
 *
 * local_energy_md evaluates the LO energy of Eq. 19 with the weights of
 * Eq. 12 by the Sherman-Morrison-Woodbury update of Eq. 20-21: from the
 * reference theta = phi (Phi_0^T phi)^{-1} (green_theta with Phi_0) and
 * T = C_av^T theta, determinant d has det(Phi_d^T phi) / det(Phi_0^T phi) =
 * det R_d with R_d = T[particles, holes], and the per-determinant four
 * vectors of Eq. 22-23 are combinations of the projections of theta's own
 * and active columns.  The weighted sum over determinants is formed once per
 * walker (two moments of the R_d^{-1}), so the per-pair cost does not grow
 * with n_det.  A determinant whose R_d is exactly singular has weight zero.
 *
 * build_md_trial:
 *   f          : LO factors of all n_cas orbitals (f->n_occ = n_cas); the
 *                handle keeps its own copy of the factor rows and tables, so
 *                f may be destroyed once this call returns
 *   n_occ      : occupied orbitals per determinant, 1 <= n_occ <= min(n_cas, 112)
 *   n_act_occ  : 1..min(6, n_occ); n_cas - n_occ <= 6; n_cas <= 128
 *   orbitals   : [M][n_cas] double (device), the orbitals C; only the active
 *                virtual columns are copied into the handle
 *   n_det      : 1..2^20;  max_exc: 0..min(n_act_occ, n_cas - n_occ)
 *   n_exc      : host int32 [n_det], 0..max_exc
 *   holes      : host int32 [n_det][max_exc], reference columns in
 *                [n_occ - n_act_occ, n_occ), distinct within a determinant
 *   particles  : host int32 [n_det][max_exc], orbitals in [n_occ, n_cas), distinct
 *   coeffs     : host double [n_det], the CI coefficients c_d (real)
 *   out        : receives a library-owned handle, released by lo_md_destroy
 * Synchronous.  LO_EINVAL for indices or sizes out of range. */
typedef struct lo_md lo_md;
int build_md_trial(lo_ctx* ctx, const lo_factors* f, int64_t n_occ, int64_t n_act_occ, const double* orbitals,
                   int64_t n_det, int64_t max_exc, const int32_t* n_exc, const int32_t* holes,
                   const int32_t* particles, const double* coeffs, lo_md** out);

int lo_md_destroy(lo_md* md);

/* Host-side description; any output may be NULL.  out_rows: pass-1 output
 * rows per walker (the workspace of local_energy_md holds out_rows x nw
 * complex values). */
int lo_md_info(const lo_md* md, int64_t* n_occ, int64_t* n_cas, int64_t* n_det, int64_t* npairs,
               int64_t* out_rows);

/* Multi-determinant LO two-body energy per walker.
 *   theta      : from green_theta with the reference determinant Phi_0
 *                ([M][n_occ] columns 0 .. n_occ-1 of the orbitals), layout
 *                as flags says
 *   info       : from that green_theta call, or NULL; walkers with info > 0
 *                get NaN energies
 *   energy     : complex [nw][2], (E_J, E_K) of E2 = sum_d w_d E2^d,
 *                w_d = c_d det(R_d)^2 / sum_d' c_d' det(R_d')^2
 *   ovlp_ratio : complex [nw] or NULL: sum_d c_d det(R_d)^2, i.e.
 *                <psi_T|phi> / det(Phi_0^T phi)^2 (zero gives NaN energies)
 * nw <= 2^24 (one workgroup per walker), else LO_EUNSUPPORTED.
 * The context workspace grows to out_rows x nw complex values plus
 * nw x (NA n_occ + NA^2 + NA^4) complex values, NA = max(n_act_occ, n_cas - n_occ),
 * plus the partial sums. */
int local_energy_md(lo_ctx* ctx, const lo_md* md, int64_t nw, const double* theta, const int32_t* info,
                    unsigned flags, double* energy, double* ovlp_ratio);

/* --------------------------------------------------- several systems at once
 *
 * Full-route energies (Eq. 16) of several systems of different size in one
 * pass, FP32 exchange contraction with FP64 Coulomb sums and FP64 reductions
 * (the LO_FP32 arithmetic of local_energy_full).  The exchange work of all
 * systems forms one list of items (4 walkers x a chunk of Cholesky vectors of
 * one system) that ONE persistent kernel launch works through; per system
 * there are the operand rewrite, the Coulomb sums and the reduction.  A
 * system that gives its trial and walkers (trial, phi) also has its theta
 * and info formed by green_theta (Eq. 11, 14, 15; FP64) at the start of every
 * evaluation, so an evaluation (and a captured graph of evaluations) goes
 * from the walkers to the energies. */
typedef struct lo_system {
  int64_t M, n_occ, n_chol, nw;
  const double* lbar;    /* device [n_chol][M][n_occ] */
  double* theta;         /* device complex [nw][M][n_occ] (walker-major): input,
                            or output when phi is given */
  int32_t* info;         /* device int32 [nw] or NULL: input, or output
                            (required) when phi is given */
  double* energy;        /* device complex [nw][2] (output) = (E_J, E_K) */
  const double* trial;   /* NULL, or device [M][n_occ] (real, orthonormal) */
  const double* phi;     /* NULL, or device complex [nw][M][n_occ] walkers */
} lo_system;

typedef struct lo_batch lo_batch;

/* Plans an evaluation of nsys systems (host array; the device arrays it
 * points to must stay valid while the plan is used; their contents may
 * change between evaluations).  chunk: optional host int64 [nsys], the
 * Cholesky vectors per work item of each system (the tile shape; <= 0 or a
 * NULL array picks a size that makes items of all systems cost about the
 * same).  precision must be LO_FP32; each system needs n_occ <= 96,
 * nw <= 65535, n_chol <= 65535, and trial and phi both or neither (with
 * them, info non-NULL).  Allocates every device buffer the evaluations need
 * (also green_theta's workspace), so lo_batch_execute allocates nothing. */
int lo_batch_create(lo_ctx* ctx, int nsys, const lo_system* sys, int precision, const int64_t* chunk,
                    lo_batch** out);
int lo_batch_destroy(lo_batch* b);

/* Work items and the chosen chunk per system (host int64 [nsys], may be NULL). */
int lo_batch_info(const lo_batch* b, int64_t* nitems, int64_t* chunk);

/* Enqueues one evaluation of every system on the context stream. */
int lo_batch_execute(lo_ctx* ctx, lo_batch* b);

/* Records `repeats` consecutive evaluations into a HIP graph (captured on a
 * stream of the plan) and instantiates it; lo_batch_replay launches it on
 * the context stream.  Capturing again replaces the graph. */
int lo_batch_capture(lo_ctx* ctx, lo_batch* b, int repeats);
int lo_batch_replay(lo_ctx* ctx, lo_batch* b);

/* ------------------------------------------------ learned residual (extension)
 *
 * Not part of the paper's method: a small network that predicts, per walker,
 * the energy that the LO truncation drops, Re(E_full - E_LO) ~ sum_i f(x_i),
 * from per-orbital features of occupied orbital i of a walker:
 *   x_i = (sum_j K_ij, sum_j m_ij, ||theta[:, i]||_2, Re(g_i . theta[:, i]))
 * with K_ij the retained rank and m_ij the sum of the discarded singular
 * values of pair block Y^[ij] (Sec. 2.3.1), and g_i the gradient of the
 * dropped energy E_HR - E_LO (Eq. 17 minus Eq. 22) with respect to column i
 * of theta at the trial, theta = Psi (lo_residual_prepare).  The first three
 * are the same for walkers whose columns have equal norms; the fourth is the
 * first-order change of the dropped energy along the walker's own deviation
 * from the trial.  f is 4 -> 128 -> 128 -> 1 with
 * tanh activations on standardised inputs z = (x - shift) * scale; the
 * parameters are one device float vector of lo_residual_nparam() entries:
 *   W1[128][4], b1[128], W2[128][128], b2[128], w3[128], b3, shift[4], scale[4]
 * (shift and scale are set by the caller and never trained).  All arrays are
 * device pointers; every call except lo_residual_prepare is asynchronous on
 * the context stream. */
int lo_residual_nparam(void);

/* Sum of the discarded singular values of every pair block, host double
 * [n_occ][n_occ] (symmetric). */
int lo_factors_discarded(const lo_factors* f, double* mass);

/* Set-up of the fourth feature: forms, in FP64 on the device and stored with
 * the factors, g[r][i] = d(E_HR - E_LO)/d theta[r][i] at theta = trial, from
 *   lbar  : [n_chol][M][n_occ] double, the vectors the factors were built from
 *   trial : [M][n_occ] double, the trial they were half-rotated with
 * (shapes M, n_occ taken from the factors); grad_out (device double
 * [M][n_occ]) receives a copy, or NULL.  Synchronous.  Must precede
 * lo_residual_features (LO_EINVAL otherwise). */
int lo_residual_prepare(lo_ctx* ctx, lo_factors* f, int64_t n_chol, const double* lbar, const double* trial,
                        double* grad_out);

/* Training target in mHa, standardised:
 *   t[w] = (1000 Re(E_J + E_K of e_exact[w] - E_J - E_K of e_lo[w]) - shift) / scale
 * e_exact, e_lo: complex [nw][2] (E_J, E_K) from an exact route and from
 * local_energy_lo for the same walkers; t: double [nw] (output).  scale must
 * be finite and non-zero. */
int lo_residual_target(lo_ctx* ctx, int64_t nw, const double* e_exact, const double* e_lo, double shift, double scale,
                       double* t);

/* Walker energy with the learned correction:
 *   out[w] = E_J + E_K + (pred[w] * scale + shift) / 1000   (the correction on the real part)
 * energy: complex [nw][2] (E_J, E_K); pred: double [nw] from
 * lo_residual_predict, whose network works on targets standardised by
 * (shift, scale) mHa, or NULL for the plain sum E_J + E_K; out: complex [nw]. */
int lo_residual_apply(lo_ctx* ctx, int64_t nw, const double* energy, const double* pred, double scale, double shift,
                      double* out);

/* x : float [nw][n_occ][4] (output), theta : complex [nw][M][n_occ]. */
int lo_residual_features(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, float* x);

/* pred[w] = sum_i f(x_wi) (double [nw], output).  precision LO_FP32 (FP32
 * throughout) or LO_BF16 (the 128 x 128 layer on BF16 MFMA from BF16-rounded
 * activations and weights, FP32 accumulation; the other layers FP32). */
int lo_residual_predict(lo_ctx* ctx, int64_t nw, int64_t n_occ, const float* params, const float* x,
                        int precision, double* pred);

/* One training step on the loss L = mean_w (sum_i f(x_wi) - target_w)^2:
 * FP32 forward and hand-written backward pass, gradients summed over rows in
 * a fixed order, then (step >= 1) one Adam update (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias correction with this step number) of params, adam_m,
 * adam_v (float [nparam] each, zero before the first step).  step == 0 only
 * evaluates.  grad (float [nparam]), loss (double [1]) and pred (double [nw])
 * are optional outputs (NULL to skip); grad and loss belong to the parameters
 * before the update. */
int lo_residual_train_step(lo_ctx* ctx, int64_t nw, int64_t n_occ, float* params, float* adam_m, float* adam_v,
                           int64_t step, double lr, const float* x, const double* target, float* grad, double* loss,
                           double* pred);

#ifdef __cplusplus
}
#endif

#endif /* LOFQMC_H */
