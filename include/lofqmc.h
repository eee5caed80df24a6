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

enum lo_status {
  LO_OK = 0,
  LO_EINVAL = -1,        /* bad argument (NULL, negative or inconsistent size, eps < 0 or NaN) */
  LO_ENOMEM = -2,        /* device or host allocation failed */
  LO_EHIP = -3,          /* a HIP runtime call failed */
  LO_EUNSUPPORTED = -4,  /* valid request outside what this build implements */
  LO_ESOLVER = -5        /* the dense SVD used while building LO factors failed */
};

/* Layout of theta (the Q matrices) produced by green_theta and read by the
 * energy calls.  Default: walker-major complex [nw][M][n_occ].  With
 * LO_THETA_ORBITAL_MAJOR: orbital-major complex [n_occ][M][nw] (walkers
 * contiguous), the layout the LO energy multiplies directly. */
enum lo_flags {
  LO_THETA_ORBITAL_MAJOR = 1u
};

enum lo_precision {
  LO_FP64 = 0,   /* FP64 contractions and FP64 sums */
  LO_FP32 = 1,   /* reserved: FP32 contractions, FP64 sums */
  LO_BF16X3 = 2  /* reserved: split-BF16 contractions, FP64 sums */
};

/* ---------------------------------------------------------------- context */

/* Creates a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream).  The context owns only small metadata and a device workspace that
 * grows on first use of a size and is reused afterwards.  No device work. */
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

/* -------------------------------------------------------- per-walker calls */

/* Green's-function intermediate Q of Eq. 15 ("theta"):
 *   O_w = trial^T phi_w (n_occ x n_occ), inverted by Gauss-Jordan elimination
 *   with partial pivoting, theta_w = phi_w O_w^{-1},
 *   log_ovlp[w] = log det O_w (one spin; imaginary part in (-pi, pi]).
 *   trial    : [M][n_occ] double (real)
 *   phi      : complex [nw][M][n_occ] walker determinants
 *   theta    : complex [nw][M][n_occ] (output), or [n_occ][M][nw] when flags
 *              holds LO_THETA_ORBITAL_MAJOR
 *   log_ovlp : complex [nw] (output; may be NULL)
 *   info     : int32 [nw] (output): 0, or k > 0 if the k-th pivot (1-based)
 *              of O_w is exactly zero; theta_w is then undefined and the
 *              energy calls return NaN for that walker.
 * Always FP64.  Supports n_occ <= 64. */
int green_theta(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t nw, const double* trial,
                const double* phi, double* theta, double* log_ovlp, int32_t* info, unsigned flags);

/* Two-body energy by the half-rotated Cholesky route (Sec. 2.2, Eq. 16):
 *   T_{wg} = Lbar_g^T theta_w (n_occ x n_occ, complex)
 *   E_J[w] = 2 sum_g (Tr T_{wg})^2,   E_K[w] = -sum_g Tr(T_{wg} T_{wg}).
 * The per-(w, g) matrix T is never written to memory.
 *   lbar   : [n_chol][M][n_occ] double
 *   theta  : complex [nw][M][n_occ] (walker-major)
 *   info   : int32 [nw] from green_theta, or NULL (all valid)
 *   energy : complex [nw][2] (output) = (E_J, E_K) per walker
 * precision must be LO_FP64; flags must be 0.  Supports n_occ <= 64. */
int local_energy_full(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, int64_t nw,
                      const double* lbar, const double* theta, const int32_t* info,
                      int precision, unsigned flags, double* energy);

/* Two-body energy by the LO route (Sec. 2.3.2, Eq. 22 with Eq. 23):
 *   for each ordered pair [ij]:  QL_i = Ubar^T Q_i, QR_j = Vbar Q_j,
 *   QL_j = Ubar^T Q_j, QR_i = Vbar Q_i (complex K_ij-vectors, bilinear),
 *   E_J = 2 sum_ij QL_i . QR_j,   E_K = -sum_ij QL_j . QR_i.
 *   factors : handle from build_lo_factors (shapes M, n_occ taken from it)
 *   theta   : complex [nw][M][n_occ], or [n_occ][M][nw] with flags
 *             LO_THETA_ORBITAL_MAJOR (the walker-major layout is transposed
 *             into the context workspace first)
 *   info    : int32 [nw] or NULL
 *   energy  : complex [nw][2] (output) = (E_J, E_K)
 * precision must be LO_FP64; flags may hold LO_THETA_ORBITAL_MAJOR only. */
int local_energy_lo(lo_ctx* ctx, const lo_factors* factors, int64_t nw, const double* theta,
                    const int32_t* info, int precision, unsigned flags, double* energy);

#ifdef __cplusplus
}
#endif

#endif /* LOFQMC_H */
