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
// work: device workspace of green_theta_workspace(n, nw) bytes (the overlap matrices)
size_t green_theta_workspace(int n, int64_t nw);
hipError_t launch_green_theta(hipStream_t s, int M, int n, int64_t nw, const double* trial, const double* phi,
                              double* theta, double* logov, int* info, int orbital_major, double* work,
                              const ProfHook* prof);

int full_num_chunks(int64_t X, int64_t nw);
hipError_t launch_energy_full(hipStream_t s, int M, int n, int64_t X, int64_t nw, const double* lbar,
                              const double* theta, double* partial, int nchunk);
hipError_t launch_reduce_partials(hipStream_t s, int64_t nw, int nchunk, const double* partial, const int* info,
                                  double* energy);

// tiles: device int [3][ntiles] (orbital, first output row, row count), tiles
// sorted by orbital; blk: device int [nblk + 1], first tile of each block of
// lo_orbital_block() orbitals; tmax: most tiles in one block.
hipError_t launch_lo_pass1(hipStream_t s, int M, int n, int64_t nw, int ntiles, const double* rows,
                           const int* rowidx, const int* tiles, const int* blk, int nblk, int tmax,
                           const double* theta, int orbital_major, double* qbar);
int lo_tile_rows();
int lo_orbital_block();
int lo_pass2_chunks(int npairs);
hipError_t launch_lo_pass2(hipStream_t s, int64_t nw, int npairs, int nchunk, const int* pK, const int64_t* offI,
                           const int64_t* offJ, const double* pw, const double* qbar, double* partial);

// ---- set-up
// C_b(m, c) = sum_k A_b(m, k) B_b(k, c), element (m, k) of A at a_base[b] + m * a_m + k * a_k, etc.
// bases: device int64 [batch][3] = (a_base, b_base, c_base).
hipError_t launch_gemm_setup(hipStream_t s, int Mr, int Nc, int K, const double* A, int64_t a_m, int64_t a_k,
                             const double* B, int64_t b_k, int64_t b_n, double* C, int64_t c_m, int64_t c_n,
                             const int64_t* bases, int batch);
// lbar[g][r][i] -> lbarT[i][g][r]
hipError_t launch_lbar_transpose(hipStream_t s, int M, int n, int64_t X, const double* lbar, double* lbarT);
// pack truncated SVD factors of a batch of column-major M x M problems
hipError_t launch_pack_factors(hipStream_t s, int M, int nb, const double* U, const double* VT, const double* S,
                               const int* K, const int64_t* row_off, double* rows);

}  // namespace lofqmc
