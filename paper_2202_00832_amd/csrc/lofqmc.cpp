// Host side of liblofqmc: argument validation, workspace, set-up of the LO
// factors (pair blocks, rocSOLVER SVD, truncation, packing, pass tables) and
// dispatch of the per-walker kernels.  See include/lofqmc.h for the contract.
#include "lofqmc.h"

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

struct lo_ctx {
  hipStream_t stream = nullptr;
  std::string err;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  rocblas_handle blas = nullptr;
  // kernel timing (lo_profile_*): events recorded before each launch, in order
  bool prof_on = false;
  std::vector<std::pair<const char*, hipEvent_t>> prof_marks;
  std::vector<hipEvent_t> prof_pool;
  std::map<std::string, std::pair<int64_t, double>> prof_acc;   // name -> (launches, ms)
};

struct lo_factors {
  int64_t M = 0, n = 0, X = 0, total_rows = 0, n_out_rows = 0;   // X: Cholesky vectors the factors came from
  double* rows = nullptr;  // device [total_rows][M]
  float* rows32 = nullptr;   // device [total_rows][Mp] (reduced-precision copies, M padded to Mp)
  __bf16* rowsbf = nullptr;  // device [total_rows][2][Mp] (hi, lo)
  std::vector<int32_t> ranks;          // [n][n]
  std::vector<double> first_dropped;   // [n][n]
  std::vector<double> discarded;       // [n][n], sum of the discarded singular values
  std::vector<int64_t> row_offset;     // [n][n], -1 for i > j
  int ntiles = 0, npairs = 0, nblk = 0, tmax = 0;
  int ntiles_lp = 0, nblk_lp = 0, tmax_lp = 0;
  int* d_rowidx = nullptr;             // [n_out_rows]
  int* d_tiles = nullptr;              // [3][ntiles]: orbital, first output row, row count;
                                       // then [nblk + 1]: first tile of each orbital block
  int* d_tiles_lp = nullptr;           // the same for the reduced-precision pass (smaller tiles)
  int64_t n_ent = 0;                   // pass-2 entries, a multiple of lo_pass2_chunk()
  int* d_ent = nullptr;                // [4][n_ent]: output rows of QL_i, QR_j, QL_j, QR_i of one rank row
  double* d_entw = nullptr;            // [n_ent]: pair weight (1 for i = j, 2 for i < j; 0 for padding)
  float* d_orbfeat = nullptr;          // [n][2]: sum_j K_ij, sum_j discarded mass (residual features)
  double* d_grad = nullptr;            // [M][n]: gradient of the dropped energy at the trial (lo_residual_prepare)
  bool diag_u_only = true;             // exact SVD: the Vbar rows of a diagonal pair equal its Ubar^T rows
};

struct lo_md {
  int64_t M = 0, n = 0, ncas = 0, nao = 0, nav = 0, ndet = 0, maxe = 0;
  int na = 0;
  double* rows = nullptr;         // device [total_rows + nav][M]: the factor rows, then C_av^T
  int* d_exc = nullptr;           // [ndet]
  int* d_holes = nullptr;         // [ndet][na], relative to the first active occupied column
  int* d_parts = nullptr;         // [ndet][na], relative to column n
  double* d_coef = nullptr;       // [ndet]
  int64_t n_out_rows = 0, act_base = 0, total_rows = 0;
  int ntiles = 0, nblk = 0, tmax = 0, npairs = 0;
  int* d_rowidx = nullptr;        // pass-1 gather table: per orbital < n its own rows then the nav C_av^T
                                  // rows (T = C_av^T theta), then every factor row once per active column
  int* d_tpos = nullptr;          // [n]: output row of T[0][o]
  int* d_tiles = nullptr;         // [3][ntiles] then [nblk + 1]
  int* d_pair = nullptr;          // [3][npairs]: i, j, K
  int64_t* d_off = nullptr;       // [3][npairs]: own rows of i and j (-1 if virtual), first active row
};

struct lo_hr {
  int64_t M = 0, n = 0, npairs = 0;
  double* Y = nullptr;     // device [npairs][M][M], row-major, pairs i <= j in row order
  int* d_pairs = nullptr;  // device [npairs][2]
};

namespace {

constexpr int kMaxOcc = 64;     // split-BF16 energies
constexpr int kMaxOccWide = 96;  // the reduced-precision energies
constexpr int kMaxOccTheta = 112;  // green_theta

int fail(lo_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_OR_FAIL(ctx, call)                                                                   \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail((ctx), LO_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  if (a < 0 || b < 0) return false;
  if (a != 0 && b > std::numeric_limits<int64_t>::max() / a) return false;
  *out = a * b;
  return true;
}

// Grows the context workspace to at least `bytes` (never shrinks).
int ensure_ws(lo_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return LO_OK;
  if (c->ws) {
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    HIP_OR_FAIL(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (hipMalloc(&c->ws, bytes) != hipSuccess) {
    c->ws = nullptr;
    return fail(c, LO_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
  }
  c->ws_bytes = bytes;
  return LO_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

template <class T>
int upload(lo_ctx* c, T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return LO_OK;
  if (hipMalloc(dst, src.size() * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return fail(c, LO_ENOMEM, "device allocation of %zu bytes failed", src.size() * sizeof(T));
  }
  HIP_OR_FAIL(c, hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return LO_OK;
}

void free_factors(lo_factors* f) {
  if (!f) return;
  (void)hipFree(f->rows);
  (void)hipFree(f->rows32);
  (void)hipFree(f->rowsbf);
  (void)hipFree(f->d_rowidx);
  (void)hipFree(f->d_tiles);
  (void)hipFree(f->d_tiles_lp);
  (void)hipFree(f->d_ent);
  (void)hipFree(f->d_entw);
  (void)hipFree(f->d_orbfeat);
  (void)hipFree(f->d_grad);
  delete f;
}

// Records an event on the context stream that opens the interval of kernel
// `name` (nullptr closes the previous one).  Timing failures are not errors
// of the computation: a mark that cannot be recorded is dropped.
void prof_record(void* vctx, const char* name) {
  lo_ctx* c = (lo_ctx*)vctx;
  if (!c->prof_on) return;
  hipEvent_t ev = nullptr;
  if (!c->prof_pool.empty()) {
    ev = c->prof_pool.back();
    c->prof_pool.pop_back();
  } else if (hipEventCreate(&ev) != hipSuccess) {
    return;
  }
  if (hipEventRecord(ev, c->stream) != hipSuccess) {
    c->prof_pool.push_back(ev);
    return;
  }
  c->prof_marks.emplace_back(name, ev);
}

// Turns the recorded marks into per-kernel sums (synchronises the stream).
int prof_collect(lo_ctx* c) {
  if (c->prof_marks.empty()) return LO_OK;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i + 1 < c->prof_marks.size(); ++i) {
    const char* name = c->prof_marks[i].first;
    if (!name) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->prof_marks[i].second, c->prof_marks[i + 1].second) != hipSuccess) continue;
    auto& a = c->prof_acc[name];
    a.first += 1;
    a.second += ms;
  }
  for (auto& m : c->prof_marks) c->prof_pool.push_back(m.second);
  c->prof_marks.clear();
  return LO_OK;
}

// RAII: closes the last kernel interval of a call on every return path.
// Fixed device scratch of local_energy_lo_noalloc: the Q-bar intermediates,
// the pass-2 partial sums and (reduced precision) the rewritten theta of one
// call.  Every GPU the library runs on holds its own copy, at its own address,
// until the process ends.  Host code never passes `scratch` itself to a kernel
// (on the host it names a stand-in, not device memory): it uses the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = LO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device.
int scratch_on_current_device(lo_ctx* c, void** out) {
  int dev = -1;
  HIP_OR_FAIL(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, LO_EUNSUPPORTED, "device index %d above %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, LO_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LO_OK;
}

struct ProfScope {
  lo_ctx* c;
  lofqmc::ProfHook hook;
  explicit ProfScope(lo_ctx* ctx, bool allow_record = true)
      : c(ctx), hook{ctx, (allow_record && ctx->prof_on) ? prof_record : nullptr} {}
  const lofqmc::ProfHook* get() const { return &hook; }
  void mark(const char* name) const { lofqmc::prof_mark(&hook, name); }
  ~ProfScope() { mark(nullptr); }
};

}  // namespace

extern "C" {

int lo_create(lo_ctx** ctx, void* hip_stream) {
  if (!ctx) return LO_EINVAL;
  lo_ctx* c = new (std::nothrow) lo_ctx();
  if (!c) return LO_ENOMEM;
  c->stream = (hipStream_t)hip_stream;
  // set-up of the fixed scratch on the current device (skipped on a host
  // without a GPU; the allocation-free call then resolves it on first use)
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    void* p = nullptr;
    int rc = scratch_on_current_device(c, &p);
    if (rc) {
      delete c;
      return rc;
    }
  } else {
    (void)hipGetLastError();
  }
  *ctx = c;
  return LO_OK;
}

int lo_set_stream(lo_ctx* ctx, void* hip_stream) {
  if (!ctx) return LO_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  if (ctx->blas) rocblas_set_stream(ctx->blas, ctx->stream);
  ctx->err.clear();
  return LO_OK;
}

int lo_synchronize(lo_ctx* ctx) {
  if (!ctx) return LO_EINVAL;
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  return LO_OK;
}

int lo_destroy(lo_ctx* ctx) {
  if (!ctx) return LO_OK;
  if (ctx->ws || !ctx->prof_marks.empty()) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  for (auto& m : ctx->prof_marks) (void)hipEventDestroy(m.second);
  for (auto ev : ctx->prof_pool) (void)hipEventDestroy(ev);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  delete ctx;
  return LO_OK;
}

const char* lo_last_error(const lo_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int lo_profile_enable(lo_ctx* ctx, int enable) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!ctx->prof_marks.empty()) {
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& m : ctx->prof_marks) ctx->prof_pool.push_back(m.second);
    ctx->prof_marks.clear();
  }
  ctx->prof_acc.clear();
  ctx->prof_on = enable != 0;
  return LO_OK;
}

int lo_profile_summary(lo_ctx* ctx, int max_kernels, char* names, int64_t* launches, double* total_ms,
                       int* count) {
  if (!ctx || max_kernels < 0 || !count || (max_kernels > 0 && (!names || !launches || !total_ms)))
    return ctx ? fail(ctx, LO_EINVAL, "bad summary arguments") : LO_EINVAL;
  ctx->err.clear();
  int rc = prof_collect(ctx);
  if (rc) return rc;
  int k = 0;
  for (const auto& kv : ctx->prof_acc) {
    if (k < max_kernels) {
      std::snprintf(names + 64 * k, 64, "%s", kv.first.c_str());
      launches[k] = kv.second.first;
      total_ms[k] = kv.second.second;
    }
    ++k;
  }
  *count = k;
  ctx->prof_acc.clear();
  return LO_OK;
}

// ------------------------------------------------------------------ set-up

int build_half_rotated_chol(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* chol,
                            const double* trial, double* lbar) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (M <= 0 || n_occ <= 0 || n_chol < 0) return fail(ctx, LO_EINVAL, "sizes must be M > 0, n_occ > 0, n_chol >= 0");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ (%lld) exceeds M (%lld)", (long long)n_occ, (long long)M);
  if (M > (1 << 20)) return fail(ctx, LO_EUNSUPPORTED, "M above 2^20");
  int64_t t;
  if (!mul_ok(M, M, &t) || !mul_ok(t, n_chol, &t)) return fail(ctx, LO_EINVAL, "n_chol*M*M overflows");
  if (n_chol == 0) return LO_OK;
  if (!chol || !trial || !lbar) return fail(ctx, LO_EINVAL, "null array");
  std::vector<int64_t> bases(3 * n_chol);
  for (int64_t g = 0; g < n_chol; ++g) {
    bases[3 * g] = g * M * M;
    bases[3 * g + 1] = 0;
    bases[3 * g + 2] = g * M * n_occ;
  }
  int64_t* d_bases = nullptr;
  int rc = upload(ctx, &d_bases, bases);
  if (rc) return rc;
  // lbar_g (M x n) = chol_g (M x M) * trial (M x n)
  const int64_t maxb = 65535;
  for (int64_t g0 = 0; g0 < n_chol; g0 += maxb) {
    const int nb = (int)std::min<int64_t>(maxb, n_chol - g0);
    hipError_t e = lofqmc::launch_gemm_setup(ctx->stream, (int)M, (int)n_occ, (int)M, chol, M, 1, trial, n_occ, 1,
                                             lbar, n_occ, 1, d_bases + 3 * g0, nb);
    if (e != hipSuccess) {
      (void)hipFree(d_bases);
      return fail(ctx, LO_EHIP, "half-rotation launch failed: %s", hipGetErrorString(e));
    }
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  HIP_OR_FAIL(ctx, hipFree(d_bases));
  return LO_OK;
}

}  // extern "C"

namespace {

// Shared by the exact and the randomized factorisation.  L = 0: full SVD of
// every pair block.  L > 0: randomized subspace iteration (Halko, Martinsson
// and Tropp 2011, Alg. 4.4) with the caller's test matrix omega [M][L] (row-
// major, device) and `power_iters` power steps, then the SVD of the L x M
// projection.
// Second half of a factor handle: the reduced-precision copies of the rows
// and the tables of the two energy passes, from M, n, X, ranks, first_dropped,
// discarded, row_offset, total_rows and the device rows.  diag_u_only: the
// rows came from the exact SVD, so the Vbar rows of a diagonal pair equal its
// Ubar^T rows.  On failure frees f and returns the error.
int finish_factors(lo_ctx* ctx, lo_factors* f, bool diag_u_only) {
  const int64_t M = f->M, n = f->n, total_rows = f->total_rows;
  int rc = LO_OK;
  auto cleanup = [&]() { (void)hipStreamSynchronize(ctx->stream); };
#define TRY_HIP(call)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      rc = fail(ctx, LO_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));                   \
      cleanup();                                                                                \
      free_factors(f);                                                                          \
      return rc;                                                                                \
    }                                                                                           \
  } while (0)
#define TRY_ALLOC(ptr, bytes)                                                                   \
  do {                                                                                          \
    if (hipMalloc(&(ptr), (bytes)) != hipSuccess) {                                             \
      ptr = nullptr;                                                                            \
      rc = fail(ctx, LO_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes));      \
      cleanup();                                                                                \
      free_factors(f);                                                                          \
      return rc;                                                                                \
    }                                                                                           \
  } while (0)
  f->diag_u_only = diag_u_only;
  if (total_rows > 0) {
    // FP32 and split-BF16 copies for the reduced-precision energy
    const size_t Mp = (size_t)lofqmc::lp_padded_m((int)M);
    TRY_ALLOC(f->rows32, sizeof(float) * (size_t)total_rows * Mp);
    TRY_ALLOC(f->rowsbf, sizeof(__bf16) * 2 * (size_t)total_rows * Mp);
    TRY_HIP(lofqmc::launch_factor_rows_lp(ctx->stream, (int)M, total_rows, f->rows, f->rows32, f->rowsbf));
  }

  // ---- tables of the two energy passes
  // A diagonal block Y^[ii] is symmetric positive semidefinite, so every left
  // singular vector with sigma > 0 equals its right one (Y v = sigma u and
  // Y v = sigma v): Vbar^[ii] = Ubar^[ii]T and QR_i = QL_i.  With the exact SVD
  // the pass-1 product of orbital i then takes only the Ubar^T rows of its
  // diagonal pair; the randomized SVD only approximates the singular vectors,
  // so its factors keep both.
  auto out_rows = [&](int o, int k) -> int64_t {
    const int64_t K = f->ranks[o * n + k];
    return (o == k && diag_u_only) ? K : 2 * K;
  };
  std::vector<int64_t> obase(n + 1, 0);
  std::vector<int64_t> loc(n * n, 0);  // local output row of pair (o, k) within orbital o
  for (int o = 0; o < n; ++o) {
    int64_t R = 0;
    for (int k = 0; k < n; ++k) {
      loc[o * n + k] = R;
      R += out_rows(o, k);
    }
    obase[o + 1] = obase[o] + R;
  }
  f->n_out_rows = obase[n];
  if (f->n_out_rows > std::numeric_limits<int>::max()) {
    rc = fail(ctx, LO_EUNSUPPORTED, "too many factor rows");
    cleanup();
    free_factors(f);
    return rc;
  }
  std::vector<int> rowidx(f->n_out_rows);
  for (int o = 0; o < n; ++o) {
    for (int k = 0; k < n; ++k) {
      const int i = std::min(o, k), j = std::max(o, k);
      const int64_t src = f->row_offset[i * n + j];
      const int64_t cnt = out_rows(o, k);
      for (int64_t q = 0; q < cnt; ++q) rowidx[obase[o] + loc[o * n + k] + q] = (int)(src + q);
    }
  }
  // pass-1 tiles: each orbital's rows split into near-equal tiles of at most
  // `cap` rows, listed by orbital as [orbital][first row][row count], then the
  // first tile of each block of lo_orbital_block() orbitals
  auto build_tiles = [&](int64_t cap, int* ntiles, int* nblk, int* tmax) {
    std::vector<int> t_orb, t_row0, t_nrows;
    for (int o = 0; o < n; ++o) {
      const int64_t R = obase[o + 1] - obase[o];
      const int64_t ntile = (R + cap - 1) / cap;
      for (int64_t q = 0; q < ntile; ++q) {
        const int64_t a = obase[o] + R * q / ntile, b = obase[o] + R * (q + 1) / ntile;
        t_orb.push_back(o);
        t_row0.push_back((int)a);
        t_nrows.push_back((int)(b - a));
      }
    }
    *ntiles = (int)t_orb.size();
    std::vector<int> tiles;
    tiles.insert(tiles.end(), t_orb.begin(), t_orb.end());
    tiles.insert(tiles.end(), t_row0.begin(), t_row0.end());
    tiles.insert(tiles.end(), t_nrows.begin(), t_nrows.end());
    const int ob = lofqmc::lo_orbital_block();
    *nblk = (int)((n + ob - 1) / ob);
    std::vector<int> blk(*nblk + 1, *ntiles);
    int t = 0;
    for (int b = 0; b < *nblk; ++b) {
      while (t < *ntiles && t_orb[t] < b * ob) ++t;
      blk[b] = t;
    }
    *tmax = 0;
    for (int b = 0; b < *nblk; ++b) *tmax = std::max(*tmax, blk[b + 1] - blk[b]);
    tiles.insert(tiles.end(), blk.begin(), blk.end());
    return tiles;
  };
  const std::vector<int> tiles = build_tiles(lofqmc::lo_tile_rows(), &f->ntiles, &f->nblk, &f->tmax);
  const std::vector<int> tiles_lp = build_tiles(lofqmc::lo_lp_tile_rows(), &f->ntiles_lp, &f->nblk_lp, &f->tmax_lp);
  // pass-2 entries: one per rank row K of every stored pair i <= j, the
  // output rows of QL_i, QR_j (Coulomb) and QL_j, QR_i (exchange), padded
  // with weight-0 entries to whole chunks
  std::vector<int> e_li, e_rj, e_lj, e_ri;
  std::vector<double> e_w;
  int nstored = 0;
  for (int i = 0; i < n; ++i) {
    for (int j = i; j < n; ++j) {
      const int K = f->ranks[i * n + j];
      if (K == 0) continue;
      ++nstored;
      const int64_t oi = obase[i] + loc[i * n + j], oj = obase[j] + loc[j * n + i];
      // the QR rows follow the QL rows, or are the QL rows (diagonal, exact SVD)
      const int64_t vr = (i == j && diag_u_only) ? 0 : K;
      for (int k = 0; k < K; ++k) {
        e_li.push_back((int)(oi + k));
        e_rj.push_back((int)(oj + vr + k));
        e_lj.push_back((int)(oj + k));
        e_ri.push_back((int)(oi + vr + k));
        e_w.push_back(i == j ? 1.0 : 2.0);
      }
    }
  }
  f->npairs = nstored;
  const int ech = lofqmc::lo_pass2_chunk();
  while (e_w.size() % ech) {
    e_li.push_back(0);
    e_rj.push_back(0);
    e_lj.push_back(0);
    e_ri.push_back(0);
    e_w.push_back(0.0);
  }
  f->n_ent = (int64_t)e_w.size();
  std::vector<int> ent(e_li);
  ent.insert(ent.end(), e_rj.begin(), e_rj.end());
  ent.insert(ent.end(), e_lj.begin(), e_lj.end());
  ent.insert(ent.end(), e_ri.begin(), e_ri.end());
  std::vector<float> orbfeat(2 * n, 0.0f);
  for (int i = 0; i < n; ++i) {
    double ks = 0.0, ms = 0.0;
    for (int j = 0; j < n; ++j) {
      ks += f->ranks[i * n + j];
      ms += f->discarded[i * n + j];
    }
    orbfeat[2 * i] = (float)ks;
    orbfeat[2 * i + 1] = (float)ms;
  }
  if ((rc = upload(ctx, &f->d_rowidx, rowidx)) || (rc = upload(ctx, &f->d_tiles, tiles)) ||
      (rc = upload(ctx, &f->d_tiles_lp, tiles_lp)) ||
      (rc = upload(ctx, &f->d_ent, ent)) || (rc = upload(ctx, &f->d_entw, e_w)) ||
      (rc = upload(ctx, &f->d_orbfeat, orbfeat))) {
    cleanup();
    free_factors(f);
    return rc;
  }
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  return LO_OK;
#undef TRY_HIP
#undef TRY_ALLOC
}

int build_factors(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar, double epsilon,
                  int64_t L, int power_iters, const double* omega, lo_factors** out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, LO_EINVAL, "null output handle");
  *out = nullptr;
  if (M <= 0 || n_occ <= 0 || n_chol <= 0) return fail(ctx, LO_EINVAL, "sizes must be positive");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (!(epsilon >= 0.0) || std::isinf(epsilon)) return fail(ctx, LO_EINVAL, "epsilon must be finite and >= 0");
  if (!lbar) return fail(ctx, LO_EINVAL, "null lbar");
  if (M > 8192) return fail(ctx, LO_EUNSUPPORTED, "M above 8192");
  if (n_occ > 4096) return fail(ctx, LO_EUNSUPPORTED, "n_occ above 4096");
  int64_t t;
  if (!mul_ok(M * n_occ, n_chol, &t)) return fail(ctx, LO_EINVAL, "n_chol*M*n_occ overflows");

  if (!ctx->blas) {
    if (rocblas_create_handle(&ctx->blas) != rocblas_status_success) {
      ctx->blas = nullptr;
      return fail(ctx, LO_ESOLVER, "rocblas_create_handle failed");
    }
  }
  rocblas_set_stream(ctx->blas, ctx->stream);

  const int64_t n = n_occ;
  const int64_t npairs = n * (n + 1) / 2;
  const size_t mm = (size_t)M * M;
  // batch of pairs: A, U, VT (3 M^2) plus S, E per pair, within ~1.5 GiB
  int64_t batch = std::max<int64_t>(1, (int64_t)((size_t(3) << 29) / (3 * mm * sizeof(double))));
  batch = std::min<int64_t>({batch, npairs, 512});

  double *d_lbarT = nullptr, *d_Y = nullptr, *d_U = nullptr, *d_VT = nullptr, *d_S = nullptr, *d_E = nullptr;
  double *d_Z = nullptr, *d_W = nullptr, *d_B = nullptr, *d_UB = nullptr;
  int *d_info = nullptr, *d_K = nullptr;
  int64_t *d_bases = nullptr, *d_roff = nullptr;
  std::vector<double*> chunks;       // packed rows per batch
  std::vector<int64_t> chunk_rows;
  lo_factors* f = nullptr;
  int rc = LO_OK;

  auto cleanup = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(d_lbarT);
    (void)hipFree(d_Y);
    (void)hipFree(d_U);
    (void)hipFree(d_VT);
    (void)hipFree(d_S);
    (void)hipFree(d_E);
    (void)hipFree(d_info);
    (void)hipFree(d_K);
    (void)hipFree(d_bases);
    (void)hipFree(d_roff);
    (void)hipFree(d_Z);
    (void)hipFree(d_W);
    (void)hipFree(d_B);
    (void)hipFree(d_UB);
    for (double* p : chunks) (void)hipFree(p);
  };
#define TRY_HIP(call)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      rc = fail(ctx, LO_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));                   \
      cleanup();                                                                                \
      free_factors(f);                                                                          \
      return rc;                                                                                \
    }                                                                                           \
  } while (0)
#define TRY_ALLOC(ptr, bytes)                                                                   \
  do {                                                                                          \
    if (hipMalloc(&(ptr), (bytes)) != hipSuccess) {                                             \
      ptr = nullptr;                                                                            \
      rc = fail(ctx, LO_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes));      \
      cleanup();                                                                                \
      free_factors(f);                                                                          \
      return rc;                                                                                \
    }                                                                                           \
  } while (0)

  TRY_ALLOC(d_lbarT, sizeof(double) * (size_t)n_chol * M * n);
  TRY_HIP(lofqmc::launch_lbar_transpose(ctx->stream, (int)M, (int)n, n_chol, lbar, d_lbarT));
  TRY_ALLOC(d_Y, sizeof(double) * mm * batch);
  TRY_ALLOC(d_U, sizeof(double) * mm * batch);
  TRY_ALLOC(d_VT, sizeof(double) * mm * batch);
  TRY_ALLOC(d_S, sizeof(double) * M * batch);
  TRY_ALLOC(d_E, sizeof(double) * M * batch);
  TRY_ALLOC(d_info, sizeof(int) * batch);
  TRY_ALLOC(d_K, sizeof(int) * batch);
  TRY_ALLOC(d_bases, sizeof(int64_t) * 3 * batch);
  TRY_ALLOC(d_roff, sizeof(int64_t) * batch);
  // randomized path: Z, W (M x L), B (L x M) and U_B (L x L) per pair
  const size_t ml = (size_t)M * L;
  if (L > 0) {
    TRY_ALLOC(d_Z, sizeof(double) * ml * batch);
    TRY_ALLOC(d_W, sizeof(double) * ml * batch);
    TRY_ALLOC(d_B, sizeof(double) * ml * batch);
    TRY_ALLOC(d_UB, sizeof(double) * (size_t)L * L * batch);
  }
  const int64_t kmax = L > 0 ? L : M;   // singular values per pair

  f = new lo_factors();
  f->M = M;
  f->n = n;
  f->X = n_chol;
  f->ranks.assign(n * n, 0);
  f->first_dropped.assign(n * n, 0.0);
  f->discarded.assign(n * n, 0.0);
  f->row_offset.assign(n * n, -1);

  std::vector<std::pair<int, int>> plist;
  plist.reserve(npairs);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) plist.emplace_back(i, j);

  std::vector<double> S_host(kmax * batch);
  std::vector<int> info_host(batch), K_host(batch);
  std::vector<int64_t> bases(3 * batch), roff_host(batch);
  int64_t total_rows = 0;

  for (int64_t p0 = 0; p0 < npairs; p0 += batch) {
    const int nb = (int)std::min<int64_t>(batch, npairs - p0);
    for (int b = 0; b < nb; ++b) {
      const auto [i, j] = plist[p0 + b];
      bases[3 * b] = (int64_t)i * n_chol * M;
      bases[3 * b + 1] = (int64_t)j * n_chol * M;
      bases[3 * b + 2] = (int64_t)b * mm;
    }
    TRY_HIP(hipMemcpyAsync(d_bases, bases.data(), sizeof(int64_t) * 3 * nb, hipMemcpyHostToDevice, ctx->stream));
    // Y^[ij](r, s) = sum_g lbarT[i][g][r] lbarT[j][g][s], stored column-major
    TRY_HIP(lofqmc::launch_gemm_setup(ctx->stream, (int)M, (int)M, (int)n_chol, d_lbarT, 1, M, d_lbarT, M, 1, d_Y, 1,
                                      M, d_bases, nb));
    rocblas_status st = rocblas_status_success;
    if (L == 0) {
      st = rocsolver_dgesvd_strided_batched(
          ctx->blas, rocblas_svect_singular, rocblas_svect_singular, (rocblas_int)M, (rocblas_int)M, d_Y,
          (rocblas_int)M, (rocblas_stride)mm, d_S, (rocblas_stride)M, d_U, (rocblas_int)M, (rocblas_stride)mm, d_VT,
          (rocblas_int)M, (rocblas_stride)mm, d_E, (rocblas_stride)M, rocblas_outofplace, d_info, nb);
    } else {
      const double one = 1.0, zero = 0.0;
      const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
      auto gemm = [&](rocblas_operation ta, rocblas_operation tb, int64_t m, int64_t nn, int64_t k, const double* A,
                      int64_t lda, int64_t sa, const double* Bm, int64_t ldb, int64_t sb, double* C, int64_t ldc,
                      int64_t sc) {
        return rocblas_dgemm_strided_batched(ctx->blas, ta, tb, (rocblas_int)m, (rocblas_int)nn, (rocblas_int)k, &one,
                                             A, (rocblas_int)lda, sa, Bm, (rocblas_int)ldb, sb, &zero, C,
                                             (rocblas_int)ldc, sc, nb);
      };
      // columns of an M x L block replaced by an orthonormal basis of their span
      auto orth = [&](double* A) {
        return lofqmc::launch_orth(ctx->stream, (int)M, (int)L, nb, A, (int64_t)ml) == hipSuccess
                   ? rocblas_status_success
                   : rocblas_status_internal_error;
      };
      // Z = Y Omega (omega is row-major M x L, i.e. column-major L x M)
      st = gemm(N_, T_, M, L, M, d_Y, M, mm, omega, L, 0, d_Z, M, ml);
      for (int q = 0; q < power_iters && st == rocblas_status_success; ++q) {
        st = orth(d_Z);
        if (st == rocblas_status_success) st = gemm(T_, N_, M, L, M, d_Y, M, mm, d_Z, M, ml, d_W, M, ml);  // Y^T Q
        if (st == rocblas_status_success) st = orth(d_W);
        if (st == rocblas_status_success) st = gemm(N_, N_, M, L, M, d_Y, M, mm, d_W, M, ml, d_Z, M, ml);  // Y Q'
      }
      if (st == rocblas_status_success) st = orth(d_Z);                                           // Q
      if (st == rocblas_status_success) st = gemm(T_, N_, L, M, M, d_Z, M, ml, d_Y, M, mm, d_B, L, ml);   // Q^T Y
      if (st == rocblas_status_success)
        st = rocsolver_dgesvd_strided_batched(
            ctx->blas, rocblas_svect_singular, rocblas_svect_singular, (rocblas_int)L, (rocblas_int)M, d_B,
            (rocblas_int)L, (rocblas_stride)ml, d_S, (rocblas_stride)L, d_UB, (rocblas_int)L,
            (rocblas_stride)(L * L), d_VT, (rocblas_int)L, (rocblas_stride)ml, d_E, (rocblas_stride)L,
            rocblas_outofplace, d_info, nb);
      if (st == rocblas_status_success) st = gemm(N_, N_, M, L, L, d_Z, M, ml, d_UB, L, L * L, d_U, M, ml);  // Q U_B
    }
    if (st != rocblas_status_success) {
      rc = fail(ctx, LO_ESOLVER, "rocBLAS/rocSOLVER call of the pair-block decomposition returned %d", (int)st);
      cleanup();
      free_factors(f);
      return rc;
    }
    TRY_HIP(hipMemcpyAsync(S_host.data(), d_S, sizeof(double) * kmax * nb, hipMemcpyDeviceToHost, ctx->stream));
    TRY_HIP(hipMemcpyAsync(info_host.data(), d_info, sizeof(int) * nb, hipMemcpyDeviceToHost, ctx->stream));
    TRY_HIP(hipStreamSynchronize(ctx->stream));
    int64_t batch_rows = 0;
    for (int b = 0; b < nb; ++b) {
      if (info_host[b] != 0) {
        rc = fail(ctx, LO_ESOLVER, "SVD of pair block %d did not converge (info %d)", (int)(p0 + b), info_host[b]);
        cleanup();
        free_factors(f);
        return rc;
      }
      const double* s = S_host.data() + (size_t)b * kmax;
      int K = 0;
      if (epsilon == 0.0) {
        K = (int)kmax;
      } else {
        while (K < kmax && s[K] >= epsilon) ++K;
      }
      const auto [i, j] = plist[p0 + b];
      if (L > 0 && K == kmax && kmax < M) {
        rc = fail(ctx, LO_EUNSUPPORTED,
                  "pair (%d, %d): all %d sketched singular values reach epsilon; a larger sketch is needed", i, j,
                  (int)kmax);
        cleanup();
        free_factors(f);
        return rc;
      }
      f->ranks[i * n + j] = f->ranks[j * n + i] = K;
      const double fd = (K < kmax) ? s[K] : 0.0;
      f->first_dropped[i * n + j] = f->first_dropped[j * n + i] = fd;
      {
        double mass = 0.0;
        for (int64_t k = K; k < kmax; ++k) mass += s[k];
        f->discarded[i * n + j] = f->discarded[j * n + i] = mass;
      }
      f->row_offset[i * n + j] = total_rows + batch_rows;
      K_host[b] = K;
      roff_host[b] = batch_rows;
      batch_rows += 2 * (int64_t)K;
    }
    double* dst = nullptr;
    if (batch_rows > 0) {
      TRY_ALLOC(dst, sizeof(double) * (size_t)batch_rows * M);
      chunks.push_back(dst);
      chunk_rows.push_back(batch_rows);
      TRY_HIP(hipMemcpyAsync(d_K, K_host.data(), sizeof(int) * nb, hipMemcpyHostToDevice, ctx->stream));
      TRY_HIP(hipMemcpyAsync(d_roff, roff_host.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, ctx->stream));
      if (L == 0)
        TRY_HIP(lofqmc::launch_pack_factors(ctx->stream, (int)M, nb, (int)M, d_U, (int64_t)mm, d_VT, (int)M,
                                            (int64_t)mm, d_S, M, d_K, d_roff, dst));
      else
        TRY_HIP(lofqmc::launch_pack_factors(ctx->stream, (int)M, nb, (int)L, d_U, (int64_t)ml, d_VT, (int)L,
                                            (int64_t)ml, d_S, L, d_K, d_roff, dst));
      TRY_HIP(hipStreamSynchronize(ctx->stream));  // host vectors are reused by the next batch
    }
    total_rows += batch_rows;
  }
  f->total_rows = total_rows;
  if (total_rows > 0) {
    TRY_ALLOC(f->rows, sizeof(double) * (size_t)total_rows * M);
    int64_t at = 0;
    for (size_t c = 0; c < chunks.size(); ++c) {
      TRY_HIP(hipMemcpyAsync(f->rows + (size_t)at * M, chunks[c], sizeof(double) * (size_t)chunk_rows[c] * M,
                             hipMemcpyDeviceToDevice, ctx->stream));
      at += chunk_rows[c];
    }
  }
  cleanup();
  const int frc = finish_factors(ctx, f, L == 0);
  if (frc) return frc;
  *out = f;
  return LO_OK;
#undef TRY_HIP
#undef TRY_ALLOC
}

// theta layout named by the layout flags (at most one may be set)
static int theta_layout_of(unsigned flags) {
  return (flags & LO_THETA_TRANSPOSED) ? lofqmc::THETA_TRANSPOSED
         : (flags & LO_THETA_ORBITAL_MAJOR) ? lofqmc::THETA_ORBITAL
                                            : lofqmc::THETA_WALKER;
}
static bool two_layouts(unsigned flags) {
  return (flags & LO_THETA_ORBITAL_MAJOR) && (flags & LO_THETA_TRANSPOSED);
}

// Argument checks of the LO energy call and the scratch bytes it needs
// (Q-bar intermediates, pass-2 partial sums, reduced-precision theta copy).
int lo_energy_check(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, const double* lbar,
                    const double* energy, int precision, unsigned flags, size_t* need) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!f) return fail(ctx, LO_EINVAL, "null factors");
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  if (precision != LO_FP64 && precision != LO_FP32 && precision != LO_BF16X3)
    return fail(ctx, LO_EINVAL, "unknown precision %d", precision);
  if (flags & ~(unsigned)(LO_THETA_ORBITAL_MAJOR | LO_THETA_TRANSPOSED | LO_EXACT_COULOMB))
    return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (two_layouts(flags)) return fail(ctx, LO_EINVAL, "two theta layouts in flags");
  const bool other_layout = theta_layout_of(flags) != lofqmc::THETA_WALKER;
  const bool exact_j = (flags & LO_EXACT_COULOMB) != 0;
  if (precision != LO_FP64 && other_layout)
    return fail(ctx, LO_EUNSUPPORTED, "reduced precision reads walker-major theta only");
  if (exact_j && other_layout) return fail(ctx, LO_EUNSUPPORTED, "LO_EXACT_COULOMB reads walker-major theta only");
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (precision != LO_FP64 && nw > 65535) return fail(ctx, LO_EUNSUPPORTED, "reduced precision: nw above 65535");
  if (precision != LO_FP64 && f->n > (precision == LO_FP32 ? kMaxOccWide : kMaxOcc))
    return fail(ctx, LO_EUNSUPPORTED, "n_occ above %d for this precision",
                precision == LO_FP32 ? kMaxOccWide : kMaxOcc);
  *need = 0;
  if (nw == 0) return LO_OK;
  if (!theta || !energy) return fail(ctx, LO_EINVAL, "null array");
  if (exact_j && !lbar) return fail(ctx, LO_EINVAL, "LO_EXACT_COULOMB needs lbar");
  const int nchunk = (int)(f->n_ent / lofqmc::lo_pass2_chunk());
  const size_t qbytes = align256(sizeof(double) * 2 * (size_t)f->n_out_rows * nw);
  const size_t pbytes = align256(sizeof(double) * 4 * (size_t)(nchunk + (exact_j ? 1 : 0)) * nw);
  const size_t tbytes =
      precision == LO_FP64 ? 0 : align256(lofqmc::lp_theta_bytes(precision, (int)f->M, (int)f->n, nw));
  const size_t cbytes = exact_j ? align256(lofqmc::coulomb_cpart_bytes((int)f->M, (int)f->n, f->X, nw)) : 0;
  *need = qbytes + pbytes + tbytes + cbytes;
  return LO_OK;
}

// Queues the LO energy kernels on the context's stream with their scratch at
// `base` (lo_energy_check's byte count); every byte they read there is
// written first by an earlier kernel of the same call.
int lo_energy_enqueue(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, const int32_t* info,
                      int precision, unsigned flags, const double* lbar, double* energy, char* base,
                      const ProfScope& prof) {
  const bool exact_j = (flags & LO_EXACT_COULOMB) != 0;
  const int64_t M = f->M, n = f->n;
  const int nchunk = (int)(f->n_ent / lofqmc::lo_pass2_chunk());
  const int nrows = nchunk + (exact_j ? 1 : 0);
  const size_t qbytes = align256(sizeof(double) * 2 * (size_t)f->n_out_rows * nw);
  const size_t pbytes = align256(sizeof(double) * 4 * (size_t)nrows * nw);
  const size_t tbytes =
      precision == LO_FP64 ? 0 : align256(lofqmc::lp_theta_bytes(precision, (int)M, (int)n, nw));
  double* qbar = (double*)base;
  double* partial = (double*)(base + qbytes);
  if (precision == LO_FP64) {
    prof.mark(lofqmc::lo_pass1_name((int)M));
    HIP_OR_FAIL(ctx, lofqmc::launch_lo_pass1(ctx->stream, (int)M, (int)n, nw, f->ntiles, f->rows, f->total_rows,
                                             f->d_rowidx,
                                             f->d_tiles, f->d_tiles + 3 * f->ntiles, f->nblk, f->tmax, theta,
                                             theta_layout_of(flags), qbar, 0));
  } else if (f->ntiles > 0) {
    void* tlp = base + qbytes + pbytes;
    prof.mark("lp_convert_kernel");
    HIP_OR_FAIL(ctx, lofqmc::launch_lp_convert_theta(ctx->stream, precision, (int)M, (int)n, nw, theta, tlp));
    prof.mark("lo_pass1_lp_kernel");
    const void* rows_lp = precision == LO_FP32 ? (const void*)f->rows32 : (const void*)f->rowsbf;
    HIP_OR_FAIL(ctx, lofqmc::launch_lo_pass1_lp(ctx->stream, precision, (int)M, (int)n, nw, f->ntiles_lp, rows_lp,
                                                f->d_rowidx, f->d_tiles_lp, f->d_tiles_lp + 3 * f->ntiles_lp,
                                                f->nblk_lp, f->tmax_lp, tlp, qbar));
  }
  prof.mark("lo_pass2_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_lo_pass2(ctx->stream, nw, f->n_ent, f->d_ent, f->d_entw, qbar, partial,
                                           exact_j ? 0 : 1));
  if (exact_j) {
    // E_J from the FP64 Cholesky traces (Eq. 16) as one more partial row
    HIP_OR_FAIL(ctx, lofqmc::launch_coulomb_fp64(ctx->stream, (int)M, (int)n, f->X, nw, theta, lbar,
                                                 base + qbytes + pbytes + tbytes, partial + (size_t)nchunk * nw * 4,
                                                 prof.get()));
  }
  prof.mark("reduce_partials_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_reduce_partials(ctx->stream, nw, nrows, partial, info, energy));
  return LO_OK;
}

}  // namespace

extern "C" {

int lo_localize_boys(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_pos, const double* positions, double* orbitals,
                     int max_sweeps, double tol, double* stats) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (M <= 0 || n_occ <= 0 || n_pos <= 0) return fail(ctx, LO_EINVAL, "sizes must be positive");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (max_sweeps < 1) return fail(ctx, LO_EINVAL, "max_sweeps must be >= 1");
  if (!(tol >= 0.0) || std::isinf(tol)) return fail(ctx, LO_EINVAL, "tol must be finite and >= 0");
  if (!positions || !orbitals) return fail(ctx, LO_EINVAL, "null array");
  if (M > (1 << 24)) return fail(ctx, LO_EUNSUPPORTED, "M above 2^24");
  if (n_pos > 3 || n_pos * n_occ * n_occ > lofqmc::boys_max_lds_doubles())
    return fail(ctx, LO_EUNSUPPORTED, "n_pos * n_occ^2 above %d (n_pos <= 3)", lofqmc::boys_max_lds_doubles());
  const size_t wbytes = lofqmc::boys_workspace((int)M, (int)n_occ, (int)n_pos);
  int rc = ensure_ws(ctx, wbytes);
  if (rc) return rc;
  double* dstats = (double*)((char*)ctx->ws + wbytes - align256(sizeof(double) * 4));
  HIP_OR_FAIL(ctx, lofqmc::launch_boys(ctx->stream, (int)M, (int)n_occ, (int)n_pos, positions, orbitals, max_sweeps,
                                       tol, ctx->ws, dstats));
  double h[3] = {0.0, 0.0, 0.0};
  HIP_OR_FAIL(ctx, hipMemcpyAsync(h, dstats, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  if (stats) std::memcpy(stats, h, sizeof(h));
  return LO_OK;
}

int build_lo_factors(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar, double epsilon,
                     lo_factors** out) {
  return build_factors(ctx, M, n_occ, n_chol, lbar, epsilon, 0, 0, nullptr, out);
}

int build_lo_factors_randomized(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar,
                                double epsilon, int64_t sketch, int power_iters, const double* omega,
                                lo_factors** out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (out) *out = nullptr;
  if (sketch <= 0 || sketch > M) return fail(ctx, LO_EINVAL, "sketch must be in 1..M");
  if (sketch > 64) return fail(ctx, LO_EUNSUPPORTED, "sketch above 64");
  if (power_iters < 0 || power_iters > 16) return fail(ctx, LO_EINVAL, "power_iters must be in 0..16");
  if (!(epsilon > 0.0) || std::isinf(epsilon)) return fail(ctx, LO_EINVAL, "epsilon must be finite and > 0");
  if (!omega) return fail(ctx, LO_EINVAL, "null omega");
  return build_factors(ctx, M, n_occ, n_chol, lbar, epsilon, sketch, power_iters, omega, out);
}

int lo_factors_destroy(lo_factors* f) {
  free_factors(f);
  return LO_OK;
}

int lo_factors_info(const lo_factors* f, int64_t* M, int64_t* n_occ, int32_t* ranks, double* first_dropped,
                    int64_t* total_rows, int64_t* bytes) {
  if (!f) return LO_EINVAL;
  if (M) *M = f->M;
  if (n_occ) *n_occ = f->n;
  if (ranks) std::memcpy(ranks, f->ranks.data(), sizeof(int32_t) * f->ranks.size());
  if (first_dropped) std::memcpy(first_dropped, f->first_dropped.data(), sizeof(double) * f->first_dropped.size());
  if (total_rows) *total_rows = f->total_rows;
  if (bytes) *bytes = f->total_rows * f->M * (int64_t)sizeof(double);
  return LO_OK;
}

int lo_factors_export(const lo_factors* f, double* rows, int64_t* row_offset) {
  if (!f) return LO_EINVAL;
  if (row_offset) std::memcpy(row_offset, f->row_offset.data(), sizeof(int64_t) * f->row_offset.size());
  if (rows && f->total_rows > 0) {
    if (hipMemcpy(rows, f->rows, sizeof(double) * (size_t)f->total_rows * f->M, hipMemcpyDeviceToHost) != hipSuccess)
      return LO_EHIP;
  }
  return LO_OK;
}

int lo_factors_import(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const int32_t* ranks,
                      const int64_t* row_offset, const double* first_dropped, const double* discarded,
                      const double* rows, unsigned flags, lo_factors** out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, LO_EINVAL, "null output handle");
  *out = nullptr;
  if (M <= 0 || n_occ <= 0 || n_chol <= 0) return fail(ctx, LO_EINVAL, "sizes must be positive");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (M > 8192 || n_occ > 4096) return fail(ctx, LO_EUNSUPPORTED, "M above 8192 or n_occ above 4096");
  if (flags & ~(unsigned)LO_FACTORS_RANDOMIZED) return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (!ranks || !row_offset) return fail(ctx, LO_EINVAL, "null ranks or row_offset");
  const int64_t n = n_occ;
  // the stored pairs i <= j must tile [0, total_rows) with 2 K rows each
  int64_t total = 0;
  std::vector<std::pair<int64_t, int64_t>> spans;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const int32_t K = ranks[i * n + j];
      if (K < 0 || K > M || K != ranks[j * n + i]) return fail(ctx, LO_EINVAL, "ranks must be symmetric, 0..M");
      if (j < i) continue;
      if (K > 0) {
        const int64_t off = row_offset[i * n + j];
        if (off < 0) return fail(ctx, LO_EINVAL, "pair (%d, %d): negative row offset", (int)i, (int)j);
        spans.emplace_back(off, 2 * (int64_t)K);
      }
      total += 2 * (int64_t)K;
    }
  std::sort(spans.begin(), spans.end());
  int64_t at = 0;
  for (const auto& sp : spans) {
    if (sp.first != at) return fail(ctx, LO_EINVAL, "row offsets do not tile the rows");
    at += sp.second;
  }
  if (total > 0 && !rows) return fail(ctx, LO_EINVAL, "null rows");
  lo_factors* f = new (std::nothrow) lo_factors();
  if (!f) return fail(ctx, LO_ENOMEM, "host allocation failed");
  f->M = M;
  f->n = n;
  f->X = n_chol;
  f->total_rows = total;
  f->ranks.assign(ranks, ranks + n * n);
  f->row_offset.assign(row_offset, row_offset + n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) f->row_offset[i * n + j] = -1;
  f->first_dropped.assign(n * n, 0.0);
  f->discarded.assign(n * n, 0.0);
  if (first_dropped) f->first_dropped.assign(first_dropped, first_dropped + n * n);
  if (discarded) f->discarded.assign(discarded, discarded + n * n);
  if (total > 0) {
    if (hipMalloc(&f->rows, sizeof(double) * (size_t)total * M) != hipSuccess) {
      f->rows = nullptr;
      free_factors(f);
      return fail(ctx, LO_ENOMEM, "device allocation of the factor rows failed");
    }
    if (hipMemcpy(f->rows, rows, sizeof(double) * (size_t)total * M, hipMemcpyHostToDevice) != hipSuccess) {
      free_factors(f);
      return fail(ctx, LO_EHIP, "upload of the factor rows failed");
    }
  }
  const int rc = finish_factors(ctx, f, (flags & LO_FACTORS_RANDOMIZED) == 0);
  if (rc) return rc;
  *out = f;
  return LO_OK;
}

int lo_factors_flags(const lo_factors* f, unsigned* flags) {
  if (!f || !flags) return LO_EINVAL;
  *flags = f->diag_u_only ? 0u : (unsigned)LO_FACTORS_RANDOMIZED;
  return LO_OK;
}

int build_hr_eri(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar, lo_hr** out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, LO_EINVAL, "null output handle");
  *out = nullptr;
  if (M <= 0 || n_occ <= 0 || n_chol < 0) return fail(ctx, LO_EINVAL, "sizes must be M > 0, n_occ > 0, n_chol >= 0");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (M > 65535 || n_chol > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "M above 65535");
  if (n_chol > 0 && !lbar) return fail(ctx, LO_EINVAL, "null lbar");
  const int64_t npairs = n_occ * (n_occ + 1) / 2;
  int64_t elems = 0, bytes = 0;
  if (!mul_ok(npairs, M * M, &elems) || !mul_ok(elems, (int64_t)sizeof(double), &bytes))
    return fail(ctx, LO_EUNSUPPORTED, "pair blocks too large");
  lo_hr* h = new (std::nothrow) lo_hr();
  if (!h) return fail(ctx, LO_ENOMEM, "host allocation failed");
  h->M = M;
  h->n = n_occ;
  h->npairs = npairs;
  double* lbarT = nullptr;
  int64_t* d_bases = nullptr;
  auto release = [&]() {
    (void)hipFree(lbarT);
    (void)hipFree(d_bases);
  };
  auto fail_all = [&](int code, const char* what) {
    (void)hipStreamSynchronize(ctx->stream);
    release();
    lo_hr_destroy(h);
    return fail(ctx, code, "%s", what);
  };
  if (hipMalloc(&h->Y, (size_t)bytes) != hipSuccess) {
    h->Y = nullptr;
    return fail_all(LO_ENOMEM, "device allocation of the pair blocks failed");
  }
  std::vector<int> pairs(2 * npairs);
  std::vector<int64_t> bases(3 * npairs);
  for (int64_t i = 0, p = 0; i < n_occ; ++i) {
    for (int64_t j = i; j < n_occ; ++j, ++p) {
      pairs[2 * p] = (int)i;
      pairs[2 * p + 1] = (int)j;
      bases[3 * p] = i * n_chol * M;
      bases[3 * p + 1] = j * n_chol * M;
      bases[3 * p + 2] = p * M * M;
    }
  }
  int rc = upload(ctx, &h->d_pairs, pairs);
  if (rc) return fail_all(rc, "device allocation failed");
  rc = upload(ctx, &d_bases, bases);
  if (rc) return fail_all(rc, "device allocation failed");
  if (n_chol > 0) {
    if (hipMalloc(&lbarT, sizeof(double) * (size_t)n_occ * n_chol * M) != hipSuccess) {
      lbarT = nullptr;
      return fail_all(LO_ENOMEM, "device allocation of the transposed Cholesky vectors failed");
    }
    if (lofqmc::launch_lbar_transpose(ctx->stream, (int)M, (int)n_occ, n_chol, lbar, lbarT) != hipSuccess)
      return fail_all(LO_EHIP, "transpose launch failed");
  }
  // Y^[ij](r, s) = sum_g lbarT[i][g][r] lbarT[j][g][s], row-major; with no
  // Cholesky vectors the K loop is empty and the blocks are written as zeros
  for (int64_t p0 = 0; p0 < npairs; p0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, npairs - p0);
    if (lofqmc::launch_gemm_setup(ctx->stream, (int)M, (int)M, (int)n_chol, lbarT, 1, M, lbarT, M, 1, h->Y, M, 1,
                                  d_bases + 3 * p0, nb) != hipSuccess)
      return fail_all(LO_EHIP, "pair-block launch failed");
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail_all(LO_EHIP, "pair-block build failed");
  release();
  *out = h;
  return LO_OK;
}

int lo_hr_destroy(lo_hr* h) {
  if (!h) return LO_OK;
  (void)hipFree(h->Y);
  (void)hipFree(h->d_pairs);
  delete h;
  return LO_OK;
}

int lo_hr_info(const lo_hr* h, int64_t* M, int64_t* n_occ, int64_t* bytes) {
  if (!h) return LO_EINVAL;
  if (M) *M = h->M;
  if (n_occ) *n_occ = h->n;
  if (bytes) *bytes = h->npairs * h->M * h->M * (int64_t)sizeof(double);
  return LO_OK;
}

int local_energy_hr(lo_ctx* ctx, const lo_hr* h, int64_t nw, const double* theta, const int32_t* info,
                    unsigned flags, double* energy) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!h) return fail(ctx, LO_EINVAL, "null pair blocks");
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  if (flags & LO_THETA_TRANSPOSED) return fail(ctx, LO_EUNSUPPORTED, "the ERI route reads [nw][M][n] or [n][M][nw] theta");
  if (flags & ~(unsigned)LO_THETA_ORBITAL_MAJOR) return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (nw == 0) return LO_OK;
  if (!theta || !energy) return fail(ctx, LO_EINVAL, "null array");
  int64_t pbytes = 0;
  if (!mul_ok(h->npairs * (int64_t)sizeof(double) * 4, nw, &pbytes))
    return fail(ctx, LO_EUNSUPPORTED, "partial sums too large");
  int rc = ensure_ws(ctx, align256((size_t)pbytes));
  if (rc) return rc;
  double* partial = (double*)ctx->ws;
  ProfScope prof(ctx);
  prof.mark("hr_energy_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_hr_energy(ctx->stream, (int)h->M, (int)h->n, nw, (int)h->npairs, h->Y, h->d_pairs,
                                            theta, (flags & LO_THETA_ORBITAL_MAJOR) ? 1 : 0, partial));
  prof.mark("reduce_partials_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_reduce_partials(ctx->stream, nw, (int)h->npairs, partial, info, energy));
  return LO_OK;
}

// ------------------------------------------------- multi-determinant trials

int lo_md_destroy(lo_md* md) {
  if (!md) return LO_OK;
  (void)hipFree(md->rows);
  (void)hipFree(md->d_tpos);
  (void)hipFree(md->d_exc);
  (void)hipFree(md->d_holes);
  (void)hipFree(md->d_parts);
  (void)hipFree(md->d_coef);
  (void)hipFree(md->d_rowidx);
  (void)hipFree(md->d_tiles);
  (void)hipFree(md->d_pair);
  (void)hipFree(md->d_off);
  delete md;
  return LO_OK;
}

int build_md_trial(lo_ctx* ctx, const lo_factors* f, int64_t n_occ, int64_t n_act_occ, const double* orbitals,
                   int64_t n_det, int64_t max_exc, const int32_t* n_exc, const int32_t* holes,
                   const int32_t* particles, const double* coeffs, lo_md** out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, LO_EINVAL, "null output handle");
  *out = nullptr;
  if (!f) return fail(ctx, LO_EINVAL, "null factors");
  const int64_t M = f->M, ncas = f->n;
  if (n_occ <= 0 || n_occ > ncas) return fail(ctx, LO_EINVAL, "n_occ must be in 1..n_cas (the factors' orbitals)");
  const int64_t nav = ncas - n_occ;
  const int amax = lofqmc::md_max_active();
  if (n_act_occ <= 0 || n_act_occ > n_occ) return fail(ctx, LO_EINVAL, "n_act_occ must be in 1..n_occ");
  if (n_act_occ > amax || nav > amax)
    return fail(ctx, LO_EUNSUPPORTED, "more than %d active occupied or active virtual orbitals", amax);
  if (n_occ > kMaxOccTheta || ncas > lofqmc::md_max_orbitals())
    return fail(ctx, LO_EUNSUPPORTED, "n_occ above %d or n_cas above %d", kMaxOccTheta, lofqmc::md_max_orbitals());
  if (n_det <= 0 || n_det > (1 << 20)) return fail(ctx, LO_EINVAL, "n_det must be in 1..2^20");
  if (max_exc < 0 || max_exc > std::min(n_act_occ, nav))
    return fail(ctx, LO_EINVAL, "max_exc must be in 0..min(n_act_occ, n_cas - n_occ)");
  if (!orbitals || !n_exc || !coeffs || (max_exc > 0 && (!holes || !particles)))
    return fail(ctx, LO_EINVAL, "null array");
  const int na = (int)std::max(n_act_occ, nav);
  const int64_t act0 = n_occ - n_act_occ;
  std::vector<int> exc(n_det), hrel((size_t)n_det * na, 0), prel((size_t)n_det * na, 0);
  std::vector<double> coef(coeffs, coeffs + n_det);
  for (int64_t d = 0; d < n_det; ++d) {
    const int e = n_exc[d];
    if (e < 0 || e > max_exc) return fail(ctx, LO_EINVAL, "determinant %lld: excitation level out of range", (long long)d);
    exc[d] = e;
    unsigned hm = 0, pm = 0;
    for (int m = 0; m < e; ++m) {
      const int h = holes[d * max_exc + m], p = particles[d * max_exc + m];
      if (h < act0 || h >= n_occ || p < n_occ || p >= ncas)
        return fail(ctx, LO_EINVAL, "determinant %lld: hole or particle outside the active space", (long long)d);
      const unsigned hb = 1u << (h - act0), pb = 1u << (p - n_occ);
      if ((hm & hb) || (pm & pb)) return fail(ctx, LO_EINVAL, "determinant %lld: repeated hole or particle", (long long)d);
      hm |= hb;
      pm |= pb;
      hrel[d * na + m] = (int)(h - act0);
      prel[d * na + m] = (int)(p - n_occ);
    }
    if (!std::isfinite(coef[d])) return fail(ctx, LO_EINVAL, "non-finite coefficient");
  }
  // output rows of pass 1: each orbital o < n_occ's own rows (as in the
  // single-determinant tables, restricted to the reference's orbitals)
  // followed by the nav rows of C_av^T, whose products with theta_o are
  // T[v][o]; then every factor row once per active occupied column
  const int64_t total = f->total_rows;
  std::vector<int64_t> obase(n_occ + 1, 0), loc(n_occ * ncas, 0);
  std::vector<int> tpos(n_occ);
  for (int64_t o = 0; o < n_occ; ++o) {
    int64_t R = 0;
    for (int64_t k = 0; k < ncas; ++k) {
      loc[o * ncas + k] = R;
      R += 2 * (int64_t)f->ranks[o * ncas + k];
    }
    tpos[o] = (int)(obase[o] + R);
    obase[o + 1] = obase[o] + R + nav;
  }
  const int64_t act_base = obase[n_occ];
  const int64_t n_out = act_base + n_act_occ * total;
  if (n_out > std::numeric_limits<int>::max()) return fail(ctx, LO_EUNSUPPORTED, "too many factor rows");
  std::vector<int> rowidx((size_t)n_out);
  for (int64_t o = 0; o < n_occ; ++o) {
    for (int64_t k = 0; k < ncas; ++k) {
      const int64_t i = std::min(o, k), j = std::max(o, k);
      const int64_t src = f->row_offset[i * ncas + j];
      const int64_t cnt = 2 * (int64_t)f->ranks[o * ncas + k];
      for (int64_t q = 0; q < cnt; ++q) rowidx[obase[o] + loc[o * ncas + k] + q] = (int)(src + q);
    }
    for (int64_t v = 0; v < nav; ++v) rowidx[tpos[o] + v] = (int)(total + v);
  }
  for (int64_t a = 0; a < n_act_occ; ++a)
    for (int64_t r = 0; r < total; ++r) rowidx[act_base + a * total + r] = (int)r;
  // pass-1 tiles: own rows per orbital in blocks of lo_orbital_block()
  // orbitals; the active-column rows in tiles of the same size, eight
  // consecutive tiles (one active column) to a block
  const int64_t cap = lofqmc::lo_tile_rows();
  const int ob = lofqmc::lo_orbital_block();
  std::vector<int> t_orb, t_row0, t_nrows, blk;
  for (int64_t o = 0; o < n_occ; ++o) {
    if (o % ob == 0) blk.push_back((int)t_orb.size());
    const int64_t R = obase[o + 1] - obase[o];
    const int64_t nt = (R + cap - 1) / cap;
    for (int64_t q = 0; q < nt; ++q) {
      t_orb.push_back((int)o);
      t_row0.push_back((int)(obase[o] + R * q / nt));
      t_nrows.push_back((int)(R * (q + 1) / nt - R * q / nt));
    }
  }
  for (int64_t a = 0; a < n_act_occ; ++a) {
    const int64_t nt = (total + cap - 1) / cap;
    for (int64_t q = 0; q < nt; ++q) {
      if (q % 8 == 0) blk.push_back((int)t_orb.size());
      t_orb.push_back((int)(act0 + a));
      t_row0.push_back((int)(act_base + a * total + total * q / nt));
      t_nrows.push_back((int)(total * (q + 1) / nt - total * q / nt));
    }
  }
  const int ntiles = (int)t_orb.size();
  const int nblk = (int)blk.size();
  blk.push_back(ntiles);
  int tmax = 0;
  for (int b = 0; b < nblk; ++b) tmax = std::max(tmax, blk[b + 1] - blk[b]);
  std::vector<int> tiles;
  tiles.insert(tiles.end(), t_orb.begin(), t_orb.end());
  tiles.insert(tiles.end(), t_row0.begin(), t_row0.end());
  tiles.insert(tiles.end(), t_nrows.begin(), t_nrows.end());
  tiles.insert(tiles.end(), blk.begin(), blk.end());
  // pairs i <= j of all n_cas orbitals with a stored block
  std::vector<int> pi, pj, pK;
  std::vector<int64_t> offI, offJ, offA;
  for (int64_t i = 0; i < ncas; ++i)
    for (int64_t j = i; j < ncas; ++j) {
      const int K = f->ranks[i * ncas + j];
      if (K == 0) continue;
      pi.push_back((int)i);
      pj.push_back((int)j);
      pK.push_back(K);
      offI.push_back(i < n_occ ? obase[i] + loc[i * ncas + j] : -1);
      offJ.push_back(j < n_occ ? obase[j] + loc[j * ncas + i] : -1);
      offA.push_back(act_base + f->row_offset[i * ncas + j]);
    }
  lo_md* md = new (std::nothrow) lo_md();
  if (!md) return fail(ctx, LO_ENOMEM, "host allocation failed");
  md->M = M;
  md->n = n_occ;
  md->ncas = ncas;
  md->nao = n_act_occ;
  md->nav = nav;
  md->ndet = n_det;
  md->maxe = max_exc;
  md->na = na;
  md->n_out_rows = n_out;
  md->act_base = act_base;
  md->total_rows = total;
  md->ntiles = ntiles;
  md->nblk = nblk;
  md->tmax = tmax;
  md->npairs = (int)pi.size();
  std::vector<int> pair(pi);
  pair.insert(pair.end(), pj.begin(), pj.end());
  pair.insert(pair.end(), pK.begin(), pK.end());
  std::vector<int64_t> off(offI);
  off.insert(off.end(), offJ.begin(), offJ.end());
  off.insert(off.end(), offA.begin(), offA.end());
  int rc = 0;
  if ((rc = upload(ctx, &md->d_exc, exc)) || (rc = upload(ctx, &md->d_holes, hrel)) ||
      (rc = upload(ctx, &md->d_parts, prel)) || (rc = upload(ctx, &md->d_coef, coef)) ||
      (rc = upload(ctx, &md->d_rowidx, rowidx)) || (rc = upload(ctx, &md->d_tiles, tiles)) ||
      (rc = upload(ctx, &md->d_tpos, tpos)) ||
      (!pair.empty() && (rc = upload(ctx, &md->d_pair, pair))) || (!off.empty() && (rc = upload(ctx, &md->d_off, off)))) {
    lo_md_destroy(md);
    return rc;
  }
  // the pass-1 rows: the factor rows, then C_av^T (row v = orbital n_occ + v)
  std::vector<double> cav((size_t)nav * M);
  if (nav > 0) {
    std::vector<double> C((size_t)M * ncas);
    if (hipMemcpy(C.data(), orbitals, sizeof(double) * C.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      lo_md_destroy(md);
      return fail(ctx, LO_EHIP, "copy of the orbitals failed");
    }
    for (int64_t v = 0; v < nav; ++v)
      for (int64_t r = 0; r < M; ++r) cav[v * M + r] = C[r * ncas + n_occ + v];
  }
  if (total + nav > 0) {
    if (hipMalloc(&md->rows, sizeof(double) * (size_t)(total + nav) * M) != hipSuccess) {
      md->rows = nullptr;
      lo_md_destroy(md);
      return fail(ctx, LO_ENOMEM, "device allocation failed");
    }
    if ((total > 0 && hipMemcpyAsync(md->rows, f->rows, sizeof(double) * (size_t)total * M, hipMemcpyDeviceToDevice,
                                     ctx->stream) != hipSuccess) ||
        (nav > 0 && hipMemcpyAsync(md->rows + (size_t)total * M, cav.data(), sizeof(double) * cav.size(),
                                   hipMemcpyHostToDevice, ctx->stream) != hipSuccess) ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      lo_md_destroy(md);
      return fail(ctx, LO_EHIP, "copy of the factor rows failed");
    }
  }
  // the uploads read host vectors that end with this call
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    lo_md_destroy(md);
    return fail(ctx, LO_EHIP, "upload of the determinant tables failed");
  }
  *out = md;
  return LO_OK;
}

int lo_md_info(const lo_md* md, int64_t* n_occ, int64_t* n_cas, int64_t* n_det, int64_t* npairs,
               int64_t* out_rows) {
  if (!md) return LO_EINVAL;
  if (n_occ) *n_occ = md->n;
  if (n_cas) *n_cas = md->ncas;
  if (n_det) *n_det = md->ndet;
  if (npairs) *npairs = md->npairs;
  if (out_rows) *out_rows = md->n_out_rows;
  return LO_OK;
}

int local_energy_md(lo_ctx* ctx, const lo_md* md, int64_t nw, const double* theta, const int32_t* info,
                    unsigned flags, double* energy, double* ovlp_ratio) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!md) return fail(ctx, LO_EINVAL, "null trial");
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  // one 256-thread workgroup per walker: the grid's work-item count must fit 32 bits
  if (nw > ((int64_t)1 << 24)) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^24");
  if (flags & ~(unsigned)(LO_THETA_ORBITAL_MAJOR | LO_THETA_TRANSPOSED))
    return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (two_layouts(flags)) return fail(ctx, LO_EINVAL, "two theta layouts in flags");
  if (nw == 0) return LO_OK;
  if (!theta || !energy) return fail(ctx, LO_EINVAL, "null array");
  const int nchunk = lofqmc::md_pair_chunks(md->npairs);
  const size_t qbytes = align256(sizeof(double) * 2 * (size_t)md->n_out_rows * nw);
  const size_t mbytes = align256(lofqmc::md_walker_bytes(md->na, (int)md->n, (int)md->ncas) * (size_t)nw);
  const size_t pbytes = align256(sizeof(double) * 4 * (size_t)nchunk * nw);
  int rc = ensure_ws(ctx, qbytes + mbytes + pbytes);
  if (rc) return rc;
  char* base = (char*)ctx->ws;
  double* qbar = (double*)base;
  void* mwork = base + qbytes;
  double* partial = (double*)(base + qbytes + mbytes);
  lofqmc::MdArgs g{};
  g.M = (int)md->M;
  g.n = (int)md->n;
  g.ncas = (int)md->ncas;
  g.nao = (int)md->nao;
  g.nav = (int)md->nav;
  g.ndet = (int)md->ndet;
  g.hstride = md->na;
  g.npairs = md->npairs;
  g.nw = nw;
  g.act_stride = md->total_rows;
  g.n_out = md->n_out_rows;
  g.tpos = md->d_tpos;
  g.exc = md->d_exc;
  g.holes = md->d_holes;
  g.parts = md->d_parts;
  g.coef = md->d_coef;
  g.pi = md->d_pair;
  g.pj = md->d_pair + md->npairs;
  g.pK = md->d_pair + 2 * md->npairs;
  g.offI = md->d_off;
  g.offJ = md->d_off + md->npairs;
  g.offA = md->d_off + 2 * md->npairs;
  g.qbar = qbar;
  ProfScope prof(ctx);
  prof.mark(lofqmc::lo_pass1_name((int)md->M));
  HIP_OR_FAIL(ctx, lofqmc::launch_lo_pass1(ctx->stream, (int)md->M, (int)md->n, nw, md->ntiles, md->rows,
                                           md->total_rows + md->nav, md->d_rowidx, md->d_tiles, md->d_tiles + 3 * md->ntiles, md->nblk,
                                           md->tmax, theta, theta_layout_of(flags), qbar, md->n_out_rows));
  prof.mark("md_prep_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_md_prep(ctx->stream, g, mwork, ovlp_ratio));
  prof.mark("md_energy_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_md_pairs(ctx->stream, g, mwork, nchunk, partial));
  prof.mark("reduce_partials_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_reduce_partials(ctx->stream, nw, md->npairs > 0 ? nchunk : 0, partial, info,
                                                  energy));
  return LO_OK;
}

// ------------------------------------------------------------- per walker

int green_theta(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t nw, const double* trial, const double* phi,
                double* theta, double* log_ovlp, int32_t* info, unsigned flags) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (M <= 0 || n_occ <= 0 || nw < 0) return fail(ctx, LO_EINVAL, "sizes must be M > 0, n_occ > 0, nw >= 0");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (n_occ > kMaxOccTheta) return fail(ctx, LO_EUNSUPPORTED, "n_occ above %d", kMaxOccTheta);
  if (M > (1 << 24)) return fail(ctx, LO_EUNSUPPORTED, "M above 2^24");
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (flags & ~(unsigned)(LO_THETA_ORBITAL_MAJOR | LO_THETA_TRANSPOSED | LO_FLAG_SMALL_PIVOT))
    return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (two_layouts(flags)) return fail(ctx, LO_EINVAL, "two theta layouts in flags");
  if (nw == 0) return LO_OK;
  if (!trial || !phi || !theta || !info) return fail(ctx, LO_EINVAL, "null array");
  int rc = ensure_ws(ctx, align256(lofqmc::green_theta_workspace((int)n_occ, nw)));
  if (rc) return rc;
  ProfScope prof(ctx);
  HIP_OR_FAIL(ctx, lofqmc::launch_green_theta(ctx->stream, (int)M, (int)n_occ, nw, 0, nw, trial, phi, theta, log_ovlp,
                                              info, theta_layout_of(flags), (double*)ctx->ws,
                                              prof.get(), (flags & LO_FLAG_SMALL_PIVOT) ? 1 : 0));
  return LO_OK;
}

int local_energy_full(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, int64_t nw, const double* lbar,
                      const double* theta, const int32_t* info, int precision, unsigned flags, double* energy) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (M <= 0 || n_occ <= 0 || n_chol < 0 || nw < 0) return fail(ctx, LO_EINVAL, "bad sizes");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (precision != LO_FP64 && precision != LO_FP32 && precision != LO_BF16X3)
    return fail(ctx, LO_EINVAL, "unknown precision %d", precision);
  if (flags == LO_THETA_ORBITAL_MAJOR || flags == LO_THETA_TRANSPOSED)
    return fail(ctx, LO_EUNSUPPORTED, "the full route reads walker-major theta only");
  if (flags != 0) return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  const int max_occ = precision == LO_FP64 ? kMaxOccTheta : (precision == LO_FP32 ? kMaxOccWide : kMaxOcc);
  if (n_occ > max_occ) return fail(ctx, LO_EUNSUPPORTED, "n_occ above %d for this precision", max_occ);
  if (M > (1 << 24)) return fail(ctx, LO_EUNSUPPORTED, "M above 2^24");
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (precision != LO_FP64 && (n_chol > 65535 || nw > 65535))
    return fail(ctx, LO_EUNSUPPORTED, "reduced precision supports nw <= 65535 and n_chol <= 65535");
  if (nw == 0) return LO_OK;
  if ((n_chol > 0 && !lbar) || !theta || !energy) return fail(ctx, LO_EINVAL, "null array");
  // with no Cholesky vectors there are no chunks and the reduction writes zeros
  const int nchunk = n_chol > 0 ? lofqmc::full_num_chunks(n_chol, nw) : 0;
  // FP64: one row per (pass, chunk); reduced precision adds one chunk row for
  // the FP64 Coulomb sums
  const int nrows = precision == LO_FP64 ? nchunk * lofqmc::full_num_passes((int)n_occ)
                                         : (n_chol > 0 ? nchunk + 1 : nchunk);
  const size_t pbytes = align256(sizeof(double) * 4 * (size_t)std::max(nrows, 1) * nw);
  const size_t lbytes = (precision != LO_FP64 && n_chol > 0)
                            ? lofqmc::full_lp_workspace(precision, (int)M, (int)n_occ, n_chol, nw)
                            : 0;
  int rc = ensure_ws(ctx, pbytes + align256(lbytes));
  if (rc) return rc;
  double* partial = (double*)ctx->ws;
  ProfScope prof(ctx);
  if (n_chol > 0) {
    if (precision == LO_FP64) {
      prof.mark("energy_full_kernel");
      HIP_OR_FAIL(ctx, lofqmc::launch_energy_full(ctx->stream, (int)M, (int)n_occ, n_chol, nw, lbar, theta,
                                                  partial, nchunk));
    } else {
      HIP_OR_FAIL(ctx, lofqmc::launch_energy_full_lp(ctx->stream, precision, (int)M, (int)n_occ, n_chol, nw, lbar,
                                                     theta, (char*)ctx->ws + pbytes, partial, nchunk,
                                                     prof.get()));
    }
  }
  prof.mark("reduce_partials_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_reduce_partials(ctx->stream, nw, nrows, partial, info, energy));
  return LO_OK;
}

int local_energy_lo(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, const int32_t* info,
                    int precision, unsigned flags, const double* lbar, double* energy) {
  size_t need = 0;
  int rc = lo_energy_check(ctx, f, nw, theta, lbar, energy, precision, flags, &need);
  if (rc || nw == 0) return rc;
  rc = ensure_ws(ctx, need);
  if (rc) return rc;
  ProfScope prof(ctx);
  return lo_energy_enqueue(ctx, f, nw, theta, info, precision, flags, lbar, energy, (char*)ctx->ws, prof);
}

int local_energy_lo_noalloc(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, const int32_t* info,
                            int precision, unsigned flags, const double* lbar, double* energy) {
  size_t need = 0;
  int rc = lo_energy_check(ctx, f, nw, theta, lbar, energy, precision, flags, &need);
  if (rc || nw == 0) return rc;
  if (need > kNoAllocScratchBytes)
    return fail(ctx, LO_EUNSUPPORTED,
                "this batch needs %zu bytes of scratch, above the fixed %zu of local_energy_lo_noalloc "
                "(use fewer walkers per call)", need, kNoAllocScratchBytes);
  void* base = nullptr;
  rc = scratch_on_current_device(ctx, &base);
  if (rc) return rc;
  ProfScope prof(ctx, /*allow_record=*/false);
  return lo_energy_enqueue(ctx, f, nw, theta, info, precision, flags, lbar, energy, (char*)base, prof);
}

// ------------------------------------------------------ several systems

}  // extern "C"

struct lo_batch {
  int nsys = 0;
  std::vector<lo_system> sys;
  std::vector<int64_t> chunk, nchunk;
  int64_t nitems = 0;
  int grid = 0;
  int nbmax = 1;                            // largest orbital-block count of the systems
  void* mem = nullptr;                      // one device allocation for everything below
  std::vector<void*> lb, tb, cpart;         // per system
  std::vector<double*> gws;                 // per system: green_theta workspace (systems given phi)
  std::vector<double*> partial;             // per system [nchunk + 1][nw][4]
  lofqmc::LpSys* d_sys = nullptr;
  unsigned* d_counter = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void batch_free(lo_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  (void)hipFree(b->mem);
  delete b;
}

hipError_t batch_enqueue(lo_batch* b, hipStream_t st) {
  hipError_t e;
  // theta of the systems given their walkers (FP64 green_theta)
  for (int k = 0; k < b->nsys; ++k) {
    const lo_system& s = b->sys[k];
    if (!s.phi) continue;
    e = lofqmc::launch_green_theta(st, (int)s.M, (int)s.n_occ, s.nw, 0, s.nw, s.trial, s.phi, s.theta, nullptr,
                                   s.info, lofqmc::THETA_WALKER, b->gws[k], nullptr, 0);
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < b->nsys; ++k) {
    const lo_system& s = b->sys[k];
    e = lofqmc::launch_lp_convert_operands(st, LO_FP32, (int)s.M, (int)s.n_occ, s.n_chol, s.nw, s.lbar, s.theta,
                                           b->lb[k], b->tb[k]);
    if (e != hipSuccess) return e;
  }
  e = lofqmc::launch_exchange_batched(st, b->nsys, b->d_sys, b->nitems, b->d_counter, b->grid, b->nbmax);
  if (e != hipSuccess) return e;
  for (int k = 0; k < b->nsys; ++k) {
    const lo_system& s = b->sys[k];
    e = lofqmc::launch_coulomb_fp64(st, (int)s.M, (int)s.n_occ, s.n_chol, s.nw, s.theta, s.lbar, b->cpart[k],
                                    b->partial[k] + (size_t)b->nchunk[k] * s.nw * 4, nullptr);
    if (e != hipSuccess) return e;
    e = lofqmc::launch_reduce_partials(st, s.nw, (int)b->nchunk[k] + 1, b->partial[k], s.info, s.energy);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int lo_batch_create(lo_ctx* ctx, int nsys, const lo_system* sys, int precision, const int64_t* chunk,
                    lo_batch** out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!out || nsys <= 0 || !sys) return fail(ctx, LO_EINVAL, "need nsys > 0 systems and an output handle");
  if (precision != LO_FP32) return fail(ctx, LO_EUNSUPPORTED, "batched evaluation is LO_FP32 only");
  if (nsys > 4096) return fail(ctx, LO_EUNSUPPORTED, "more than 4096 systems");
  for (int k = 0; k < nsys; ++k) {
    const lo_system& s = sys[k];
    if (s.M <= 0 || s.n_occ <= 0 || s.n_chol <= 0 || s.nw <= 0 || s.n_occ > s.M)
      return fail(ctx, LO_EINVAL, "system %d: bad sizes", k);
    if (s.n_occ > kMaxOccWide || s.nw > 65535 || s.n_chol > 65535 || s.M > (1 << 20))
      return fail(ctx, LO_EUNSUPPORTED, "system %d: outside n_occ <= 96, nw, n_chol <= 65535", k);
    if (!s.lbar || !s.theta || !s.energy) return fail(ctx, LO_EINVAL, "system %d: null array", k);
    if (!s.trial != !s.phi) return fail(ctx, LO_EINVAL, "system %d: trial and phi go together", k);
    if (s.phi && !s.info) return fail(ctx, LO_EINVAL, "system %d: green_theta needs an info array", k);
  }
  int dev = 0, ncu = 0;
  HIP_OR_FAIL(ctx, hipGetDevice(&dev));
  HIP_OR_FAIL(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  lo_batch* b = new (std::nothrow) lo_batch();
  if (!b) return fail(ctx, LO_ENOMEM, "host allocation failed");
  b->nsys = nsys;
  b->sys.assign(sys, sys + nsys);
  b->grid = std::max(ncu, 1);
  // cost of one Cholesky vector for 4 walkers ~ Mp * NB^2; default chunks make
  // all items cost about total / (16 * grid)
  std::vector<double> unit(nsys);
  double total = 0.0;
  for (int k = 0; k < nsys; ++k) {
    const lo_system& s = b->sys[k];
    const double nb = lofqmc::lp_orbital_blocks((int)s.n_occ);
    unit[k] = (double)lofqmc::lp_padded_m((int)s.M) * nb * nb;
    total += unit[k] * (double)s.n_chol * (double)((s.nw + 3) / 4);
  }
  const double target = total / (16.0 * b->grid);
  b->chunk.resize(nsys);
  b->nchunk.resize(nsys);
  for (int k = 0; k < nsys; ++k) {
    const lo_system& s = b->sys[k];
    int64_t c = (chunk && chunk[k] > 0) ? chunk[k] : (int64_t)std::llround(target / unit[k]);
    c = std::min<int64_t>(std::max<int64_t>(c, 1), s.n_chol);
    b->chunk[k] = c;
    b->nchunk[k] = (s.n_chol + c - 1) / c;
  }
  // item order: systems by decreasing cost per item, so the largest items
  // are taken first by the persistent kernel
  std::vector<int> order(nsys);
  for (int k = 0; k < nsys; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return unit[a] * b->chunk[a] > unit[c] * b->chunk[c]; });
  // one allocation: per system lb, tb, cpart, partial; then the table and the counter
  std::vector<size_t> off_lb(nsys), off_tb(nsys), off_cp(nsys), off_pa(nsys), off_gw(nsys);
  size_t at = 0;
  for (int k = 0; k < nsys; ++k) {
    const lo_system& s = b->sys[k];
    off_gw[k] = at;
    if (s.phi) at += align256(lofqmc::green_theta_workspace((int)s.n_occ, s.nw));
    off_lb[k] = at;
    at += align256(lofqmc::lp_lbar_bytes(LO_FP32, (int)s.M, (int)s.n_occ, s.n_chol));
    off_tb[k] = at;
    at += align256(lofqmc::lp_theta_bytes(LO_FP32, (int)s.M, (int)s.n_occ, s.nw));
    off_cp[k] = at;
    at += align256(lofqmc::coulomb_cpart_bytes((int)s.M, (int)s.n_occ, s.n_chol, s.nw));
    off_pa[k] = at;
    at += align256(sizeof(double) * 4 * (size_t)(b->nchunk[k] + 1) * s.nw);
  }
  const size_t off_sys = at;
  at += align256(sizeof(lofqmc::LpSys) * nsys);
  const size_t off_cnt = at;
  at += 256;
  if (hipMalloc(&b->mem, at) != hipSuccess) {
    b->mem = nullptr;
    batch_free(b);
    return fail(ctx, LO_ENOMEM, "batch allocation of %zu bytes failed", at);
  }
  char* base = (char*)b->mem;
  b->lb.resize(nsys);
  b->tb.resize(nsys);
  b->cpart.resize(nsys);
  b->partial.resize(nsys);
  b->gws.assign(nsys, nullptr);
  for (int k = 0; k < nsys; ++k)
    if (b->sys[k].phi) b->gws[k] = (double*)(base + off_gw[k]);
  std::vector<lofqmc::LpSys> table(nsys);
  int64_t item = 0;
  for (int q = 0; q < nsys; ++q) {
    const int k = order[q];
    const lo_system& s = b->sys[k];
    b->lb[k] = base + off_lb[k];
    b->tb[k] = base + off_tb[k];
    b->cpart[k] = base + off_cp[k];
    b->partial[k] = (double*)(base + off_pa[k]);
    lofqmc::LpSys& d = table[q];
    d.Mp = lofqmc::lp_padded_m((int)s.M);
    d.nb = lofqmc::lp_orbital_blocks((int)s.n_occ);
    b->nbmax = std::max(b->nbmax, d.nb);
    d.X = s.n_chol;
    d.nw = s.nw;
    d.gchunk = b->chunk[k];
    d.nchunk = b->nchunk[k];
    d.item0 = item;
    d.lb = b->lb[k];
    d.tb = b->tb[k];
    d.partial = b->partial[k];
    item += d.nchunk * ((s.nw + 3) / 4);
  }
  b->nitems = item;
  if (b->nitems > ((int64_t)1 << 31)) {
    batch_free(b);
    return fail(ctx, LO_EUNSUPPORTED, "more than 2^31 work items");
  }
  b->d_sys = (lofqmc::LpSys*)(base + off_sys);
  b->d_counter = (unsigned*)(base + off_cnt);
  if (hipMemcpy(b->d_sys, table.data(), sizeof(lofqmc::LpSys) * nsys, hipMemcpyHostToDevice) != hipSuccess) {
    batch_free(b);
    return fail(ctx, LO_EHIP, "upload of the batch table failed");
  }
  *out = b;
  return LO_OK;
}

int lo_batch_destroy(lo_batch* b) {
  batch_free(b);
  return LO_OK;
}

int lo_batch_info(const lo_batch* b, int64_t* nitems, int64_t* chunk) {
  if (!b) return LO_EINVAL;
  if (nitems) *nitems = b->nitems;
  if (chunk) std::memcpy(chunk, b->chunk.data(), sizeof(int64_t) * b->nsys);
  return LO_OK;
}

int lo_batch_execute(lo_ctx* ctx, lo_batch* b) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!b) return fail(ctx, LO_EINVAL, "null batch");
  ProfScope prof(ctx);
  prof.mark("batch_evaluation");
  HIP_OR_FAIL(ctx, batch_enqueue(b, ctx->stream));
  return LO_OK;
}

int lo_batch_capture(lo_ctx* ctx, lo_batch* b, int repeats) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!b || repeats <= 0) return fail(ctx, LO_EINVAL, "need a batch and repeats > 0");
  if (b->exec) {
    HIP_OR_FAIL(ctx, hipGraphExecDestroy(b->exec));
    b->exec = nullptr;
  }
  if (b->graph) {
    HIP_OR_FAIL(ctx, hipGraphDestroy(b->graph));
    b->graph = nullptr;
  }
  if (!b->cap) HIP_OR_FAIL(ctx, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  // everything queued before capture must be complete: the capture stream
  // does not order against the context stream
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int r = 0; r < repeats && e == hipSuccess; ++r) e = batch_enqueue(b, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(ctx, LO_EHIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  b->graph = g;
  HIP_OR_FAIL(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return LO_OK;
}

int lo_batch_replay(lo_ctx* ctx, lo_batch* b) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!b || !b->exec) return fail(ctx, LO_EINVAL, "no captured graph");
  ProfScope prof(ctx);
  prof.mark("batch_graph");
  HIP_OR_FAIL(ctx, hipGraphLaunch(b->exec, ctx->stream));
  return LO_OK;
}

// ------------------------------------------------------ learned residual

int lo_residual_nparam(void) { return lofqmc::residual_nparam(); }

int lo_factors_discarded(const lo_factors* f, double* mass) {
  if (!f || !mass) return LO_EINVAL;
  std::memcpy(mass, f->discarded.data(), sizeof(double) * f->discarded.size());
  return LO_OK;
}

int lo_residual_features(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, float* x) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!f) return fail(ctx, LO_EINVAL, "null factors");
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  if (nw == 0) return LO_OK;
  if (!theta || !x) return fail(ctx, LO_EINVAL, "null array");
  if (!f->d_orbfeat) return fail(ctx, LO_EINVAL, "factors hold no orbital table");
  if (!f->d_grad) return fail(ctx, LO_EINVAL, "lo_residual_prepare has not been called for these factors");
  ProfScope prof(ctx);
  prof.mark("residual_features_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_residual_features(ctx->stream, (int)f->M, (int)f->n, nw, theta, f->d_orbfeat,
                                                    f->d_grad, x));
  return LO_OK;
}

int lo_residual_target(lo_ctx* ctx, int64_t nw, const double* e_exact, const double* e_lo, double shift, double scale,
                       double* t) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  if (!(scale != 0.0) || !std::isfinite(scale) || !std::isfinite(shift))
    return fail(ctx, LO_EINVAL, "scale must be finite and non-zero, shift finite");
  if (nw == 0) return LO_OK;
  if (!e_exact || !e_lo || !t) return fail(ctx, LO_EINVAL, "null array");
  HIP_OR_FAIL(ctx, lofqmc::launch_residual_target(ctx->stream, nw, e_exact, e_lo, shift, scale, t));
  return LO_OK;
}

int lo_residual_apply(lo_ctx* ctx, int64_t nw, const double* energy, const double* pred, double scale, double shift,
                      double* out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  if (!std::isfinite(scale) || !std::isfinite(shift)) return fail(ctx, LO_EINVAL, "scale and shift must be finite");
  if (nw == 0) return LO_OK;
  if (!energy || !out) return fail(ctx, LO_EINVAL, "null array");
  HIP_OR_FAIL(ctx, lofqmc::launch_residual_apply(ctx->stream, nw, energy, pred, scale, shift, out));
  return LO_OK;
}

int lo_residual_prepare(lo_ctx* ctx, lo_factors* f, int64_t n_chol, const double* lbar, const double* trial,
                        double* grad_out) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!f) return fail(ctx, LO_EINVAL, "null factors");
  if (n_chol < 0) return fail(ctx, LO_EINVAL, "n_chol < 0");
  if ((n_chol > 0 && !lbar) || !trial) return fail(ctx, LO_EINVAL, "null array");
  const int64_t M = f->M, n = f->n;
  // host tables: the pair of every stored row, first row and rank of every pair a <= b
  std::vector<int> pair_of_row(2 * (size_t)f->total_rows, 0);
  std::vector<int64_t> pair_off(n * n, 0);
  std::vector<int> pair_k(n * n, 0);
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = a; b < n; ++b) {
      const int64_t off = f->row_offset[a * n + b];
      const int K = f->ranks[a * n + b];
      pair_off[a * n + b] = off;
      pair_k[a * n + b] = K;
      for (int64_t k = 0; k < 2 * (int64_t)K; ++k) {
        pair_of_row[2 * (off + k)] = (int)a;
        pair_of_row[2 * (off + k) + 1] = (int)b;
      }
    }
  if (!f->d_grad && hipMalloc(&f->d_grad, sizeof(double) * (size_t)(M * n)) != hipSuccess) {
    f->d_grad = nullptr;
    return fail(ctx, LO_ENOMEM, "gradient allocation failed");
  }
  int rc = ensure_ws(ctx, lofqmc::residual_gradient_workspace((int)n, n_chol, f->total_rows));
  if (rc) return rc;
  int* d_por = nullptr;
  int64_t* d_off = nullptr;
  int* d_k = nullptr;
  if ((rc = upload(ctx, &d_por, pair_of_row)) || (rc = upload(ctx, &d_off, pair_off)) ||
      (rc = upload(ctx, &d_k, pair_k))) {
    (void)hipFree(d_por);
    (void)hipFree(d_off);
    (void)hipFree(d_k);
    return rc;
  }
  hipError_t e = lofqmc::launch_residual_gradient(ctx->stream, (int)M, (int)n, n_chol, lbar, trial, f->total_rows,
                                                  f->rows, d_por, d_off, d_k, ctx->ws, f->d_grad);
  if (e == hipSuccess && grad_out)
    e = hipMemcpyAsync(grad_out, f->d_grad, sizeof(double) * (size_t)(M * n), hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(d_por);
  (void)hipFree(d_off);
  (void)hipFree(d_k);
  if (e != hipSuccess) return fail(ctx, LO_EHIP, "residual gradient: %s", hipGetErrorString(e));
  return LO_OK;
}

int lo_residual_predict(lo_ctx* ctx, int64_t nw, int64_t n_occ, const float* params, const float* x, int precision,
                        double* pred) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (nw < 0 || n_occ <= 0) return fail(ctx, LO_EINVAL, "bad sizes");
  if (precision != LO_FP32 && precision != LO_BF16) return fail(ctx, LO_EINVAL, "precision must be FP32 or BF16");
  if (nw * n_occ > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw * n_occ above 2^31-1");
  if (nw == 0) return LO_OK;
  if (!params || !x || !pred) return fail(ctx, LO_EINVAL, "null array");
  const int bf = precision == LO_BF16 ? 1 : 0;
  int rc = ensure_ws(ctx, lofqmc::residual_predict_workspace(bf, nw, (int)n_occ));
  if (rc) return rc;
  ProfScope prof(ctx);
  prof.mark(bf ? "residual_infer_bf16_kernel" : "residual_forward_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_residual_predict(ctx->stream, bf, nw, (int)n_occ, params, x, ctx->ws, pred));
  return LO_OK;
}

int lo_residual_train_step(lo_ctx* ctx, int64_t nw, int64_t n_occ, float* params, float* adam_m, float* adam_v,
                           int64_t step, double lr, const float* x, const double* target, float* grad, double* loss,
                           double* pred) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (nw < 0 || n_occ <= 0 || step < 0) return fail(ctx, LO_EINVAL, "bad sizes or step");
  if (!(lr >= 0.0)) return fail(ctx, LO_EINVAL, "lr must be >= 0");
  if (nw * n_occ > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw * n_occ above 2^31-1");
  if (nw == 0) return LO_OK;
  if (!params || !x || !target || (step > 0 && (!adam_m || !adam_v))) return fail(ctx, LO_EINVAL, "null array");
  int rc = ensure_ws(ctx, lofqmc::residual_train_workspace(nw, (int)n_occ));
  if (rc) return rc;
  ProfScope prof(ctx);
  prof.mark("residual_train_step");
  HIP_OR_FAIL(ctx, lofqmc::launch_residual_train_step(ctx->stream, nw, (int)n_occ, params, adam_m, adam_v, step,
                                                      (float)lr, x, target, ctx->ws, grad, loss, pred));
  return LO_OK;
}

}  // extern "C"
