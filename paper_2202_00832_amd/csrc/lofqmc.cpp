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
  int64_t M = 0, n = 0, total_rows = 0, n_out_rows = 0;
  double* rows = nullptr;  // device [total_rows][M]
  std::vector<int32_t> ranks;          // [n][n]
  std::vector<double> first_dropped;   // [n][n]
  std::vector<int64_t> row_offset;     // [n][n], -1 for i > j
  int ntiles = 0, npairs = 0, nblk = 0, tmax = 0;
  int* d_rowidx = nullptr;             // [n_out_rows]
  int* d_tiles = nullptr;              // [3][ntiles]: orbital, first output row, row count;
                                       // then [nblk + 1]: first tile of each orbital block
  int* d_pK = nullptr;                 // [npairs]
  int64_t* d_off = nullptr;            // [2][npairs]: output rows of the pair for orbital i and j
  double* d_pw = nullptr;              // [npairs]
};

namespace {

constexpr int kMaxOcc = 64;

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
  (void)hipFree(f->d_rowidx);
  (void)hipFree(f->d_tiles);
  (void)hipFree(f->d_pK);
  (void)hipFree(f->d_off);
  (void)hipFree(f->d_pw);
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
struct ProfScope {
  lo_ctx* c;
  lofqmc::ProfHook hook;
  explicit ProfScope(lo_ctx* ctx) : c(ctx), hook{ctx, ctx->prof_on ? prof_record : nullptr} {}
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

int build_lo_factors(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, const double* lbar, double epsilon,
                     lo_factors** out) {
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

  f = new lo_factors();
  f->M = M;
  f->n = n;
  f->ranks.assign(n * n, 0);
  f->first_dropped.assign(n * n, 0.0);
  f->row_offset.assign(n * n, -1);

  std::vector<std::pair<int, int>> plist;
  plist.reserve(npairs);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) plist.emplace_back(i, j);

  std::vector<double> S_host(M * batch);
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
    rocblas_status st = rocsolver_dgesvd_strided_batched(
        ctx->blas, rocblas_svect_singular, rocblas_svect_singular, (rocblas_int)M, (rocblas_int)M, d_Y,
        (rocblas_int)M, (rocblas_stride)mm, d_S, (rocblas_stride)M, d_U, (rocblas_int)M, (rocblas_stride)mm, d_VT,
        (rocblas_int)M, (rocblas_stride)mm, d_E, (rocblas_stride)M, rocblas_outofplace, d_info, nb);
    if (st != rocblas_status_success) {
      rc = fail(ctx, LO_ESOLVER, "rocsolver_dgesvd_strided_batched returned %d", (int)st);
      cleanup();
      free_factors(f);
      return rc;
    }
    TRY_HIP(hipMemcpyAsync(S_host.data(), d_S, sizeof(double) * M * nb, hipMemcpyDeviceToHost, ctx->stream));
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
      const double* s = S_host.data() + (size_t)b * M;
      int K = 0;
      if (epsilon == 0.0) {
        K = (int)M;
      } else {
        while (K < M && s[K] >= epsilon) ++K;
      }
      const auto [i, j] = plist[p0 + b];
      f->ranks[i * n + j] = f->ranks[j * n + i] = K;
      const double fd = (K < M) ? s[K] : 0.0;
      f->first_dropped[i * n + j] = f->first_dropped[j * n + i] = fd;
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
      TRY_HIP(lofqmc::launch_pack_factors(ctx->stream, (int)M, nb, d_U, d_VT, d_S, d_K, d_roff, dst));
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

  // ---- tables of the two energy passes
  std::vector<int64_t> obase(n + 1, 0);
  std::vector<int64_t> loc(n * n, 0);  // local output row of pair (o, k) within orbital o
  for (int o = 0; o < n; ++o) {
    int64_t R = 0;
    for (int k = 0; k < n; ++k) {
      loc[o * n + k] = R;
      R += 2 * (int64_t)f->ranks[o * n + k];
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
  std::vector<int> t_orb, t_row0, t_nrows;
  for (int o = 0; o < n; ++o) {
    for (int k = 0; k < n; ++k) {
      const int i = std::min(o, k), j = std::max(o, k);
      const int64_t src = f->row_offset[i * n + j];
      const int64_t cnt = 2 * (int64_t)f->ranks[o * n + k];
      for (int64_t q = 0; q < cnt; ++q) rowidx[obase[o] + loc[o * n + k] + q] = (int)(src + q);
    }
    // split the orbital's rows into near-equal tiles of at most lo_tile_rows()
    const int64_t R = obase[o + 1] - obase[o];
    const int64_t cap = lofqmc::lo_tile_rows();
    const int64_t ntile = (R + cap - 1) / cap;
    for (int64_t q = 0; q < ntile; ++q) {
      const int64_t a = obase[o] + R * q / ntile, b = obase[o] + R * (q + 1) / ntile;
      t_orb.push_back(o);
      t_row0.push_back((int)a);
      t_nrows.push_back((int)(b - a));
    }
  }
  f->ntiles = (int)t_orb.size();
  std::vector<int> tiles;
  tiles.insert(tiles.end(), t_orb.begin(), t_orb.end());
  tiles.insert(tiles.end(), t_row0.begin(), t_row0.end());
  tiles.insert(tiles.end(), t_nrows.begin(), t_nrows.end());
  // orbital blocks of pass 1: first tile of each block (tiles are sorted by orbital)
  const int ob = lofqmc::lo_orbital_block();
  f->nblk = (int)((n + ob - 1) / ob);
  {
    std::vector<int> blk(f->nblk + 1, f->ntiles);
    int t = 0;
    for (int b = 0; b < f->nblk; ++b) {
      while (t < f->ntiles && t_orb[t] < b * ob) ++t;
      blk[b] = t;
    }
    f->tmax = 0;
    for (int b = 0; b < f->nblk; ++b) f->tmax = std::max(f->tmax, blk[b + 1] - blk[b]);
    tiles.insert(tiles.end(), blk.begin(), blk.end());
  }
  std::vector<int> pK;
  std::vector<int64_t> off;
  std::vector<double> pw;
  std::vector<int64_t> offJ;
  for (int i = 0; i < n; ++i) {
    for (int j = i; j < n; ++j) {
      const int K = f->ranks[i * n + j];
      if (K == 0) continue;
      pK.push_back(K);
      off.push_back(obase[i] + loc[i * n + j]);
      offJ.push_back(obase[j] + loc[j * n + i]);
      pw.push_back(i == j ? 1.0 : 2.0);
    }
  }
  f->npairs = (int)pK.size();
  off.insert(off.end(), offJ.begin(), offJ.end());
  if ((rc = upload(ctx, &f->d_rowidx, rowidx)) || (rc = upload(ctx, &f->d_tiles, tiles)) ||
      (rc = upload(ctx, &f->d_pK, pK)) || (rc = upload(ctx, &f->d_off, off)) || (rc = upload(ctx, &f->d_pw, pw))) {
    cleanup();
    free_factors(f);
    return rc;
  }
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  cleanup();
  *out = f;
  return LO_OK;
#undef TRY_HIP
#undef TRY_ALLOC
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

// ------------------------------------------------------------- per walker

int green_theta(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t nw, const double* trial, const double* phi,
                double* theta, double* log_ovlp, int32_t* info, unsigned flags) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (M <= 0 || n_occ <= 0 || nw < 0) return fail(ctx, LO_EINVAL, "sizes must be M > 0, n_occ > 0, nw >= 0");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (n_occ > kMaxOcc) return fail(ctx, LO_EUNSUPPORTED, "n_occ above %d", kMaxOcc);
  if (M > (1 << 24)) return fail(ctx, LO_EUNSUPPORTED, "M above 2^24");
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (flags & ~(unsigned)LO_THETA_ORBITAL_MAJOR) return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (nw == 0) return LO_OK;
  if (!trial || !phi || !theta || !info) return fail(ctx, LO_EINVAL, "null array");
  int rc = ensure_ws(ctx, align256(lofqmc::green_theta_workspace((int)n_occ, nw)));
  if (rc) return rc;
  ProfScope prof(ctx);
  HIP_OR_FAIL(ctx, lofqmc::launch_green_theta(ctx->stream, (int)M, (int)n_occ, nw, trial, phi, theta, log_ovlp,
                                              info, (flags & LO_THETA_ORBITAL_MAJOR) ? 1 : 0, (double*)ctx->ws,
                                              prof.get()));
  return LO_OK;
}

int local_energy_full(lo_ctx* ctx, int64_t M, int64_t n_occ, int64_t n_chol, int64_t nw, const double* lbar,
                      const double* theta, const int32_t* info, int precision, unsigned flags, double* energy) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (M <= 0 || n_occ <= 0 || n_chol < 0 || nw < 0) return fail(ctx, LO_EINVAL, "bad sizes");
  if (n_occ > M) return fail(ctx, LO_EINVAL, "n_occ exceeds M");
  if (precision != LO_FP64) return fail(ctx, LO_EUNSUPPORTED, "precision %d not implemented", precision);
  if (flags != 0) return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (n_occ > kMaxOcc) return fail(ctx, LO_EUNSUPPORTED, "n_occ above %d", kMaxOcc);
  if (M > (1 << 24)) return fail(ctx, LO_EUNSUPPORTED, "M above 2^24");
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (nw == 0) return LO_OK;
  if ((n_chol > 0 && !lbar) || !theta || !energy) return fail(ctx, LO_EINVAL, "null array");
  // with no Cholesky vectors there are no chunks and the reduction writes zeros
  const int nchunk = n_chol > 0 ? lofqmc::full_num_chunks(n_chol, nw) : 0;
  const size_t pbytes = align256(sizeof(double) * 4 * (size_t)std::max(nchunk, 1) * nw);
  int rc = ensure_ws(ctx, pbytes);
  if (rc) return rc;
  double* partial = (double*)ctx->ws;
  ProfScope prof(ctx);
  if (n_chol > 0) {
    prof.mark("energy_full_kernel");
    HIP_OR_FAIL(ctx, lofqmc::launch_energy_full(ctx->stream, (int)M, (int)n_occ, n_chol, nw, lbar, theta, partial,
                                                nchunk));
  }
  prof.mark("reduce_partials_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_reduce_partials(ctx->stream, nw, nchunk, partial, info, energy));
  return LO_OK;
}

int local_energy_lo(lo_ctx* ctx, const lo_factors* f, int64_t nw, const double* theta, const int32_t* info,
                    int precision, unsigned flags, double* energy) {
  if (!ctx) return LO_EINVAL;
  ctx->err.clear();
  if (!f) return fail(ctx, LO_EINVAL, "null factors");
  if (nw < 0) return fail(ctx, LO_EINVAL, "nw < 0");
  if (precision != LO_FP64) return fail(ctx, LO_EUNSUPPORTED, "precision %d not implemented", precision);
  if (flags & ~(unsigned)LO_THETA_ORBITAL_MAJOR) return fail(ctx, LO_EINVAL, "unknown flags 0x%x", flags);
  if (nw > ((int64_t)1 << 31) - 1) return fail(ctx, LO_EUNSUPPORTED, "nw above 2^31-1");
  if (nw == 0) return LO_OK;
  if (!theta || !energy) return fail(ctx, LO_EINVAL, "null array");
  const bool orbital_major = (flags & LO_THETA_ORBITAL_MAJOR) != 0;
  const int64_t M = f->M, n = f->n;
  const int nchunk = lofqmc::lo_pass2_chunks(f->npairs);
  const size_t qbytes = align256(sizeof(double) * 2 * (size_t)f->n_out_rows * nw);
  const size_t pbytes = align256(sizeof(double) * 4 * (size_t)nchunk * nw);
  int rc = ensure_ws(ctx, qbytes + pbytes);
  if (rc) return rc;
  char* base = (char*)ctx->ws;
  double* qbar = (double*)base;
  double* partial = (double*)(base + qbytes);
  ProfScope prof(ctx);
  prof.mark("lo_pass1_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_lo_pass1(ctx->stream, (int)M, (int)n, nw, f->ntiles, f->rows, f->d_rowidx,
                                           f->d_tiles, f->d_tiles + 3 * f->ntiles, f->nblk, f->tmax, theta,
                                           orbital_major ? 1 : 0, qbar));
  prof.mark("lo_pass2_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_lo_pass2(ctx->stream, nw, f->npairs, nchunk, f->d_pK, f->d_off,
                                           f->d_off + f->npairs, f->d_pw, qbar, partial));
  prof.mark("reduce_partials_kernel");
  HIP_OR_FAIL(ctx, lofqmc::launch_reduce_partials(ctx->stream, nw, nchunk, partial, info, energy));
  return LO_OK;
}

}  // extern "C"
