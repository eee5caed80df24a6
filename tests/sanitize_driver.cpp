// Host-side argument validation of liblofqmc under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py with the
// sanitizers on the host code only).  Runs on a host without a GPU: every
// call below must fail its checks before touching the device.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "lofqmc.h"

static int failures = 0;
#define EXPECT(call, code)                                                                        \
  do {                                                                                            \
    const int rc_ = (call);                                                                       \
    if (rc_ != (code)) {                                                                          \
      std::printf("FAIL %s: got %d, want %d\n", #call, rc_, (int)(code));                         \
      ++failures;                                                                                 \
    }                                                                                             \
  } while (0)

int main() {
  lo_ctx* h = nullptr;
  EXPECT(lo_create(&h, nullptr), LO_OK);
  EXPECT(lo_create(nullptr, nullptr), LO_EINVAL);
  double* fake = reinterpret_cast<double*>(0x1000);   // never dereferenced
  int32_t* ifake = reinterpret_cast<int32_t*>(0x1000);
  lo_factors* out = nullptr;
  EXPECT(green_theta(h, 0, 2, 1, fake, fake, fake, nullptr, ifake, 0), LO_EINVAL);
  EXPECT(green_theta(h, 200, 113, 1, fake, fake, fake, nullptr, ifake, 0), LO_EUNSUPPORTED);
  EXPECT(green_theta(h, 8, 2, 3, fake, fake, fake, nullptr, ifake, 2), LO_EINVAL);
  EXPECT(local_energy_full(h, 200, 113, 3, 4, fake, fake, nullptr, LO_FP64, 0, fake), LO_EUNSUPPORTED);
  EXPECT(local_energy_full(h, 8, 2, 3, 4, fake, fake, nullptr, 7, 0, fake), LO_EINVAL);
  EXPECT(local_energy_lo(h, nullptr, 4, fake, nullptr, LO_FP64, 0, nullptr, fake), LO_EINVAL);
  EXPECT(local_energy_lo_noalloc(h, nullptr, 4, fake, nullptr, LO_FP64, 0, nullptr, fake), LO_EINVAL);
  EXPECT(build_lo_factors(h, 8, 2, 3, fake, -1.0, &out), LO_EINVAL);
  EXPECT(build_lo_factors(h, 8, 2, 3, fake, NAN, &out), LO_EINVAL);
  EXPECT(build_lo_factors(h, 8, 9, 3, fake, 1e-4, &out), LO_EINVAL);
  // factor import: the tiling of the rows by the pairs' offsets
  const int32_t rk[4] = {1, 0, 0, 1}, rk_asym[4] = {1, 1, 0, 1};
  const int64_t ro[4] = {0, -1, -1, 2}, ro_bad[4] = {0, -1, -1, 3}, ro_neg[4] = {-5, -1, -1, 2};
  EXPECT(lo_factors_import(h, 8, 2, 3, rk, ro_bad, nullptr, nullptr, fake, 0, &out), LO_EINVAL);
  EXPECT(lo_factors_import(h, 8, 2, 3, rk, ro_neg, nullptr, nullptr, fake, 0, &out), LO_EINVAL);
  EXPECT(lo_factors_import(h, 8, 2, 3, rk_asym, ro, nullptr, nullptr, fake, 0, &out), LO_EINVAL);
  EXPECT(lo_factors_import(h, 8, 2, 3, rk, ro, nullptr, nullptr, nullptr, 0, &out), LO_EINVAL);
  // localization, learned residual, multi-determinant and HR-ERI checks
  EXPECT(lo_localize_boys(h, 10, 11, 1, fake, fake, 5, 1e-12, nullptr), LO_EINVAL);
  EXPECT(lo_localize_boys(h, 200, 72, 3, fake, fake, 5, 1e-12, nullptr), LO_EUNSUPPORTED);
  EXPECT(lo_residual_target(h, 4, fake, fake, 0.0, 0.0, fake), LO_EINVAL);
  EXPECT(lo_residual_apply(h, 4, nullptr, nullptr, 1.0, 0.0, fake), LO_EINVAL);
  EXPECT(lo_residual_prepare(h, nullptr, 3, fake, fake, nullptr), LO_EINVAL);
  EXPECT(build_hr_eri(h, 70000, 2, 3, fake, reinterpret_cast<lo_hr**>(&out)), LO_EUNSUPPORTED);
  EXPECT(local_energy_md(h, nullptr, 4, fake, nullptr, 0, fake, nullptr), LO_EINVAL);
  EXPECT(lo_batch_create(h, 0, nullptr, LO_FP32, nullptr, nullptr), LO_EINVAL);
  // the error text of the last failure is a valid string
  std::printf("last error: %s\n", lo_last_error(h));
  EXPECT(lo_destroy(h), LO_OK);
  EXPECT(lo_destroy(nullptr), LO_OK);
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
  return failures ? 1 : 0;
}
