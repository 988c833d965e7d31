// abi_sanitize.cpp -- drives the host-side argument validation of every entry
// point of include/lyaf.h with invalid and empty arguments, for a build of the
// library's host code with AddressSanitizer and UndefinedBehaviorSanitizer.
// Every call here must return before any HIP call (no GPU is needed); the
// program exits non-zero on the first unexpected return code.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "lyaf.h"

#define EXPECT(call, code)                                                         \
  do {                                                                             \
    const int rc_ = (call);                                                        \
    if (rc_ != (code)) {                                                           \
      fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, rc_, \
              (int)(code));                                                        \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

int main() {
  // fake device addresses: never dereferenced on the host, and every call
  // below is rejected (or is empty) before anything is enqueued
  float *fp = reinterpret_cast<float *>(uintptr_t(0x1000));
  double *dp = reinterpret_cast<double *>(uintptr_t(0x2000));
  int64_t *ip = reinterpret_cast<int64_t *>(uintptr_t(0x3000));
  std::vector<int64_t> off = {0, 16, 40, 40};
  lyaf_skewers sk{3, off.data(), fp, fp, fp, fp, fp};
  lyaf_params prm{1.0, 10.0, 6.0, 0u};

  EXPECT(lyaf_tau(nullptr, &prm, fp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_tau(&sk, nullptr, fp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_tau(&sk, &prm, nullptr, nullptr), LYAF_EINVAL);
  for (double bad : {0.0, -1.0, (double)NAN, (double)INFINITY}) {
    lyaf_params q = prm;
    q.tau_ref = bad;
    EXPECT(lyaf_tau(&sk, &q, fp, nullptr), LYAF_EINVAL);
  }
  {
    lyaf_params q = prm;
    q.window_k = -1.0;
    EXPECT(lyaf_tau(&sk, &q, fp, nullptr), LYAF_EINVAL);
    q = prm;
    q.delta_pivot = 0.0;
    EXPECT(lyaf_tau(&sk, &q, fp, nullptr), LYAF_EINVAL);
    q = prm;
    q.flags = 1u << 20;
    EXPECT(lyaf_tau(&sk, &q, fp, nullptr), LYAF_EINVAL);
    q = prm;
    q.flags = LYAF_FLAG_SHAPE(LYAF_NUM_SHAPES);
    EXPECT(lyaf_tau(&sk, &q, fp, nullptr), LYAF_EINVAL);
  }
  {
    std::vector<int64_t> o = {1, 16, 40, 40};  // offsets[0] != 0
    lyaf_skewers b = sk;
    b.offsets = o.data();
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    o = {0, 16, 8, 40};  // decreasing
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    o = {0, 16, 16 + (int64_t(1) << 24) + 1, 16 + (int64_t(1) << 24) + 1};  // N > 2^24
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    b = sk;
    b.n_skewers = -1;
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    b = sk;
    b.offsets = nullptr;
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    b = sk;
    b.delta = nullptr;
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    b = sk;
    b.gamma = nullptr;
    EXPECT(lyaf_tau(&b, &prm, fp, nullptr), LYAF_EINVAL);
    std::vector<int64_t> z = {0, 0, 0};  // empty batch: nothing to do
    lyaf_skewers e{2, z.data(), nullptr, nullptr, fp, fp, fp};
    EXPECT(lyaf_tau(&e, &prm, nullptr, nullptr), LYAF_OK);
  }
  EXPECT(lyaf_normalise_mean_flux(-1, fp, fp, 0.8, dp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_normalise_mean_flux(10, nullptr, fp, 0.8, dp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_normalise_mean_flux(10, fp, fp, 0.8, dp, nullptr), LYAF_EINVAL);  // aliasing
  for (double F : {0.0, 1.0, -0.1, (double)NAN})
    EXPECT(lyaf_normalise_mean_flux(10, fp, fp + 64, F, dp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_normalise_mean_flux(10, fp, fp + 64, 0.8, nullptr, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_normalise_mean_flux_backward(-1, fp, dp, fp, fp, 1, fp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_normalise_mean_flux_backward(0, nullptr, nullptr, nullptr, nullptr, 1, nullptr,
                                           nullptr),
         LYAF_OK);
  EXPECT(lyaf_normalise_mean_flux_backward(10, nullptr, dp, fp, fp, 1, fp, nullptr),
         LYAF_EINVAL);
  EXPECT(lyaf_tau_backward(&sk, &prm, nullptr, fp, fp, dp, dp, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_tau_backward(nullptr, &prm, fp, fp, fp, dp, dp, nullptr), LYAF_EINVAL);
  lyaf_plan *plan = nullptr;
  EXPECT(lyaf_plan_create(&sk, &prm, 0.8, fp, fp, dp, 0u, nullptr, &plan), LYAF_EINVAL);
  EXPECT(lyaf_plan_create(&sk, &prm, 1.2, fp, fp + 64, dp, 0u, nullptr, &plan), LYAF_EINVAL);
  EXPECT(lyaf_plan_create(&sk, &prm, 0.8, fp, fp + 64, dp, 1u << 9, nullptr, &plan),
         LYAF_EINVAL);
  EXPECT(lyaf_plan_create(&sk, &prm, 0.8, fp, fp + 64, dp, 0u, nullptr, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_plan_execute(nullptr, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_plan_status(nullptr, nullptr, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_plan_describe(nullptr, nullptr, 0), LYAF_EINVAL);
  EXPECT(lyaf_plan_destroy(nullptr), LYAF_OK);

  lyaf_instrument_params ins{7.0, 3.0, 0.0, 0.02, 6.0};
  std::vector<int64_t> oo = {0, 4, 10, 10};
  EXPECT(lyaf_instrument(3, off.data(), fp, fp, nullptr, oo.data(), fp, fp, nullptr),
         LYAF_EINVAL);
  EXPECT(lyaf_instrument(3, off.data(), fp, fp, &ins, oo.data(), nullptr, fp, nullptr),
         LYAF_EINVAL);  // noise required when noise_sigma > 0
  for (int field = 0; field < 5; ++field) {
    lyaf_instrument_params q = ins;
    double *f[5] = {&q.fwhm_kms, &q.bin_kms, &q.v_start_kms, &q.noise_sigma, &q.window_k};
    *f[field] = field == 2 ? INFINITY : -1.0;
    EXPECT(lyaf_instrument(3, off.data(), fp, fp, &q, oo.data(), fp, fp, nullptr), LYAF_EINVAL);
  }
  {
    std::vector<int64_t> bad_oo = {0, 4, 10, 11};  // bins for a skewer without pixels
    EXPECT(lyaf_instrument(3, off.data(), fp, fp, &ins, bad_oo.data(), fp, fp, nullptr),
           LYAF_EINVAL);
  }
  EXPECT(lyaf_instrument_backward(3, off.data(), fp, &ins, oo.data(), fp, nullptr, nullptr),
         LYAF_EINVAL);
  EXPECT(lyaf_flux_pdf(-1, fp, ip, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_flux_pdf(10, nullptr, ip, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_flux_pdf(10, fp, nullptr, nullptr), LYAF_EINVAL);
  {
    std::vector<int64_t> po = {0, 16, 40};  // 24 is not a power of two
    EXPECT(lyaf_flux_power(2, po.data(), fp, fp, 0.8, fp, nullptr), LYAF_EINVAL);
    po = {0, 16, 16 + 16384};  // longer than 8192
    EXPECT(lyaf_flux_power(2, po.data(), fp, fp, 0.8, fp, nullptr), LYAF_EINVAL);
    po = {0, 16, 32};
    EXPECT(lyaf_flux_power(2, po.data(), fp, fp, 0.0, fp, nullptr), LYAF_EINVAL);
    EXPECT(lyaf_flux_power(0, nullptr, nullptr, nullptr, 0.8, nullptr, nullptr), LYAF_OK);
  }
  EXPECT(lyaf_status_read(nullptr, nullptr), LYAF_EINVAL);
  EXPECT(lyaf_kernel_timing(1), LYAF_OK);
  double ms = -1.0;
  int64_t n = -1;
  EXPECT(lyaf_kernel_timing_read("tau", &ms, &n), LYAF_OK);
  if (ms != 0.0 || n != 0) return 1;
  EXPECT(lyaf_kernel_timing_read(nullptr, &ms, &n), LYAF_EINVAL);
  EXPECT(lyaf_kernel_timing(0), LYAF_OK);
  for (int code = 1; code >= -8; --code)
    if (!lyaf_strerror(code) || !*lyaf_strerror(code)) return 1;
  if (fabs(lyaf_angstrom_to_kms(3.63, 3.0) - 223.8) > 0.1) return 1;
  if (!(lyaf_lya_lyb_path_kms(3000.0) > 40000.0)) return 1;
  if (lyaf_version() < 100) return 1;
  puts("abi_sanitize: ok");
  return 0;
}
