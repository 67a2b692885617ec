// Host sanitizer driver for the C ABI's argument validation (include/cme.h):
// linked against a build of cme_api.hip whose host code carries
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py),
// it drives every entry point through its refusal paths and the static
// tables on a machine without a GPU.  Each call must return the documented
// status without touching memory it does not own.  Test infrastructure only.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "cme.h"

static int fails = 0;
#define EXPECT(call, code)                                                           \
  do {                                                                               \
    const int rc_ = (call);                                                          \
    if (rc_ != (code)) {                                                             \
      std::fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, \
                   rc_, (int)(code));                                                \
      ++fails;                                                                       \
    }                                                                                \
  } while (0)

static cme_instance inst(int n, long long off) {
  cme_instance x;
  std::memset(&x, 0, sizeof x);
  x.n_modes = n;
  x.mode_offset = off;
  x.kappa_ext = 0.5;
  x.g0 = 1.0;
  x.a_in_re = 0.5;
  x.sigma0 = x.sigma1 = 1.0;
  return x;
}

int main() {
  for (int c = -12; c <= 2; ++c)
    if (!cme_strerror(c) || !std::strlen(cme_strerror(c))) ++fails;
  if (cme_version() < 10000) ++fails;
  std::vector<int32_t> ids(256);
  int total_ids = 0;
  for (int prec = 0; prec < 2; ++prec)
    for (int n = 8; n <= 131072; n *= 2) {
      const int k = cme_list_kernels(prec, n, ids.data(), 2);  // capped
      const int k2 = cme_list_kernels(prec, n, ids.data(), (int)ids.size());
      if (k != k2 || k2 < 0) ++fails;
      total_ids += k2;
      for (int i = 0; i < k2; ++i) {
        int32_t info[10];
        if (cme_kernel_info(ids[i], info, 10) != 10 || info[1] != n) ++fails;
        if (cme_kernel_info(ids[i], info, 3) != 10) ++fails;  // short buffer
      }
    }
  if (total_ids == 0) ++fails;
  int32_t info[10];
  EXPECT(cme_kernel_info(-1, info, 10), CME_EINVAL);
  EXPECT(cme_kernel_info(1 << 20, info, 10), CME_EINVAL);
  EXPECT(cme_kernel_info(0, nullptr, 10), CME_EINVAL);

  const double kap[64] = {1.0}, om[64] = {0.0};
  cme_plan *plan = reinterpret_cast<cme_plan *>(1);
  cme_instance one = inst(16, 0);
  EXPECT(cme_init(nullptr, 1, &one, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 0, &one, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
         CME_EINVAL);
  if (plan != nullptr) ++fails;  // cleared on error
  EXPECT(cme_init(&plan, 1, nullptr, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, nullptr, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, kap, om, 7, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, kap, om, CME_F64, 9, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, kap, om, CME_F64, CME_RK4, 5, 1e-3, nullptr, 0), CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, kap, om, CME_F32, CME_RK4, CME_FWM_PADDED, 1e-3, nullptr, 0),
         CME_EUNSUPPORTED);
  EXPECT(cme_init(&plan, 1, &one, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 0.0, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, NAN, nullptr, 0),
         CME_EINVAL);
  EXPECT(cme_init(&plan, 1, &one, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 64),
         CME_EINVAL);
  for (int n : {0, 8, 24, 100, 131072, -16}) {
    cme_instance x = inst(n, 0);
    EXPECT(cme_init(&plan, 1, &x, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
           CME_EINVAL);
  }
  {
    cme_instance x = inst(16, 0);
    x.reserved = 3;
    EXPECT(cme_init(&plan, 1, &x, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
           CME_EINVAL);
    x = inst(16, -1);
    EXPECT(cme_init(&plan, 1, &x, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
           CME_EINVAL);
    x = inst(16, 0);
    x.g0 = NAN;
    EXPECT(cme_init(&plan, 1, &x, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
           CME_ENONFINITE);
    x = inst(16, 0);
    x.kappa_ext = -1.0;
    EXPECT(cme_init(&plan, 1, &x, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
           CME_EINVAL);
    cme_instance two[2] = {inst(16, 0), inst(16, 8)};  // overlapping ranges
    EXPECT(cme_init(&plan, 2, two, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0),
           CME_EINVAL);
    x = inst(65536, 0);  // padded: 2N-point transforms beyond the largest
    EXPECT(cme_init(&plan, 1, &x, kap, om, CME_F64, CME_RK4, CME_FWM_PADDED, 1e-3, nullptr, 0),
           CME_EUNSUPPORTED);
  }
  // a valid request reaches the device query and is refused there (no GPU)
  {
    cme_instance two[2] = {inst(16, 0), inst(32, 16)};
    const int rc =
        cme_init(&plan, 2, two, kap, om, CME_F64, CME_RK4, CME_FWM_CYCLIC, 1e-3, nullptr, 0);
    if (rc != CME_ENODEVICE && rc != CME_EHIP) ++fails;
    if (plan != nullptr) ++fails;
  }
  // every entry point refuses a null plan
  char buf[64];
  int32_t flags[4], kid = 0;
  double g[4];
  EXPECT(cme_step(nullptr, buf, 0), CME_EINVAL);
  EXPECT(cme_run(nullptr, buf, 0, 1, 0, nullptr), CME_EINVAL);
  EXPECT(cme_fwm(nullptr, buf, buf), CME_EINVAL);
  EXPECT(cme_adjoint(nullptr, buf, nullptr, 0, 1, 0, buf, buf, g, g, g), CME_EINVAL);
  EXPECT(cme_adjoint_noalloc(nullptr, buf, nullptr, 0, 1, 0, buf, buf, g, g, g), CME_EINVAL);
  EXPECT(cme_status(nullptr, flags), CME_EINVAL);
  EXPECT(cme_set_stream(nullptr, nullptr), CME_EINVAL);
  EXPECT(cme_plan_kernel(nullptr, 16, &kid), CME_EINVAL);
  EXPECT(cme_plan_select(nullptr, 16, 0), CME_EINVAL);
  EXPECT(cme_destroy(nullptr), CME_OK);
  if (fails) {
    std::fprintf(stderr, "%d failures\n", fails);
    return 1;
  }
  std::printf("abi sanitizer driver: ok\n");
  return 0;
}
