// host_driver.cpp -- drives the host-side planning and validation of the HIP
// library (make_plan, plan_segments, the workspace and LDS figures, argument
// checks of every entry point, the batched plan's validation) over a wide
// grid of valid, extreme and invalid arguments, for an AddressSanitizer +
// UndefinedBehaviorSanitizer build of the host code (tests/test_sanitizers.py).
// Device pointers are all NULL, so every call returns before any device
// work; no GPU is needed.  Any out-of-bounds access, signed overflow, bad
// shift or other undefined behaviour aborts the run.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "fmgsr.h"

static int failures = 0;

static void expect_fail(int st, const char* what) {
  if (st >= 0) {
    std::fprintf(stderr, "%s: accepted (%d)\n", what, st);
    ++failures;
  }
}

int main() {
  fmgsr_options o;
  const int64_t ns[] = {0, 1, 2, 3, 6, 64, 1000, 1024, 4096, 5 << 12, (int64_t)1 << 20,
                        (int64_t)1 << 28, (int64_t)1 << 34, (int64_t)1 << 40, INT64_MAX,
                        -1, INT64_MIN};
  const int32_t levels_v[] = {-1, 0, 1, 2, 3, 11, 13, 21, 29, 35, 40, 41, 64, INT32_MAX};
  const int64_t segs_v[] = {-1, 0, 1, 2, 3, 4, 16, 4096, 65536, (int64_t)1 << 40, INT64_MAX};
  const int32_t buf_v[] = {-1, 0, 1, 2, 8, 64, 1024, 1025, INT32_MAX};
  const int nus[][2] = {{2, 1}, {0, 0}, {16, 16}, {17, 1}, {-1, 2}};
  long calls = 0;
  for (int64_t n : ns)
    for (int32_t L : levels_v)
      for (int sr = -1; sr <= 4; ++sr)
        for (int tau = 0; tau <= 2; ++tau)
          for (int prec = 0; prec <= 2; ++prec)
            for (const auto& nu : nus) {
              fmgsr_default_options(&o);
              o.nu1 = nu[0];
              o.nu2 = nu[1];
              o.sr_levels = sr;
              o.tau_mode = tau;
              o.precision = prec;
              (void)fmgsr_workspace_bytes(n, L, &o);
              for (int64_t S : segs_v)
                for (int32_t b : buf_v) {
                  const size_t w = fmgsr_workspace_bytes_for(n, L, S, b, &o);
                  const size_t lds = fmgsr_launch_lds_bytes(n, L, S, b, &o);
                  if (w > 0 && w > fmgsr_workspace_bytes(n, L, &o)) {
                    std::fprintf(stderr, "workspace_for > workspace (n %lld)\n", (long long)n);
                    ++failures;
                  }
                  if (lds > 160 * 1024) {
                    std::fprintf(stderr, "LDS request %zu\n", lds);
                    ++failures;
                  }
                  // NULL device arrays: every call must be refused on the host
                  expect_fail(fmgsr_solve(nullptr, nullptr, 0.0, 0.0, n, L, S, b, &o, nullptr,
                                          nullptr), "fmgsr_solve");
                  expect_fail(fmgsr_decompress(nullptr, nullptr, 0.0, 0.0, n, S, b, &o, 0,
                                               n > 0 ? n : 0, nullptr, nullptr),
                              "fmgsr_decompress");
                  calls += 4;
                }
            }
  // options with functionals / kept coarse level (never dereferenced: the
  // arrays are refused before use)
  fmgsr_default_options(&o);
  double dummy[4] = {0, 0, 0, 0};
  o.functionals = dummy;
  expect_fail(fmgsr_solve(nullptr, nullptr, 0, 0, 1024, 11, 4, 4, &o, nullptr, nullptr),
              "host functionals");
  o.functionals = nullptr;
  o.coarse_out = dummy;
  expect_fail(fmgsr_solve(nullptr, nullptr, 0, 0, 1024, 11, 4, 4, &o, nullptr, nullptr),
              "host coarse_out");
  for (int st = -10; st <= 10; ++st) (void)fmgsr_status_string(st);
  (void)fmgsr_version();

  // batched plans: invalid problem sets are refused before any device work
  struct Case {
    std::vector<int64_t> n;
    std::vector<int32_t> L;
    std::vector<int64_t> segs;
    int32_t buffer;
  };
  const Case cases[] = {
      {{1000}, {5}, {}, 8},       {{4096}, {0}, {}, 8},        {{4096}, {13}, {3}, 8},
      {{4096}, {13}, {4096}, 8},  {{4096}, {13}, {}, 65},      {{4096}, {13}, {}, -1},
      {{0}, {1}, {}, 8},          {{-5}, {1}, {}, 8},          {{INT64_MAX}, {40}, {}, 8},
      {{4096, 1000}, {13, 5}, {}, 8}, {{1 << 20}, {64}, {}, 8}, {{4096}, {13}, {-2}, 8},
  };
  for (const Case& c : cases) {
    fmgsr_batch plan = nullptr;
    fmgsr_default_options(&o);
    expect_fail(fmgsr_batch_create((int32_t)c.n.size(), c.n.data(), nullptr, c.L.data(),
                                   c.segs.empty() ? nullptr : c.segs.data(), c.buffer, nullptr,
                                   FMGSR_OP_CUBIC_REACTION, &o, &plan),
                "fmgsr_batch_create");
    if (plan) ++failures;
  }
  expect_fail(fmgsr_batch_create(0, nullptr, nullptr, nullptr, nullptr, 8, nullptr, 1, &o, nullptr),
              "empty batch");
  expect_fail(fmgsr_batch_solve(nullptr, nullptr, nullptr, nullptr, nullptr), "batch_solve");
  expect_fail(fmgsr_batch_destroy(nullptr), "batch_destroy");
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("host driver: %ld planning and validation calls clean\n", calls);
  return 0;
}
