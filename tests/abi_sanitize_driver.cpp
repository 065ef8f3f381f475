// Host-side checks of the C ABI (include/drot.h) that need no GPU, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code of
// the library (tests/test_host_sanitizers.py).  Every call here must be
// rejected by argument validation before any device work; the program
// prints each failed check and exits with the number of failures.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "drot.h"

static int failures = 0;

static void expect(const char* what, int got, int want) {
  if (got != want) {
    std::printf("FAIL %s: got %d, want %d (%s)\n", what, got, want, drot_last_error());
    ++failures;
  } else if (want < 0 && std::strlen(drot_last_error()) == 0) {
    std::printf("FAIL %s: no error message\n", what);
    ++failures;
  }
}

static drot_params params() {
  drot_params p;
  std::memset(&p, 0, sizeof p);
  p.rho = 1e-4;
  p.tol = 0.0;
  p.max_iter = 10;
  return p;
}

int main() {
  if (!drot_version() || !std::strlen(drot_version())) ++failures;
  for (int s = -8; s <= 2; ++s)
    if (!drot_strerror(s) || !std::strlen(drot_strerror(s))) ++failures;

  // Fake, aligned, non-overlapping device addresses: validation only.
  const int64_t m = 300, n = 260;
  void* C = reinterpret_cast<void*>(uintptr_t(1) << 40);
  void* X = reinterpret_cast<void*>(uintptr_t(1) << 41);
  void* p = reinterpret_cast<void*>(uintptr_t(1) << 42);
  void* q = reinterpret_cast<void*>(uintptr_t(1) << 43);
  double mu0_dummy = 0.0;
  drot_result r;
  drot_params prm = params();

  expect("out NULL", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &prm, X, n, nullptr, nullptr,
                                        nullptr, nullptr, nullptr, nullptr), DROT_EINVAL);
  expect("m = 0", drot_solve_noalloc(0, n, DROT_F32, C, n, p, q, &prm, X, n, nullptr, nullptr,
                                     nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("dtype", drot_solve_noalloc(m, n, 7, C, n, p, q, &prm, X, n, nullptr, nullptr, nullptr,
                                     nullptr, &r, nullptr), DROT_EINVAL);
  expect("params NULL", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, nullptr, X, n, nullptr,
                                           nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("ldc < n", drot_solve_noalloc(m, n, DROT_F32, C, n - 1, p, q, &prm, X, n, nullptr,
                                       nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("ldx < n", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &prm, X, n - 1, nullptr,
                                       nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("C NULL", drot_solve_noalloc(m, n, DROT_F32, nullptr, n, p, q, &prm, X, n, nullptr,
                                      nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("X misaligned",
         drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &prm, static_cast<char*>(X) + 2, n,
                            nullptr, nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("C and X overlap",
         drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &prm, static_cast<char*>(C) + 64, n,
                            nullptr, nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  expect("mu0 without nu0", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &prm, X, n, nullptr,
                                               nullptr, &mu0_dummy, nullptr, &r, nullptr),
         DROT_EINVAL);
  {
    drot_params b = params();
    b.rho = -1.0;
    expect("rho < 0", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr, nullptr,
                                         nullptr, nullptr, &r, nullptr), DROT_EINVAL);
    b = params();
    b.tol = std::nan("");
    expect("tol NaN", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr, nullptr,
                                         nullptr, nullptr, &r, nullptr), DROT_EINVAL);
    b = params();
    b.max_iter = 0;
    expect("max_iter 0", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr,
                                            nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
    b = params();
    b.flags = 0x100;
    expect("unknown flag", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr,
                                              nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
    b = params();
    b.flags = DROT_FLAG_SKIP_C | DROT_FLAG_COMPENSATED;
    expect("skip-C + compensated",
           drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr, nullptr, nullptr,
                              nullptr, &r, nullptr), DROT_EUNSUPPORTED);
    b = params();
    b.flags = DROT_FLAG_TIME_SWEEP;
    expect("sweep timing", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr,
                                              nullptr, nullptr, nullptr, &r, nullptr),
           DROT_EUNSUPPORTED);
    b = params();
    b.tile_chunks = 3;
    expect("tile chunks", drot_solve_noalloc(m, n, DROT_F32, C, n, p, q, &b, X, n, nullptr,
                                             nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  }
  expect("beyond the static scratch",
         drot_solve_noalloc(20000, 20000, DROT_F32, C, 20000, p, q, &prm,
                            reinterpret_cast<void*>(uintptr_t(1) << 44), 20000, nullptr, nullptr,
                            nullptr, nullptr, &r, nullptr), DROT_EINVAL);

  // Context-less calls.
  expect("ctx destroy NULL", drot_ctx_destroy(nullptr), DROT_OK);
  expect("iterate NULL ctx", drot_iterate(nullptr, 1, nullptr), DROT_EINVAL);
  int64_t done = 0;
  int32_t stopped = 0;
  expect("poll NULL ctx", drot_poll(nullptr, &done, &stopped, nullptr), DROT_EINVAL);
  expect("finish NULL ctx", drot_finish(nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  size_t bytes = 0;
  expect("checkpoint size NULL ctx", drot_checkpoint_size(nullptr, &bytes), DROT_EINVAL);
  double trace[8];
  expect("trace NULL ctx", drot_get_trace(nullptr, 1, 1, trace), DROT_EINVAL);
  expect("solve NULL ctx", drot_solve(nullptr, m, n, DROT_F32, C, n, p, q, &prm, X, n, nullptr,
                                      nullptr, nullptr, nullptr, &r, nullptr), DROT_EINVAL);
  drot_problem prob;
  std::memset(&prob, 0, sizeof prob);
  drot_result outs[1];
  expect("batched count 0", drot_solve_batched(nullptr, 0, DROT_F32, &prob, &prm, outs, nullptr),
         DROT_EINVAL);
  expect("batched NULL problem arrays",
         drot_solve_batched(nullptr, 1, DROT_F32, &prob, &prm, outs, nullptr), DROT_EINVAL);

  // The warm-start network's argument checks.
  drot_mlp* net = nullptr;
  expect("mlp widths", drot_mlp_create(&net, 0, 100, 64, 64, 64, 1), DROT_EINVAL);
  expect("mlp destroy NULL", drot_mlp_destroy(nullptr), DROT_OK);
  int64_t count = 0;
  expect("mlp params NULL", drot_mlp_num_params(nullptr, &count), DROT_EINVAL);
  expect("mlp apply NULL", drot_mlp_apply_gradients(nullptr, nullptr, 1e-3f, nullptr), DROT_EINVAL);

  // A context: DROT_EDEVICE without a GPU, a working one with.
  drot_ctx* ctx = nullptr;
  const int rc = drot_ctx_create(&ctx, 0);
  if (rc == DROT_OK) {
    expect("iterate before bind", drot_iterate(ctx, 1, nullptr), DROT_ESTATE);
    drot_ctx_destroy(ctx);
  } else {
    expect("ctx create without a GPU", rc, DROT_EDEVICE);
  }
  std::printf("%d failures\n", failures);
  return failures;
}
