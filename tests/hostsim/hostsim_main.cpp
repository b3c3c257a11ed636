// Scenarios for the plan/scheduler code of the library built on the host (no GPU): the
// kernels are stubs that only record their launches, so numbers are meaningless, but the
// control flow is the library's own: workspace set-up and release, the pass schedule, the
// panel order of streamed sources, callbacks, and the error paths under injected
// allocation, copy and launch failures.  Run under AddressSanitizer/UBSan, a leak or an
// out-of-range host access fails the run.  Prints one "PASS <name>" line per scenario.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/rpca.h"
#include "hostsim.h"

static int g_failures = 0;

#define CHECK(cond)                                                                       \
  do {                                                                                    \
    if (!(cond)) {                                                                        \
      std::printf("FAIL %s:%d %s (%s)\n", __FILE__, __LINE__, #cond, g_scenario.c_str()); \
      ++g_failures;                                                                       \
      return;                                                                             \
    }                                                                                     \
  } while (0)

static std::string g_scenario;

struct Dev {  // device buffers of one problem (host memory under the stand-in)
  float *A = nullptr, *U = nullptr, *S = nullptr, *V = nullptr, *G = nullptr;
  int64_t m, n, k, l;
  Dev(int64_t m_, int64_t n_, int64_t k_, int64_t l_) : m(m_), n(n_), k(k_), l(l_) {
    hipMalloc(&A, sizeof(float) * m * n);
    hipMalloc(&U, sizeof(float) * m * k);
    hipMalloc(&S, sizeof(float) * k);
    hipMalloc(&V, sizeof(float) * n * k);
    hipMalloc(&G, sizeof(float) * (m < n ? m : n) * l);
  }
  ~Dev() {
    hipFree(A);
    hipFree(U);
    hipFree(S);
    hipFree(V);
    hipFree(G);
  }
};

static rpca_desc desc_of(int64_t m, int64_t n, int k, int l, int i, int storage, int source, int center,
                         uint32_t flags, int64_t panel_rows = 0) {
  rpca_desc d;
  std::memset(&d, 0, sizeof d);
  d.m = m;
  d.n = n;
  d.k = k;
  d.l = l;
  d.i = i;
  d.storage = storage;
  d.source = source;
  d.center = center;
  d.panel_rows = panel_rows;
  d.seed = 7;
  d.flags = flags;
  d.device = 0;
  return d;
}

// ---------------------------------------------------------------- in-core plans
static void incore(int storage, int center, uint32_t flags, int64_t m, int64_t n) {
  g_scenario = "incore storage " + std::to_string(storage) + " center " + std::to_string(center) + " flags " +
               std::to_string(flags) + " " + std::to_string(m) + "x" + std::to_string(n);
  hostsim::reset();
  const long live0 = hostsim::record().live_device;
  const int k = 8, l = 12, i = 2;
  Dev d(m, n, k, l);
  rpca_desc ds = desc_of(m, n, k, l, i, storage, RPCA_SRC_DEVICE, center, flags);
  rpca_plan_t p = nullptr;
  CHECK(rpca_plan(&ds, nullptr, &p) == RPCA_OK && p != nullptr);
  float* cs = nullptr;
  void* A = d.A;
  int64_t lda = n;
  void* stored = nullptr;
  if (storage != RPCA_A_F32) {
    lda = (n + 15) / 16 * 16;
    hipMalloc(&stored, (size_t)m * lda * 4 * 2);
    hipMalloc(&cs, sizeof(float) * n);
    A = stored;
  }
  for (int rep = 0; rep < 2; ++rep) {
    const rpca_status st = rpca_factor(p, A, lda, storage == RPCA_A_FP8_E4M3 ? cs : nullptr, nullptr, nullptr,
                                       rep ? d.G : nullptr, d.U, k, d.S, d.V, k);
    CHECK(st == RPCA_OK);
  }
  rpca_stats s;
  CHECK(rpca_get_stats(p, &s) == RPCA_OK);
  CHECK(s.passes >= i + 2);
  if (m >= n) CHECK(s.a_reads == 2 * i + 2 || ((flags & RPCA_FLAG_FP64_STEP1) && s.a_reads >= i + 2));
  if (flags & RPCA_FLAG_KEEP_STATE) {
    float* dA = nullptr;
    hipMalloc(&dA, sizeof(float) * m * n);
    const rpca_status sb = rpca_backward(p, d.S, d.U, k, d.V, k, dA, n);
    CHECK(sb == RPCA_OK || (storage != RPCA_A_F32 && sb == RPCA_ERR_UNSUPPORTED));
    double* H = nullptr;
    const int64_t L = (int64_t)(i + 1) * l;
    hipMalloc(&H, sizeof(double) * m * L);
    CHECK(rpca_get_state(p, RPCA_STATE_Q, H, L) == RPCA_OK);
    hipFree(H);
    hipFree(dA);
  }
  rpca_destroy(p);
  hipFree(stored);
  hipFree(cs);
  CHECK(hostsim::record().live_device == live0 + 5);  // only the Dev buffers remain
  std::printf("PASS %s\n", g_scenario.c_str());
}

// ---------------------------------------------------------------- allocation failures
static void alloc_failures() {
  g_scenario = "plan creation with the n-th device allocation failing";
  const int64_t m = 3000, n = 700;
  // count the allocations of a successful plan
  hostsim::reset();
  rpca_desc ds = desc_of(m, n, 8, 12, 2, RPCA_A_F32, RPCA_SRC_DEVICE, 1, RPCA_FLAG_KEEP_STATE | RPCA_FLAG_PROFILE);
  rpca_plan_t p = nullptr;
  const long live0 = hostsim::record().live_device;
  CHECK(rpca_plan(&ds, nullptr, &p) == RPCA_OK);
  const long total = hostsim::record().mallocs;
  rpca_destroy(p);
  CHECK(hostsim::record().live_device == live0);
  CHECK(total > 5);
  for (long f = 0; f < total; ++f) {
    hostsim::reset();
    hostsim::faults().malloc_fail_at = f;
    rpca_plan_t q = reinterpret_cast<rpca_plan_t>(0x1);
    const rpca_status st = rpca_plan(&ds, nullptr, &q);
    CHECK(st == RPCA_ERR_OUT_OF_MEMORY || st == RPCA_ERR_HIP);
    CHECK(q == nullptr);
    CHECK(hostsim::record().live_device == live0);  // everything allocated before the failure is freed
  }
  std::printf("PASS %s (%ld allocations)\n", g_scenario.c_str(), total);
}

// ---------------------------------------------------------------- launch failures
static void launch_failures() {
  g_scenario = "factor with the first launch of each launcher failing";
  const int64_t m = 3000, n = 700;
  const int k = 8, l = 12, i = 2;
  Dev d(m, n, k, l);
  rpca_desc ds = desc_of(m, n, k, l, i, RPCA_A_F32, RPCA_SRC_DEVICE, 1, RPCA_FLAG_PROFILE);
  hostsim::reset();
  rpca_plan_t p = nullptr;
  CHECK(rpca_plan(&ds, nullptr, &p) == RPCA_OK);
  hostsim::reset();
  CHECK(rpca_factor(p, d.A, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k) == RPCA_OK);
  const std::map<std::string, long> used = hostsim::record().launches;
  CHECK(used.size() > 10);
  for (const auto& kv : used) {
    hostsim::reset();
    hostsim::faults().launch_fail_name = kv.first;
    hostsim::faults().launch_fail_at = 0;
    const rpca_status st = rpca_factor(p, d.A, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k);
    if (st != RPCA_ERR_HIP) {
      std::printf("FAIL launcher %s: status %d\n", kv.first.c_str(), (int)st);
      ++g_failures;
      continue;
    }
    rpca_stats s;
    rpca_get_stats(p, &s);
    if (s.hip_error != hipErrorLaunchFailure) {
      std::printf("FAIL launcher %s: hip_error %d\n", kv.first.c_str(), s.hip_error);
      ++g_failures;
    }
    // the plan stays usable after the failed call
    hostsim::reset();
    CHECK(rpca_factor(p, d.A, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k) == RPCA_OK);
  }
  rpca_destroy(p);
  std::printf("PASS %s (%zu launchers)\n", g_scenario.c_str(), used.size());
}

// ---------------------------------------------------------------- streamed sources
struct PanelLog {
  int64_t n;
  std::vector<std::pair<int64_t, int64_t>> calls;
  long fail_at = -1;
  int scale_calls = 0;
};

static int host_cb(void* user, int64_t row0, int64_t nrows, void* dst, int64_t ld, float* col_scale) {
  PanelLog* lg = static_cast<PanelLog*>(user);
  if (lg->fail_at >= 0 && (long)lg->calls.size() == lg->fail_at) return 3;
  lg->calls.push_back({row0, nrows});
  // touch every byte the plan says it owns (AddressSanitizer checks the range)
  std::memset(dst, 0, (size_t)nrows * ld * sizeof(float));
  if (col_scale != nullptr) {
    ++lg->scale_calls;
    for (int64_t c = 0; c < lg->n; ++c) col_scale[c] = 1.f;
  }
  return 0;
}

static int dev_cb(void* user, int64_t row0, int64_t nrows, float* dst, int64_t ld, void*) {
  PanelLog* lg = static_cast<PanelLog*>(user);
  if (lg->fail_at >= 0 && (long)lg->calls.size() == lg->fail_at) return 5;
  lg->calls.push_back({row0, nrows});
  std::memset(dst, 0, (size_t)nrows * ld * sizeof(float));
  return 0;
}

static bool panels_cover(const PanelLog& lg, int64_t m, int64_t pr, int passes) {
  const int64_t np = (m + pr - 1) / pr;
  if ((int64_t)lg.calls.size() != np * passes) return false;
  for (int ps = 0; ps < passes; ++ps)
    for (int64_t b = 0; b < np; ++b) {
      const auto& c = lg.calls[ps * np + b];
      if (c.first != b * pr || c.second != (b + 1 < np ? pr : m - b * pr)) return false;
    }
  return true;
}

static void streamed(int source, int center) {
  g_scenario = "streamed source " + std::to_string(source) + " center " + std::to_string(center);
  const int64_t m = 5000, n = 600, pr = 1024;
  const int k = 6, l = 10, i = 2;
  Dev d(m, n, k, l);
  hostsim::reset();
  const long live0 = hostsim::record().live_device;
  rpca_desc ds = desc_of(m, n, k, l, i, RPCA_A_F32, source, center, RPCA_FLAG_PROFILE, pr);
  rpca_plan_t p = nullptr;
  CHECK(rpca_plan(&ds, nullptr, &p) == RPCA_OK);
  PanelLog lg;
  lg.n = n;
  float* pinned = nullptr;
  if (source == RPCA_SRC_HOST_PINNED) hipHostMalloc(&pinned, sizeof(float) * m * n);
  if (source == RPCA_SRC_DEVICE_CALLBACK) CHECK(rpca_set_device_panel_cb(p, dev_cb, &lg) == RPCA_OK);
  hostsim::reset();
  rpca_status st = rpca_factor(p, pinned, n, nullptr, source == RPCA_SRC_CALLBACK ? host_cb : nullptr, &lg, nullptr,
                               d.U, k, d.S, d.V, k);
  CHECK(st == RPCA_OK);
  rpca_stats s;
  CHECK(rpca_get_stats(p, &s) == RPCA_OK);
  CHECK(s.passes == i + 2 + (center ? 1 : 0));
  CHECK(s.a_reads == s.passes);
  if (source != RPCA_SRC_DEVICE_CALLBACK) {
    CHECK(s.h2d_bytes == (int64_t)s.passes * m * n * 4);
    CHECK(hostsim::record().h2d_bytes >= (uint64_t)s.h2d_bytes);
  }
  if (source != RPCA_SRC_HOST_PINNED) CHECK(panels_cover(lg, m, pr, s.passes));
  // a callback failing in the middle of a pass aborts with CALLBACK, and the plan stays usable
  if (source != RPCA_SRC_HOST_PINNED) {
    const int64_t np = (m + pr - 1) / pr;
    for (long f : {0L, 1L, (long)np + 2, (long)(s.passes * np - 1)}) {
      lg.calls.clear();
      lg.fail_at = f;
      st = rpca_factor(p, nullptr, n, nullptr, source == RPCA_SRC_CALLBACK ? host_cb : nullptr, &lg, nullptr, d.U, k,
                       d.S, d.V, k);
      CHECK(st == RPCA_ERR_CALLBACK);
      CHECK((long)lg.calls.size() == f);
    }
    lg.calls.clear();
    lg.fail_at = -1;
    CHECK(rpca_factor(p, nullptr, n, nullptr, source == RPCA_SRC_CALLBACK ? host_cb : nullptr, &lg, nullptr, d.U, k,
                      d.S, d.V, k) == RPCA_OK);
    CHECK(panels_cover(lg, m, pr, s.passes));
  } else {
    // a failing host-to-device copy surfaces as HIP
    for (long f : {0L, 3L, 9L}) {
      hostsim::reset();
      hostsim::faults().copy_fail_at = f;
      st = rpca_factor(p, pinned, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k);
      CHECK(st == RPCA_ERR_HIP);
    }
    hostsim::reset();
    CHECK(rpca_factor(p, pinned, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k) == RPCA_OK);
  }
  rpca_destroy(p);
  hipHostFree(pinned);
  CHECK(hostsim::record().live_device == live0);
  std::printf("PASS %s (%zu panel calls)\n", g_scenario.c_str(), lg.calls.size());
}

// ---------------------------------------------------------------- argument errors on a live plan
static void argument_errors() {
  g_scenario = "argument errors on a live plan";
  const int64_t m = 2000, n = 500;
  const int k = 5, l = 8, i = 1;
  Dev d(m, n, k, l);
  rpca_desc ds = desc_of(m, n, k, l, i, RPCA_A_F32, RPCA_SRC_DEVICE, 0, 0);
  rpca_plan_t p = nullptr;
  CHECK(rpca_plan(&ds, nullptr, &p) == RPCA_OK);
  CHECK(rpca_factor(p, nullptr, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k) == RPCA_ERR_INVALID_ARG);
  CHECK(rpca_factor(p, d.A, n - 1, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k) == RPCA_ERR_INVALID_ARG);
  CHECK(rpca_factor(p, d.A, n, nullptr, nullptr, nullptr, nullptr, d.U, k - 1, d.S, d.V, k) == RPCA_ERR_INVALID_ARG);
  CHECK(rpca_factor(p, d.A, n, nullptr, nullptr, nullptr, nullptr, nullptr, k, d.S, d.V, k) == RPCA_ERR_INVALID_ARG);
  float* dA = nullptr;
  hipMalloc(&dA, sizeof(float) * m * n);
  CHECK(rpca_backward(p, d.S, d.U, k, d.V, k, dA, n) == RPCA_ERR_NO_STATE);
  double* Q = nullptr;
  hipMalloc(&Q, sizeof(double) * m * (i + 1) * l);
  CHECK(rpca_get_state(p, RPCA_STATE_Q, Q, (i + 1) * l) == RPCA_ERR_NO_STATE);
  CHECK(rpca_set_device_panel_cb(p, dev_cb, nullptr) == RPCA_ERR_UNSUPPORTED);
  hipFree(Q);
  hipFree(dA);
  CHECK(rpca_factor(p, d.A, n, nullptr, nullptr, nullptr, nullptr, d.U, k, d.S, d.V, k) == RPCA_OK);
  rpca_destroy(p);
  std::printf("PASS %s\n", g_scenario.c_str());
}

int main() {
  incore(RPCA_A_F32, 0, 0, 3000, 700);
  incore(RPCA_A_F32, 1, RPCA_FLAG_KEEP_STATE | RPCA_FLAG_PROFILE, 3000, 700);
  incore(RPCA_A_F32, 1, RPCA_FLAG_FORCE_FALLBACK, 3000, 700);
  incore(RPCA_A_F32, 0, RPCA_FLAG_FORCE_HOUSEHOLDER | RPCA_FLAG_KEEP_STATE, 3000, 700);
  incore(RPCA_A_F32, 1, RPCA_FLAG_SPLIT_BF16, 3000, 700);
  incore(RPCA_A_F32, 1, RPCA_FLAG_FP64_STEP1, 3000, 700);
  incore(RPCA_A_F32, 1, 0, 700, 3000);  // m < n: the plan factors A^T
  incore(RPCA_A_BF16, 1, 0, 3000, 700);
  incore(RPCA_A_FP8_E4M3, 1, RPCA_FLAG_PROFILE, 3000, 700);
  incore(RPCA_A_BF16_HILO, 0, 0, 3000, 700);
  alloc_failures();
  launch_failures();
  streamed(RPCA_SRC_HOST_PINNED, 0);
  streamed(RPCA_SRC_HOST_PINNED, 1);
  streamed(RPCA_SRC_CALLBACK, 1);
  streamed(RPCA_SRC_DEVICE_CALLBACK, 0);
  argument_errors();
  std::printf("%s: %d failure(s)\n", g_failures ? "FAILED" : "ALL PASSED", g_failures);
  return g_failures ? 1 : 0;
}
