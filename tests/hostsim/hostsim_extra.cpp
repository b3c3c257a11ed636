// Host-side planning helpers of the kernel files, stood in for the host-only build: split
// policies that keep the invariants plan.cpp relies on (row splits a multiple of 64 rows,
// K chunks a multiple of 64) and exercise the multi-split paths, and fit predicates.
#include <hip/hip_runtime.h>

#include "../../paper_1007_5510_amd/csrc/kernels.h"

namespace rpca {

static int64_t up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

static void ksplit2(int64_t n, int* ks, int64_t* kchunk) {
  const int64_t c = n >= 128 ? up((n + 1) / 2, 64) : up(n, 64);
  *kchunk = c;
  *ks = (int)((n + c - 1) / c);
}

static void rsplit3(int64_t m, int* ns, int64_t* rps) {
  const int64_t r = up((m + 2) / 3 > 0 ? (m + 2) / 3 : 1, 64);
  *rps = r;
  *ns = (int)((m + r - 1) / r);
}

void fwd_split(int64_t, int64_t n, int64_t, int* ksplit, int64_t* kchunk) { ksplit2(n, ksplit, kchunk); }
void adj_split(int64_t m, int64_t, int, int64_t, int* nsplit, int64_t* rows_per_split) { rsplit3(m, nsplit, rows_per_split); }
void fwd_split_lp(int, int64_t, int64_t n, int64_t, int* ksplit, int64_t* kchunk) { ksplit2(n, ksplit, kchunk); }
void adj_split_lp(int, int64_t m, int64_t, int, int64_t, int* nsplit, int64_t* rows_per_split) {
  rsplit3(m, nsplit, rows_per_split);
}
void fwd64_split(int64_t, int64_t n, int, int64_t, int* ksplit, int64_t* kchunk) { ksplit2(n, ksplit, kchunk); }
void adj64_split(int64_t m, int64_t, int, int64_t, int* nsplit, int64_t* rows_per_split) {
  rsplit3(m, nsplit, rows_per_split);
}

size_t fused_ws_words() { return 4096; }
size_t fused_xpart_floats(int) { return 4096; }
size_t fused_xred_floats() { return 4096; }
bool fused_fits(int64_t, int, bool, int, int) { return false; }

bool cholinv_fits(int L) { return L >= 1 && L <= 1024; }
bool hh_fits(int, int64_t) { return true; }
void set_hh_lds_limit(size_t) {}
void set_max_lds(size_t) {}
size_t syev_small_work(int L, int kk) { return (size_t)L * (L + 1) / 2 + 4 * (size_t)L + 8 + (size_t)L * kk + 64; }

}  // namespace rpca
