// C ABI and host orchestration of the randomized block-Lanczos PCA
// (Section 3, Steps 1-6; Section 4 out-of-core structure).  Every arithmetic
// step runs in the library's HIP kernels; the host only validates, sizes the
// workspace, launches, and makes the one decision that needs a value from
// the device (whether Step 2 must take its fallback).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rpca.h"
#include "kernels.h"
#include "storage.h"

using namespace rpca;

namespace {

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct rpca_plan_s {
  rpca_desc d{};
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t m = 0, n = 0;
  int k = 0, l = 0, i = 0, L = 0;
  int64_t ldx = 0;  // row stride of transposed blocks (n rounded up to 4)
  int64_t ldp = 0;  // row stride of split partials
  size_t max_lds = 65536;

  // split configuration of the adjoint products
  int ns_y = 1, ns_t = 1;
  int64_t rps_y = 0, rps_t = 0;
  int ns_cs = 1;  // column-sum splits over A
  int64_t rps_cs = 0;
  int ns_cn = 1;  // column-sum splits over the narrow m-row blocks (H, Q)
  int64_t rps_cn = 0;
  int ns_g = 1;   // Gram splits over H / Q rows
  int64_t rps_g = 0;
  int ns_gt = 1;  // Gram splits over T rows
  int64_t rps_gt = 0;
  int fwd_ks = 1;  // K split of the forward product
  int64_t fwd_kchunk = 0;
  int64_t ldpf = 0;  // row stride of the forward split partials
  int storage = RPCA_A_F32;
  // streamed sources (A in pinned host memory or produced by a callback), Section 4
  bool streamed = false;
  int64_t panel_rows = 0;       // rows per panel
  int64_t ldb = 0;              // leading dimension of the device panel buffers
  hipStream_t cstream = nullptr;  // host -> device copies
  hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  float* dbuf[2] = {nullptr, nullptr};    // device panel buffers
  float* staging[2] = {nullptr, nullptr};  // pinned host staging (callback source)
  int ns_py = 1, ns_pt = 1, ns_pcs = 1;    // per-panel split counts (adjoint l / L columns, column sums)
  int64_t rps_py = 0, rps_pt = 0, rps_pcs = 0;
  int fwd_ks_p = 1;
  int64_t fwd_kchunk_p = 0;
  double* acc = nullptr;        // float64 accumulator of the adjoint products (L x ldp) or column sums
  rpca_device_panel_cb dcb = nullptr;  // DEVICE_CALLBACK source: row generator and its argument
  void* dcb_user = nullptr;
  // low-precision storage: bfloat16 hi/lo planes of the float operand
  int64_t ldxs = 0;  // X planes: cpad_x rows of ldxs (n rounded up to 64)
  int cpad_x = 0;
  int64_t ldzs = 0;  // transposed Z planes: cpad_z rows of ldzs (m rounded up to 64)
  int cpad_z = 0;

  std::vector<void*> allocs;
  // device buffers
  float* X = nullptr;       // (i+1) blocks of l x ldx (transposed X_j, X_0 = G)
  float* shift = nullptr;   // ldx
  double* mu = nullptr;     // n
  double* dres = nullptr;   // n: mu - fl32(mu)
  double* d0 = nullptr;     // n: colsum(A - 1 s0^T) / m of pass 0 (centring fused into pass 0)
  float* H = nullptr;       // m x L
  double* Q1 = nullptr;     // m x L
  double* Q = nullptr;      // m x L
  float* Q32 = nullptr;     // m x L
  float* P = nullptr;       // adjoint split partials
  float* Pf = nullptr;      // forward split partials
  double* T = nullptr;      // n x L
  double* csp = nullptr;    // column-sum partials
  double* gp = nullptr;     // Gram partials
  double* Wg = nullptr;     // L x L Gram
  double* R1 = nullptr;     // L x L
  double* R2 = nullptr;
  double* R3 = nullptr;
  double* Rtmp = nullptr;
  double* Rfull = nullptr;
  double* Rinv = nullptr;
  double* Mg = nullptr;     // T^T T
  double* eigwork = nullptr;  // Step 4 eigensolver scratch
  double* lam = nullptr;      // eigenvalues of T^T T, descending
  double* Wsorted = nullptr;  // eigenvectors (columns), same order
  double* sigL = nullptr;     // S~ = sqrt(lam)
  double* Vk = nullptr;     // n x k
  double* sig = nullptr;    // k
  double* sgn = nullptr;    // k
  double* alpha = nullptr;  // i+1
  double* zsum = nullptr;   // L
  double* sqp = nullptr;    // sum of squares partials
  float* corr = nullptr;    // L
  int* flags = nullptr;     // [0] nonfinite, [1..3] Cholesky breakdown in the first, second, third Cholesky QR
  uint16_t* Xh = nullptr;   // low-precision storage only
  uint16_t* Xl = nullptr;
  uint16_t* Zh = nullptr;
  uint16_t* Zl = nullptr;
  // float32 products on bfloat16 matrix cores (RPCA_FLAG_SPLIT_BF16): three-way
  // operand planes and the row splits of the adjoint in multiples of 32
  bool x6 = false;
  uint16_t* Xp3 = nullptr;
  uint16_t* Zp3 = nullptr;
  int64_t ldxs3 = 0, xplane3 = 0, ldzs3 = 0, zplane3 = 0;
  int cpadx3 = 0, cpadz3 = 0;
  int ns_y6 = 1, ns_t6 = 1;
  int64_t rps_y6 = 0, rps_t6 = 0;
  int64_t sqp_cap = 0;
  // Step 1 in float64 (RPCA_FLAG_FP64_STEP1): float64 blocks X_j and H, their
  // split partial sums, and the split configuration of those kernels
  bool f64s1 = false;
  int64_t ldx64 = 0, ldp64 = 0;
  double* X64 = nullptr;   // (i+1) blocks of l x ldx64 (zero past n)
  double* H64 = nullptr;   // m x L
  double* P64 = nullptr;   // adjoint partials [ns_y64][l][ldp64]
  double* Pf64 = nullptr;  // forward partials [fwd_ks64][m][l]
  double* corr64 = nullptr;  // l: mu^T X_j (centring)
  int ns_y64 = 1, fwd_ks64 = 1;
  int64_t rps_y64 = 0, fwd_kchunk64 = 0;

  // m < n (Section 3: the algorithm runs on the transpose).  The plan's m, n, k, l, i are those
  // of B = A~^T (n x m); Steps 1 and 3 run the A-kernels with the roles of the products swapped:
  // B X = A~^T X is an adjoint launch over A, B^T Y = A~ Y a forward launch.  Buffers over A's
  // shape (am x an, am < an):
  struct Trans {
    bool on = false;
    int64_t am = 0, an = 0;
    int64_t ldxa = 0;            // an rounded up to 4
    float* shift = nullptr;      // ldxa, zero tail
    double* mu = nullptr;        // an
    double* dres = nullptr;      // an
    float* Z = nullptr;          // am x L: the blocks X_B^(j) (row-major), then T_B in float32
    float* HBt = nullptr;        // L x ldxa: a block of H_B (or Q_B) transposed, zero past an
    double* H64 = nullptr;       // an x L: H_B in float64 (Step 2 input)
    float* P = nullptr;          // adjoint partials [ns_y][l][ldxa]
    float* Pf = nullptr;         // forward partials [fwd_ks][am][ldpf]
    double* sqp = nullptr;       // sums of squares of a transposed block
    int ns_y = 1, fwd_ks = 1, ns_cs = 1, ns_cz = 1;
    int64_t rps_y = 0, fwd_kchunk = 0, ldpf = 0, rps_cs = 0, rps_cz = 0;
  } tr;

  // single-read power steps (panel_fused.hip): groups of compute units (one or two XCDs each)
  // split the columns; rows of a group in blocks of 16; adjoint partial sums per row segment
  bool fused = false;
  int fu_ngroups = 0, fu_xpg = 0, fu_cpx = 0, fu_nseg = 1;
  int64_t fu_rpg = 0, fu_segrows = 0;
  unsigned* fu_ws = nullptr;
  float* fu_xpart = nullptr;
  float* fu_xred = nullptr;
  std::vector<EventPair> ev_fused;
  int nev_fused = 0;

  bool have_state = false;
  bool Qfinal_is_Q1 = false;
  const void* A_last = nullptr;  // matrix of the last factorisation (for the backward passes)
  int64_t lda_last = 0;

  // Householder TSQR workspace of Step 2, allocated on first use: per level of
  // the tree the stacked triangles of the level below (levels >= 1; level 0
  // works in place on Q1), the reflector scalars, two buffers for the top-down
  // formation of Q, and the final triangle
  struct Tsqr {
    bool ready = false;
    std::vector<int64_t> rows, bu;
    std::vector<int> nb;
    std::vector<double*> X, tau;
    double* O[2] = {nullptr, nullptr};
    double* Rtop = nullptr;
  } tsqr;

  // reverse-mode workspace, allocated by the first rpca_backward
  struct Backward {
    bool ready = false;
    int R = 0;                                       // rank of dA = P Y^T: (3i + 2) l
    double *Qbar = nullptr, *Hbar = nullptr;         // m x L
    float *Zf = nullptr, *Zin = nullptr;             // m x L, m x l
    double *Pm = nullptr, *Yt = nullptr;             // m x R, R x ldx
    float* Xbar = nullptr;                           // i blocks of l x ldx (transposed)
    double* Tbar = nullptr;                          // n x L
    float* TbarT = nullptr;                          // L x ldx
    double *NtV = nullptr, *Wbar = nullptr, *XV = nullptr, *YW = nullptr;  // L x k
    double *WT = nullptr, *Wsc = nullptr, *Nm = nullptr, *Tmp = nullptr, *Bmat = nullptr;  // L x L
    double *M2 = nullptr, *Smat = nullptr, *Rf = nullptr, *Rt = nullptr, *RfInv = nullptr, *RinvT = nullptr;
    double *Ck = nullptr, *Bp = nullptr;             // k x L
    double* ppart = nullptr;                         // column-sum partials of P
    int Rp = 0;                                      // R rounded up to 4 (zero padding)
    float *P32 = nullptr, *Y32 = nullptr;            // m x Rp, n x Rp: float32 factors of dA
    uint16_t *P3 = nullptr, *Y3 = nullptr;           // their three-part bfloat16 splits (K-step-major,
    int kp3 = 0;                                     // kp3 = R rounded up to 32, rows padded to 256:
    int64_t mpad3 = 0, npad3 = 0;                    // mpad3 and npad3)
    int ns_x = 1;                                    // row splits of the m-row X^T Y products
    int64_t rps_x = 0;                               // (short splits: they are latency bound)
    double* xpart = nullptr;                         // their partials, ns_x x L x L
  } bw;
  rpca_stats stats{};
  std::vector<EventPair> ev_fwd, ev_adj;
  hipEvent_t stage_ev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // PROFILE stage marks
  int nev_fwd = 0, nev_adj = 0;
  int tp_ev0 = 0, tp_ev1 = 0;  // adjoint events [tp_ev0, tp_ev1) belong to the T pass

  ~rpca_plan_s() {
    DevGuard g(device);
    if (cstream != nullptr) (void)hipStreamSynchronize(cstream);
    if (stream != nullptr || streamed) (void)hipStreamSynchronize(stream);
    for (void* p : allocs) (void)hipFree(p);
    for (int q = 0; q < 2; ++q) {
      if (staging[q]) (void)hipHostFree(staging[q]);
      if (ev_ready[q]) (void)hipEventDestroy(ev_ready[q]);
      if (ev_free[q]) (void)hipEventDestroy(ev_free[q]);
    }
    if (cstream != nullptr) (void)hipStreamDestroy(cstream);
    for (auto& e : ev_fwd) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
    for (auto& e : ev_adj) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
    for (auto& e : ev_fused) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
    for (hipEvent_t e : stage_ev)
      if (e) (void)hipEventDestroy(e);
  }

  template <typename T>
  hipError_t alloc(T** p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)count * sizeof(T));
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *p = reinterpret_cast<T*>(q);
    return hipSuccess;
  }
};

#define RPCA_TRY(expr)                                  \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) {                             \
      plan->stats.hip_error = (int32_t)e_;              \
      (void)hipGetLastError();                          \
      return e_ == hipErrorOutOfMemory ? RPCA_ERR_OUT_OF_MEMORY : RPCA_ERR_HIP; \
    }                                                   \
  } while (0)

namespace {

// Section 3 parameter rules (reading: enforce l >= k and (i+1) l <= n - k).
rpca_status validate_desc(const rpca_desc* d) {
  if (d == nullptr) return RPCA_ERR_INVALID_ARG;
  if (d->m <= 0 || d->n <= 0) return RPCA_ERR_INVALID_ARG;
  const int64_t small = d->m < d->n ? d->m : d->n;  // m < n: the rules apply to A^T (n x m)
  if (d->k < 1 || (int64_t)d->k >= small) return RPCA_ERR_INVALID_ARG;
  if (d->l < d->k || d->i < 0) return RPCA_ERR_INVALID_ARG;
  if ((int64_t)(d->i + 1) * d->l > small - d->k) return RPCA_ERR_INVALID_ARG;
  if (d->storage < RPCA_A_F32 || d->storage > RPCA_A_BF16_HILO) return RPCA_ERR_UNSUPPORTED;
  if (d->source < RPCA_SRC_DEVICE || d->source > RPCA_SRC_DEVICE_CALLBACK) return RPCA_ERR_UNSUPPORTED;
  if ((int64_t)(d->i + 1) * d->l > 1024) return RPCA_ERR_UNSUPPORTED;
  return RPCA_OK;
}

void choose_rows(int64_t rows, int64_t per, int maxs, int* ns, int64_t* rps) {
  int64_t s = std::max<int64_t>(1, std::min<int64_t>(maxs, (rows + per - 1) / per));
  int64_t r = round_up((rows + s - 1) / s, 16);
  s = (rows + r - 1) / r;
  *ns = (int)std::max<int64_t>(1, s);
  *rps = std::max<int64_t>(r, 16);
}

}  // namespace

extern "C" {

const char* rpca_status_str(rpca_status s) {
  switch (s) {
    case RPCA_OK: return "ok";
    case RPCA_ERR_INVALID_ARG: return "invalid argument";
    case RPCA_ERR_UNSUPPORTED: return "unsupported";
    case RPCA_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RPCA_ERR_HIP: return "HIP runtime error";
    case RPCA_ERR_CALLBACK: return "panel callback failed";
    case RPCA_ERR_NONFINITE: return "non-finite value in data or iterates";
    case RPCA_ERR_QR_BREAKDOWN: return "QR breakdown (numerically rank-deficient block)";
    case RPCA_ERR_NO_STATE: return "no kept forward state";
    case RPCA_ERR_SCRATCH_LIMIT: return "request needs more scratch than the fixed no-allocation array holds";
  }
  return "unknown status";
}

void rpca_destroy(rpca_plan_t plan) { delete plan; }

rpca_status rpca_plan(const rpca_desc* desc, void* hip_stream, rpca_plan_t* out) {
  if (out == nullptr) return RPCA_ERR_INVALID_ARG;
  *out = nullptr;
  rpca_status vs = validate_desc(desc);
  if (vs != RPCA_OK) return vs;
  // streamed sources carry float32 data
  if (desc->source != RPCA_SRC_DEVICE && desc->storage != RPCA_A_F32) return RPCA_ERR_UNSUPPORTED;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device < 0 || desc->device >= ndev) {
    (void)hipGetLastError();
    return RPCA_ERR_INVALID_ARG;
  }
  rpca_plan_s* plan = new (std::nothrow) rpca_plan_s();
  if (plan == nullptr) return RPCA_ERR_OUT_OF_MEMORY;
  plan->d = *desc;
  plan->device = desc->device;
  plan->stream = reinterpret_cast<hipStream_t>(hip_stream);
  DevGuard g(plan->device);
  auto fail = [&](rpca_status s) {
    delete plan;
    return s;
  };
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, plan->device) != hipSuccess) return fail(RPCA_ERR_HIP);
  plan->max_lds = prop.sharedMemPerBlock;
  set_max_lds(plan->max_lds);
  set_hh_lds_limit(plan->max_lds);

  // m < n: plan the problem of B = A~^T (n x m); float32 A in device memory, no reverse sweep
  const bool trans = desc->m < desc->n;
  if (trans && (desc->storage != RPCA_A_F32 || desc->source != RPCA_SRC_DEVICE ||
                (desc->flags & (RPCA_FLAG_SPLIT_BF16 | RPCA_FLAG_FP64_STEP1 | RPCA_FLAG_KEEP_STATE)) != 0))
    return fail(RPCA_ERR_UNSUPPORTED);
  const int64_t m = trans ? desc->n : desc->m, n = trans ? desc->m : desc->n;
  const int k = desc->k, l = desc->l, i = desc->i, L = (i + 1) * l;
  plan->m = m;
  plan->n = n;
  plan->k = k;
  plan->l = l;
  plan->i = i;
  plan->L = L;
  plan->ldx = round_up(n, 4);
  plan->ldp = round_up(n, 4);

  const int64_t slots = (int64_t)prop.multiProcessorCount * 2;  // two 256-thread blocks per CU
  plan->storage = desc->storage;
  const bool lowp = desc->storage != RPCA_A_F32;
  if (lowp) {
    const int64_t lp_slots = prop.multiProcessorCount;  // one low-precision workgroup per CU (LDS)
    adj_split_lp(desc->storage, m, n, l, lp_slots, &plan->ns_y, &plan->rps_y);
    adj_split_lp(desc->storage, m, n, L, lp_slots, &plan->ns_t, &plan->rps_t);
    fwd_split_lp(desc->storage, m, n, lp_slots, &plan->fwd_ks, &plan->fwd_kchunk);
    plan->ldxs = round_up(n, 64);
    plan->cpad_x = (int)round_up(l, 64);
    plan->ldzs = round_up(m, 64);
    plan->cpad_z = (int)round_up(L, L > 64 ? 192 : 64);  // whole Z tiles of the adjoint
  } else {
    adj_split(m, n, l, slots, &plan->ns_y, &plan->rps_y);
    adj_split(m, n, L, slots, &plan->ns_t, &plan->rps_t);
    fwd_split(m, n, slots, &plan->fwd_ks, &plan->fwd_kchunk);
  }
  choose_rows(m, 4096, 256, &plan->ns_cs, &plan->rps_cs);
  choose_rows(m, 512, 1024, &plan->ns_cn, &plan->rps_cn);
  {
    // Gram / X^T Y row splits over H and Q: short splits (the products are latency bound), as
    // many as keep the float64 partial matrices within 64 MB
    const int64_t cap = std::max<int64_t>(64, std::min<int64_t>(1024, ((int64_t)64 << 20) / (8 * (int64_t)L * L)));
    choose_rows(m, 128, (int)cap, &plan->ns_g, &plan->rps_g);
  }
  choose_rows(n, 80, 256, &plan->ns_gt, &plan->rps_gt);
  if (desc->flags & RPCA_FLAG_SPLIT_BF16) {
    // the split products read A in float pairs from device memory
    if (desc->storage != RPCA_A_F32 || desc->source != RPCA_SRC_DEVICE || n % 2 != 0) return fail(RPCA_ERR_UNSUPPORTED);
    plan->x6 = true;
    plan->ldxs3 = round_up(n + 64, 64);
    plan->cpadx3 = (int)round_up(l, 64);
    plan->xplane3 = (int64_t)plan->cpadx3 * plan->ldxs3;
    plan->ldzs3 = round_up(m, 64);
    plan->cpadz3 = (int)round_up(std::max(L, l + 1), 64);
    plan->zplane3 = (int64_t)plan->cpadz3 * plan->ldzs3;
    plan->rps_y6 = round_up(plan->rps_y, 32);
    plan->ns_y6 = (int)((m + plan->rps_y6 - 1) / plan->rps_y6);
    plan->rps_t6 = round_up(plan->rps_t, 32);
    plan->ns_t6 = (int)((m + plan->rps_t6 - 1) / plan->rps_t6);
  }
  if (desc->flags & RPCA_FLAG_FP64_STEP1) {
    // float64 Step 1 reads float32 A from device memory and keeps no state for
    // the reverse sweep
    if (desc->storage != RPCA_A_F32 || desc->source != RPCA_SRC_DEVICE ||
        (desc->flags & (RPCA_FLAG_SPLIT_BF16 | RPCA_FLAG_KEEP_STATE)) != 0)
      return fail(RPCA_ERR_UNSUPPORTED);
    plan->f64s1 = true;
    plan->ldx64 = round_up(n + F64_KST, 4);
    plan->ldp64 = round_up(n, 4);
    adj64_split(m, n, l, slots, &plan->ns_y64, &plan->rps_y64);
    fwd64_split(m, n, l, slots, &plan->fwd_ks64, &plan->fwd_kchunk64);
  }
  plan->ldpf = ((int64_t)l + 63) / 64 * 64;
  plan->streamed = desc->source != RPCA_SRC_DEVICE;
  if (plan->streamed) {
    const int64_t pr = desc->panel_rows > 0 ? desc->panel_rows : 16384;
    plan->panel_rows = pr < m ? pr : m;
    plan->ldb = round_up(n, 4);
    adj_split(plan->panel_rows, n, l, slots, &plan->ns_py, &plan->rps_py);
    adj_split(plan->panel_rows, n, L, slots, &plan->ns_pt, &plan->rps_pt);
    fwd_split(plan->panel_rows, n, slots, &plan->fwd_ks_p, &plan->fwd_kchunk_p);
    choose_rows(plan->panel_rows, 1024, 64, &plan->ns_pcs, &plan->rps_pcs);
  }

  // Single-read power steps (RPCA_FLAG_FUSED) on float32 A in device memory: a cooperative launch
  // over every CU of a device laid out as 8 XCDs of 32 CUs (MI355X); groups of one XCD when the column
  // slices fit, else of two.  The kernel checks the layout it finds (plan-time dry run below).
  if (!lowp && !plan->x6 && !plan->f64s1 && !trans && !plan->streamed && i > 0 && m >= 32768 &&
      (desc->flags & RPCA_FLAG_FUSED) != 0 && prop.cooperativeLaunch && prop.multiProcessorCount == 256 &&
      plan->max_lds >= 160 * 1024) {
    const int nx = 8, cpx = 32;
    for (int xpg = 1; xpg <= 2 && !plan->fused; ++xpg) {
      const int gs = xpg * cpx, ng = nx / xpg;
      if (!fused_fits(n, l, true, ng, gs)) continue;
      plan->fused = true;
      plan->fu_ngroups = ng;
      plan->fu_xpg = xpg;
      plan->fu_cpx = cpx;
      plan->fu_rpg = round_up((m + ng - 1) / ng, 16);
      plan->fu_nseg = (int)((plan->fu_rpg + 8191) / 8192);
      plan->fu_segrows = round_up((plan->fu_rpg + plan->fu_nseg - 1) / plan->fu_nseg, 16);
    }
  }

  const int64_t ldx = plan->ldx;
  int64_t pcount = std::max<int64_t>((int64_t)plan->ns_y * (l + 1), (int64_t)plan->ns_t * L) * plan->ldp;
  if (plan->fused)
    pcount = std::max<int64_t>(pcount, (int64_t)plan->fu_ngroups * plan->fu_nseg * (l + 1) * plan->ldp);
  if (plan->streamed)
    pcount = std::max<int64_t>(pcount, std::max<int64_t>((int64_t)plan->ns_py * l, (int64_t)plan->ns_pt * L) *
                                           plan->ldp);
  const int64_t LL = (int64_t)L * L;
  plan->sqp_cap = ((n + 255) / 256) * (int64_t)std::max(l, 1) + 16;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, cnt)                                                    \
  do {                                                                     \
    e = plan->alloc(&plan->ptr, (cnt));                                    \
    if (e != hipSuccess)                                                   \
      return fail(e == hipErrorOutOfMemory ? RPCA_ERR_OUT_OF_MEMORY : RPCA_ERR_HIP); \
  } while (0)
  ALLOC(X, (int64_t)(i + 1) * l * ldx);
  ALLOC(shift, ldx);
  ALLOC(mu, n);
  ALLOC(dres, n);
  ALLOC(d0, n);
  ALLOC(H, m * L);
  ALLOC(Q1, m * L);
  ALLOC(Q, m * L);
  ALLOC(Q32, m * L);
  ALLOC(P, pcount);
  if (plan->streamed)
    ALLOC(Pf, plan->fwd_ks_p > 1 ? (int64_t)plan->fwd_ks_p * plan->panel_rows * plan->ldpf : 1);
  else
    ALLOC(Pf, plan->fwd_ks > 1 ? (int64_t)plan->fwd_ks * m * plan->ldpf : 1);
  ALLOC(T, n * L);
  ALLOC(csp, std::max<int64_t>((int64_t)std::max(plan->ns_cs, plan->ns_pcs) * (ldx + L),
                                (int64_t)plan->ns_cn * std::max(L, 1024)));
  ALLOC(gp, (int64_t)std::max(plan->ns_g, plan->ns_gt) * LL);
  ALLOC(Wg, LL);
  ALLOC(R1, LL);
  ALLOC(R2, LL);
  ALLOC(R3, LL);
  ALLOC(Rtmp, LL);
  ALLOC(Rfull, LL);
  ALLOC(Rinv, LL);
  ALLOC(Mg, LL);
  ALLOC(eigwork, (int64_t)syev_small_work(L, L));
  ALLOC(lam, L);
  ALLOC(Wsorted, LL);
  ALLOC(sigL, L);
  ALLOC(Vk, n * k);
  ALLOC(sig, k);
  ALLOC(sgn, k);
  ALLOC(alpha, i + 1);
  ALLOC(zsum, L);
  ALLOC(sqp, plan->sqp_cap);
  ALLOC(corr, L);
  ALLOC(flags, 8);
  if (plan->streamed) {
    ALLOC(dbuf[0], plan->panel_rows * plan->ldb);
    ALLOC(dbuf[1], plan->panel_rows * plan->ldb);
    ALLOC(acc, (int64_t)L * plan->ldp);
    if (desc->source == RPCA_SRC_CALLBACK) {
      for (int q = 0; q < 2; ++q) {
        void* hp = nullptr;
        if (hipHostMalloc(&hp, sizeof(float) * (size_t)(plan->panel_rows * plan->ldb), hipHostMallocDefault) !=
            hipSuccess) {
          (void)hipGetLastError();
          return fail(RPCA_ERR_OUT_OF_MEMORY);
        }
        plan->staging[q] = static_cast<float*>(hp);
      }
    }
    if (hipStreamCreateWithFlags(&plan->cstream, hipStreamNonBlocking) != hipSuccess) return fail(RPCA_ERR_HIP);
    for (int q = 0; q < 2; ++q)
      if (hipEventCreateWithFlags(&plan->ev_ready[q], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&plan->ev_free[q], hipEventDisableTiming) != hipSuccess)
        return fail(RPCA_ERR_HIP);
  }
  if (plan->f64s1) {
    ALLOC(X64, (int64_t)(i + 1) * l * plan->ldx64);
    ALLOC(H64, m * L);
    ALLOC(P64, (int64_t)plan->ns_y64 * l * plan->ldp64);
    ALLOC(Pf64, plan->fwd_ks64 > 1 ? (int64_t)plan->fwd_ks64 * m * l : 1);
    ALLOC(corr64, l);
    if (hipMemset(plan->X64, 0, sizeof(double) * (size_t)((int64_t)(i + 1) * l * plan->ldx64)) != hipSuccess)
      return fail(RPCA_ERR_HIP);
  }
  if (plan->x6) {
    ALLOC(Xp3, 3 * plan->xplane3);
    ALLOC(Zp3, 3 * plan->zplane3);
  }
  if (trans) {
    auto& t = plan->tr;
    t.on = true;
    t.am = n;  // A is am x an with am = the plan's n, an = the plan's m
    t.an = m;
    t.ldxa = round_up(t.an, 4);
    adj_split(t.am, t.an, l, slots, &t.ns_y, &t.rps_y);
    fwd_split(t.am, t.an, slots, &t.fwd_ks, &t.fwd_kchunk);
    t.ldpf = round_up(L, 64);
    choose_rows(t.am, 4096, 256, &t.ns_cs, &t.rps_cs);
    choose_rows(t.am, 512, 1024, &t.ns_cz, &t.rps_cz);
    ALLOC(tr.shift, t.ldxa);
    ALLOC(tr.mu, t.an);
    ALLOC(tr.dres, t.an);
    ALLOC(tr.Z, t.am * L);
    ALLOC(tr.HBt, (int64_t)L * t.ldxa);
    ALLOC(tr.H64, t.an * L);
    ALLOC(tr.P, (int64_t)t.ns_y * l * t.ldxa);
    ALLOC(tr.Pf, t.fwd_ks > 1 ? (int64_t)t.fwd_ks * t.am * t.ldpf : 1);
    ALLOC(tr.sqp, ((t.an + 255) / 256) * (int64_t)l + 16);
    ALLOC(csp, (int64_t)std::max(t.ns_cs, t.ns_cz) * (t.ldxa + L));
    if (hipMemset(plan->tr.shift, 0, sizeof(float) * (size_t)t.ldxa) != hipSuccess ||
        hipMemset(plan->tr.HBt, 0, sizeof(float) * (size_t)(L * t.ldxa)) != hipSuccess)
      return fail(RPCA_ERR_HIP);
  }
  if (lowp) {
    ALLOC(Xh, (int64_t)plan->cpad_x * plan->ldxs);
    ALLOC(Xl, (int64_t)plan->cpad_x * plan->ldxs);
    ALLOC(Zh, (int64_t)plan->cpad_z * plan->ldzs);
    ALLOC(Zl, (int64_t)plan->cpad_z * plan->ldzs);
  }
  if (plan->fused) {
    ALLOC(fu_ws, (int64_t)fused_ws_words());
    ALLOC(fu_xpart, (int64_t)fused_xpart_floats(plan->fu_xpg * plan->fu_cpx));
    ALLOC(fu_xred, (int64_t)fused_xred_floats());
  }
#undef ALLOC
  // zero the padded transposed blocks and the shift once (padding must stay 0)
  if (hipMemset(plan->X, 0, sizeof(float) * (size_t)(i + 1) * l * ldx) != hipSuccess ||
      hipMemset(plan->shift, 0, sizeof(float) * (size_t)ldx) != hipSuccess ||
      hipMemset(plan->P, 0, sizeof(float) * (size_t)pcount) != hipSuccess)
    return fail(RPCA_ERR_HIP);
  if (hipDeviceSynchronize() != hipSuccess) return fail(RPCA_ERR_HIP);
  if (plan->fused) {
    // dry run without rows: the kernel's group set-up checks the XCD layout it meets; any
    // mismatch (or a refused cooperative launch) leaves the plan on the two-launch power steps
    FusedArgs fa;
    fa.A = plan->X;
    fa.lda = ldx;
    fa.m = 0;
    fa.n = n;
    fa.shift = plan->shift;
    fa.Xt = plan->X;
    fa.ldx = ldx;
    fa.ncols = l;
    fa.ones = true;
    fa.Z = plan->H;
    fa.ldz = L;
    fa.P = plan->P;
    fa.ldp = plan->ldp;
    fa.split_stride = (int64_t)(l + 1) * plan->ldp;
    fa.ngroups = plan->fu_ngroups;
    fa.xcc_per_group = plan->fu_xpg;
    fa.cu_per_xcc = plan->fu_cpx;
    fa.gsize = plan->fu_xpg * plan->fu_cpx;
    fa.rows_per_group = plan->fu_rpg;
    fa.nseg = plan->fu_nseg;
    fa.seg_rows = plan->fu_segrows;
    fa.ws = plan->fu_ws;
    fa.xpart = plan->fu_xpart;
    fa.xred = plan->fu_xred;
    unsigned herr = 1u;
    hipError_t le = launch_fused_f32(fa, nullptr);
    if (le == hipSuccess) le = hipDeviceSynchronize();
    if (le == hipSuccess) le = hipMemcpy(&herr, plan->fu_ws + 257, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (le != hipSuccess) (void)hipGetLastError();
    if (le != hipSuccess || herr != 0u) plan->fused = false;
    if (hipMemset(plan->P, 0, sizeof(float) * (size_t)pcount) != hipSuccess) return fail(RPCA_ERR_HIP);
  }
  plan->ev_fwd.resize(16);
  plan->ev_adj.resize(16);
  plan->ev_fused.resize(plan->fused ? 8 : 0);
  for (auto* vec : {&plan->ev_fwd, &plan->ev_adj, &plan->ev_fused})
    for (auto& ev : *vec)
      if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) return fail(RPCA_ERR_HIP);
  if (desc->flags & RPCA_FLAG_PROFILE)
    for (hipEvent_t& e : plan->stage_ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(RPCA_ERR_HIP);
  *out = plan;
  return RPCA_OK;
}

rpca_status rpca_set_device_panel_cb(rpca_plan_t plan, rpca_device_panel_cb cb, void* user) {
  if (plan == nullptr || cb == nullptr) return RPCA_ERR_INVALID_ARG;
  if (plan->d.source != RPCA_SRC_DEVICE_CALLBACK) return RPCA_ERR_UNSUPPORTED;
  plan->dcb = cb;
  plan->dcb_user = user;
  return RPCA_OK;
}

rpca_status rpca_get_stats(rpca_plan_t plan, rpca_stats* out) {
  if (plan == nullptr || out == nullptr) return RPCA_ERR_INVALID_ARG;
  *out = plan->stats;
  return RPCA_OK;
}

}  // extern "C"

namespace {

// Event pair for the next timed panel kernel (null when not profiling or out of pairs).
EventPair* next_fwd_events(rpca_plan_s* plan) {
  if (!(plan->d.flags & RPCA_FLAG_PROFILE) || plan->nev_fwd >= (int)plan->ev_fwd.size()) return nullptr;
  return &plan->ev_fwd[plan->nev_fwd++];
}

// Stage mark q of the PROFILE timing (0 entry, 1 centring, 2 Step 1, 3 Step 2,
// 4 Step 3, 5 Step 4, 6 Steps 5-6), recorded on the plan's stream.
hipError_t mark_stage(rpca_plan_s* plan, int q) {
  if (!(plan->d.flags & RPCA_FLAG_PROFILE) || plan->stage_ev[q] == nullptr) return hipSuccess;
  return hipEventRecord(plan->stage_ev[q], plan->stream);
}

// A bounded wait of the fused power step gave up: its output is not valid.  The plan
// keeps to the two-launch power steps from now on; the call reports the failure.
rpca_status fused_failed(rpca_plan_s* plan) {
  plan->fused = false;
  plan->stats.hip_error = (int32_t)hipErrorLaunchTimeOut;
  return RPCA_ERR_HIP;
}

EventPair* next_fused_events(rpca_plan_s* plan) {
  if (!(plan->d.flags & RPCA_FLAG_PROFILE) || plan->nev_fused >= (int)plan->ev_fused.size()) return nullptr;
  return &plan->ev_fused[plan->nev_fused++];
}

EventPair* next_adj_events(rpca_plan_s* plan) {
  if (!(plan->d.flags & RPCA_FLAG_PROFILE) || plan->nev_adj >= (int)plan->ev_adj.size()) return nullptr;
  return &plan->ev_adj[plan->nev_adj++];
}

// One CholQR round: W = X^T X (+ shift), R = chol(W), Xout = X R^-1.
rpca_status cholqr_round(rpca_plan_s* plan, bool x_f64, const void* X, double* Xout, float* Xout32, double* R,
                         double shift_coef, int* flag) {
  const int L = plan->L;
  const int64_t m = plan->m;
  hipStream_t st = plan->stream;
  RPCA_TRY(launch_gram(x_f64, X, L, m, L, plan->rps_g, plan->ns_g, plan->gp, st));
  RPCA_TRY(launch_gram_reduce(plan->gp, plan->ns_g, L, R, shift_coef, st));
  if (cholinv_fits(L)) {
    RPCA_TRY(launch_cholinv(R, L, 1e-14, flag, plan->Rinv, st));
  } else {
    RPCA_TRY(launch_cholesky(R, L, 1e-14, flag, st));
    RPCA_TRY(launch_triinv(R, L, plan->Rinv, st));
  }
  RPCA_TRY(launch_gemm64(x_f64, X, L, plan->Rinv, L, m, L, L, true, nullptr, Xout, L, Xout32, L, st));
  return RPCA_OK;
}

// Step 2 of last resort, for a basis that is numerically rank deficient beyond
// what one shifted round repairs (condition of H above ~1/u, as the Krylov
// blocks of a spectrum spanning many orders of magnitude are): shifted
// Cholesky QR rounds repeated until the Gram matrix of the current basis has a
// plain Cholesky factorisation, then two plain rounds.  Every round
// right-multiplies by an upper-triangular matrix, so the span is kept up to
// rounding, and each shifted round lifts the directions at rounding level
// towards full rank; they end as an orthonormal completion, the part that the
// trailing columns of a pivoted QR (Step 2) play for such an H.  The product of
// the round factors is kept in Rfull (H = Q Rfull) for the reverse sweep.
rpca_status cholqr_repeated(rpca_plan_s* plan, bool x_f64, const void* H, double** Qout) {
  const int L = plan->L;
  const int64_t m = plan->m, LL = (int64_t)L * L;
  hipStream_t st = plan->stream;
  const double u = 1.1102230246251565e-16;
  const double coef = 11.0 * ((double)m * L + (double)L * (L + 1)) * u;
  const void* X = H;
  bool xf = x_f64;
  double* bufs[2] = {plan->Q1, plan->Q};
  int nb = 0, plain = 0;
  for (int r = 0; r < 12; ++r) {
    RPCA_TRY(launch_gram(xf, X, L, m, L, plan->rps_g, plan->ns_g, plan->gp, st));
    RPCA_TRY(launch_gram_reduce(plan->gp, plan->ns_g, L, plan->R1, 0.0, st));
    RPCA_TRY(hipMemsetAsync(plan->flags + 1, 0, 2 * sizeof(int), st));
    RPCA_TRY(launch_cholinv(plan->R1, L, 1e-14, plan->flags + 1, plan->Rinv, st));
    int hf[2] = {0, 0};
    RPCA_TRY(hipMemcpyAsync(hf, plan->flags + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    RPCA_TRY(hipStreamSynchronize(st));
    if (hf[0] != 0) {
      // W + s I, s = coef trace(W): positive definite in floating point
      RPCA_TRY(launch_gram_reduce(plan->gp, plan->ns_g, L, plan->R1, coef, st));
      RPCA_TRY(launch_cholinv(plan->R1, L, 1e-14, plan->flags + 2, plan->Rinv, st));
      RPCA_TRY(hipMemcpyAsync(hf + 1, plan->flags + 2, sizeof(int), hipMemcpyDeviceToHost, st));
      RPCA_TRY(hipStreamSynchronize(st));
      if (hf[1] != 0) return RPCA_ERR_QR_BREAKDOWN;
      plain = 0;
    } else {
      ++plain;
    }
    double* Xn = bufs[nb];
    nb ^= 1;
    RPCA_TRY(launch_gemm64(xf, X, L, plan->Rinv, L, m, L, L, true, nullptr, Xn, L, plain == 2 ? plan->Q32 : nullptr,
                           L, st));
    if (r == 0) {
      RPCA_TRY(hipMemcpyAsync(plan->Rfull, plan->R1, sizeof(double) * (size_t)LL, hipMemcpyDeviceToDevice, st));
    } else {
      RPCA_TRY(launch_trmm_upper(plan->R1, plan->Rfull, L, plan->Rtmp, st));
      RPCA_TRY(hipMemcpyAsync(plan->Rfull, plan->Rtmp, sizeof(double) * (size_t)LL, hipMemcpyDeviceToDevice, st));
    }
    X = Xn;
    xf = true;
    if (plain == 2) {
      *Qout = Xn;
      return RPCA_OK;
    }
  }
  return RPCA_ERR_QR_BREAKDOWN;
}

// Step 2 by Householder TSQR (qr_householder.hip): orthonormal to rounding for
// any H.  Level 0 takes blocks of at least 2L rows (at most 2048 blocks); each
// higher level stacks the triangles of the level below in pairs.  One
// workgroup per block keeps the block's reflector and its partial sums in LDS:
// (block rows + 16 (L + 1)) doubles, which the device's LDS (160 KB per
// workgroup on gfx950) holds for every L <= 1024 the plan accepts.
rpca_status householder_qr(rpca_plan_s* plan, bool x_f64, const void* H, double** Qout) {
  const int L = plan->L;
  const int64_t m = plan->m, LL = (int64_t)L * L;
  hipStream_t st = plan->stream;
  auto& t = plan->tsqr;
  if (!t.ready) {
    int64_t bu0 = (m + 2047) / 2048;
    if (bu0 < 2 * L) bu0 = 2 * L;
    int nb0 = (int)(m / bu0);
    if (nb0 < 1) nb0 = 1;
    const int64_t last0 = m - (int64_t)(nb0 - 1) * bu0;
    if (!hh_fits(L, last0 > bu0 ? last0 : bu0) || !hh_fits(L, 2 * (int64_t)L)) return RPCA_ERR_QR_BREAKDOWN;
    t.rows.push_back(m);
    t.bu.push_back(bu0);
    t.nb.push_back(nb0);
    while (t.nb.back() > 1) {
      const int prev = t.nb.back();
      t.rows.push_back((int64_t)prev * L);
      t.bu.push_back(2 * (int64_t)L);
      t.nb.push_back(prev / 2 > 1 ? prev / 2 : 1);
    }
    const size_t nl = t.rows.size();
    t.X.assign(nl, nullptr);
    t.tau.assign(nl, nullptr);
    for (size_t q = 0; q < nl; ++q) {
      if (q > 0 && plan->alloc(&t.X[q], t.rows[q] * L) != hipSuccess) return RPCA_ERR_OUT_OF_MEMORY;
      if (plan->alloc(&t.tau[q], (int64_t)t.nb[q] * L) != hipSuccess) return RPCA_ERR_OUT_OF_MEMORY;
    }
    const int64_t orows = nl > 1 ? t.rows[1] : L;
    if (plan->alloc(&t.O[0], orows * L) != hipSuccess || plan->alloc(&t.O[1], orows * L) != hipSuccess ||
        plan->alloc(&t.Rtop, LL) != hipSuccess)
      return RPCA_ERR_OUT_OF_MEMORY;
    t.ready = true;
  }
  const size_t nl = t.rows.size();
  // level 0 works on a float64 copy of H in Q1
  if (x_f64)
    RPCA_TRY(hipMemcpyAsync(plan->Q1, H, sizeof(double) * (size_t)(m * L), hipMemcpyDeviceToDevice, st));
  else
    RPCA_TRY(launch_widen(static_cast<const float*>(H), L, (int)std::min<int64_t>(m, 1 << 30), L, plan->Q1, L, st));
  t.X[0] = plan->Q1;
  for (size_t q = 0; q < nl; ++q)
    RPCA_TRY(launch_hh_factor(t.X[q], t.rows[q], t.bu[q], t.nb[q], L, t.tau[q], q + 1 < nl ? t.X[q + 1] : t.Rtop,
                              st));
  // Q = Q_0 (Q_1 (... Q_top [I; 0])), one level at a time from the top
  const double* C = nullptr;
  for (size_t q = nl; q-- > 0;) {
    double* Y = q == 0 ? plan->Q : t.O[q & 1];
    RPCA_TRY(launch_hh_apply(t.X[q], t.rows[q], t.bu[q], t.nb[q], L, t.tau[q], C, Y, st));
    C = Y;
  }
  RPCA_TRY(launch_to_f32(plan->Q, m, L, L, nullptr, plan->Q32, L, st));
  RPCA_TRY(hipMemcpyAsync(plan->Rfull, t.Rtop, sizeof(double) * (size_t)LL, hipMemcpyDeviceToDevice, st));
  *Qout = plan->Q;
  return RPCA_OK;
}

}  // namespace

namespace {

// One pass over A in row panels (Section 4: rows as they fit), double
// buffered: the copy stream moves panel b into device buffer b % 2 while the
// compute stream works on panel b - 1; `fn(panel, ldb, row0, rows)` enqueues
// the panel's kernels on the compute stream.
template <typename Fn>
rpca_status stream_panels(rpca_plan_s* plan, const float* Ahost, int64_t lda, rpca_panel_cb cb, void* user,
                          Fn&& fn) {
  const int64_t m = plan->m, n = plan->n, pr = plan->panel_rows, ldb = plan->ldb;
  hipStream_t st = plan->stream, cs = plan->cstream;
  const int64_t np = (m + pr - 1) / pr;
  // the buffers may still be read by work already queued on the compute stream
  RPCA_TRY(hipEventRecord(plan->ev_free[0], st));
  RPCA_TRY(hipStreamWaitEvent(cs, plan->ev_free[0], 0));
  // the staging buffers may still be read by the last copies of the previous pass
  if (cb != nullptr) RPCA_TRY(hipStreamSynchronize(cs));
  const bool on_device = plan->d.source == RPCA_SRC_DEVICE_CALLBACK;
  for (int64_t b = 0; b < np; ++b) {
    const int s = (int)(b & 1);
    const int64_t row0 = b * pr;
    const int64_t rows = pr < m - row0 ? pr : m - row0;
    if (b >= 2) RPCA_TRY(hipStreamWaitEvent(cs, plan->ev_free[s], 0));
    const float* src = nullptr;
    int64_t sld = lda;
    if (on_device) {
      // rows generated in place on the fill stream, after panel b - 2 has released the buffer
      if (plan->dcb(plan->dcb_user, row0, rows, plan->dbuf[s], ldb, reinterpret_cast<void*>(cs)) != 0) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamSynchronize(st);
        return RPCA_ERR_CALLBACK;
      }
    } else if (cb != nullptr) {
      // the staging buffer's previous copy must be done before the callback refills it
      if (b >= 2) RPCA_TRY(hipEventSynchronize(plan->ev_ready[s]));
      if (cb(user, row0, rows, plan->staging[s], ldb, nullptr) != 0) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamSynchronize(st);
        return RPCA_ERR_CALLBACK;
      }
      src = plan->staging[s];
      sld = ldb;
    } else {
      src = Ahost + row0 * lda;
    }
    if (on_device) {
    } else if (sld == ldb) {
      RPCA_TRY(hipMemcpyAsync(plan->dbuf[s], src, sizeof(float) * (size_t)(rows * ldb), hipMemcpyHostToDevice, cs));
    } else {
      RPCA_TRY(hipMemcpy2DAsync(plan->dbuf[s], sizeof(float) * (size_t)ldb, src, sizeof(float) * (size_t)sld,
                                sizeof(float) * (size_t)n, (size_t)rows, hipMemcpyHostToDevice, cs));
    }
    RPCA_TRY(hipEventRecord(plan->ev_ready[s], cs));
    RPCA_TRY(hipStreamWaitEvent(st, plan->ev_ready[s], 0));
    rpca_status r = fn(plan->dbuf[s], ldb, row0, rows);
    if (r != RPCA_OK) return r;
    RPCA_TRY(hipEventRecord(plan->ev_free[s], st));
    if (!on_device) plan->stats.h2d_bytes += rows * n * (int64_t)sizeof(float);
  }
  return RPCA_OK;
}

}  // namespace

extern "C" rpca_status rpca_factor(rpca_plan_t plan, const void* A, int64_t lda, const float* col_scale,
                                   rpca_panel_cb cb, void* user, const float* G, float* U, int64_t ldu, float* S,
                                   float* V, int64_t ldv) {
  if (plan == nullptr) return RPCA_ERR_INVALID_ARG;
  const int64_t m = plan->m, n = plan->n;
  const int k = plan->k, l = plan->l, i = plan->i, L = plan->L;
  const int source = plan->d.source;
  if (U == nullptr || S == nullptr || V == nullptr || ldu < k || ldv < k) return RPCA_ERR_INVALID_ARG;
  if (source == RPCA_SRC_CALLBACK) {
    if (cb == nullptr) return RPCA_ERR_INVALID_ARG;
  } else if (source == RPCA_SRC_DEVICE_CALLBACK) {
    if (plan->dcb == nullptr) return RPCA_ERR_INVALID_ARG;
    cb = nullptr;
  } else {
    if (A == nullptr || lda < (plan->tr.on ? plan->tr.an : n)) return RPCA_ERR_INVALID_ARG;
    cb = nullptr;
  }
  const bool streamed = plan->streamed;
  const float* Ahost = streamed ? static_cast<const float*>(A) : nullptr;
  DevGuard g(plan->device);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = plan->stream;
  rpca_stats& sx = plan->stats;
  sx = rpca_stats{};
  plan->have_state = false;
  plan->nev_fwd = plan->nev_adj = plan->nev_fused = 0;
  plan->tp_ev0 = plan->tp_ev1 = 0;
  plan->A_last = streamed ? nullptr : A;
  plan->lda_last = lda;
  const bool center = plan->d.center != 0;
  const bool rescale = !(plan->d.flags & RPCA_FLAG_NO_RESCALE);
  // streamed panels sit in 16-byte aligned device buffers with ldb % 4 == 0
  const bool vec = streamed || (((reinterpret_cast<uintptr_t>(A) & 15) == 0) && (lda % 4 == 0));
  // split products on bfloat16 matrix cores when planned and A is 16-byte aligned with lda % 4 == 0
  const bool x6 = plan->x6 && !streamed && plan->storage == RPCA_A_F32 && vec;
  const int ns_y = x6 ? plan->ns_y6 : plan->ns_y;
  const int64_t ldx = plan->ldx;
  const int storage = plan->storage;
  const bool lowp = storage != RPCA_A_F32;
  // low-precision formats are read 16 bytes at a time from 16-byte aligned rows
  if (lowp && (!vec || lda % 16 != 0)) return RPCA_ERR_INVALID_ARG;
  if (storage == RPCA_A_FP8_E4M3 && col_scale == nullptr) return RPCA_ERR_INVALID_ARG;
  const float* cs = storage == RPCA_A_FP8_E4M3 ? col_scale : nullptr;
  const int64_t plane = storage == RPCA_A_BF16_HILO ? m * lda : 0;
  // bytes per stored element
  const int64_t bpe = storage == RPCA_A_FP8_E4M3 ? 1 : (storage == RPCA_A_BF16 ? 2 : 4);

  RPCA_TRY(hipMemsetAsync(plan->flags, 0, 8 * sizeof(int), st));
  RPCA_TRY(mark_stage(plan, 0));

  // centring: mu = column means (FP64), shift = fl32(mu), d = mu - shift.
  // The panel kernels always read a shift vector: without centring it is the
  // plan's zero-filled buffer (never written for such a plan).
  const float* shift = plan->shift;
  const double* dres = nullptr;
  // Low-precision storage has no in-register shift: d is the whole mean.
  // In-core storage folds the column sums into pass 0's adjoint (no separate
  // pass over A).
  const bool trans = plan->tr.on;
  auto& tr = plan->tr;
  const bool fuse0 = center && !streamed && i >= 1 && !plan->f64s1 && !trans;
  if (center && trans) {
    // column means of A (am x an): shift = fl32(mu), dres = mu - fl32(mu)
    RPCA_TRY(launch_colsum(ST_F32, A, lda, tr.am, tr.an, nullptr, 0, tr.rps_cs, tr.ns_cs, plan->csp, st));
    RPCA_TRY(launch_colsum_reduce(plan->csp, tr.ns_cs, tr.an, 1.0 / (double)tr.am, tr.mu, tr.shift, tr.dres, st));
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  } else if (center && streamed) {
    // a streamed pass of column sums (float64, accumulated over the panels)
    RPCA_TRY(launch_fill_f64(plan->acc, n, 0.0, st));
    rpca_status r = stream_panels(plan, Ahost, lda, cb, user, [&](const float* P, int64_t ldb, int64_t, int64_t rows) {
      RPCA_TRY(launch_colsum(ST_F32, P, ldb, rows, n, nullptr, 0, plan->rps_pcs, plan->ns_pcs, plan->csp, st));
      RPCA_TRY(launch_accumulate_parts(true, plan->csp, plan->ns_pcs, n, 1, n, n, plan->acc, st));
      return RPCA_OK;
    });
    if (r != RPCA_OK) return r;
    RPCA_TRY(launch_colsum_reduce(plan->acc, 1, n, 1.0 / (double)m, plan->mu, plan->shift, plan->dres, st));
    dres = plan->dres;
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  } else if (fuse0) {
    if (!lowp) {
      // shift of pass 0: the column means of the first row panel
      const int64_t rows0 = m < 4096 ? m : 4096;
      int ns0 = 1;
      int64_t rps0 = 0;
      choose_rows(rows0, 1024, 64, &ns0, &rps0);
      RPCA_TRY(launch_colsum(ST_F32, A, lda, rows0, n, nullptr, 0, rps0, ns0, plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, ns0, n, 1.0 / (double)rows0, plan->mu, plan->shift, nullptr, st));
      sx.a_bytes_read += rows0 * n * bpe;
    }
  } else if (center) {
    RPCA_TRY(launch_colsum(storage, A, lda, m, n, cs, plane, plan->rps_cs, plan->ns_cs, plan->csp, st));
    if (lowp) {
      RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cs, n, 1.0 / (double)m, plan->mu, nullptr, nullptr, st));
      dres = plan->mu;
    } else {
      RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cs, n, 1.0 / (double)m, plan->mu, plan->shift, plan->dres,
                                    st));
      dres = plan->dres;
    }
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  }

  RPCA_TRY(mark_stage(plan, 1));

  // Step 1: X_0 = G
  float* X0 = plan->X;
  if (G != nullptr)
    RPCA_TRY(launch_transpose_G(G, l, n, l, X0, ldx, st));
  else
    RPCA_TRY(launch_gen_G(plan->d.seed, n, l, X0, ldx, st));
  RPCA_TRY(launch_fill_f64(plan->alpha, i + 1, 1.0, st));

  // float64 Step 1: H^(j) = alpha_j A~ X_j and X_{j+1} = A~^T H^(j) on the FP64
  // matrix cores, X_0 = G widened exactly; alpha_{j+1} = 1/||X_{j+1}||_F.  With
  // centring A~ = A - 1 mu^T enters as the exact rank-one corrections
  // A~ X = A X - 1 (mu^T X) and A~^T H = A^T H - mu (1^T H) in float64.
  const bool f64s1 = plan->f64s1;
  if (f64s1) {
    const int64_t ldx64 = plan->ldx64;
    RPCA_TRY(launch_widen(X0, ldx, l, n, plan->X64, ldx64, st));
    for (int j = 0; j <= i; ++j) {
      Fwd64Args fa;
      fa.A = static_cast<const float*>(A);
      fa.lda = lda;
      fa.m = m;
      fa.n = n;
      fa.Xt = plan->X64 + (int64_t)j * l * ldx64;
      fa.ldx = ldx64;
      fa.ncols = l;
      fa.alpha = plan->alpha + j;
      if (center) {
        RPCA_TRY(launch_dot_rows64(plan->mu, fa.Xt, ldx64, n, l, plan->corr64, st));
        fa.corr = plan->corr64;
      }
      fa.Z = plan->H64 + (int64_t)j * l;
      fa.ldz = L;
      fa.vec = vec;
      fa.ksplit = plan->fwd_ks64;
      fa.kchunk = plan->fwd_kchunk64;
      fa.P = plan->Pf64;
      fa.ldp = l;
      fa.split_stride = m * l;
      if (EventPair* ev = next_fwd_events(plan)) {
        fa.ev_begin = ev->a;
        fa.ev_end = ev->b;
      }
      RPCA_TRY(launch_fwd64(fa, st));
      sx.passes += 1;
      sx.a_reads += 1;
      sx.a_bytes_read += m * n * bpe;
      if (j == i) break;
      Adj64Args aa;
      aa.A = static_cast<const float*>(A);
      aa.lda = lda;
      aa.m = m;
      aa.n = n;
      aa.Z = fa.Z;
      aa.ldz = L;
      aa.ncols = l;
      aa.rows_per_split = plan->rps_y64;
      aa.nsplit = plan->ns_y64;
      aa.P = plan->P64;
      aa.ldp = plan->ldp64;
      aa.split_stride = (int64_t)l * plan->ldp64;
      aa.vec = vec;
      if (EventPair* ev = next_adj_events(plan)) {
        aa.ev_begin = ev->a;
        aa.ev_end = ev->b;
      }
      RPCA_TRY(launch_adj64(aa, st));
      sx.a_reads += 1;
      sx.a_bytes_read += m * n * bpe;
      if (center) {  // 1^T H^(j)
        RPCA_TRY(launch_colsum_f64(fa.Z, L, m, l, plan->rps_cn, plan->ns_cn, plan->csp, st));
        RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, l, 1.0, plan->zsum, nullptr, nullptr, st));
      }
      int npart = 0;
      RPCA_TRY(launch_reduce_x64(plan->P64, plan->ns_y64, aa.split_stride, plan->ldp64, l, n,
                                 center ? plan->mu : nullptr, center ? plan->zsum : nullptr,
                                 plan->X64 + (int64_t)(j + 1) * l * ldx64, ldx64, plan->sqp, &npart, st));
      RPCA_TRY(launch_finish_scale(plan->sqp, npart, rescale, plan->alpha + j + 1, plan->flags, st));
    }
    RPCA_TRY(launch_check_finite_f64(plan->H64, m, L, L, plan->flags, st));
  }

  // m < n: Step 1 on B = A~^T (the plan's m x n is an x am).  H_B^(j) = A~^T X_B^(j) is an adjoint
  // launch over A with Z = X_B^(j) (am x l, row-major); X_B^(j+1) = alpha_{j+1} A~ H_B^(j) a forward
  // launch with H_B^(j) transposed, alpha_{j+1} = 1/||H_B^(j)||_F.  Centring: A~^T Z =
  // (A - 1 s^T)^T Z - d (1^T Z) and A~ Y = (A - 1 s^T) Y - 1 (d^T Y), s = fl32(mu), d = mu - s.
  for (int j = 0; trans && j <= i; ++j) {
    float* Zj = tr.Z + (int64_t)j * l;
    if (j == 0) {
      if (G != nullptr)
        RPCA_TRY(hipMemcpy2DAsync(tr.Z, sizeof(float) * (size_t)L, G, sizeof(float) * (size_t)l,
                                  sizeof(float) * (size_t)l, (size_t)tr.am, hipMemcpyDeviceToDevice, st));
      else
        RPCA_TRY(launch_transpose_G(X0, ldx, l, (int)tr.am, tr.Z, L, st));
    }
    if (center) {
      RPCA_TRY(launch_colsum(ST_F32, Zj, L, tr.am, l, nullptr, 0, tr.rps_cz, tr.ns_cz, plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, tr.ns_cz, l, 1.0, plan->zsum, nullptr, nullptr, st));
    }
    AdjArgs aa;
    aa.A = A;
    aa.lda = lda;
    aa.m = tr.am;
    aa.n = tr.an;
    aa.shift = tr.shift;
    aa.Z = Zj;
    aa.ldz = L;
    aa.ncols = l;
    aa.rows_per_split = tr.rps_y;
    aa.nsplit = tr.ns_y;
    aa.P = tr.P;
    aa.ldp = tr.ldxa;
    aa.split_stride = (int64_t)l * tr.ldxa;
    aa.vec = vec;
    if (EventPair* ev = next_adj_events(plan)) {
      aa.ev_begin = ev->a;
      aa.ev_end = ev->b;
    }
    RPCA_TRY(launch_adj_f32(aa, st));
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
    const double* dz = center ? tr.dres : nullptr;
    const double* zs = center ? plan->zsum : nullptr;
    RPCA_TRY(launch_reduce_t(tr.P, tr.ns_y, aa.split_stride, tr.ldxa, l, tr.an, nullptr, dz, zs, tr.H64 + (int64_t)j * l,
                             L, st));
    if (j == i) break;
    int npart = 0;
    RPCA_TRY(launch_reduce_y(tr.P, tr.ns_y, aa.split_stride, tr.ldxa, l, tr.an, nullptr, dz, zs, tr.HBt, tr.ldxa,
                             tr.sqp, &npart, st));
    RPCA_TRY(launch_finish_scale(tr.sqp, npart, rescale, plan->alpha + j + 1, plan->flags, st));
    if (center) RPCA_TRY(launch_dot_rows(tr.dres, tr.HBt, tr.ldxa, tr.an, l, plan->corr, st));
    FwdArgs fa;
    fa.A = A;
    fa.lda = lda;
    fa.m = tr.am;
    fa.n = tr.an;
    fa.shift = tr.shift;
    fa.Xt = tr.HBt;
    fa.ldx = tr.ldxa;
    fa.ncols = l;
    fa.corr = center ? plan->corr : nullptr;
    fa.alpha = plan->alpha + j + 1;
    fa.Z = tr.Z + (int64_t)(j + 1) * l;
    fa.ldz = L;
    fa.vec = vec;
    fa.ksplit = tr.fwd_ks;
    fa.kchunk = tr.fwd_kchunk;
    fa.P = tr.Pf;
    fa.ldp = tr.ldpf;
    fa.split_stride = tr.am * tr.ldpf;
    if (EventPair* ev = next_fwd_events(plan)) {
      fa.ev_begin = ev->a;
      fa.ev_end = ev->b;
    }
    RPCA_TRY(launch_fwd_f32(fa, st));
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  }
  if (trans) RPCA_TRY(launch_check_finite_f64(tr.H64, m, L, L, plan->flags, st));

  // streamed: one host-link transfer per pass; each panel runs the forward
  // product and the adjoint of its own rows while it is resident in HBM
  for (int j = 0; streamed && j <= i; ++j) {
    float* Xj = plan->X + (int64_t)j * l * ldx;
    if (center) RPCA_TRY(launch_dot_rows(dres, Xj, ldx, n, l, plan->corr, st));
    if (j < i) RPCA_TRY(launch_fill_f64(plan->acc, (int64_t)l * plan->ldp, 0.0, st));
    rpca_status r = stream_panels(plan, Ahost, lda, cb, user,
                                  [&](const float* P, int64_t ldb, int64_t row0, int64_t rows) {
      FwdArgs fa;
      fa.A = P;
      fa.lda = ldb;
      fa.m = rows;
      fa.n = n;
      fa.shift = shift;
      fa.Xt = Xj;
      fa.ldx = ldx;
      fa.ncols = l;
      fa.corr = center ? plan->corr : nullptr;
      fa.alpha = plan->alpha + j;
      fa.Z = plan->H + row0 * L + (int64_t)j * l;
      fa.ldz = L;
      fa.vec = true;
      fa.ksplit = plan->fwd_ks_p;
      fa.kchunk = plan->fwd_kchunk_p;
      fa.P = plan->Pf;
      fa.ldp = plan->ldpf;
      fa.split_stride = rows * plan->ldpf;
      RPCA_TRY(launch_fwd_f32(fa, st));
      if (j < i) {
        AdjArgs aa;
        aa.A = P;
        aa.lda = ldb;
        aa.m = rows;
        aa.n = n;
        aa.shift = shift;
        aa.Z = fa.Z;
        aa.ldz = L;
        aa.ncols = l;
        aa.rows_per_split = plan->rps_py;
        aa.nsplit = plan->ns_py;
        aa.P = plan->P;
        aa.ldp = plan->ldp;
        aa.split_stride = (int64_t)l * plan->ldp;
        aa.vec = true;
        RPCA_TRY(launch_adj_f32(aa, st));
        RPCA_TRY(launch_accumulate_parts(false, plan->P, plan->ns_py, aa.split_stride, l, n, plan->ldp, plan->acc,
                                         st));
      }
      return RPCA_OK;
    });
    if (r != RPCA_OK) return r;
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
    if (j == i) break;
    if (center) {
      RPCA_TRY(launch_colsum(ST_F32, plan->H + (int64_t)j * l, L, m, l, nullptr, 0, plan->rps_cn, plan->ns_cn,
                             plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, l, 1.0, plan->zsum, nullptr, nullptr, st));
    }
    float* Xn = plan->X + (int64_t)(j + 1) * l * ldx;
    int npart = 0;
    RPCA_TRY(launch_reduce_y64(plan->acc, plan->ldp, l, n, dres, center ? plan->zsum : nullptr, Xn, ldx, plan->sqp,
                               &npart, st));
    RPCA_TRY(launch_finish_scale(plan->sqp, npart, rescale, plan->alpha + j + 1, plan->flags, st));
  }

  // single-read power steps: float32 A in device memory, not the split products
  const bool fused = plan->fused && !lowp && !x6 && !streamed && !f64s1 && !trans;
  for (int j = 0; !streamed && !f64s1 && !trans && j <= i; ++j) {
    float* Xj = plan->X + (int64_t)j * l * ldx;
    // with fused centring, pass 0 writes the uncorrected product (A - 1 s0^T) G and corrects it below
    const bool p0 = fuse0 && j == 0;
    if (center && !p0) RPCA_TRY(launch_dot_rows(dres, Xj, ldx, n, l, plan->corr, st));
    if (fused && j < i) {
      // H^(j) = alpha_j ((A - 1 s^T) X_j - 1 corr^T) and the row-segment partial sums of
      // (A - 1 s^T)^T H^(j) (plus the ones column in pass 0) from one read of A
      FusedArgs fu;
      fu.A = A;
      fu.lda = lda;
      fu.m = m;
      fu.n = n;
      fu.shift = shift;
      fu.Xt = Xj;
      fu.ldx = ldx;
      fu.ncols = l;
      fu.ones = p0;
      fu.corr = (center && !p0) ? plan->corr : nullptr;
      fu.alpha = plan->alpha + j;
      fu.Z = plan->H + (int64_t)j * l;
      fu.ldz = L;
      fu.P = plan->P;
      fu.ldp = plan->ldp;
      fu.split_stride = (int64_t)(p0 ? l + 1 : l) * plan->ldp;
      fu.ngroups = plan->fu_ngroups;
      fu.xcc_per_group = plan->fu_xpg;
      fu.cu_per_xcc = plan->fu_cpx;
      fu.gsize = plan->fu_xpg * plan->fu_cpx;
      fu.rows_per_group = plan->fu_rpg;
      fu.nseg = plan->fu_nseg;
      fu.seg_rows = plan->fu_segrows;
      fu.vec = vec;
      fu.ws = plan->fu_ws;
      fu.xpart = plan->fu_xpart;
      fu.xred = plan->fu_xred;
      if (EventPair* ev = next_fused_events(plan)) {
        fu.ev_begin = ev->a;
        fu.ev_end = ev->b;
      }
      RPCA_TRY(launch_fused_f32(fu, st));
      // a timeout of the kernel's bounded waits is reported through flags[5]
      RPCA_TRY(hipMemcpyAsync(plan->flags + 5, plan->fu_ws + 257, sizeof(int), hipMemcpyDeviceToDevice, st));
      sx.passes += 1;
      sx.a_reads += 1;
      sx.a_bytes_read += m * n * bpe;
      const int nsp = plan->fu_ngroups * plan->fu_nseg;
      if (center) {
        RPCA_TRY(launch_colsum(ST_F32, plan->H + (int64_t)j * l, L, m, l, nullptr, 0, plan->rps_cn, plan->ns_cn,
                               plan->csp, st));
        RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, l, 1.0, plan->zsum, nullptr, nullptr, st));
      }
      if (p0) {
        RPCA_TRY(launch_pass0_center(plan->P, nsp, fu.split_stride, plan->ldp, l, n, m, plan->shift, plan->d0,
                                     plan->mu, plan->dres, st));
        dres = plan->dres;
      }
      float* Xn = plan->X + (int64_t)(j + 1) * l * ldx;
      int npart = 0;
      RPCA_TRY(launch_reduce_y(plan->P, nsp, fu.split_stride, plan->ldp, l, n, nullptr, p0 ? plan->d0 : dres,
                               center ? plan->zsum : nullptr, Xn, ldx, plan->sqp, &npart, st));
      if (p0) {  // H^(0) = (A - 1 s0^T) G - 1 (d0^T G)  (block scale 1)
        RPCA_TRY(launch_dot_rows(plan->d0, Xj, ldx, n, l, plan->corr, st));
        RPCA_TRY(launch_sub_cols(plan->H, L, m, l, plan->corr, st));
      }
      RPCA_TRY(launch_finish_scale(plan->sqp, npart, rescale, plan->alpha + j + 1, plan->flags, st));
      continue;
    }
    FwdArgs fa;
    fa.A = A;
    fa.lda = lda;
    fa.m = m;
    fa.n = n;
    fa.shift = shift;
    fa.Xt = Xj;
    fa.ldx = ldx;
    fa.ncols = l;
    fa.corr = (center && !p0) ? plan->corr : nullptr;
    fa.alpha = plan->alpha + j;
    fa.Z = plan->H + (int64_t)j * l;
    fa.ldz = L;
    fa.vec = vec;
    fa.ksplit = plan->fwd_ks;
    fa.kchunk = plan->fwd_kchunk;
    fa.P = plan->Pf;
    fa.ldp = plan->ldpf;
    fa.split_stride = m * plan->ldpf;
    if (EventPair* ev = next_fwd_events(plan)) {
      fa.ev_begin = ev->a;
      fa.ev_end = ev->b;
    }
    if (lowp) {
      RPCA_TRY(launch_split_x(Xj, ldx, n, l, cs, plan->Xh, plan->Xl, plan->ldxs, plan->cpad_x, st));
      fa.Xh = plan->Xh;
      fa.Xl = plan->Xl;
      fa.ldxs = plan->ldxs;
      fa.plane = plane;
      RPCA_TRY(launch_fwd_lowp(storage, fa, st));
    } else if (x6) {
      RPCA_TRY(launch_split3_x(Xj, ldx, n, l, plan->cpadx3, plan->Xp3, plan->ldxs3, plan->xplane3, st));
      fa.X3 = plan->Xp3;
      fa.ldxs3 = plan->ldxs3;
      fa.xplane3 = plan->xplane3;
      RPCA_TRY(launch_fwd_x6(fa, st));
    } else {
      RPCA_TRY(launch_fwd_f32(fa, st));
    }
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
    if (j == i) break;
    // fused half of the pass: X_{j+1} = A~^T H^(j)
    if (center)
      RPCA_TRY(launch_colsum(ST_F32, plan->H + (int64_t)j * l, L, m, l, nullptr, 0, plan->rps_cn, plan->ns_cn,
                             plan->csp, st));
    if (center) RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, l, 1.0, plan->zsum, nullptr, nullptr, st));
    AdjArgs aa;
    aa.A = A;
    aa.lda = lda;
    aa.m = m;
    aa.n = n;
    aa.shift = shift;
    aa.Z = plan->H + (int64_t)j * l;
    aa.ldz = L;
    aa.ncols = l;
    aa.rows_per_split = x6 ? plan->rps_y6 : plan->rps_y;
    aa.nsplit = ns_y;
    aa.P = plan->P;
    aa.ldp = plan->ldp;
    aa.split_stride = (int64_t)(p0 ? l + 1 : l) * plan->ldp;
    aa.vec = vec;
    aa.ones = p0;
    if (EventPair* ev = next_adj_events(plan)) {
      aa.ev_begin = ev->a;
      aa.ev_end = ev->b;
    }
    if (lowp) {
      // pass 0: an implicit ones column after the l columns of Z gives the column sums
      RPCA_TRY(launch_split_zt(aa.Z, L, m, l, plan->Zh, plan->Zl, plan->ldzs, plan->cpad_z, st, p0));
      aa.Zh = plan->Zh;
      aa.Zl = plan->Zl;
      aa.ldzs = plan->ldzs;
      aa.cpad_z = plan->cpad_z;
      aa.plane = plane;
      if (p0) aa.ncols = l + 1;
      RPCA_TRY(launch_adj_lowp(storage, aa, st));
    } else if (x6) {
      RPCA_TRY(launch_split3_zt(aa.Z, L, m, l, p0, (int)round_up(l + 1, 64), plan->Zp3, plan->ldzs3, plan->zplane3,
                                st));
      aa.Z3 = plan->Zp3;
      aa.ldzs3 = plan->ldzs3;
      aa.zplane3 = plan->zplane3;
      RPCA_TRY(launch_adj_x6(aa, st));
    } else {
      RPCA_TRY(launch_adj_f32(aa, st));
    }
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
    if (p0 && lowp) {
      // mu = column sums / m of the stored matrix; the rank-one correction uses all of it
      RPCA_TRY(launch_pass0_mean_lp(plan->P, ns_y, aa.split_stride, plan->ldp, l, n, m, cs, plan->mu, st));
      dres = plan->mu;
    } else if (p0) {
      // d0 = colsum(A - 1 s0^T)/m; the later passes shift by fl32(s0 + d0)
      RPCA_TRY(launch_pass0_center(plan->P, ns_y, aa.split_stride, plan->ldp, l, n, m, plan->shift, plan->d0,
                                   plan->mu, plan->dres, st));
      dres = plan->dres;
    }
    const double* d0 = lowp ? plan->mu : plan->d0;  // pass 0's correction (s0 = 0 in low precision)
    float* Xn = plan->X + (int64_t)(j + 1) * l * ldx;
    int npart = 0;
    // X_1 = (A - 1 s0^T)^T Z - d0 (1^T Z)^T with Z the uncorrected block (exact: colsum(A - 1 s0^T) = m d0)
    RPCA_TRY(launch_reduce_y(plan->P, ns_y, aa.split_stride, plan->ldp, l, n, cs, p0 ? d0 : dres,
                             center ? plan->zsum : nullptr, Xn, ldx, plan->sqp, &npart, st));
    if (p0) {  // H^(0) = (A - 1 s0^T) G - 1 (d0^T G)  (block scale 1)
      RPCA_TRY(launch_dot_rows(d0, Xj, ldx, n, l, plan->corr, st));
      RPCA_TRY(launch_sub_cols(plan->H, L, m, l, plan->corr, st));
    }
    RPCA_TRY(launch_finish_scale(plan->sqp, npart, rescale, plan->alpha + j + 1, plan->flags, st));
  }
  if (!f64s1 && !trans) RPCA_TRY(launch_check_finite_f32(plan->H, m, L, L, plan->flags, st));
  RPCA_TRY(mark_stage(plan, 2));

  // Step 2: Cholesky QR twice; shifted Cholesky QR three times as the first
  // fallback, repeated shifted rounds as the second, Householder TSQR as the
  // third
  int level = (plan->d.flags & RPCA_FLAG_FORCE_HOUSEHOLDER) != 0 ? 3
              : (plan->d.flags & RPCA_FLAG_FORCE_FALLBACK) != 0 ? 1 : 0;
  double* Qfinal = nullptr;
  // With centring every exact block A~ X_j has zero column sums; the float32
  // rounding of H leaves a component along 1 that the conditioning of H would
  // amplify inside span(Q), so it is removed in float64 before the QR (a no-op
  // in exact arithmetic).
  const bool x_f64 = center || f64s1 || trans;
  const void* Hqr = f64s1    ? static_cast<const void*>(plan->H64)
                    : trans  ? static_cast<const void*>(tr.H64)
                    : center ? static_cast<const void*>(plan->Q)
                             : static_cast<const void*>(plan->H);
  for (int attempt = 0; attempt < 4; ++attempt) {
    RPCA_TRY(hipMemsetAsync(plan->flags + 1, 0, 3 * sizeof(int), st));
    if (center && !f64s1 && !trans) {
      RPCA_TRY(launch_colsum(ST_F32, plan->H, L, m, L, nullptr, 0, plan->rps_cn, plan->ns_cn, plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, L, 1.0, plan->zsum, nullptr, nullptr, st));
      RPCA_TRY(launch_center_cols(plan->H, L, m, L, plan->zsum, 1.0 / (double)m, plan->Q, L, st));
    }
    rpca_status s;
    if (level == 3) {
      s = householder_qr(plan, x_f64, Hqr, &Qfinal);
      if (s != RPCA_OK) return s;
      int hf0[6] = {0, 0, 0, 0, 0, 0};
      RPCA_TRY(hipMemcpyAsync(hf0, plan->flags, 6 * sizeof(int), hipMemcpyDeviceToHost, st));
      RPCA_TRY(hipStreamSynchronize(st));
      if (hf0[5] != 0) return fused_failed(plan);
      if (hf0[0] != 0) return RPCA_ERR_NONFINITE;
      break;
    }
    if (level == 2) {
      s = cholqr_repeated(plan, x_f64, Hqr, &Qfinal);
      if (s == RPCA_ERR_QR_BREAKDOWN) {
        level = 3;
        continue;
      }
      if (s != RPCA_OK) return s;
      int hf0[6] = {0, 0, 0, 0, 0, 0};
      RPCA_TRY(hipMemcpyAsync(hf0, plan->flags, 6 * sizeof(int), hipMemcpyDeviceToHost, st));
      RPCA_TRY(hipStreamSynchronize(st));
      if (hf0[5] != 0) return fused_failed(plan);
      if (hf0[0] != 0) return RPCA_ERR_NONFINITE;
      break;
    }
    if (level == 0) {
      s = cholqr_round(plan, x_f64, Hqr, plan->Q1, nullptr, plan->R1, 0.0, plan->flags + 1);
      if (s != RPCA_OK) return s;
      s = cholqr_round(plan, true, plan->Q1, plan->Q, plan->Q32, plan->R2, 0.0, plan->flags + 2);
      if (s != RPCA_OK) return s;
      Qfinal = plan->Q;
    } else {
      // shift = 11 (m L + L (L+1)) u ||H||_F^2 (shifted Cholesky QR)
      const double u = 1.1102230246251565e-16;
      const double coef = 11.0 * ((double)m * L + (double)L * (L + 1)) * u;
      s = cholqr_round(plan, x_f64, Hqr, plan->Q1, nullptr, plan->R1, coef, plan->flags + 1);
      if (s != RPCA_OK) return s;
      s = cholqr_round(plan, true, plan->Q1, plan->Q, nullptr, plan->R2, 0.0, plan->flags + 2);
      if (s != RPCA_OK) return s;
      s = cholqr_round(plan, true, plan->Q, plan->Q1, plan->Q32, plan->R3, 0.0, plan->flags + 3);
      if (s != RPCA_OK) return s;
      Qfinal = plan->Q1;
    }
    int hf[6] = {0, 0, 0, 0, 0, 0};
    RPCA_TRY(hipMemcpyAsync(hf, plan->flags, 6 * sizeof(int), hipMemcpyDeviceToHost, st));
    RPCA_TRY(hipStreamSynchronize(st));
    if (hf[5] != 0) return fused_failed(plan);
    if (hf[0] != 0) return RPCA_ERR_NONFINITE;
    const bool broke = hf[1] != 0 || hf[2] != 0 || hf[3] != 0;
    if (!broke) break;
    ++level;
  }
  sx.qr_fallback = level;
  RPCA_TRY(mark_stage(plan, 3));

  // Step 3: T = A~^T Q  (n x L, FP64 after the ordered split reduction)
  plan->tp_ev0 = plan->nev_adj;
  if (center && !trans) {
    RPCA_TRY(launch_colsum(ST_F32, plan->Q32, L, m, L, nullptr, 0, plan->rps_cn, plan->ns_cn, plan->csp, st));
    RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, L, 1.0, plan->zsum, nullptr, nullptr, st));
  }
  if (trans) {
    // T_B = B^T Q_B = A~ Q_B (am x L): a forward launch with Q_B transposed, corrected by d^T Q_B;
    // centred, T_B's columns lie in range(A~), orthogonal to 1, so the float32 rounding component
    // along 1 is removed in float64 (a no-op in exact arithmetic)
    RPCA_TRY(launch_transpose_G(plan->Q32, L, tr.an, L, tr.HBt, tr.ldxa, st));
    if (center) RPCA_TRY(launch_dot_rows(tr.dres, tr.HBt, tr.ldxa, tr.an, L, plan->corr, st));
    FwdArgs fa;
    fa.A = A;
    fa.lda = lda;
    fa.m = tr.am;
    fa.n = tr.an;
    fa.shift = tr.shift;
    fa.Xt = tr.HBt;
    fa.ldx = tr.ldxa;
    fa.ncols = L;
    fa.corr = center ? plan->corr : nullptr;
    fa.Z = tr.Z;
    fa.ldz = L;
    fa.vec = vec;
    fa.ksplit = tr.fwd_ks;
    fa.kchunk = tr.fwd_kchunk;
    fa.P = tr.Pf;
    fa.ldp = tr.ldpf;
    fa.split_stride = tr.am * tr.ldpf;
    RPCA_TRY(launch_fwd_f32(fa, st));
    if (center) {
      RPCA_TRY(launch_colsum(ST_F32, tr.Z, L, tr.am, L, nullptr, 0, tr.rps_cz, tr.ns_cz, plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, tr.ns_cz, L, 1.0, plan->zsum, nullptr, nullptr, st));
      RPCA_TRY(launch_center_cols(tr.Z, L, tr.am, L, plan->zsum, 1.0 / (double)tr.am, plan->T, L, st));
    } else {
      RPCA_TRY(launch_widen(tr.Z, L, (int)tr.am, L, plan->T, L, st));
    }
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  } else if (streamed) {
    RPCA_TRY(launch_fill_f64(plan->acc, (int64_t)L * plan->ldp, 0.0, st));
    rpca_status r = stream_panels(plan, Ahost, lda, cb, user,
                                  [&](const float* P, int64_t ldb, int64_t row0, int64_t rows) {
      AdjArgs aa;
      aa.A = P;
      aa.lda = ldb;
      aa.m = rows;
      aa.n = n;
      aa.shift = shift;
      aa.Z = plan->Q32 + row0 * L;
      aa.ldz = L;
      aa.ncols = L;
      aa.rows_per_split = plan->rps_pt;
      aa.nsplit = plan->ns_pt;
      aa.P = plan->P;
      aa.ldp = plan->ldp;
      aa.split_stride = (int64_t)L * plan->ldp;
      aa.vec = true;
      RPCA_TRY(launch_adj_f32(aa, st));
      RPCA_TRY(launch_accumulate_parts(false, plan->P, plan->ns_pt, aa.split_stride, L, n, plan->ldp, plan->acc, st));
      return RPCA_OK;
    });
    if (r != RPCA_OK) return r;
    RPCA_TRY(launch_reduce_t64(plan->acc, plan->ldp, L, n, dres, center ? plan->zsum : nullptr, plan->T, L, st));
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  } else {
    AdjArgs aa;
    aa.A = A;
    aa.lda = lda;
    aa.m = m;
    aa.n = n;
    aa.shift = shift;
    aa.Z = plan->Q32;
    aa.ldz = L;
    aa.ncols = L;
    aa.rows_per_split = x6 ? plan->rps_t6 : plan->rps_t;
    aa.nsplit = x6 ? plan->ns_t6 : plan->ns_t;
    aa.P = plan->P;
    aa.ldp = plan->ldp;
    aa.split_stride = (int64_t)L * plan->ldp;
    aa.vec = vec;
    if (EventPair* ev = next_adj_events(plan)) {
      aa.ev_begin = ev->a;
      aa.ev_end = ev->b;
    }
    if (lowp) {
      RPCA_TRY(launch_split_zt(plan->Q32, L, m, L, plan->Zh, plan->Zl, plan->ldzs, plan->cpad_z, st));
      aa.Zh = plan->Zh;
      aa.Zl = plan->Zl;
      aa.ldzs = plan->ldzs;
      aa.cpad_z = plan->cpad_z;
      aa.plane = plane;
      RPCA_TRY(launch_adj_lowp(storage, aa, st));
    } else if (x6) {
      RPCA_TRY(launch_split3_zt(plan->Q32, L, m, L, false, plan->cpadz3, plan->Zp3, plan->ldzs3, plan->zplane3, st));
      aa.Z3 = plan->Zp3;
      aa.ldzs3 = plan->ldzs3;
      aa.zplane3 = plan->zplane3;
      RPCA_TRY(launch_adj_x6(aa, st));
    } else {
      RPCA_TRY(launch_adj_f32(aa, st));
    }
    RPCA_TRY(launch_reduce_t(plan->P, aa.nsplit, aa.split_stride, plan->ldp, L, n, cs, dres,
                             center ? plan->zsum : nullptr, plan->T, L, st));
    sx.passes += 1;
    sx.a_reads += 1;
    sx.a_bytes_read += m * n * bpe;
  }
  plan->tp_ev1 = plan->nev_adj;
  RPCA_TRY(mark_stage(plan, 4));

  // Step 4: T^T T = W diag(S~^2) W^T (tridiagonal reduction, bisection, inverse iteration)
  RPCA_TRY(launch_gram(true, plan->T, L, n, L, plan->rps_gt, plan->ns_gt, plan->gp, st));
  RPCA_TRY(launch_gram_reduce(plan->gp, plan->ns_gt, L, plan->Mg, 0.0, st));
  const int kvec = (plan->d.flags & RPCA_FLAG_KEEP_STATE) ? L : k;
  RPCA_TRY(launch_syev_small(plan->Mg, L, kvec, plan->eigwork, plan->lam, plan->sigL, plan->Wsorted, L, plan->max_lds,
                             st));
  sx.eig_vectors = kvec;
  RPCA_TRY(mark_stage(plan, 5));

  // Steps 5-6: V = T W_k / ||T W_k|| (signed), S = ||T W_k||, U = Q W_k (signed)
  // (m < n: the plan's U is A's V and the plan's V is A's U)
  float* Uo = trans ? V : U;
  float* Vo = trans ? U : V;
  const int64_t lduo = trans ? ldv : ldu, ldvo = trans ? ldu : ldv;
  RPCA_TRY(launch_gemm64(true, plan->T, L, plan->Wsorted, L, n, k, L, false, nullptr, plan->Vk, k, nullptr, 0, st));
  RPCA_TRY(launch_normalize_sign(plan->Vk, n, k, k, plan->sig, plan->sgn, st));
  RPCA_TRY(launch_gemm64(true, Qfinal, L, plan->Wsorted, L, m, k, L, false, plan->sgn, nullptr, 0, Uo, lduo, st));
  RPCA_TRY(launch_to_f32(plan->Vk, n, k, k, nullptr, Vo, ldvo, st));
  RPCA_TRY(launch_to_f32(plan->sig, 1, k, k, nullptr, S, k, st));
  RPCA_TRY(mark_stage(plan, 6));
  RPCA_TRY(hipStreamSynchronize(st));
  const auto t_end = std::chrono::steady_clock::now();
  sx.ms_total = std::chrono::duration<double, std::milli>(t_end - t0).count();
  if (plan->d.flags & RPCA_FLAG_PROFILE) {
    double* stage_ms[6] = {&sx.ms_colmean, &sx.ms_power, &sx.ms_qr, &sx.ms_tpass, &sx.ms_small_svd, &sx.ms_assemble};
    for (int q = 0; q < 6; ++q) {
      float t = 0.f;
      RPCA_TRY(hipEventElapsedTime(&t, plan->stage_ev[q], plan->stage_ev[q + 1]));
      *stage_ms[q] = t;
    }
    for (int q = 0; q < plan->nev_fwd; ++q) {
      float t = 0.f;
      RPCA_TRY(hipEventElapsedTime(&t, plan->ev_fwd[q].a, plan->ev_fwd[q].b));
      sx.ms_fwd_kernel += t;
    }
    for (int q = 0; q < plan->nev_adj; ++q) {
      float t = 0.f;
      RPCA_TRY(hipEventElapsedTime(&t, plan->ev_adj[q].a, plan->ev_adj[q].b));
      sx.ms_adj_kernel += t;
      if (q >= plan->tp_ev0 && q < plan->tp_ev1) sx.ms_tpass_kernel += t;
    }
    for (int q = 0; q < plan->nev_fused; ++q) {
      float t = 0.f;
      RPCA_TRY(hipEventElapsedTime(&t, plan->ev_fused[q].a, plan->ev_fused[q].b));
      sx.ms_fused_kernel += t;
    }
    sx.fused_launches = plan->nev_fused;
    sx.fwd_launches = plan->nev_fwd;
    sx.adj_launches = plan->nev_adj;
    sx.tpass_launches = plan->tp_ev1 - plan->tp_ev0;
  }
  plan->have_state = true;
  plan->Qfinal_is_Q1 = (Qfinal == plan->Q1);
  return RPCA_OK;
}

extern "C" rpca_status rpca_get_state(rpca_plan_t plan, int32_t which, void* dst, int64_t ld) {
  if (plan == nullptr || dst == nullptr) return RPCA_ERR_INVALID_ARG;
  if (plan->tr.on) return RPCA_ERR_UNSUPPORTED;  // m < n: intermediates belong to A^T's problem
  if (!plan->have_state) return RPCA_ERR_NO_STATE;
  DevGuard g(plan->device);
  const int64_t m = plan->m, n = plan->n;
  const int L = plan->L;
  const void* src = nullptr;
  int64_t rows = 0, cols = 0, lds = 0, esz = 0;
  switch (which) {
    case RPCA_STATE_H:
      if (plan->f64s1) return RPCA_ERR_NO_STATE;
      src = plan->H; rows = m; cols = L; lds = L; esz = 4; break;
    case RPCA_STATE_H64:
      if (!plan->f64s1) return RPCA_ERR_NO_STATE;
      src = plan->H64; rows = m; cols = L; lds = L; esz = 8; break;
    case RPCA_STATE_HSCALE: src = plan->alpha; rows = 1; cols = plan->i + 1; lds = cols; esz = 8; break;
    case RPCA_STATE_Q: src = plan->Qfinal_is_Q1 ? plan->Q1 : plan->Q; rows = m; cols = L; lds = L; esz = 8; break;
    case RPCA_STATE_T: src = plan->T; rows = n; cols = L; lds = L; esz = 8; break;
    case RPCA_STATE_SIGMA: src = plan->sigL; rows = 1; cols = L; lds = L; esz = 8; break;
    case RPCA_STATE_W: src = plan->Wsorted; rows = L; cols = L; lds = L; esz = 8; break;
    case RPCA_STATE_MU:
      if (!plan->d.center) return RPCA_ERR_NO_STATE;
      src = plan->mu; rows = 1; cols = n; lds = n; esz = 8; break;
    default: return RPCA_ERR_INVALID_ARG;
  }
  if (ld < cols) return RPCA_ERR_INVALID_ARG;
  hipError_t e = hipMemcpy2DAsync(dst, (size_t)(ld * esz), src, (size_t)(lds * esz), (size_t)(cols * esz),
                                  (size_t)rows, hipMemcpyDeviceToDevice, plan->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess) {
    plan->stats.hip_error = (int32_t)e;
    (void)hipGetLastError();
    return RPCA_ERR_HIP;
  }
  return RPCA_OK;
}

namespace {

rpca_status backward_alloc(rpca_plan_s* plan) {
  auto& b = plan->bw;
  if (b.ready) return RPCA_OK;
  const int64_t m = plan->m, ldx = plan->ldx;
  const int k = plan->k, l = plan->l, i = plan->i, L = plan->L;
  b.R = (3 * i + 2) * l;
  const int64_t LL = (int64_t)L * L;
  hipError_t e = hipSuccess;
#define BALLOC(ptr, cnt)                                                   \
  do {                                                                     \
    e = plan->alloc(&b.ptr, (cnt));                                        \
    if (e != hipSuccess)                                                   \
      return e == hipErrorOutOfMemory ? RPCA_ERR_OUT_OF_MEMORY : RPCA_ERR_HIP; \
  } while (0)
  BALLOC(Qbar, m * L);
  BALLOC(Hbar, m * L);
  BALLOC(Zf, m * L);
  BALLOC(Zin, m * l);
  BALLOC(Pm, m * b.R);
  BALLOC(Yt, (int64_t)b.R * ldx);
  BALLOC(Xbar, (int64_t)(i > 0 ? i : 1) * l * ldx);
  BALLOC(Tbar, plan->n * L);
  BALLOC(TbarT, (int64_t)L * ldx);
  BALLOC(NtV, (int64_t)L * k);
  BALLOC(Wbar, (int64_t)L * k);
  BALLOC(XV, (int64_t)L * k);
  BALLOC(YW, (int64_t)L * k);
  BALLOC(WT, LL);
  BALLOC(Wsc, LL);
  BALLOC(Nm, LL);
  BALLOC(Tmp, LL);
  BALLOC(Bmat, LL);
  BALLOC(M2, LL);
  BALLOC(Smat, LL);
  BALLOC(Rf, LL);
  BALLOC(Rt, LL);
  BALLOC(RfInv, LL);
  BALLOC(RinvT, LL);
  BALLOC(Ck, (int64_t)k * L);
  BALLOC(Bp, (int64_t)k * L);
  BALLOC(ppart, (int64_t)plan->ns_cs * b.R);
  b.Rp = (b.R + 3) / 4 * 4;
  BALLOC(P32, m * b.Rp);
  BALLOC(Y32, plan->n * b.Rp);
  b.kp3 = (int)round_up(b.R, 32);
  choose_rows(m, 128, 1024, &b.ns_x, &b.rps_x);
  BALLOC(xpart, (int64_t)b.ns_x * LL);
  b.mpad3 = round_up(m, 256);
  b.npad3 = round_up(plan->n, 256);
  BALLOC(P3, 3 * b.mpad3 * b.kp3);
  BALLOC(Y3, 3 * b.npad3 * b.kp3);
#undef BALLOC
  // the K padding of the float32 factors stays zero
  if (hipMemset(b.P32, 0, sizeof(float) * (size_t)(m * b.Rp)) != hipSuccess ||
      hipMemset(b.Y32, 0, sizeof(float) * (size_t)(plan->n * b.Rp)) != hipSuccess)
    return RPCA_ERR_HIP;
  b.ready = true;
  return RPCA_OK;
}

}  // namespace

// Reverse sweep of Steps 1-6 (reading: exact derivative of the computed
// function with G fixed).  Small steps in float64, passes over A on the
// float32 panel kernels, the rank-R factors of dA = P Y^T assembled in float64
// and their product formed from three-part bfloat16 splits of the float32
// factors (six products per K-step on the bfloat16 matrix cores, one 128 x 128
// tile of dA per block, the finiteness check in its epilogue), with
//   P = [Q | a_0 Z_0 .. a_i Z_i | H^(0) .. H^(i-1)],  Y = [T_bar | X_0 .. X_i | X_bar_1 .. X_bar_i]
// where Z_i = H_bar_i, Z_j = H_bar_j + A~ X_bar_{j+1}, X_bar_j = a_j A~^T Z_j, and
// a_j are the positive block scales of the forward (constants: Q does not depend on them).
extern "C" rpca_status rpca_backward(rpca_plan_t plan, const float* gS, const float* gU, int64_t ldgu,
                                     const float* gV, int64_t ldgv, float* dA, int64_t ldda) {
  if (plan == nullptr || dA == nullptr) return RPCA_ERR_INVALID_ARG;
  if (plan->streamed) return RPCA_ERR_UNSUPPORTED;  // the reverse sweep reads A from HBM
  if (!plan->have_state || !(plan->d.flags & RPCA_FLAG_KEEP_STATE) || plan->A_last == nullptr)
    return RPCA_ERR_NO_STATE;
  if (plan->storage != RPCA_A_F32) return RPCA_ERR_UNSUPPORTED;
  const int64_t m = plan->m, n = plan->n, ldx = plan->ldx;
  const int k = plan->k, l = plan->l, i = plan->i, L = plan->L;
  if (ldda < n || (gU != nullptr && ldgu < k) || (gV != nullptr && ldgv < k)) return RPCA_ERR_INVALID_ARG;
  DevGuard g(plan->device);
  rpca_status as = backward_alloc(plan);
  if (as != RPCA_OK) return as;
  auto& b = plan->bw;
  hipStream_t st = plan->stream;
  const int R = b.R;
  const bool center = plan->d.center != 0;
  const double* dres = center ? plan->dres : nullptr;
  const float* A = static_cast<const float*>(plan->A_last);
  const int64_t lda = plan->lda_last;
  const bool vec = ((reinterpret_cast<uintptr_t>(A) & 15) == 0) && (lda % 4 == 0);
  const double* Q = plan->Qfinal_is_Q1 ? plan->Q1 : plan->Q;
  const int64_t LL = (int64_t)L * L;

  // ---- small SVD adjoint: T_bar = T B + V_bar S~^-1 W^T
  if (gU != nullptr)
    RPCA_TRY(launch_xty(true, Q, L, L, false, gU, ldgu, k, m, b.rps_x, b.ns_x, plan->sgn, b.xpart, b.Wbar, st));
  else
    RPCA_TRY(hipMemsetAsync(b.Wbar, 0, sizeof(double) * (size_t)L * k, st));
  if (gV != nullptr)
    RPCA_TRY(launch_xty(true, plan->T, L, L, false, gV, ldgv, k, n, plan->rps_gt, plan->ns_gt, plan->sgn, plan->gp,
                        b.NtV, st));
  else
    RPCA_TRY(hipMemsetAsync(b.NtV, 0, sizeof(double) * (size_t)L * k, st));
  RPCA_TRY(launch_svdadj_prep(plan->Wsorted, plan->sigL, plan->sgn, L, k, b.WT, b.Wsc, b.Ck, b.Bp, st));
  RPCA_TRY(launch_gemm64(true, b.WT, L, b.NtV, k, L, k, L, false, nullptr, b.XV, k, nullptr, 0, st));
  RPCA_TRY(launch_gemm64(true, b.WT, L, b.Wbar, k, L, k, L, false, nullptr, b.YW, k, nullptr, 0, st));
  RPCA_TRY(launch_svdadj_mid(b.XV, b.YW, plan->sigL, gS, L, k, b.Nm, st));
  RPCA_TRY(launch_gemm64(true, b.Wsc, L, b.Nm, L, L, L, L, false, nullptr, b.Tmp, L, nullptr, 0, st));
  RPCA_TRY(launch_gemm64(true, b.Tmp, L, b.WT, L, L, L, L, false, nullptr, b.Bmat, L, nullptr, 0, st));
  RPCA_TRY(launch_gemm64(true, plan->T, L, b.Bmat, L, n, L, L, false, nullptr, b.Tbar, L, nullptr, 0, st));
  if (gV != nullptr)
    RPCA_TRY(launch_gemm64(false, gV, ldgv, b.Ck, L, n, L, k, false, nullptr, b.Tbar, L, nullptr, 0, st, b.Tbar, L));
  // T_bar^T: float32 for the panel product, float64 into the first L rows of Y^T
  RPCA_TRY(launch_transpose_out(b.Tbar, L, n, L, b.TbarT, b.Yt, ldx, st));

  // ---- T = A~^T Q:  Q_bar = G_U' W_k^T + A~ T_bar
  {
    if (center) RPCA_TRY(launch_dot_rows(dres, b.TbarT, ldx, n, L, plan->corr, st));
    // L columns as launches of at most 64 (the last one narrower: 32 columns of matrix-core
    // work for a remainder of up to 32), each with the K split of the l-column products
    for (int c0 = 0; c0 < L; c0 += 64) {
      FwdArgs fa;
      fa.A = A;
      fa.lda = lda;
      fa.m = m;
      fa.n = n;
      fa.shift = plan->shift;
      fa.Xt = b.TbarT + (int64_t)c0 * ldx;
      fa.ldx = ldx;
      fa.ncols = L - c0 < 64 ? L - c0 : 64;
      fa.corr = center ? plan->corr + c0 : nullptr;
      fa.Z = b.Zf + c0;
      fa.ldz = L;
      fa.vec = vec;
      fa.ksplit = plan->fwd_ks;
      fa.kchunk = plan->fwd_kchunk;
      fa.P = plan->Pf;
      fa.ldp = plan->ldpf;
      fa.split_stride = m * plan->ldpf;
      RPCA_TRY(launch_fwd_f32(fa, st));
    }
  }
  if (gU != nullptr) {
    RPCA_TRY(launch_gemm64(false, gU, ldgu, b.Bp, L, m, L, k, false, nullptr, b.Qbar, L, nullptr, 0, st));
    RPCA_TRY(launch_add_f32(b.Zf, L, m, L, b.Qbar, L, true, st));
  } else {
    RPCA_TRY(launch_add_f32(b.Zf, L, m, L, b.Qbar, L, false, st));
  }

  // ---- QR adjoint: H_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T, R = R2 R1 (R3 R2 R1 after the fallback)
  RPCA_TRY(launch_xty(true, b.Qbar, L, L, true, Q, L, L, m, b.rps_x, b.ns_x, nullptr, b.xpart, b.M2, st));
  RPCA_TRY(launch_copyltu_neg(b.M2, L, b.Smat, st));
  RPCA_TRY(launch_gemm64(true, Q, L, b.Smat, L, m, L, L, false, nullptr, b.Qbar, L, nullptr, 0, st, b.Qbar, L));
  if (plan->stats.qr_fallback >= 2) {
    RPCA_TRY(hipMemcpyAsync(b.Rf, plan->Rfull, sizeof(double) * (size_t)LL, hipMemcpyDeviceToDevice, st));
  } else {
    RPCA_TRY(launch_trmm_upper(plan->R2, plan->R1, L, b.Rf, st));
    if (plan->stats.qr_fallback) {
      RPCA_TRY(launch_trmm_upper(plan->R3, b.Rf, L, b.Rt, st));
      RPCA_TRY(hipMemcpyAsync(b.Rf, b.Rt, sizeof(double) * (size_t)LL, hipMemcpyDeviceToDevice, st));
    }
  }
  RPCA_TRY(launch_triinv(b.Rf, L, b.RfInv, st));
  RPCA_TRY(launch_transpose_sq(b.RfInv, L, true, b.RinvT, st));
  RPCA_TRY(launch_gemm64(true, b.Qbar, L, b.RinvT, L, m, L, L, false, nullptr, b.Hbar, L, nullptr, 0, st));

  // ---- reverse power sweep
  const int64_t ldp = R;
  RPCA_TRY(launch_combine(b.Hbar + (int64_t)i * l, L, nullptr, 0, m, l, plan->alpha + i, b.Pm + L + (int64_t)i * l,
                          ldp, b.Zin, l, st));
  for (int j = i; j >= 1; --j) {
    // X_bar_j = A~^T (a_j Z_j)
    if (center) {
      RPCA_TRY(launch_colsum(ST_F32, b.Zin, l, m, l, nullptr, 0, plan->rps_cn, plan->ns_cn, plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, l, 1.0, plan->zsum, nullptr, nullptr, st));
    }
    AdjArgs aa;
    aa.A = A;
    aa.lda = lda;
    aa.m = m;
    aa.n = n;
    aa.shift = plan->shift;
    aa.Z = b.Zin;
    aa.ldz = l;
    aa.ncols = l;
    aa.rows_per_split = plan->rps_y;
    aa.nsplit = plan->ns_y;
    aa.P = plan->P;
    aa.ldp = plan->ldp;
    aa.split_stride = (int64_t)l * plan->ldp;
    aa.vec = vec;
    RPCA_TRY(launch_adj_f32(aa, st));
    float* Xb = b.Xbar + (int64_t)(j - 1) * l * ldx;
    int npart = 0;
    RPCA_TRY(launch_reduce_y(plan->P, plan->ns_y, aa.split_stride, plan->ldp, l, n, nullptr, dres,
                             center ? plan->zsum : nullptr, Xb, ldx, plan->sqp, &npart, st));
    // Z_{j-1} = H_bar_{j-1} + A~ X_bar_j
    if (center) RPCA_TRY(launch_dot_rows(dres, Xb, ldx, n, l, plan->corr, st));
    FwdArgs fa;
    fa.A = A;
    fa.lda = lda;
    fa.m = m;
    fa.n = n;
    fa.shift = plan->shift;
    fa.Xt = Xb;
    fa.ldx = ldx;
    fa.ncols = l;
    fa.corr = center ? plan->corr : nullptr;
    fa.Z = b.Zf;
    fa.ldz = l;
    fa.vec = vec;
    fa.ksplit = plan->fwd_ks;
    fa.kchunk = plan->fwd_kchunk;
    fa.P = plan->Pf;
    fa.ldp = plan->ldpf;
    fa.split_stride = m * plan->ldpf;
    RPCA_TRY(launch_fwd_f32(fa, st));
    RPCA_TRY(launch_combine(b.Hbar + (int64_t)(j - 1) * l, L, b.Zf, l, m, l, plan->alpha + (j - 1),
                            b.Pm + L + (int64_t)(j - 1) * l, ldp, b.Zin, l, st));
  }

  // ---- factors of dA and the dense product
  RPCA_TRY(launch_copy_cols(true, Q, L, m, L, b.Pm, ldp, st));
  if (i > 0) RPCA_TRY(launch_copy_cols(false, plan->H, L, m, i * l, b.Pm + 2 * L, ldp, st));
  RPCA_TRY(launch_widen(plan->X, ldx, L, n, b.Yt + (int64_t)L * ldx, ldx, st));
  if (i > 0) RPCA_TRY(launch_widen(b.Xbar, ldx, i * l, n, b.Yt + (int64_t)2 * L * ldx, ldx, st));
  if (center) RPCA_TRY(launch_center_f64(b.Pm, ldp, m, R, plan->rps_cs, plan->ns_cs, b.ppart, st));
  // dA = P Y^T: P (m x R) and Y = (Y^T)^T (n x R) rounded to float32, the product as the sum
  // of the six bfloat16 products of order <= 2 of their three-part splits (float32-level
  // products on the bfloat16 matrix cores, float32 accumulation over K = R)
  RPCA_TRY(launch_to_f32(b.Pm, m, R, ldp, nullptr, b.P32, b.Rp, st));
  RPCA_TRY(launch_transpose_out(b.Yt, ldx, R, (int)n, b.Y32, nullptr, b.Rp, st));
  RPCA_TRY(launch_split3_rows(b.P32, b.Rp, m, R, b.mpad3, b.kp3, b.P3, st));
  RPCA_TRY(launch_split3_rows(b.Y32, b.Rp, n, R, b.npad3, b.kp3, b.Y3, st));
  // a derivative that is not defined at this A (tied leading S~, or a Step 2 factor that is
  // singular to working precision) shows as non-finite entries, flagged as they are written
  RPCA_TRY(hipMemsetAsync(plan->flags + 4, 0, sizeof(int), st));
  RPCA_TRY(launch_outer_x6(b.P3, b.mpad3, b.Y3, b.npad3, b.kp3, m, n, dA, ldda, plan->flags + 4, st));
  int bad = 0;
  RPCA_TRY(hipMemcpyAsync(&bad, plan->flags + 4, sizeof(int), hipMemcpyDeviceToHost, st));
  RPCA_TRY(hipStreamSynchronize(st));
  return bad != 0 ? RPCA_ERR_NONFINITE : RPCA_OK;
}

// Appendix estimator p_{j,q}(D) of ||D||_2 for D = A~ - U S V^T: the q start
// vectors (Philox stream 9, iid N(0,1)) run through j products with D^T D as
// one block; each column is divided by its norm after every product (which
// changes neither the ratios nor their maximum), the last norms are the
// ratios ||(D^T D)^j w|| / ||(D^T D)^(j-1) w||, and the estimate is the square
// root of the largest.  Passes over A use the float32 panel kernels; the
// rank-k correction and the normalisation run in float64.
extern "C" rpca_status rpca_residual(rpca_plan_t plan, const void* A, int64_t lda, const float* col_scale,
                                     const float* U, int64_t ldu, const float* S, const float* V, int64_t ldv,
                                     int32_t j, int32_t q, uint64_t seed, double* estimate) {
  (void)col_scale;
  if (plan == nullptr || A == nullptr || U == nullptr || S == nullptr || V == nullptr || estimate == nullptr)
    return RPCA_ERR_INVALID_ARG;
  if (plan->storage != RPCA_A_F32 || plan->streamed || plan->tr.on) return RPCA_ERR_UNSUPPORTED;
  const int64_t m = plan->m, n = plan->n, ldx = plan->ldx, ldp = plan->ldp;
  const int k = plan->k;
  if (j < 1 || q < 1 || q > 1024 || lda < n || ldu < k || ldv < k) return RPCA_ERR_INVALID_ARG;
  DevGuard g(plan->device);
  hipStream_t st = plan->stream;
  const bool center = plan->d.center != 0;
  const float* Af = static_cast<const float*>(A);
  const bool vec = ((reinterpret_cast<uintptr_t>(A) & 15) == 0) && (lda % 4 == 0);
  hipDeviceProp_t prop;
  RPCA_TRY(hipGetDeviceProperties(&prop, plan->device));
  int ns = 1;
  int64_t rps = 0;
  adj_split(m, n, q, (int64_t)prop.multiProcessorCount * 2, &ns, &rps);
  // workspace (freed on return)
  if (center && !plan->have_state) return RPCA_ERR_NO_STATE;  // the column means come from rpca_factor
  std::vector<void*> mem;
  bool ok = true;
  auto grab = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
      (void)hipGetLastError();
      ok = false;
      return nullptr;
    }
    mem.push_back(p);
    return p;
  };
  struct Free {
    std::vector<void*>* v;
    ~Free() {
      for (void* p : *v) (void)hipFree(p);
    }
  } freer{&mem};
  double* x = static_cast<double*>(grab(sizeof(double) * (size_t)(n * q)));
  float* xt = static_cast<float*>(grab(sizeof(float) * (size_t)(q * ldx)));
  float* z = static_cast<float*>(grab(sizeof(float) * (size_t)(m * q)));
  double* dx = static_cast<double*>(grab(sizeof(double) * (size_t)(m * q)));
  float* yt = static_cast<float*>(grab(sizeof(float) * (size_t)(q * ldx)));
  double* y = static_cast<double*>(grab(sizeof(double) * (size_t)(n * q)));
  double* c = static_cast<double*>(grab(sizeof(double) * (size_t)(k * q)));
  double* nrm = static_cast<double*>(grab(sizeof(double) * (size_t)q));
  double* sg = static_cast<double*>(grab(sizeof(double) * (size_t)q));
  double* est = static_cast<double*>(grab(sizeof(double)));
  float* part = static_cast<float*>(grab(sizeof(float) * (size_t)(ns * q * ldp)));
  double* xpart = static_cast<double*>(grab(sizeof(double) * (size_t)(std::max(plan->ns_g, plan->ns_gt) * k * q)));
  float* corr = static_cast<float*>(grab(sizeof(float) * (size_t)q));
  double* zsum = static_cast<double*>(grab(sizeof(double) * (size_t)q));
  double* sq = static_cast<double*>(grab(sizeof(double) * (size_t)(((n + 255) / 256) * q + 16)));
  if (!ok) return RPCA_ERR_OUT_OF_MEMORY;
  const double* dres = center ? plan->dres : nullptr;

  RPCA_TRY(launch_gen_normal64(seed, 9u, n, q, x, q, st));
  RPCA_TRY(launch_normalize_sign(x, n, q, q, nrm, sg, st));
  for (int step = 0; step < j; ++step) {
    // D x = A~ x - U (S o (V^T x))
    RPCA_TRY(launch_transpose_out(x, q, n, q, xt, nullptr, ldx, st));
    if (center) RPCA_TRY(launch_dot_rows(dres, xt, ldx, n, q, corr, st));
    FwdArgs fa;
    fa.A = Af;
    fa.lda = lda;
    fa.m = m;
    fa.n = n;
    fa.shift = plan->shift;
    fa.Xt = xt;
    fa.ldx = ldx;
    fa.ncols = q;
    fa.corr = center ? corr : nullptr;
    fa.Z = z;
    fa.ldz = q;
    fa.vec = vec;
    RPCA_TRY(launch_fwd_f32(fa, st));
    RPCA_TRY(launch_add_f32(z, q, m, q, dx, q, false, st));
    RPCA_TRY(launch_xty(false, V, ldv, k, true, x, q, q, n, plan->rps_gt, plan->ns_gt, nullptr, xpart, c, st));
    RPCA_TRY(launch_neg_rowscale(c, S, k, q, st));
    RPCA_TRY(launch_gemm64(false, U, ldu, c, q, m, q, k, false, nullptr, dx, q, z, q, st, dx, q));
    // y = A~^T (D x) - V (S o (U^T D x))
    if (center) {
      RPCA_TRY(launch_colsum(ST_F32, z, q, m, q, nullptr, 0, plan->rps_cn, plan->ns_cn, plan->csp, st));
      RPCA_TRY(launch_colsum_reduce(plan->csp, plan->ns_cn, q, 1.0, zsum, nullptr, nullptr, st));
    }
    AdjArgs aa;
    aa.A = Af;
    aa.lda = lda;
    aa.m = m;
    aa.n = n;
    aa.shift = plan->shift;
    aa.Z = z;
    aa.ldz = q;
    aa.ncols = q;
    aa.rows_per_split = rps;
    aa.nsplit = ns;
    aa.P = part;
    aa.ldp = ldp;
    aa.split_stride = (int64_t)q * ldp;
    aa.vec = vec;
    RPCA_TRY(launch_adj_f32(aa, st));
    int npart = 0;
    RPCA_TRY(launch_reduce_y(part, ns, aa.split_stride, ldp, q, n, nullptr, dres, center ? zsum : nullptr, yt, ldx,
                             sq, &npart, st));
    RPCA_TRY(launch_widen(yt, ldx, q, n, y, n, st));  // y^T (q x n) in float64
    RPCA_TRY(launch_transpose_out(y, n, q, (int)n, nullptr, x, q, st));  // x = y (n x q)
    RPCA_TRY(launch_xty(false, U, ldu, k, true, dx, q, q, m, plan->rps_g, plan->ns_g, nullptr, xpart, c, st));
    RPCA_TRY(launch_neg_rowscale(c, S, k, q, st));
    RPCA_TRY(launch_gemm64(false, V, ldv, c, q, n, q, k, false, nullptr, x, q, nullptr, 0, st, x, q));
    RPCA_TRY(launch_normalize_sign(x, n, q, q, nrm, sg, st));
  }
  RPCA_TRY(launch_sqrt_max(nrm, q, est, st));
  RPCA_TRY(hipMemcpyAsync(estimate, est, sizeof(double), hipMemcpyDeviceToHost, st));
  RPCA_TRY(hipStreamSynchronize(st));
  return RPCA_OK;
}

namespace rpca {
// Row splits of the quantiser's column reductions and the bytes of its scratch:
// column-sum partials [ns][n] float64 and the means [n] float64 (shift_mode 2),
// column-maximum partials [ns][n] float (FP8).  Both quantise entry points use
// this layout, so they reduce in the same split order and store the same bits.
size_t quantize_scratch(int64_t m, int64_t n, int* ns, int64_t* rps) {
  choose_rows(m, 4096, 256, ns, rps);
  return (size_t)*ns * (size_t)n * (sizeof(double) + sizeof(float)) + (size_t)n * sizeof(double);
}

hipError_t quantize_run(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda, void* out, int64_t ldo,
                        float* col_scale, float* shift, int32_t shift_mode, void* scratch, int ns, int64_t rps,
                        hipStream_t st) {
  double* csp = reinterpret_cast<double*>(scratch);
  double* mu = csp + (size_t)ns * n;
  float* amax = reinterpret_cast<float*>(mu + n);
  hipError_t e = hipSuccess;
  if (shift_mode == 2) {
    e = launch_colsum(ST_F32, A, lda, m, n, nullptr, 0, rps, ns, csp, st);
    if (e == hipSuccess) e = launch_colsum_reduce(csp, ns, n, 1.0 / (double)m, mu, shift, nullptr, st);
  }
  if (e == hipSuccess)
    e = launch_quantize(storage, m, n, A, lda, shift_mode != 0 ? shift : nullptr, out, ldo, col_scale, amax, ns, rps,
                        st);
  return e;
}

int quantize_check(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda, const void* out, int64_t ldo,
                   const float* col_scale, const float* shift, int32_t shift_mode) {
  if (storage != RPCA_A_BF16 && storage != RPCA_A_FP8_E4M3 && storage != RPCA_A_BF16_HILO)
    return RPCA_ERR_INVALID_ARG;
  if (m <= 0 || n <= 0 || A == nullptr || out == nullptr || lda < n || ldo < n || ldo % 16 != 0 ||
      (reinterpret_cast<uintptr_t>(out) & 15) != 0)
    return RPCA_ERR_INVALID_ARG;
  if (storage == RPCA_A_FP8_E4M3 && col_scale == nullptr) return RPCA_ERR_INVALID_ARG;
  if (shift_mode < 0 || shift_mode > 2 || (shift_mode != 0 && shift == nullptr)) return RPCA_ERR_INVALID_ARG;
  return RPCA_OK;
}
}  // namespace rpca

extern "C" rpca_status rpca_quantize(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda, void* out,
                                     int64_t ldo, float* col_scale, float* shift, int32_t shift_mode,
                                     void* hip_stream) {
  const int vs = quantize_check(storage, m, n, A, lda, out, ldo, col_scale, shift, shift_mode);
  if (vs != RPCA_OK) return static_cast<rpca_status>(vs);
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  int ns = 1;
  int64_t rps = 0;
  const size_t nbytes = quantize_scratch(m, n, &ns, &rps);
  void* scratch = nullptr;
  hipError_t e = hipMalloc(&scratch, nbytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? RPCA_ERR_OUT_OF_MEMORY : RPCA_ERR_HIP;
  }
  e = quantize_run(storage, m, n, A, lda, out, ldo, col_scale, shift, shift_mode, scratch, ns, rps, st);
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  (void)hipFree(scratch);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return RPCA_ERR_HIP;
  }
  return RPCA_OK;
}
