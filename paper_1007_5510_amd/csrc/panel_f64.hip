// Passes over the float32 data matrix of Step 1 (eqs. first_prod .. last_prod)
// carried in float64 on the gfx950 FP64 matrix cores (v_mfma_f64_16x16x4_f64),
// the arithmetic the paper's experiments use (matrix stored in single
// precision, every computation in double precision, Section 6):
//
//   fwd:  Z = alpha * A X            m x c, X held transposed (Xt, c x n)
//   adj:  P_s = (A_s^T Z_s)^T        c x n per row split s
//
// Every float32 entry of A is exact in float64, so each product is formed
// exactly and only the float64 accumulation rounds.  The float32 kernels
// round every product and chain to 24 bits, which hides the directions that
// the later Krylov blocks carry at relative size below ~1e-7 of the leading
// ones; spectra that need them (a wide range above sigma_{k+1} and a long,
// heavy tail) reach sigma_{k+1} only with this arithmetic.
//
// v_mfma_f64_16x16x4_f64 layout (wave64): A operand lane i + 16 kk holds
// A[i][kk], B operand lane j + 16 kk holds B[kk][j], and the result lane
// j + 16 g, register v holds D[4 v + g][j].
//
// Forward: M = rows of A, N = columns of X, K = columns of A.  Each lane
// loads a float4 of a row of A along K; the four MFMAs of a K-step take its
// four entries, so lane group g covers K = 4 g + t in MFMA t, and X is read
// in the same permuted order from LDS (the sum is unchanged).  A wave owns
// 16 * F64_RT rows and 16 * CT columns; a block of four waves shares each
// staged slice of X.  The K range may be split over blockIdx.y, the partial
// sums then reduced in a fixed order.
//
// Adjoint: M = columns of Z (the Z slice is the A operand), N = columns of A,
// K = rows.  Each lane loads a float4 of a row of A, four consecutive
// columns, one per MFMA of the K-step; the result of MFMA t at lane j + 16 g,
// register v is P[c0 + 4 v + g][cb + 4 j + t], so a lane owns four consecutive
// output columns and sixteen lanes a contiguous run of 64: the partial sums
// are written as 32-byte vectors, coalesced.  Z rows are staged per block in
// LDS.  Rows are split over blocks; the split partial sums are reduced in a
// fixed order.
//
// Rows and columns past the ends are read at clamped, valid addresses and
// never stored; the K (or row) tail shorter than one stage is masked.
#include "common.h"
#include "kernels.h"

namespace rpca {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

namespace {

RPCA_DEV f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool VEC>
RPCA_DEV floatx4 ld4f(const float* __restrict__ p) {
  if (VEC) return *reinterpret_cast<const floatx4*>(p);
  return floatx4{p[0], p[1], p[2], p[3]};
}

// p[k..k+3], entries at or beyond `end` read as zero
RPCA_DEV floatx4 ld4f_masked(const float* __restrict__ p, int64_t k, int64_t end) {
  floatx4 v = {0.f, 0.f, 0.f, 0.f};
  if (k < end) v.x = p[k];
  if (k + 1 < end) v.y = p[k + 1];
  if (k + 2 < end) v.z = p[k + 2];
  if (k + 3 < end) v.w = p[k + 3];
  return v;
}

// logical block b of `total` placed so that consecutive logical blocks share
// an XCD (hardware dispatch is round-robin over the eight XCDs)
RPCA_DEV int64_t f64_xcd_remap(int64_t b, int64_t total) {
  const int64_t q = total / 8, r = total % 8;
  const int64_t x = b % 8, local = b / 8;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

}  // namespace

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
template <int CT, bool VEC>
__global__ __launch_bounds__(256, 2) void fwd64_kernel(const float* __restrict__ A, int64_t lda, int64_t m,
                                                       int64_t n, const double* __restrict__ Xt, int64_t ldx,
                                                       int ncols, int64_t kchunk,
                                                       const double* __restrict__ alpha_ptr,
                                                       const double* __restrict__ corr, double* __restrict__ Z,
                                                       int64_t ldz, int64_t split_stride, int direct) {
  constexpr int RT = F64_RT, KST = F64_KST;
  constexpr int NC = 16 * CT;          // columns of X per block
  constexpr int XP = KST + 2;          // padded LDS row (doubles)
  constexpr int XE = NC * KST / 256;   // doubles of X staged per thread (2 or 4)
  constexpr int TPR = KST / XE;        // threads per staged row of X
  constexpr int KH = KST / 16;         // float4 of A per row tile and stage
  __shared__ double Xs[2][NC][XP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * (64 * RT) + wave * (16 * RT);
  const int sk = blockIdx.y;
  const int c0 = blockIdx.z * NC;
  const int64_t kbeg = (int64_t)sk * kchunk;
  const int64_t kend = kbeg + kchunk < n ? kbeg + kchunk : n;
  const float* __restrict__ arow[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int64_t row = r0 + 16 * r + li;
    arow[r] = A + (row < m ? row : m - 1) * lda;
  }
  const int xc = tid / TPR, xo = (tid % TPR) * XE;
  const double* __restrict__ xsrc = Xt + (int64_t)(c0 + xc < ncols ? c0 + xc : ncols - 1) * ldx;

  f64x4 acc[RT][CT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = f64x4{0.0, 0.0, 0.0, 0.0};

  struct AStage {
    floatx4 a[RT][KH];
  };
  struct XStage {
    f64x2 x[XE / 2];
  };
  auto load_a = [&](AStage& b, int64_t kb) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int h = 0; h < KH; ++h) b.a[r][h] = ld4f<VEC>(arow[r] + kb + 16 * h + 4 * g);
  };
  auto load_x = [&](XStage& b, int64_t kb) {
#pragma unroll
    for (int e = 0; e < XE / 2; ++e) b.x[e] = *reinterpret_cast<const f64x2*>(xsrc + kb + xo + 2 * e);
  };
  auto store_x = [&](const XStage& b, int buf) {
#pragma unroll
    for (int e = 0; e < XE / 2; ++e) *reinterpret_cast<f64x2*>(&Xs[buf][xc][xo + 2 * e]) = b.x[e];
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int h = 0; h < KH; ++h) {
      f64x2 xb[CT][2];
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const double* src = &Xs[buf][16 * c + li][16 * h + 4 * g];
        xb[c][0] = *reinterpret_cast<const f64x2*>(src);
        xb[c][1] = *reinterpret_cast<const f64x2*>(src + 2);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const double a = (double)b.a[r][h][t];
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[r][c] = mfma64(a, xb[c][t >> 1][t & 1], acc[r][c]);
        }
      }
    }
  };

  const int64_t nfull = (kend - kbeg) / KST;
  if (nfull > 0) {
    AStage ac, an;
    XStage xr;
    load_x(xr, kbeg);
    load_a(ac, kbeg);
    store_x(xr, 0);
    __syncthreads();
    for (int64_t st = 0; st < nfull; ++st) {
      const int64_t kn = kbeg + (st + 1 < nfull ? st + 1 : st) * KST;
      load_x(xr, kn);
      load_a(an, kn);
      __builtin_amdgcn_sched_barrier(0);
      compute(ac, (int)(st & 1));
      store_x(xr, (int)((st + 1) & 1));
      __syncthreads();
      ac = an;
    }
  }
  // K tail shorter than one stage: A masked to zero past kend; X is read from
  // its zero-padded rows (ldx >= n + KST), finite everywhere
  const int64_t kt = kbeg + nfull * KST;
  if (kt < kend) {
    const int buf = (int)(nfull & 1);
    AStage at;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int h = 0; h < KH; ++h) at.a[r][h] = ld4f_masked(arow[r], kt + 16 * h + 4 * g, kend);
    XStage xr;
    load_x(xr, kt);
    store_x(xr, buf);
    __syncthreads();
    compute(at, buf);
  }

  const double al = (direct && alpha_ptr != nullptr) ? *alpha_ptr : 1.0;
  double* __restrict__ out = Z + (direct ? 0 : (int64_t)sk * split_stride);
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int col = c0 + 16 * c + li;
      const double cr = (direct && corr != nullptr && col < ncols) ? corr[col] : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * r + 4 * v + g;
        if (row < m && col < ncols) out[row * ldz + col] = direct ? al * (acc[r][c][v] - cr) : acc[r][c][v];
      }
    }
}

// Z[r][c] = alpha * (sum_s P[s][r][c] - corr[c]), splits summed in order
__global__ __launch_bounds__(256) void fwd64_reduce_kernel(const double* __restrict__ P, int nsplit,
                                                           int64_t split_stride, int64_t ldp, int64_t m, int ncols,
                                                           const double* __restrict__ alpha_ptr,
                                                           const double* __restrict__ corr,
                                                           double* __restrict__ Z, int64_t ldz) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * ncols) return;
  const int64_t r = e / ncols;
  const int c = (int)(e % ncols);
  double v = 0.0;
  v += sum_strided(P + r * ldp + c, nsplit, split_stride);
  if (corr != nullptr) v -= corr[c];
  Z[r * ldz + c] = (alpha_ptr != nullptr ? *alpha_ptr : 1.0) * v;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
template <int CT, bool VEC>
__global__ __launch_bounds__(256, 2) void adj64_kernel(const float* __restrict__ A, int64_t lda, int64_t m,
                                                       int64_t n, const double* __restrict__ Z, int64_t ldz,
                                                       int ncols, int64_t rows_per_split, int nsplit, int ctiles,
                                                       double* __restrict__ P, int64_t ldp,
                                                       int64_t split_stride) {
  constexpr int RS = F64_RS;
  constexpr int NC = 16 * CT;         // Z columns per block
  constexpr int ZP = NC + 2;          // padded LDS row (doubles)
  constexpr int ZE = RS * NC / 256;   // Z entries staged per thread (2 or 4)
  constexpr int TPR = NC / ZE;        // threads per staged Z row
  __shared__ double Zs[2][RS][ZP];
  const int64_t total = (int64_t)ctiles * nsplit;
  const int64_t logical = f64_xcd_remap(blockIdx.x, total);
  const int ct = (int)(logical % ctiles);
  const int sp = (int)(logical / ctiles);
  const int c0 = blockIdx.y * NC;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, kk = lane >> 4;
  const int64_t cb = (int64_t)ct * 256 + wave * 64;
  const int64_t cl = cb + 4 * lj;
  const int64_t clc = cl < n ? cl : 0;  // clamped column for the unmasked path
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  const int zr = tid / TPR, zo = (tid % TPR) * ZE;
  int zcol[ZE];
#pragma unroll
  for (int e = 0; e < ZE; ++e) zcol[e] = c0 + zo + e < ncols ? c0 + zo + e : ncols - 1;

  f64x4 acc[CT][4];
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[c][t] = f64x4{0.0, 0.0, 0.0, 0.0};

  struct AStage {
    floatx4 a[RS / 4];
  };
  struct ZStage {
    double z[ZE];
  };
  auto load_a = [&](AStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const float* arow = A + (rb + 4 * q + kk) * lda;
      b.a[q] = VEC ? ld4f<true>(arow + clc) : ld4f_masked(arow, cl, n);
    }
  };
  auto load_z = [&](ZStage& b, int64_t rb) {
    const double* zrow = Z + (rb + zr) * ldz;
#pragma unroll
    for (int e = 0; e < ZE; ++e) b.z[e] = zrow[zcol[e]];
  };
  auto store_z = [&](const ZStage& b, int buf) {
#pragma unroll
    for (int e = 0; e < ZE; ++e) Zs[buf][zr][zo + e] = b.z[e];
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      double za[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) za[c] = Zs[buf][4 * q + kk][16 * c + lj];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double a = (double)b.a[q][t];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c][t] = mfma64(za[c], a, acc[c][t]);
      }
    }
  };

  const int64_t nfull = (rend - rbeg) / RS;
  if (nfull > 0) {
    AStage ac, an;
    ZStage zs;
    load_z(zs, rbeg);
    load_a(ac, rbeg);
    store_z(zs, 0);
    __syncthreads();
    for (int64_t st = 0; st < nfull; ++st) {
      const int64_t rn = rbeg + (st + 1 < nfull ? st + 1 : st) * RS;
      load_z(zs, rn);
      load_a(an, rn);
      __builtin_amdgcn_sched_barrier(0);
      compute(ac, (int)(st & 1));
      store_z(zs, (int)((st + 1) & 1));
      __syncthreads();
      ac = an;
    }
  }
  // tail rows: Z zero past rend, A read at the last row of the split (finite)
  const int64_t rt = rbeg + nfull * RS;
  if (rt < rend) {
    const int buf = (int)(nfull & 1);
    {
      const int64_t r = rt + zr;
      const double* zrow = Z + (r < rend ? r : rend - 1) * ldz;
#pragma unroll
      for (int e = 0; e < ZE; ++e) Zs[buf][zr][zo + e] = r < rend ? zrow[zcol[e]] : 0.0;
    }
    AStage at;
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const int64_t r = rt + 4 * q + kk;
      const float* arow = A + (r < rend ? r : rend - 1) * lda;
      at.a[q] = VEC ? ld4f<true>(arow + clc) : ld4f_masked(arow, cl, n);
    }
    __syncthreads();
    compute(at, buf);
  }

  double* __restrict__ Ps = P + (int64_t)sp * split_stride;
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = c0 + 16 * c + 4 * v + kk;
      if (j >= ncols) continue;
      double* __restrict__ prow = Ps + (int64_t)j * ldp;
      if (cl + 3 < n) {
        *reinterpret_cast<f64x4*>(prow + cl) = f64x4{acc[c][0][v], acc[c][1][v], acc[c][2][v], acc[c][3][v]};
      } else {
        if (cl < n) prow[cl] = acc[c][0][v];
        if (cl + 1 < n) prow[cl + 1] = acc[c][1][v];
        if (cl + 2 < n) prow[cl + 2] = acc[c][2][v];
      }
    }
}

// Xt[j][c] = sum_s P[s][j][c] - d[c] zsum[j] (float64, splits in order); per-block sums of squares
// into sq_part
__global__ __launch_bounds__(256) void reduce_x64_kernel(const double* __restrict__ P, int nsplit,
                                                         int64_t split_stride, int64_t ldp, int64_t n,
                                                         const double* __restrict__ d,
                                                         const double* __restrict__ zsum, double* __restrict__ Xt,
                                                         int64_t ldx, double* __restrict__ sq_part) {
  __shared__ double sh[4];
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  double sq = 0.0;
  if (c < n) {
    const double* p = P + (int64_t)j * ldp + c;
    double v = 0.0;
    v += sum_strided(p, nsplit, split_stride);
    if (d != nullptr) v -= d[c] * zsum[j];
    Xt[(int64_t)j * ldx + c] = v;
    sq = v * v;
  }
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) sq_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// corr[j] = sum_c d[c] Xt[j][c], one block per j, fixed order within a block
__global__ __launch_bounds__(256) void dot_rows64_kernel(const double* __restrict__ d, const double* __restrict__ Xt,
                                                         int64_t ldx, int64_t n, double* __restrict__ corr) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < n; c += 256) s += d[c] * Xt[(int64_t)j * ldx + c];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) corr[j] = sh[0] + sh[1] + sh[2] + sh[3];
}

// part[s][c] = sum of X[r][c] over the rows of split s (one block per split and 64 columns)
__global__ __launch_bounds__(256) void colsum_f64_kernel(const double* __restrict__ X, int64_t ld, int64_t rows,
                                                         int cols, int64_t rows_per_split,
                                                         double* __restrict__ part) {
  __shared__ double sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  const int s = blockIdx.y;
  const int64_t r0 = (int64_t)s * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < rows ? r0 + rows_per_split : rows;
  double v = 0.0;
  if (c < cols)
    for (int64_t r = r0 + w; r < r1; r += 4) v += X[r * ld + c];
  sh[w][threadIdx.x & 63] = v;
  __syncthreads();
  if (w == 0 && c < cols)
    part[(int64_t)s * cols + c] = sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// flag |= 1 when any entry of X (rows x cols, ld) is not finite
__global__ __launch_bounds__(256) void check_finite64_kernel(const double* __restrict__ X, int64_t rows, int cols,
                                                             int64_t ld, int* __restrict__ flag) {
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t tot = rows * cols;
  bool bad = false;
  for (int64_t e = e0; e < tot; e += (int64_t)gridDim.x * 256) {
    const double v = X[(e / cols) * ld + e % cols];
    bad |= !isfinite(v);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void fwd64_split(int64_t m, int64_t n, int ncols, int64_t slots, int* ksplit, int64_t* kchunk) {
  const int64_t rb = (m + 64 * F64_RT - 1) / (64 * F64_RT);
  const int64_t cb = ncols <= 16 ? 1 : (ncols + 31) / 32;
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= 16; ++s) {
    const int64_t chunk = ((n + s - 1) / s + F64_KST - 1) / F64_KST * F64_KST;
    const int64_t ns = (n + chunk - 1) / chunk;
    const int64_t blocks = rb * cb * ns;
    const int64_t rounds = (blocks + slots - 1) / slots;
    const double eff = (double)blocks / (double)(rounds * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = (int)ns;
    }
    if (eff >= 0.94 || chunk <= 4 * F64_KST) break;
  }
  const int64_t chunk = ((n + best - 1) / best + F64_KST - 1) / F64_KST * F64_KST;
  *ksplit = (int)((n + chunk - 1) / chunk);
  *kchunk = chunk;
}

void adj64_split(int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit, int64_t* rows_per_split) {
  const int64_t per = (int64_t)(ncols <= 16 ? 1 : (ncols + 31) / 32) * ((n + 255) / 256);
  int64_t lo = (2 * slots + per - 1) / per;
  int64_t hi = lo * 4 + 8;
  const int64_t maxs = m / 64 > 0 ? m / 64 : 1;
  if (lo > maxs) lo = maxs;
  if (hi > maxs) hi = maxs;
  if (lo < 1) lo = 1;
  double best = -1.0;
  int64_t bs = 1, br = (m + F64_RS - 1) / F64_RS * F64_RS;
  for (int64_t s = lo; s <= hi; ++s) {
    const int64_t r = ((m + s - 1) / s + F64_RS - 1) / F64_RS * F64_RS;
    const int64_t ns = (m + r - 1) / r;
    const int64_t blocks = per * ns;
    const int64_t rounds = (blocks + slots - 1) / slots;
    const double eff = (double)blocks / (double)(rounds * slots);
    if (eff > best + 1e-3) {
      best = eff;
      bs = ns;
      br = r;
    }
  }
  *nsplit = (int)bs;
  *rows_per_split = br;
}

template <int CT>
static void launch_fwd64_ct(const Fwd64Args& a, dim3 grid, double* out, int64_t ldo, int64_t kchunk, bool direct,
                            hipStream_t st) {
  if (a.vec)
    hipLaunchKernelGGL((fwd64_kernel<CT, true>), grid, dim3(256), 0, st, a.A, a.lda, a.m, a.n, a.Xt, a.ldx, a.ncols,
                       kchunk, a.alpha, a.corr, out, ldo, a.split_stride, direct ? 1 : 0);
  else
    hipLaunchKernelGGL((fwd64_kernel<CT, false>), grid, dim3(256), 0, st, a.A, a.lda, a.m, a.n, a.Xt, a.ldx,
                       a.ncols, kchunk, a.alpha, a.corr, out, ldo, a.split_stride, direct ? 1 : 0);
}

hipError_t launch_fwd64(const Fwd64Args& a, hipStream_t st) {
  if (a.m <= 0 || a.ncols <= 0) return hipSuccess;
  if (a.A == nullptr || a.Xt == nullptr || a.Z == nullptr || a.n <= 0) return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldz < a.ncols || a.ldx < a.n + F64_KST || a.ldx % 2 != 0) return hipErrorInvalidValue;
  if (a.vec && (a.lda % 4 != 0 || (reinterpret_cast<uintptr_t>(a.A) & 15) != 0)) return hipErrorInvalidValue;
  const int ns = a.ksplit > 0 ? a.ksplit : 1;
  const int64_t kchunk = ns > 1 ? a.kchunk : a.n;
  if (ns > 1 && (a.P == nullptr || a.kchunk % F64_KST != 0 || (int64_t)ns * a.kchunk < a.n ||
                 a.ldp < a.ncols || a.split_stride < a.m * a.ldp))
    return hipErrorInvalidValue;
  const bool direct = ns == 1;
  const int ct = a.ncols <= 16 ? 1 : 2;
  const int nc = 16 * ct;
  dim3 grid((unsigned)((a.m + 64 * F64_RT - 1) / (64 * F64_RT)), (unsigned)ns, (unsigned)((a.ncols + nc - 1) / nc));
  double* out = direct ? a.Z : a.P;
  const int64_t ldo = direct ? a.ldz : a.ldp;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  if (ct == 1)
    launch_fwd64_ct<1>(a, grid, out, ldo, kchunk, direct, st);
  else
    launch_fwd64_ct<2>(a, grid, out, ldo, kchunk, direct, st);
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  if (e != hipSuccess || direct) return e;
  const int64_t tot = a.m * a.ncols;
  hipLaunchKernelGGL(fwd64_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a.P, ns,
                     a.split_stride, a.ldp, a.m, a.ncols, a.alpha, a.corr, a.Z, a.ldz);
  return hipGetLastError();
}

template <int CT>
static void launch_adj64_ct(const Adj64Args& a, bool vec, int ctiles, hipStream_t st) {
  const int nc = 16 * CT;
  dim3 grid((unsigned)((int64_t)ctiles * a.nsplit), (unsigned)((a.ncols + nc - 1) / nc));
  if (vec)
    hipLaunchKernelGGL((adj64_kernel<CT, true>), grid, dim3(256), 0, st, a.A, a.lda, a.m, a.n, a.Z, a.ldz, a.ncols,
                       a.rows_per_split, a.nsplit, ctiles, a.P, a.ldp, a.split_stride);
  else
    hipLaunchKernelGGL((adj64_kernel<CT, false>), grid, dim3(256), 0, st, a.A, a.lda, a.m, a.n, a.Z, a.ldz,
                       a.ncols, a.rows_per_split, a.nsplit, ctiles, a.P, a.ldp, a.split_stride);
}

hipError_t launch_adj64(const Adj64Args& a, hipStream_t st) {
  if (a.n <= 0 || a.ncols <= 0 || a.nsplit <= 0 || a.m <= 0) return hipSuccess;
  if (a.A == nullptr || a.Z == nullptr || a.P == nullptr) return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldp < a.n || a.ldp % 4 != 0 || a.ldz < a.ncols) return hipErrorInvalidValue;
  if (a.rows_per_split <= 0 || (int64_t)a.nsplit * a.rows_per_split < a.m ||
      (int64_t)(a.nsplit - 1) * a.rows_per_split >= a.m || a.split_stride < (int64_t)a.ncols * a.ldp ||
      a.split_stride % 4 != 0)
    return hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(a.P) & 31) != 0) return hipErrorInvalidValue;
  const bool vec = a.vec && a.n % 4 == 0 && a.lda % 4 == 0 && (reinterpret_cast<uintptr_t>(a.A) & 15) == 0;
  const int ctiles = (int)((a.n + 255) / 256);
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  if (a.ncols <= 16)
    launch_adj64_ct<1>(a, vec, ctiles, st);
  else
    launch_adj64_ct<2>(a, vec, ctiles, st);
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  return e;
}

hipError_t launch_reduce_x64(const double* P, int nsplit, int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                             const double* d, const double* zsum, double* Xt, int64_t ldx, double* sq_part,
                             int* n_sq_part, hipStream_t st) {
  if ((d == nullptr) != (zsum == nullptr)) return hipErrorInvalidValue;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  *n_sq_part = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(reduce_x64_kernel, grid, dim3(256), 0, st, P, nsplit, split_stride, ldp, n, d, zsum, Xt, ldx,
                     sq_part);
  return hipGetLastError();
}

hipError_t launch_dot_rows64(const double* d, const double* Xt, int64_t ldx, int64_t n, int ncols, double* corr,
                             hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(dot_rows64_kernel, dim3((unsigned)ncols), dim3(256), 0, st, d, Xt, ldx, n, corr);
  return hipGetLastError();
}

hipError_t launch_colsum_f64(const double* X, int64_t ld, int64_t rows, int cols, int64_t rows_per_split,
                             int nsplit, double* part, hipStream_t st) {
  if (rows <= 0 || cols <= 0 || nsplit <= 0) return hipSuccess;
  if ((int64_t)nsplit * rows_per_split < rows) return hipErrorInvalidValue;
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)nsplit);
  hipLaunchKernelGGL(colsum_f64_kernel, grid, dim3(256), 0, st, X, ld, rows, cols, rows_per_split, part);
  return hipGetLastError();
}

hipError_t launch_check_finite_f64(const double* X, int64_t rows, int cols, int64_t ld, int* flag, hipStream_t st) {
  const int64_t tot = rows * cols;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(check_finite64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, rows, cols, ld, flag);
  return hipGetLastError();
}

}  // namespace rpca
