// Float64 dense steps that touch only O((i+1) l (m+n)) entries (Section 4:
// Steps 2, 4, 5 and 6 run "in RAM"):
//   Step 2  H = Q R by Cholesky QR applied twice (Gram, Cholesky, Q = H R^-1),
//           with a shifted first round as the fallback for ill-conditioned H;
//   Step 4  the SVD of T through the symmetric eigenproblem of T^T T (the
//           eigensolver itself is in small_eig.hip);
//   Step 5/6 U = Q W_k and V = T W_k / ||T W_k|| with the sign convention.
#include "common.h"
#include "kernels.h"

namespace rpca {

// ---------------------------------------------------------------- Gram X^T X
template <typename TX>
__global__ __launch_bounds__(256) void gram_kernel(const TX* __restrict__ X, int64_t ldx, int64_t rows, int L,
                                                   int64_t rps, int tiles, double* __restrict__ part) {
  __shared__ double XI[16][65];
  __shared__ double XJ[16][65];
  const int ti = blockIdx.x / tiles, tj = blockIdx.x % tiles;
  const int s = blockIdx.y;
  const int I0 = ti * 64, J0 = tj * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int64_t rb = (int64_t)s * rps;
  const int64_t re = rb + rps < rows ? rb + rps : rows;
  for (int64_t r0 = rb; r0 < re; r0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int rr = e >> 6, cc = e & 63;
      const int64_t r = r0 + rr;
      const bool rok = r < re;
      XI[rr][cc] = (rok && I0 + cc < L) ? (double)X[r * ldx + I0 + cc] : 0.0;
      XJ[rr][cc] = (rok && J0 + cc < L) ? (double)X[r * ldx + J0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
      double xi[4], xj[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xi[a] = XI[rr][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) xj[b] = XJ[rr][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xi[a], xj[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)s * L * L;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = I0 + ty + 16 * a, j = J0 + tx + 16 * b;
      if (i < L && j < L) out[(int64_t)i * L + j] = acc[a][b];
    }
}

static size_t g_max_lds_gram();

// ---------------------------------------------------------------- Gram on FP64 matrix cores
// v_mfma_f64_16x16x4_f64: A operand lane i + 16 kk holds A[i][kk], B operand lane j + 16 kk holds
// B[kk][j], D: lane j + 16 g, register v holds D[4 v + g][j] (rows interleaved by lane group,
// unlike the float32 16x16x4 form).  For W = X^T X both operands are
// 16-column slices of the same 4 rows of X.  One workgroup (8 waves) takes a split of rows and up
// to GM_TILES upper-triangular 16 x 16 tiles (ta <= tb); grid.y walks groups of tiles when L is
// large.  Rows are staged 16 at a time in LDS as float64 with a row stride of Lp doubles,
// Lp = 16 (mod 32), so the 4 rows x 16 columns of an operand read hit distinct banks.  Each tile
// is written to the split's partial W and mirrored (the reduction then sums full matrices).
constexpr int GM_WAVES = 8;
constexpr int GM_PER_WAVE = 10;
constexpr int GM_TILES = GM_WAVES * GM_PER_WAVE;
constexpr int GM_ROWS = 16;

typedef double doublex4 __attribute__((ext_vector_type(4)));

static int gram_lp(int L) {
  const int T = (L + 15) / 16;
  const int lp = 16 * T;
  return lp % 32 == 16 ? lp : lp + 16;
}

// GQ >= GM_ROWS * Lp / 512: staged elements per thread (a stage buffer holds
// 512 GQ doubles, the part past GM_ROWS * Lp being padding that every thread
// may write, so the staging has no branches)
template <typename TX, int GQ>
__global__ __launch_bounds__(512) void gram_mfma_kernel(const TX* __restrict__ X, int64_t ldx, int64_t rows, int L,
                                                        int Lp, int64_t rps, int T, int NT,
                                                        double* __restrict__ part) {
  extern __shared__ double gs[];  // [2][512 GQ]
  constexpr int SB = 512 * GQ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = blockIdx.x;
  const int grp = blockIdx.y;
  const int64_t rb = (int64_t)s * rps;
  const int64_t re = rb + rps < rows ? rb + rps : rows;
  // this wave's tiles: t = grp * GM_TILES + q * GM_WAVES + wave, upper triangle in row-major order;
  // slots past the last tile compute tile (0, 0) and are not written
  int ta[GM_PER_WAVE], tb[GM_PER_WAVE];
  bool ok[GM_PER_WAVE];
#pragma unroll
  for (int q = 0; q < GM_PER_WAVE; ++q) {
    int t = grp * GM_TILES + q * GM_WAVES + wave;
    ok[q] = t < NT;
    int a = 0;
    if (!ok[q]) t = 0;
    while (t >= T - a) {
      t -= T - a;
      ++a;
    }
    ta[q] = a;
    tb[q] = a + t;
  }
  // staging: element e = tid + 512 q -> (row e / Lp, column e % Lp) when e < GM_ROWS * Lp
  int srow[GQ], scol[GQ];
#pragma unroll
  for (int q = 0; q < GQ; ++q) {
    const int e = tid + 512 * q;
    srow[q] = e < GM_ROWS * Lp ? e / Lp : GM_ROWS;  // GM_ROWS marks padding
    scol[q] = e < GM_ROWS * Lp ? e % Lp : Lp;
  }
  // raw loads from clamped addresses, masked when stored so that they stay in flight meanwhile
  TX pre[GQ];
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
      const int64_t r = r0 + srow[q];
      pre[q] = X[(r < re ? r : re - 1) * ldx + (scol[q] < L ? scol[q] : L - 1)];
    }
  };
  auto store = [&](double* xs, int64_t r0) {
#pragma unroll
    for (int q = 0; q < GQ; ++q)
      xs[tid + 512 * q] = (r0 + srow[q] < re && scol[q] < L) ? (double)pre[q] : 0.0;
  };
  doublex4 acc[GM_PER_WAVE];
#pragma unroll
  for (int q = 0; q < GM_PER_WAVE; ++q) acc[q] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int kr = lane >> 4, jc = lane & 15;
  if (rb < re) {
    load(rb);
    store(gs, rb);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t r0 = rb; r0 < re; r0 += GM_ROWS) {
    const bool more = r0 + GM_ROWS < re;
    if (more) load(r0 + GM_ROWS);  // next stage in flight during this one
    const double* xs = gs + buf * SB;
#pragma unroll
    for (int kk = 0; kk < GM_ROWS / 4; ++kk) {
      const double* row = xs + (4 * kk + kr) * Lp + jc;
      double av[GM_PER_WAVE], bv[GM_PER_WAVE];
#pragma unroll
      for (int q = 0; q < GM_PER_WAVE; ++q) {
        av[q] = row[16 * ta[q]];
        bv[q] = row[16 * tb[q]];
      }
#pragma unroll
      for (int q = 0; q < GM_PER_WAVE; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc[q], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) store(gs + (buf ^ 1) * SB, r0 + GM_ROWS);
    __syncthreads();
    buf ^= 1;
  }
  double* out = part + (int64_t)s * L * L;
#pragma unroll
  for (int q = 0; q < GM_PER_WAVE; ++q) {
    if (!ok[q]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ta[q] + 4 * v + (lane >> 4);
      const int j = 16 * tb[q] + (lane & 15);
      if (i < L && j < L) {
        out[(int64_t)i * L + j] = acc[q][v];
        if (ta[q] != tb[q]) out[(int64_t)j * L + i] = acc[q][v];
      }
    }
  }
}

hipError_t launch_gram(bool x_is_f64, const void* X, int64_t ldx, int64_t rows, int L, int64_t rows_per_split,
                       int nsplit, double* part, hipStream_t st) {
  const int T = (L + 15) / 16;
  const int NT = T * (T + 1) / 2;
  const int Lp = gram_lp(L);
  const int gq = Lp <= 224 ? 7 : (Lp <= 416 ? 13 : 21);
  const size_t lds = sizeof(double) * 2 * 512 * (size_t)gq;
  if (Lp <= 656 && lds <= g_max_lds_gram()) {
    dim3 grid((unsigned)nsplit, (unsigned)((NT + GM_TILES - 1) / GM_TILES));
#define RPCA_GRAM(GQ)                                                                                           \
  do {                                                                                                          \
    if (x_is_f64)                                                                                               \
      hipLaunchKernelGGL((gram_mfma_kernel<double, GQ>), grid, dim3(512), lds, st, (const double*)X, ldx, rows, L, \
                         Lp, rows_per_split, T, NT, part);                                                      \
    else                                                                                                        \
      hipLaunchKernelGGL((gram_mfma_kernel<float, GQ>), grid, dim3(512), lds, st, (const float*)X, ldx, rows, L,  \
                         Lp, rows_per_split, T, NT, part);                                                      \
  } while (0)
    if (Lp <= 224)
      RPCA_GRAM(7);
    else if (Lp <= 416)
      RPCA_GRAM(13);
    else
      RPCA_GRAM(21);
#undef RPCA_GRAM
    return hipGetLastError();
  }
  const int tiles = (L + 63) / 64;
  dim3 grid((unsigned)(tiles * tiles), (unsigned)nsplit);
  if (x_is_f64)
    hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, st, (const double*)X, ldx, rows, L,
                       rows_per_split, tiles, part);
  else
    hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(256), 0, st, (const float*)X, ldx, rows, L, rows_per_split,
                       tiles, part);
  return hipGetLastError();
}

// 16 elements per block, 16 groups of threads each summing every 16th split, combined in a fixed order
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part, int nsplit, int L,
                                                          double* __restrict__ W) {
  __shared__ double sh[16][16];
  const int t = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t LL = (int64_t)L * L;
  const int64_t e = (int64_t)blockIdx.x * 16 + t;
  double s = 0.0;
  if (e < LL)
    for (int k = g; k < nsplit; k += 16) s += part[(int64_t)k * LL + e];
  sh[g][t] = s;
  __syncthreads();
  if (g != 0 || e >= LL) return;
  double tot = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) tot += sh[q][t];
  W[e] = tot;
}

// diag += coef * trace(W)  (shift of the shifted Cholesky QR)
__global__ __launch_bounds__(256) void add_trace_shift_kernel(double* __restrict__ W, int L, double coef) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < L; i += 256) s += W[(int64_t)i * L + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double shift = coef * sh[0];
  for (int i = threadIdx.x; i < L; i += 256) W[(int64_t)i * L + i] += shift;
}

hipError_t launch_gram_reduce(const double* part, int nsplit, int L, double* W, double shift_coef,
                              hipStream_t st) {
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((LL + 15) / 16)), dim3(256), 0, st, part, nsplit, L, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || shift_coef == 0.0) return e;
  hipLaunchKernelGGL(add_trace_shift_kernel, dim3(1), dim3(256), 0, st, W, L, shift_coef);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Cholesky
// Right-looking Cholesky of the symmetric positive definite W = R^T R (upper
// R) by one workgroup.  With PACKED the upper triangle lives in LDS, else the
// factorisation runs in place in global memory (visible to the whole
// workgroup after each barrier).  A pivot at or below rel_tol times the
// original diagonal entry marks breakdown (flag = first bad column + 1); the
// factorisation then continues with a unit pivot so the kernel always ends.
struct TriAcc {
  double* p;
  int L;
  bool packed;
  RPCA_DEV double& at(int i, int j) const {
    return packed ? p[(int64_t)i * L - (int64_t)i * (i - 1) / 2 + (j - i)] : p[(int64_t)i * L + j];
  }
};

template <bool PACKED>
__global__ __launch_bounds__(1024) void cholesky_kernel(double* __restrict__ W, int L, double rel_tol,
                                                        int* __restrict__ flag) {
  extern __shared__ double smem[];
  __shared__ double s_piv;
  double* d0 = smem;  // L original diagonal entries
  TriAcc a{PACKED ? smem + L : W, L, PACKED};
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < L; i += nt) d0[i] = W[(int64_t)i * L + i];
  if (PACKED) {
    for (int64_t e = tid; e < (int64_t)L * L; e += nt) {
      const int i = (int)(e / L), j = (int)(e % L);
      if (j >= i) a.at(i, j) = W[e];
    }
  }
  __syncthreads();
  for (int k = 0; k < L; ++k) {
    if (tid == 0) {
      double p = a.at(k, k);
      const bool ok = isfinite(p) && p > rel_tol * d0[k] && p > 0.0;
      if (!ok) {
        atomicCAS(flag, 0, k + 1);
        p = 1.0;
      }
      s_piv = sqrt(p);
    }
    __syncthreads();
    const double piv = s_piv;
    const double inv = 1.0 / piv;
    for (int j = k + tid; j < L; j += nt) a.at(k, j) = (j == k) ? piv : a.at(k, j) * inv;
    __syncthreads();
    const int mrem = L - k - 1;
    const int64_t tot = (int64_t)mrem * mrem;
    for (int64_t e = tid; e < tot; e += nt) {
      const int ii = (int)(e / mrem), jj = (int)(e % mrem);
      if (jj >= ii) {
        const int i = k + 1 + ii, j = k + 1 + jj;
        a.at(i, j) -= a.at(k, i) * a.at(k, j);
      }
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < (int64_t)L * L; e += nt) {
    const int i = (int)(e / L), j = (int)(e % L);
    if (j < i)
      W[e] = 0.0;
    else if (PACKED)
      W[e] = a.at(i, j);
  }
}

static size_t g_max_lds = 65536;  // per-workgroup LDS limit of the current device
void set_max_lds(size_t bytes) { g_max_lds = bytes; }
static size_t g_max_lds_gram() { return g_max_lds; }

hipError_t launch_cholesky(double* W, int L, double rel_tol, int* flag, hipStream_t st) {
  const size_t bytes = ((size_t)L + (size_t)L * (L + 1) / 2) * sizeof(double);
  if (bytes <= g_max_lds) {
    hipLaunchKernelGGL(cholesky_kernel<true>, dim3(1), dim3(1024), bytes, st, W, L, rel_tol, flag);
  } else {
    hipLaunchKernelGGL(cholesky_kernel<false>, dim3(1), dim3(1024), (size_t)L * sizeof(double), st, W, L, rel_tol,
                       flag);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- R^-1
// Rows of X = R^-1 (upper triangular) are produced from the bottom up:
// X[i][i] = 1/R[i][i] and X[i][j] = -(sum_{p=i+1..j} R[i][p] X[p][j]) / R[i][i]
// only needs rows below i, so every column j of row i is computed in
// parallel, with a power-of-two group of threads splitting each dot product.
__global__ __launch_bounds__(1024) void triinv_kernel(const double* __restrict__ R, int L, double* __restrict__ X) {
  extern __shared__ double rrow[];  // row i of R
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t t = tid; t < (int64_t)L * L; t += nt) {
    const int i = (int)(t / L), j = (int)(t % L);
    if (j < i) X[t] = 0.0;
  }
  for (int i = L - 1; i >= 0; --i) {
    __syncthreads();
    for (int j = i + tid; j < L; j += nt) rrow[j] = R[(int64_t)i * L + j];
    __syncthreads();
    const int ncol = L - i;
    int G = 1;
    while (G * 2 * ncol <= nt && G < 64) G *= 2;
    const double inv = 1.0 / rrow[i];
    for (int base = 0; base < ncol * G; base += nt) {
      const int t = base + tid;
      const int c = t / G, part = t % G;
      const int j = i + c;
      double s = 0.0;
      if (c < ncol) {
        for (int p = i + 1 + part; p <= j; p += G) s = fma(rrow[p], X[(int64_t)p * L + j], s);
      }
      for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (c < ncol && part == 0) X[(int64_t)i * L + j] = (j == i) ? inv : -s * inv;
    }
  }
}

// ---------------------------------------------------------------- Cholesky and R^-1 in one workgroup
// W (L x L symmetric, upper triangle read) = R^T R.  Each of the 1024 threads keeps up to E entries
// (i <= j) of the upper triangle in registers, fixed at the start; step k publishes row k through
// a double-buffered LDS row and every thread applies the rank-one update to its own entries with
// i > k, using the unscaled pivot row (a_ij -= a_ki a_kj / p_k), so one barrier per step suffices;
// rows are scaled by 1/sqrt(p_k) at the end.  A pivot that is not finite, not positive or below
// rel_tol times the original diagonal sets *flag = k + 1 (first such k) and is replaced by 1.
// Then R^-1 (upper) is formed by columns, thread j back-substituting column j against R held packed
// in LDS (no barriers); its entries live in Rinv (each thread touches only its own column).
template <int E, bool INV>
__global__ __launch_bounds__(1024) void cholinv_kernel(double* __restrict__ W, int L, double rel_tol,
                                                       int* __restrict__ flag, double* __restrict__ Rinv) {
  extern __shared__ double cs[];
  double* row = cs;              // [2][L]
  double* piv = cs + 2 * L;      // [L]
  double* dorig = cs + 3 * L;    // [L]
  double* rp = cs + 4 * L;       // packed R (upper, row-major), L (L + 1) / 2
  const int tid = threadIdx.x;
  const int64_t NT = (int64_t)L * (L + 1) / 2;
  double a[E];
  int ij[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    int64_t e = tid + 1024 * (int64_t)q;
    int i = 0;
    if (e < NT) {
      while (e >= L - i) {
        e -= L - i;
        ++i;
      }
      const int j = i + (int)e;
      ij[q] = (i << 16) | j;
      a[q] = W[(int64_t)i * L + j];
    } else {
      ij[q] = -1;
      a[q] = 0.0;
    }
  }
  for (int k = tid; k < L; k += 1024) dorig[k] = W[(int64_t)k * L + k];
  for (int k = 0; k < L; ++k) {
    double* rb = row + (k & 1) * L;
#pragma unroll
    for (int q = 0; q < E; ++q)
      if (ij[q] >= 0 && (ij[q] >> 16) == k) rb[ij[q] & 0xFFFF] = a[q];
    __syncthreads();
    double p = rb[k];
    const bool ok = isfinite(p) && p > 0.0 && p > rel_tol * dorig[k];
    if (!ok) p = 1.0;
    if (tid == 0) {
      piv[k] = p;
      if (!ok) atomicCAS(flag, 0, k + 1);
    }
    const double ip = 1.0 / p;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (ij[q] >= 0 && (ij[q] >> 16) > k) a[q] -= rb[ij[q] >> 16] * rb[ij[q] & 0xFFFF] * ip;
    }
  }
  __syncthreads();
  // R = D^-1/2 (unscaled rows); write R (lower triangle zero) and its packed copy
#pragma unroll
  for (int q = 0; q < E; ++q) {
    if (ij[q] < 0) continue;
    const int i = ij[q] >> 16, j = ij[q] & 0xFFFF;
    const double sq = sqrt(piv[i]);
    const double r = (i == j) ? sq : a[q] / sq;
    W[(int64_t)i * L + j] = r;
    if (j > i) W[(int64_t)j * L + i] = 0.0;
    if (INV) rp[(int64_t)i * L - (int64_t)i * (i - 1) / 2 + (j - i)] = r;
  }
  if (!INV) return;
  __syncthreads();
  for (int j = tid; j < L; j += 1024) {
    double* x = Rinv + j;  // column j, stride L
    for (int i = j + 1; i < L; ++i) x[(int64_t)i * L] = 0.0;
    const double* rjj = rp + (int64_t)j * L - (int64_t)j * (j - 1) / 2;
    x[(int64_t)j * L] = 1.0 / rjj[0];
    for (int i = j - 1; i >= 0; --i) {
      const double* ri = rp + (int64_t)i * L - (int64_t)i * (i - 1) / 2;  // ri[p - i] = R(i, p)
      double s = 0.0;
      for (int pp = i + 1; pp <= j; ++pp) s = fma(ri[pp - i], x[(int64_t)pp * L], s);
      x[(int64_t)i * L] = -s / ri[0];
    }
  }
}

static size_t cholinv_lds(int L) { return sizeof(double) * (4 * (size_t)L + (size_t)L * (L + 1) / 2); }

// the triangle must fit 16 entries per thread (L <= 180) and R packed must fit in LDS
// ---------------------------------------------------------------- blocked
// Cholesky and triangular inverse in LDS for L <= 192, by 16 x 16 blocks on
// FP64 matrix cores (v_mfma_f64_16x16x4f64).  The matrix is padded to
// Lp = 16 ceil(L / 16) with an identity block, which leaves the leading
// L x L factor and inverse unchanged, and kept as its packed upper triangle
// (row i holds columns i .. Lp-1).
//   Cholesky W = R^T R (right-looking, block column k): the diagonal block is
//   factored by one wave, column c of the block in the registers of lane c;
//   the block row R_kj = R_kk^-T W_kj by forward substitution, one thread per
//   column; the trailing upper blocks W_jl -= R_kj^T R_kl with MFMAs.  A
//   pivot at or below rel_tol times the original diagonal entry is breakdown
//   (flag = first bad column + 1) and is replaced by a unit pivot.
//   Inverse X = R^-1 (left to right, block column j): X_jj = R_jj^-1 by back
//   substitution in one wave; Y_k = R_kj X_jj, then X_ij = -sum_{k>=i} X_ik Y_k
//   for i < j, both with MFMAs, the results held in registers until every
//   wave has read its operands, then written in place.
// W (L x L, row-major) receives R with zeros below the diagonal (CHOL) or is
// read as R (inverse only); Rinv receives R^-1 with zeros below.
// f64 16x16x4 operands: lane m + 16 k holds A[m][k] and B[k][m]; D: lane
// n + 16 g, register v holds D[4 v + g][n].
constexpr int CB = 16;

static int blk_lp(int L) { return (L + CB - 1) / CB * CB; }

static size_t chol_blk_lds(int L) {
  const size_t lp = (size_t)blk_lp(L);
  return sizeof(double) * (lp * (lp + 1) / 2 + (size_t)L + CB * CB + CB + 8);
}

bool chol_blk_fits(int L) { return L >= 1 && blk_lp(L) <= 192 && chol_blk_lds(L) <= g_max_lds; }

template <bool CHOL>
__global__ __launch_bounds__(1024) void chol_blk_kernel(double* __restrict__ W, int L, double rel_tol,
                                                        int* __restrict__ flag, double* __restrict__ Rinv) {
  extern __shared__ double smem[];
  const int Lp = (L + CB - 1) / CB * CB, NB = Lp / CB;
  const int64_t np = (int64_t)Lp * (Lp + 1) / 2;
  double* P = smem;         // packed upper, np
  double* d0 = P + np;      // L original diagonal entries
  double* Tm = d0 + L;      // 16 x 16 diagonal-block inverse, row-major
  double* rinv = Tm + CB * CB;  // 1 / R(t, t) of the current diagonal block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  auto off = [&](int i) { return i * Lp - (i * (i - 1)) / 2; };
  auto at = [&](int i, int j) -> double& { return P[off(i) + j - i]; };  // j >= i

  for (int i = wave; i < Lp; i += 16)
    for (int j = i + lane; j < Lp; j += 64) at(i, j) = (i < L && j < L) ? W[(int64_t)i * L + j] : (i == j ? 1.0 : 0.0);
  if (CHOL)
    for (int i = tid; i < L; i += 1024) d0[i] = W[(int64_t)i * L + i];
  __syncthreads();

  if (CHOL) {
    for (int kb = 0; kb < NB; ++kb) {
      const int k0 = kb * CB;
      if (wave == 0) {  // diagonal block: lane c holds column c
        const int c = c16;
        double w[CB];
#pragma unroll
        for (int t = 0; t < CB; ++t) w[t] = t <= c ? at(k0 + t, k0 + c) : 0.0;
#pragma unroll
        for (int t = 0; t < CB; ++t) {
          double p = __shfl(w[t], t, 64);
          const int col = k0 + t;
          const bool ok = col >= L || (isfinite(p) && p > 0.0 && p > rel_tol * d0[col]);
          if (!ok) {
            p = 1.0;
            if (lane == 0) atomicCAS(flag, 0, col + 1);
          }
          const double r = sqrt(p), ir = 1.0 / r;
          if (c == t) w[t] = r;
          else if (c > t) w[t] *= ir;
#pragma unroll
          for (int u = t + 1; u < CB; ++u) {
            const double rtu = __shfl(w[t], u, 64);
            if (c >= u) w[u] -= rtu * w[t];
          }
        }
        if (lane < CB) {
#pragma unroll
          for (int t = 0; t < CB; ++t) {
            if (t <= c) at(k0 + t, k0 + c) = w[t];
            if (t == c) rinv[t] = 1.0 / w[t];
          }
        }
      }
      __syncthreads();
      // block row: R_kj = R_kk^-T W_kj, one thread per column
      const int c = k0 + CB + tid;
      if (c < Lp) {
        double x[CB];
#pragma unroll
        for (int t = 0; t < CB; ++t) x[t] = at(k0 + t, c);
#pragma unroll
        for (int t = 0; t < CB; ++t) {
          double sacc = x[t];
#pragma unroll
          for (int q = 0; q < t; ++q) sacc -= at(k0 + q, k0 + t) * x[q];
          x[t] = sacc * rinv[t];
        }
#pragma unroll
        for (int t = 0; t < CB; ++t) at(k0 + t, c) = x[t];
      }
      __syncthreads();
      // trailing upper blocks (jb, lb), kb < jb <= lb
      const int nrem = NB - kb - 1;
      const int ntile = nrem * (nrem + 1) / 2;
      for (int q = wave; q < ntile; q += 16) {
        int rem = q, jb = kb + 1;
        while (rem >= NB - jb) {
          rem -= NB - jb;
          ++jb;
        }
        const int lb = jb + rem;
        const int j0 = jb * CB, l0 = lb * CB;
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double a = at(k0 + 4 * s + g, j0 + c16);
          const double b = at(k0 + 4 * s + g, l0 + c16);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = j0 + 4 * v + g, col = l0 + c16;
          if (jb < lb || col >= row) at(row, col) -= acc[v];
        }
      }
      __syncthreads();
    }
    for (int i = wave; i < L; i += 16)
      for (int j = lane; j < L; j += 64) W[(int64_t)i * L + j] = j >= i ? at(i, j) : 0.0;
  }

  for (int jb = 0; jb < NB; ++jb) {
    const int j0 = jb * CB;
    if (wave == 0) {  // X_jj = R_jj^-1, lane c computes column c
      const int c = c16;
      double x[CB];
#pragma unroll
      for (int i = CB - 1; i >= 0; --i) {
        const double rii = at(j0 + i, j0 + i);
        double sacc = 0.0;
#pragma unroll
        for (int q = i + 1; q < CB; ++q) sacc += at(j0 + i, j0 + q) * x[q];
        x[i] = i > c ? 0.0 : (i == c ? 1.0 / rii : -sacc / rii);
      }
      if (lane < CB) {
#pragma unroll
        for (int i = 0; i < CB; ++i) Tm[i * CB + c] = x[i];
      }
    }
    __syncthreads();
    // Y_w = R_wj X_jj for block rows w < jb
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    if (wave < jb) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = at(CB * wave + c16, j0 + 4 * s + g);
        const double b = Tm[(4 * s + g) * CB + c16];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
    }
    __syncthreads();
    if (wave < jb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) at(CB * wave + 4 * v + g, j0 + c16) = acc[v];
    }
    __syncthreads();
    // X_ij = -sum_{k = i}^{jb-1} X_ik Y_k for block rows i < jb
    acc = doublex4{0.0, 0.0, 0.0, 0.0};
    if (wave < jb) {
      const int row = CB * wave + c16;
      for (int kb = wave; kb < jb; ++kb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int col = CB * kb + 4 * s + g;
          const double a = col >= row ? at(row, col) : 0.0;
          const double b = at(CB * kb + 4 * s + g, j0 + c16);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (wave < jb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) at(CB * wave + 4 * v + g, j0 + c16) = -acc[v];
    }
    if (wave == 15) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, r = e >> 4, cc = e & 15;
        if (cc >= r) at(j0 + r, j0 + cc) = Tm[e];
      }
    }
    __syncthreads();
  }
  for (int i = wave; i < L; i += 16)
    for (int j = lane; j < L; j += 64) Rinv[(int64_t)i * L + j] = j >= i ? at(i, j) : 0.0;
}

// ---------------------------------------------------------------- blocked, in global memory
// The same blocked Cholesky and inverse for 192 < L <= 1024, where the packed triangle no longer
// fits in LDS: the matrix stays in global memory (at most 8 MiB, resident in L2) and one workgroup
// of 16 waves walks it by 16 x 16 blocks exactly as above.  W is factored in place (lower
// triangle zeroed); R is then copied to Rinv and inverted there.  Entries past L read as the
// identity and are never written, which is the identity padding of the LDS version.  Block
// results are held in registers (up to 4 block rows per wave) until every wave has read its
// operands; barriers order the global-memory updates within the workgroup.
constexpr int CBG_MAXNB = 64;

bool chol_blkg_fits(int L) { return L >= 1 && L <= CB * CBG_MAXNB; }

// RB: block rows per wave in the inverse (NB <= 16 RB)
template <bool CHOL, int RB>
__global__ __launch_bounds__(1024) void chol_blkg_kernel(double* __restrict__ W, int L, double rel_tol,
                                                         int* __restrict__ flag, double* __restrict__ Rinv) {
  __shared__ double d0[CB * CBG_MAXNB];
  __shared__ double Tm[CB * CB];  // R_kk (factor) or X_jj (inverse), row-major
  __shared__ double rinv[CB];
  const int Lp = (L + CB - 1) / CB * CB, NB = Lp / CB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  // 32-bit element offsets (L <= 1024) keep one address register per access
  auto get = [&](const double* A, int i, int j) -> double {
    return (i < L && j < L) ? A[(unsigned)(i * L + j)] : (i == j ? 1.0 : 0.0);
  };
  auto put = [&](double* A, int i, int j, double v) {
    if (i < L && j < L) A[(unsigned)(i * L + j)] = v;
  };

  if (CHOL) {
    for (int i = tid; i < L; i += 1024) d0[i] = W[(int64_t)i * L + i];
    __syncthreads();
    for (int kb = 0; kb < NB; ++kb) {
      const int k0 = kb * CB;
      if (wave == 0) {  // diagonal block: lane c holds column c
        const int c = c16;
        double w[CB];
#pragma unroll
        for (int t = 0; t < CB; ++t) w[t] = t <= c ? get(W, k0 + t, k0 + c) : 0.0;
#pragma unroll
        for (int t = 0; t < CB; ++t) {
          double p = __shfl(w[t], t, 64);
          const int col = k0 + t;
          const bool ok = col >= L || (isfinite(p) && p > 0.0 && p > rel_tol * d0[col]);
          if (!ok) {
            p = 1.0;
            if (lane == 0) atomicCAS(flag, 0, col + 1);
          }
          const double r = sqrt(p), ir = 1.0 / r;
          if (c == t) w[t] = r;
          else if (c > t) w[t] *= ir;
#pragma unroll
          for (int u = t + 1; u < CB; ++u) {
            const double rtu = __shfl(w[t], u, 64);
            if (c >= u) w[u] -= rtu * w[t];
          }
        }
        if (lane < CB) {
#pragma unroll
          for (int t = 0; t < CB; ++t) {
            if (t <= c) put(W, k0 + t, k0 + c, w[t]);
            Tm[t * CB + c] = t <= c ? w[t] : 0.0;
            if (t == c) rinv[t] = 1.0 / w[t];
          }
        }
      }
      __syncthreads();
      // block row: R_kj = R_kk^-T W_kj, one thread per column c < L (R_kk from LDS; padding
      // columns are zero in R and are skipped; c < L puts every row k0 + t below L)
      const int c = k0 + CB + tid;
      if (c < L) {
        double* wc = W + (unsigned)(k0 * L + c);
        double x[CB];
#pragma unroll
        for (int t = 0; t < CB; ++t) x[t] = wc[t * L];
#pragma unroll
        for (int t = 0; t < CB; ++t) {
          double sacc = x[t];
#pragma unroll
          for (int q = 0; q < t; ++q) sacc -= Tm[q * CB + t] * x[q];
          x[t] = sacc * rinv[t];
        }
#pragma unroll
        for (int t = 0; t < CB; ++t) wc[t * L] = x[t];
      }
      __syncthreads();
      // trailing upper blocks (jb, lb), kb < jb <= lb; two tiles per wave at a time, so
      // their operand loads are in flight together
      const int nrem = NB - kb - 1;
      const int ntile = nrem * (nrem + 1) / 2;
      auto tile_of = [&](int q, int& jb, int& lb) {
        int rem = q;
        jb = kb + 1;
        while (rem >= NB - jb) {
          rem -= NB - jb;
          ++jb;
        }
        lb = jb + rem;
      };
      for (int q = wave; q < ntile; q += 32) {
        const bool two = q + 16 < ntile;
        int jb0, lb0, jb1 = kb + 1, lb1 = kb + 1;
        tile_of(q, jb0, lb0);
        if (two) tile_of(q + 16, jb1, lb1);
        double a0[4], b0[4], a1[4], b1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a0[s] = get(W, k0 + 4 * s + g, jb0 * CB + c16);
          b0[s] = get(W, k0 + 4 * s + g, lb0 * CB + c16);
          a1[s] = two ? get(W, k0 + 4 * s + g, jb1 * CB + c16) : 0.0;
          b1[s] = two ? get(W, k0 + 4 * s + g, lb1 * CB + c16) : 0.0;
        }
        doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b0[s], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b1[s], acc1, 0, 0, 0);
        }
        double c0[4], c1[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          c0[v] = get(W, jb0 * CB + 4 * v + g, lb0 * CB + c16);
          c1[v] = two ? get(W, jb1 * CB + 4 * v + g, lb1 * CB + c16) : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row0 = jb0 * CB + 4 * v + g, col0 = lb0 * CB + c16;
          if (jb0 < lb0 || col0 >= row0) put(W, row0, col0, c0[v] - acc0[v]);
          const int row1 = jb1 * CB + 4 * v + g, col1 = lb1 * CB + c16;
          if (two && (jb1 < lb1 || col1 >= row1)) put(W, row1, col1, c1[v] - acc1[v]);
        }
      }
      __syncthreads();
    }
    for (int i = wave; i < L; i += 16)
      for (int j = lane; j < i; j += 64) W[(int64_t)i * L + j] = 0.0;
  }
  // Rinv = R (upper, zeros below), then inverted in place
  for (int i = wave; i < L; i += 16)
    for (int j = lane; j < L; j += 64) Rinv[(int64_t)i * L + j] = j >= i ? W[(int64_t)i * L + j] : 0.0;
  __syncthreads();
  double* X = Rinv;
  for (int jb = 0; jb < NB; ++jb) {
    const int j0 = jb * CB;
    if (wave == 0) {  // X_jj = R_jj^-1, lane c computes column c
      const int c = c16;
      double x[CB];
#pragma unroll
      for (int i = CB - 1; i >= 0; --i) {
        const double rii = get(X, j0 + i, j0 + i);
        double sacc = 0.0;
#pragma unroll
        for (int q = i + 1; q < CB; ++q) sacc += get(X, j0 + i, j0 + q) * x[q];
        x[i] = i > c ? 0.0 : (i == c ? 1.0 / rii : -sacc / rii);
      }
      if (lane < CB) {
#pragma unroll
        for (int i = 0; i < CB; ++i) Tm[i * CB + c] = x[i];
      }
    }
    __syncthreads();
    // Y_w = R_wj X_jj for block rows w < jb (w = wave + 16 r)
    doublex4 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      acc[r] = doublex4{0.0, 0.0, 0.0, 0.0};
      const int w = wave + 16 * r;
      if (w < jb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double a = get(X, CB * w + c16, j0 + 4 * s + g);
          const double b = Tm[(4 * s + g) * CB + c16];
          acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r], 0, 0, 0);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int w = wave + 16 * r;
      if (w < jb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) put(X, CB * w + 4 * v + g, j0 + c16, acc[r][v]);
      }
    }
    __syncthreads();
    // X_ij = -sum_{k = i}^{jb-1} X_ik Y_k for block rows i < jb
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      acc[r] = doublex4{0.0, 0.0, 0.0, 0.0};
      const int w = wave + 16 * r;
      if (w < jb) {
        const int row = CB * w + c16;
        // two block columns at a time (their loads in flight together), then the odd one
        int kb = w;
        for (; kb + 1 < jb; kb += 2) {
          double a[8], b[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int col = CB * kb + 4 * s + g;
            a[s] = col >= row ? get(X, row, col) : 0.0;
            b[s] = get(X, CB * kb + 4 * s + g, j0 + c16);
          }
#pragma unroll
          for (int s = 0; s < 8; ++s) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc[r], 0, 0, 0);
        }
        if (kb < jb) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int col = CB * kb + 4 * s + g;
            const double a = col >= row ? get(X, row, col) : 0.0;
            const double b = get(X, CB * kb + 4 * s + g, j0 + c16);
            acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int w = wave + 16 * r;
      if (w < jb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) put(X, CB * w + 4 * v + g, j0 + c16, -acc[r][v]);
      }
    }
    if (wave == 15) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, r = e >> 4, cc = e & 15;
        if (cc >= r) put(X, j0 + r, j0 + cc, Tm[e]);
      }
    }
    __syncthreads();
  }
}

bool cholinv_fits(int L) {
  return chol_blk_fits(L) || chol_blkg_fits(L) ||
         ((int64_t)L * (L + 1) / 2 <= 16 * 1024 && cholinv_lds(L) <= g_max_lds);
}

hipError_t launch_cholinv(double* W, int L, double rel_tol, int* flag, double* Rinv, hipStream_t st) {
  if (chol_blk_fits(L)) {
    hipLaunchKernelGGL((chol_blk_kernel<true>), dim3(1), dim3(1024), chol_blk_lds(L), st, W, L, rel_tol, flag, Rinv);
    return hipGetLastError();
  }
  if (chol_blkg_fits(L)) {
    if (L <= 32 * CB)
      hipLaunchKernelGGL((chol_blkg_kernel<true, 2>), dim3(1), dim3(1024), 0, st, W, L, rel_tol, flag, Rinv);
    else
      hipLaunchKernelGGL((chol_blkg_kernel<true, 4>), dim3(1), dim3(1024), 0, st, W, L, rel_tol, flag, Rinv);
    return hipGetLastError();
  }
  if (!cholinv_fits(L)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cholinv_kernel<16, false>), dim3(1), dim3(1024), cholinv_lds(L), st, W, L, rel_tol, flag,
                     Rinv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_triinv(W, L, Rinv, st);
}

hipError_t launch_triinv(const double* R, int L, double* Rinv, hipStream_t st) {
  if (chol_blk_fits(L)) {
    hipLaunchKernelGGL((chol_blk_kernel<false>), dim3(1), dim3(1024), chol_blk_lds(L), st, const_cast<double*>(R), L,
                       0.0, nullptr, Rinv);
    return hipGetLastError();
  }
  if (chol_blkg_fits(L)) {
    if (L <= 32 * CB)
      hipLaunchKernelGGL((chol_blkg_kernel<false, 2>), dim3(1), dim3(1024), 0, st, const_cast<double*>(R), L, 0.0,
                         nullptr, Rinv);
    else
      hipLaunchKernelGGL((chol_blkg_kernel<false, 4>), dim3(1), dim3(1024), 0, st, const_cast<double*>(R), L, 0.0,
                         nullptr, Rinv);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(triinv_kernel, dim3(1), dim3(1024), (size_t)L * sizeof(double), st, R, L, Rinv);
  return hipGetLastError();
}

// C (L x L) = A B for upper triangular A, B
__global__ void trmm_upper_kernel(const double* __restrict__ A, const double* __restrict__ B, int L,
                                  double* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L * L) return;
  const int i = (int)(e / L), j = (int)(e % L);
  double s = 0.0;
  for (int p = i; p <= j; ++p) s = fma(A[(int64_t)i * L + p], B[(int64_t)p * L + j], s);
  C[e] = s;
}

hipError_t launch_trmm_upper(const double* A, const double* B, int L, double* C, hipStream_t st) {
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(trmm_upper_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st, A, B, L, C);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP64 GEMM
// C[M x N] = A[M x K] B[K x N] (* colscale) (+ Cin); 64 x 64 tiles, 4 x 4 per thread.
// Cin may alias C (each element is read and written by the same thread).
template <typename TA>
__global__ __launch_bounds__(256) void gemm64_kernel(const TA* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ B, int64_t ldb, int64_t M, int N,
                                                     int K, int b_upper, const double* __restrict__ colscale,
                                                     const double* Cin, int64_t ldcin, double* C, int64_t ldc,
                                                     float* __restrict__ C32, int64_t ldc32) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int64_t R0 = (int64_t)blockIdx.x * 64;
  const int J0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int kmax = b_upper ? (J0 + 64 < K ? J0 + 64 : K) : K;
  for (int k0 = 0; k0 < kmax; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int row = e >> 4, kk = e & 15;
      const int64_t r = R0 + row;
      const int k = k0 + kk;
      As[kk][row] = (r < M && k < kmax) ? (double)A[r * lda + k] : 0.0;
      const int kb = e >> 6, col = e & 63;
      const int kb2 = k0 + kb, c = J0 + col;
      Bs[kb][col] = (kb2 < kmax && c < N) ? B[(int64_t)kb2 * ldb + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double xa[4], xb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = As[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) xb[b] = Bs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xa[a], xb[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = J0 + tx + 16 * b;
    if (c >= N) continue;
    const double sc = colscale != nullptr ? colscale[c] : 1.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t r = R0 + ty + 16 * a;
      if (r >= M) continue;
      double v = acc[a][b] * sc;
      if (Cin != nullptr) v += Cin[r * ldcin + c];
      if (C != nullptr) C[r * ldc + c] = v;
      if (C32 != nullptr) C32[r * ldc32 + c] = (float)v;
    }
  }
}

// C[M x N] = A[M x K] B[K x N] on FP64 matrix cores: a workgroup (4 waves)
// takes 64 rows and 16 NT columns, K in stages of 16 staged in LDS (A
// transposed, both with a row stride of 16 (mod 32) doubles so the 4 x 16
// operand reads of a wave hit distinct banks), the next stage loaded into
// registers during the current one.  With b_upper the stages and tiles that
// only meet zeros of B are skipped.
template <typename TA, int NT>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const TA* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ B, int64_t ldb, int64_t M, int N,
                                                        int K, int b_upper, const double* __restrict__ colscale,
                                                        const double* Cin, int64_t ldcin, double* C, int64_t ldc,
                                                        float* __restrict__ C32, int64_t ldc32) {
  constexpr int NP = 16 * NT;   // columns per workgroup
  constexpr int BST = NP + 16;  // B stage row stride
  constexpr int AST = 64 + 16;  // A^T stage row stride
  __shared__ double Bs[2][16][BST];
  __shared__ double At[2][16][AST];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  const int64_t R0 = (int64_t)blockIdx.x * 64;
  const int J0 = blockIdx.y * NP;
  const int kend = b_upper ? (J0 + NP < K ? J0 + NP : K) : K;
  // loaders: A row ar, K quad aq; B row br, columns bc + 16 q (consecutive lanes, consecutive columns)
  const int ar = tid >> 2, aq = (tid & 3) * 4;
  const int64_t arow = R0 + ar < M ? R0 + ar : M - 1;
  const int br = tid >> 4, bc = tid & 15;
  // two register sets: the stage two ahead is loaded while the next one is stored
  struct Regs {
    TA a[4];
    double b[NT];
  };
  Regs r0, r1;
  // unconditional loads from clamped addresses; the values outside the
  // ranges are zeroed when stored, so the loads stay in flight meanwhile
  auto load = [&](Regs& r, int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + aq + q;
      r.a[q] = A[arow * lda + (k < kend ? k : kend - 1)];
    }
    const int k = k0 + br;
    const int64_t kr = k < kend ? k : kend - 1;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int c = J0 + bc + 16 * q;
      r.b[q] = B[kr * ldb + (c < N ? c : N - 1)];
    }
  };
  auto store = [&](const Regs& r, int buf, int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) At[buf][aq + q][ar] = k0 + aq + q < kend ? (double)r.a[q] : 0.0;
    const bool kin = k0 + br < kend;
#pragma unroll
    for (int q = 0; q < NT; ++q) Bs[buf][br][bc + 16 * q] = (kin && J0 + bc + 16 * q < N) ? r.b[q] : 0.0;
  };
  doublex4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  auto compute = [&](int buf, int k0) {
    double a4[4], bcur[4], bnext[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      a4[s4] = At[buf][4 * s4 + g][16 * wave + n16];
      bcur[s4] = Bs[buf][4 * s4 + g][n16];
    }
    // tile by tile, the B operands of the next tile read during this one's MFMAs
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t + 1 < NT) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) bnext[s4] = Bs[buf][4 * s4 + g][16 * (t + 1) + n16];
      }
      if (!b_upper || J0 + 16 * t + 15 >= k0) {  // tile t meets nonzero rows of B in this stage
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[s4], bcur[s4], acc[t], 0, 0, 0);
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) bcur[s4] = bnext[s4];
    }
  };
  const int nst = (kend + 15) / 16;
  if (nst > 0) {
    load(r0, 0);
    store(r0, 0, 0);
  }
  if (nst > 1) load(r1, 16);
  __syncthreads();
  // stage st in buffer st & 1; a buffer is rewritten only after the barrier that ends its last reads
  for (int st = 0; st < nst; st += 2) {
    if (st + 2 < nst) load(r0, (st + 2) * 16);
    compute(0, st * 16);
    if (st + 1 < nst) store(r1, 1, (st + 1) * 16);
    __syncthreads();
    if (st + 1 >= nst) break;
    if (st + 3 < nst) load(r1, (st + 3) * 16);
    compute(1, (st + 1) * 16);
    if (st + 2 < nst) store(r0, 0, (st + 2) * 16);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = J0 + 16 * t + n16;
    if (c >= N) continue;
    const double sc = colscale != nullptr ? colscale[c] : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = R0 + 16 * wave + 4 * v + g;
      if (r >= M) continue;
      double val = acc[t][v] * sc;
      if (Cin != nullptr) val += Cin[r * ldcin + c];
      if (C != nullptr) C[r * ldc + c] = val;
      if (C32 != nullptr) C32[r * ldc32 + c] = (float)val;
    }
  }
}

template <typename TA, int NT>
static void launch_gemm_mfma(const TA* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int N, int K,
                             bool b_upper, const double* colscale, double* C, int64_t ldc, float* C32, int64_t ldc32,
                             hipStream_t st, const double* Cin, int64_t ldcin) {
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 16 * NT - 1) / (16 * NT)));
  hipLaunchKernelGGL((gemm_mfma_kernel<TA, NT>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, b_upper ? 1 : 0,
                     colscale, Cin, ldcin, C, ldc, C32, ldc32);
}

template <typename TA>
static void launch_gemm_mfma_any(const TA* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int N, int K,
                                 bool b_upper, const double* colscale, double* C, int64_t ldc, float* C32,
                                 int64_t ldc32, hipStream_t st, const double* Cin, int64_t ldcin) {
  if (N <= 64)
    launch_gemm_mfma<TA, 4>(A, lda, B, ldb, M, N, K, b_upper, colscale, C, ldc, C32, ldc32, st, Cin, ldcin);
  else if (N <= 128)
    launch_gemm_mfma<TA, 8>(A, lda, B, ldb, M, N, K, b_upper, colscale, C, ldc, C32, ldc32, st, Cin, ldcin);
  else
    launch_gemm_mfma<TA, 12>(A, lda, B, ldb, M, N, K, b_upper, colscale, C, ldc, C32, ldc32, st, Cin, ldcin);
}

hipError_t launch_gemm64(bool a_is_f64, const void* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int N,
                         int K, bool b_upper, const double* colscale, double* C, int64_t ldc, float* C32,
                         int64_t ldc32, hipStream_t st, const double* Cin, int64_t ldcin) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K >= 1) {
    if (a_is_f64)
      launch_gemm_mfma_any<double>((const double*)A, lda, B, ldb, M, N, K, b_upper, colscale, C, ldc, C32, ldc32, st,
                                   Cin, ldcin);
    else
      launch_gemm_mfma_any<float>((const float*)A, lda, B, ldb, M, N, K, b_upper, colscale, C, ldc, C32, ldc32, st,
                                  Cin, ldcin);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  if (a_is_f64)
    hipLaunchKernelGGL(gemm64_kernel<double>, grid, dim3(256), 0, st, (const double*)A, lda, B, ldb, M, N, K,
                       b_upper ? 1 : 0, colscale, Cin, ldcin, C, ldc, C32, ldc32);
  else
    hipLaunchKernelGGL(gemm64_kernel<float>, grid, dim3(256), 0, st, (const float*)A, lda, B, ldb, M, N, K,
                       b_upper ? 1 : 0, colscale, Cin, ldcin, C, ldc, C32, ldc32);
  return hipGetLastError();
}

// ---------------------------------------------------------------- outputs
// One workgroup per column: norm, first index of the largest |entry|, then
// V[:, j] <- V[:, j] * sign / norm.
__global__ __launch_bounds__(256) void normalize_sign_kernel(double* __restrict__ V, int64_t rows, int64_t ldv,
                                                             double* __restrict__ sig, double* __restrict__ sgn) {
  __shared__ double s_sum[256];
  __shared__ double s_max[256];
  __shared__ int64_t s_idx[256];
  const int j = blockIdx.x;
  double s = 0.0, best = -1.0;
  int64_t bi = 0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) {
    const double x = V[r * ldv + j];
    s = fma(x, x, s);
    const double ax = fabs(x);
    if (ax > best) {
      best = ax;
      bi = r;
    }
  }
  s_sum[threadIdx.x] = s;
  s_max[threadIdx.x] = best;
  s_idx[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
      const double m2 = s_max[threadIdx.x + o];
      const int64_t i2 = s_idx[threadIdx.x + o];
      if (m2 > s_max[threadIdx.x] || (m2 == s_max[threadIdx.x] && i2 < s_idx[threadIdx.x])) {
        s_max[threadIdx.x] = m2;
        s_idx[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const double nrm = sqrt(s_sum[0]);
  const double piv = V[s_idx[0] * ldv + j];
  const double sg = piv < 0.0 ? -1.0 : 1.0;
  const double f = nrm > 0.0 ? sg / nrm : sg;
  __syncthreads();
  for (int64_t r = threadIdx.x; r < rows; r += 256) V[r * ldv + j] *= f;
  if (threadIdx.x == 0) {
    sig[j] = nrm;
    sgn[j] = sg;
  }
}

hipError_t launch_normalize_sign(double* V, int64_t rows, int k, int64_t ldv, double* sig, double* sgn,
                                 hipStream_t st) {
  hipLaunchKernelGGL(normalize_sign_kernel, dim3((unsigned)k), dim3(256), 0, st, V, rows, ldv, sig, sgn);
  return hipGetLastError();
}

__global__ void to_f32_kernel(const double* __restrict__ X, int64_t rows, int cols, int64_t ldx,
                              const double* __restrict__ colscale, float* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  const double sc = colscale != nullptr ? colscale[c] : 1.0;
  out[r * ldo + c] = (float)(X[r * ldx + c] * sc);
}

hipError_t launch_to_f32(const double* X, int64_t rows, int cols, int64_t ldx, const double* colscale, float* out,
                         int64_t ldo, hipStream_t st) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, rows, cols, ldx,
                     colscale, out, ldo);
  return hipGetLastError();
}

}  // namespace rpca
