// Householder QR of the tall, skinny m x L block H for Step 2 (the paper's
// QR of H, Section 3), as a reduction tree over row blocks (TSQR): the row
// blocks of H are factored independently, their L x L triangles stacked in
// pairs and factored again, up to one triangle R, and Q is formed explicitly
// by applying the reflectors of every level top-down to [I; 0].  Every step
// is an orthogonal transformation in float64, so Q is orthonormal to
// rounding whatever the condition of H (a rank-deficient H gets an
// orthonormal completion in place of its null directions).  Column pivoting
// is not applied: it permutes R's columns and leaves span(Q), on which Steps
// 3-6 depend, unchanged.
//
// One workgroup (sixteen waves) per block.  A reflector step on a block of nr
// rows: the sum of squares of the column below the diagonal (block
// reduction), v and tau as in LAPACK's dlarfg (beta = -sign(alpha) ||x||,
// tau = (beta - alpha) / beta, v = x / (alpha - beta), v_j = 1), v cached in
// LDS, then w = v^T B for the trailing columns with the rows split over the
// waves and the columns over the lanes (coalesced row segments), and the
// rank-one update B -= tau v w^T.  The block lives in global memory (it is
// revisited L times and stays in the caches); this path is a fallback.
#include "common.h"
#include "kernels.h"

namespace rpca {

constexpr int HH_WAVES = 16;  // waves per workgroup: the rows of a block are split over them
constexpr int HH_THREADS = 64 * HH_WAVES;

namespace {

// rows [r0, r0 + nr) of block k of a level: blocks of bu rows, the last one
// taking the remainder
RPCA_DEV void hh_block_rows(int64_t rows_total, int64_t bu, int nb, int k, int64_t* r0, int64_t* nr) {
  *r0 = (int64_t)k * bu;
  *nr = k == nb - 1 ? rows_total - *r0 : bu;
}

RPCA_DEV double hh_block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < HH_WAVES; ++q) t += red[q];
  return t;
}

// sum over the waves' partial dot products of column c
RPCA_DEV double hh_part_sum(const double* part, int L, int c) {
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < HH_WAVES; ++q) t += part[q * L + c];
  return t;
}

}  // namespace

// Factor block k in place (reflectors below the diagonal, R on and above it),
// tau[k L + j], and write R (upper, zeros below) to Rout + k L L.  Requires
// nr >= L for every block.  LDS: maxrows + HH_WAVES (L + 1) doubles.
__global__ __launch_bounds__(HH_THREADS) void hh_factor_kernel(double* __restrict__ X, int64_t rows_total, int64_t bu,
                                                        int nb, int L, int maxrows, double* __restrict__ tau,
                                                        double* __restrict__ Rout) {
  extern __shared__ double hsh[];
  double* v = hsh;
  double* part = hsh + maxrows;
  double* red = part + HH_WAVES * L;
  const int k = blockIdx.x;
  int64_t r0, nr64;
  hh_block_rows(rows_total, bu, nb, k, &r0, &nr64);
  const int nr = (int)nr64;
  double* __restrict__ B = X + r0 * L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = 0; j < L; ++j) {
    double s = 0.0;
    for (int i = j + 1 + tid; i < nr; i += HH_THREADS) {
      const double x = B[(int64_t)i * L + j];
      s += x * x;
    }
    // alpha is read before the barriers of the reduction; thread 0 overwrites it below
    const double alpha = B[(int64_t)j * L + j];
    s = hh_block_sum(s, red);
    double t = 0.0, scale = 0.0, beta = alpha;
    if (s > 0.0) {
      const double nrm = sqrt(alpha * alpha + s);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    for (int i = j + 1 + tid; i < nr; i += HH_THREADS) {
      const double vi = B[(int64_t)i * L + j] * scale;
      B[(int64_t)i * L + j] = vi;
      v[i] = vi;
    }
    if (tid == 0) {
      v[j] = 1.0;
      B[(int64_t)j * L + j] = beta;
      tau[(int64_t)k * L + j] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      // rows [j, nr) split into HH_WAVES contiguous ranges, one per wave
      const int span = nr - j;
      const int ib = j + (span * w) / HH_WAVES, ie = j + (span * (w + 1)) / HH_WAVES;
      for (int c = j + 1 + lane; c < L; c += 64) {
        double p = 0.0;
#pragma unroll 8
        for (int i = ib; i < ie; ++i) p += v[i] * B[(int64_t)i * L + c];
        part[w * L + c] = p;
      }
      __syncthreads();
      for (int c = j + 1 + lane; c < L; c += 64) {
        const double wc = t * hh_part_sum(part, L, c);
#pragma unroll 8
        for (int i = ib; i < ie; ++i) B[(int64_t)i * L + c] -= v[i] * wc;
      }
    }
    __syncthreads();
  }
  double* __restrict__ R = Rout + (int64_t)k * L * L;
  for (int e = tid; e < L * L; e += HH_THREADS) {
    const int i = e / L, c = e % L;
    R[e] = c >= i ? B[(int64_t)i * L + c] : 0.0;
  }
}

// Block k of a level: Y (its nr rows of Yout) = Q_k [C_k; 0], with C_k rows
// [k L, (k+1) L) of Cin (the identity when Cin is null) and Q_k the product
// of the block's reflectors, applied last-to-first.  LDS: maxrows + HH_WAVES (L + 1).
__global__ __launch_bounds__(HH_THREADS) void hh_apply_kernel(const double* __restrict__ X, int64_t rows_total, int64_t bu,
                                                       int nb, int L, int maxrows, const double* __restrict__ tau,
                                                       const double* __restrict__ Cin, double* __restrict__ Yout) {
  extern __shared__ double hsh[];
  double* v = hsh;
  double* part = hsh + maxrows;
  const int k = blockIdx.x;
  int64_t r0, nr64;
  hh_block_rows(rows_total, bu, nb, k, &r0, &nr64);
  const int nr = (int)nr64;
  const double* __restrict__ B = X + r0 * L;
  double* __restrict__ Y = Yout + r0 * L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int64_t e = tid; e < (int64_t)nr * L; e += HH_THREADS) {
    const int i = (int)(e / L), c = (int)(e % L);
    double y = 0.0;
    if (i < L) y = Cin != nullptr ? Cin[((int64_t)k * L + i) * L + c] : (i == c ? 1.0 : 0.0);
    Y[e] = y;
  }
  __syncthreads();
  for (int j = L - 1; j >= 0; --j) {
    const double t = tau[(int64_t)k * L + j];
    if (t == 0.0) continue;  // uniform across the workgroup
    for (int i = j + 1 + tid; i < nr; i += HH_THREADS) v[i] = B[(int64_t)i * L + j];
    if (tid == 0) v[j] = 1.0;
    __syncthreads();
    const int span = nr - j;
    const int ib = j + (span * w) / HH_WAVES, ie = j + (span * (w + 1)) / HH_WAVES;
    for (int c = lane; c < L; c += 64) {
      double p = 0.0;
#pragma unroll 8
      for (int i = ib; i < ie; ++i) p += v[i] * Y[(int64_t)i * L + c];
      part[w * L + c] = p;
    }
    __syncthreads();
    for (int c = lane; c < L; c += 64) {
      const double wc = t * hh_part_sum(part, L, c);
#pragma unroll 8
      for (int i = ib; i < ie; ++i) Y[(int64_t)i * L + c] -= v[i] * wc;
    }
    __syncthreads();
  }
}

static size_t hh_lds(int L, int maxrows) { return sizeof(double) * (size_t)(maxrows + HH_WAVES * (L + 1)); }

// LDS one workgroup may use on this device (160 KB on gfx950), set by the plan
static size_t g_hh_lds_limit = 65536;
void set_hh_lds_limit(size_t bytes) { g_hh_lds_limit = bytes; }
bool hh_fits(int L, int64_t maxrows) { return maxrows <= (1 << 20) && hh_lds(L, (int)maxrows) <= g_hh_lds_limit; }

hipError_t launch_hh_factor(double* X, int64_t rows_total, int64_t bu, int nb, int L, double* tau, double* Rout,
                            hipStream_t st) {
  if (nb <= 0 || L <= 0) return hipSuccess;
  if (rows_total - (int64_t)(nb - 1) * bu < L || (nb > 1 && bu < L)) return hipErrorInvalidValue;
  const int64_t maxrows = rows_total - (int64_t)(nb - 1) * bu > bu ? rows_total - (int64_t)(nb - 1) * bu : bu;
  if (!hh_fits(L, maxrows)) return hipErrorInvalidValue;
  const size_t lds = hh_lds(L, (int)maxrows);
  hipLaunchKernelGGL(hh_factor_kernel, dim3((unsigned)nb), dim3(HH_THREADS), lds, st, X, rows_total, bu, nb, L,
                     (int)maxrows, tau, Rout);
  return hipGetLastError();
}

hipError_t launch_hh_apply(const double* X, int64_t rows_total, int64_t bu, int nb, int L, const double* tau,
                           const double* Cin, double* Yout, hipStream_t st) {
  if (nb <= 0 || L <= 0) return hipSuccess;
  if (rows_total - (int64_t)(nb - 1) * bu < L || (nb > 1 && bu < L)) return hipErrorInvalidValue;
  const int64_t maxrows = rows_total - (int64_t)(nb - 1) * bu > bu ? rows_total - (int64_t)(nb - 1) * bu : bu;
  if (!hh_fits(L, maxrows)) return hipErrorInvalidValue;
  const size_t lds = hh_lds(L, (int)maxrows);
  hipLaunchKernelGGL(hh_apply_kernel, dim3((unsigned)nb), dim3(HH_THREADS), lds, st, X, rows_total, bu, nb, L,
                     (int)maxrows, tau, Cin, Yout);
  return hipGetLastError();
}

}  // namespace rpca
