// Auxiliary kernels around the panel products: column means for centring,
// the Gaussian test matrix G of Step 1, the ordered reduction of the split
// adjoint partial sums (with the rank-one centring correction), and the
// positive block scale that keeps the power iterates in range (Section 3,
// remark on over/underflow).
#include "common.h"
#include "kernels.h"
#include "storage.h"

namespace rpca {

// ---------------------------------------------------------------- column sums
// part[s][c] = sum of X[r][c] over the rows r of split s.  A block takes 64
// columns (one per lane) and its four waves take every fourth row, eight
// rows in flight per lane; the wave sums are combined in a fixed order.
template <int ST>
__global__ __launch_bounds__(256) void colsum_kernel(const void* __restrict__ X, int64_t ld, int64_t rows,
                                                     int64_t cols, const float* __restrict__ cs, int64_t plane,
                                                     int64_t rps, double* __restrict__ part) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const int s = blockIdx.y;
  const int64_t r0 = (int64_t)s * rps;
  const int64_t r1 = r0 + rps < rows ? r0 + rps : rows;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  if (c < cols) {
    int64_t r = r0 + w;
    for (; r + 28 < r1; r += 32) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = load_elem<ST>(X, (r + 4 * u) * ld + c, plane);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += (double)v[u];
    }
    for (; r < r1; r += 4) acc[0] += (double)load_elem<ST>(X, r * ld + c, plane);
  }
  sh[w][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (w != 0 || c >= cols) return;
  double tot = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
  if (ST == ST_FP8) tot *= (double)cs[c];
  part[(int64_t)s * cols + c] = tot;
}

hipError_t launch_colsum(int storage, const void* X, int64_t ld, int64_t rows, int64_t cols,
                         const float* col_scale, int64_t plane, int64_t rows_per_split, int nsplit,
                         double* part, hipStream_t st) {
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)nsplit);
  switch (storage) {
    case ST_F32:
      hipLaunchKernelGGL(colsum_kernel<ST_F32>, grid, dim3(256), 0, st, X, ld, rows, cols, col_scale, plane,
                         rows_per_split, part);
      break;
    case ST_BF16:
      hipLaunchKernelGGL(colsum_kernel<ST_BF16>, grid, dim3(256), 0, st, X, ld, rows, cols, col_scale, plane,
                         rows_per_split, part);
      break;
    case ST_FP8:
      hipLaunchKernelGGL(colsum_kernel<ST_FP8>, grid, dim3(256), 0, st, X, ld, rows, cols, col_scale, plane,
                         rows_per_split, part);
      break;
    case ST_HILO:
      hipLaunchKernelGGL(colsum_kernel<ST_HILO>, grid, dim3(256), 0, st, X, ld, rows, cols, col_scale, plane,
                         rows_per_split, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// 16 columns per block, 16 groups of threads each summing every 16th split (a split count of
// several hundred leaves each thread a short chain), combined in a fixed order
__global__ __launch_bounds__(256) void colsum_reduce_kernel(const double* __restrict__ part, int nsplit,
                                                            int64_t cols, double scale, double* __restrict__ out,
                                                            float* __restrict__ out32, double* __restrict__ resid) {
  __shared__ double sh[16][16];
  const int t = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t c = (int64_t)blockIdx.x * 16 + t;
  double s = 0.0;
  if (c < cols)
    for (int k = g; k < nsplit; k += 16) s += part[(int64_t)k * cols + c];
  sh[g][t] = s;
  __syncthreads();
  if (g != 0 || c >= cols) return;
  s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += sh[q][t];
  s *= scale;
  out[c] = s;
  if (out32 != nullptr) {
    const float f = (float)s;
    out32[c] = f;
    if (resid != nullptr) resid[c] = s - (double)f;
  }
}

hipError_t launch_colsum_reduce(const double* part, int nsplit, int64_t cols, double scale, double* out,
                                float* out_f32, double* resid, hipStream_t st) {
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((unsigned)((cols + 15) / 16)), dim3(256), 0, st, part, nsplit, cols,
                     scale, out, out_f32, resid);
  return hipGetLastError();
}

// ---------------------------------------------------------------- G
__global__ void gen_G_kernel(uint64_t seed, int64_t n, int l, float* __restrict__ Xt, int64_t ldx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * l) return;
  const int64_t r = e / l;
  const int c = (int)(e % l);
  Xt[(int64_t)c * ldx + r] = (float)normal_elem(seed, 1u, (uint64_t)e);
}

hipError_t launch_gen_G(uint64_t seed, int64_t n, int l, float* Xt, int64_t ldx, hipStream_t st) {
  const int64_t tot = n * l;
  hipLaunchKernelGGL(gen_G_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, seed, n, l, Xt, ldx);
  return hipGetLastError();
}

__global__ void transpose_G_kernel(const float* __restrict__ G, int64_t ldg, int64_t n, int l,
                                   float* __restrict__ Xt, int64_t ldx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * l) return;
  const int64_t r = e / l;
  const int c = (int)(e % l);
  Xt[(int64_t)c * ldx + r] = G[r * ldg + c];
}

hipError_t launch_transpose_G(const float* G, int64_t ldg, int64_t n, int l, float* Xt, int64_t ldx,
                              hipStream_t st) {
  const int64_t tot = n * l;
  hipLaunchKernelGGL(transpose_G_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, G, ldg, n, l,
                     Xt, ldx);
  return hipGetLastError();
}

// ---------------------------------------------------------------- block reductions
template <typename T>
RPCA_DEV T block_sum_256(T v, T* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T tot = T(0);
  if (threadIdx.x == 0) {
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += sh[k];
  }
  return tot;  // valid in thread 0
}

__global__ __launch_bounds__(256) void dot_rows_kernel(const double* __restrict__ d, const float* __restrict__ Xt,
                                                       int64_t ldx, int64_t n, float* __restrict__ corr) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  const float* x = Xt + (int64_t)j * ldx;
  // the loads of four strides go out together; the products are added in the same order
  double s = 0.0;
  int64_t c = threadIdx.x;
  for (; c + 768 < n; c += 1024) {
    double dv[4];
    float xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dv[u] = d[c + 256 * u];
      xv[u] = x[c + 256 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += dv[u] * (double)xv[u];
  }
  for (; c < n; c += 256) s += d[c] * (double)x[c];
  s = block_sum_256(s, sh);
  if (threadIdx.x == 0) corr[j] = (float)s;
}

hipError_t launch_dot_rows(const double* d, const float* Xt, int64_t ldx, int64_t n, int ncols, float* corr,
                           hipStream_t st) {
  hipLaunchKernelGGL(dot_rows_kernel, dim3((unsigned)ncols), dim3(256), 0, st, d, Xt, ldx, n, corr);
  return hipGetLastError();
}

template <typename TP>
__global__ __launch_bounds__(256) void reduce_y_kernel(const TP* __restrict__ P, int nsplit,
                                                       int64_t split_stride, int64_t ldp, int64_t n,
                                                       const float* __restrict__ cs, const double* __restrict__ d,
                                                       const double* __restrict__ zsum, float* __restrict__ Xt,
                                                       int64_t ldx, double* __restrict__ sq_part) {
  __shared__ double sh[4];
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  double sq = 0.0;
  if (c < n) {
    double v = 0.0;
    const TP* p = P + (int64_t)j * ldp + c;
    v += sum_strided(p, nsplit, split_stride);
    if (cs != nullptr) v *= (double)cs[c];
    if (d != nullptr) v -= d[c] * zsum[j];
    const float f = (float)v;
    Xt[(int64_t)j * ldx + c] = f;
    sq = (double)f * (double)f;
  }
  sq = block_sum_256(sq, sh);
  if (threadIdx.x == 0) sq_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sq;
}

hipError_t launch_reduce_y(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                           const float* col_scale, const double* d, const double* zsum, float* Xt, int64_t ldx,
                           double* sq_part, int* n_sq_part, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  *n_sq_part = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(reduce_y_kernel<float>, grid, dim3(256), 0, st, P, nsplit, split_stride, ldp, n, col_scale, d,
                     zsum, Xt, ldx, sq_part);
  return hipGetLastError();
}

hipError_t launch_reduce_y64(const double* P, int64_t ldp, int ncols, int64_t n, const double* d, const double* zsum,
                             float* Xt, int64_t ldx, double* sq_part, int* n_sq_part, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  *n_sq_part = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(reduce_y_kernel<double>, grid, dim3(256), 0, st, P, 1, (int64_t)0, ldp, n, nullptr, d, zsum,
                     Xt, ldx, sq_part);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void finish_scale_kernel(const double* __restrict__ sq_part, int n_part,
                                                           int rescale, double* __restrict__ alpha,
                                                           int* __restrict__ flag) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < n_part; k += 256) s += sq_part[k];
  s = block_sum_256(s, sh);
  if (threadIdx.x == 0) {
    if (!isfinite(s)) {
      atomicOr(flag, 1);
      *alpha = 1.0;
    } else {
      *alpha = (rescale && s > 0.0) ? 1.0 / sqrt(s) : 1.0;
    }
  }
}

hipError_t launch_finish_scale(const double* sq_part, int n_part, bool rescale, double* alpha, int* flag,
                               hipStream_t st) {
  hipLaunchKernelGGL(finish_scale_kernel, dim3(1), dim3(256), 0, st, sq_part, n_part, rescale ? 1 : 0, alpha,
                     flag);
  return hipGetLastError();
}

template <typename TP>
__global__ __launch_bounds__(256) void reduce_t_kernel(const TP* __restrict__ P, int nsplit,
                                                       int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                                                       const float* __restrict__ cs, const double* __restrict__ d,
                                                       const double* __restrict__ qsum, double* __restrict__ T,
                                                       int64_t ldt) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (c >= n) return;
  double v = 0.0;
  const TP* p = P + (int64_t)j * ldp + c;
  v += sum_strided(p, nsplit, split_stride);
  if (cs != nullptr) v *= (double)cs[c];
  if (d != nullptr) v -= d[c] * qsum[j];
  T[c * ldt + j] = v;
}

hipError_t launch_reduce_t(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                           const float* col_scale, const double* d, const double* qsum, double* T, int64_t ldt,
                           hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  hipLaunchKernelGGL(reduce_t_kernel<float>, grid, dim3(256), 0, st, P, nsplit, split_stride, ldp, ncols, n,
                     col_scale, d, qsum, T, ldt);
  return hipGetLastError();
}

hipError_t launch_reduce_t64(const double* P, int64_t ldp, int ncols, int64_t n, const double* d, const double* qsum,
                             double* T, int64_t ldt, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  hipLaunchKernelGGL(reduce_t_kernel<double>, grid, dim3(256), 0, st, P, 1, (int64_t)0, ldp, ncols, n, nullptr, d,
                     qsum, T, ldt);
  return hipGetLastError();
}

// Centring fused into pass 0.  Pass 0 runs with the shift s0 (mean of a first
// row panel) and its adjoint also forms the column sums of A - 1 s0^T (row
// `row` of each split partial).  Then d0 = those sums / m, mu = s0 + d0, and
// the shift of the later passes becomes fl32(mu) with residual mu - fl32(mu).
__global__ __launch_bounds__(256) void pass0_center_kernel(const float* __restrict__ P, int nsplit,
                                                           int64_t split_stride, int64_t ldp, int row, int64_t n,
                                                           double inv_m, float* __restrict__ shift,
                                                           double* __restrict__ d0, double* __restrict__ mu,
                                                           double* __restrict__ dres) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  double v = 0.0;
  const float* p = P + (int64_t)row * ldp + c;
  v += sum_strided(p, nsplit, split_stride);
  const double d = v * inv_m;
  const double u = (double)shift[c] + d;
  const float s1 = (float)u;
  d0[c] = d;
  mu[c] = u;
  shift[c] = s1;
  dres[c] = u - (double)s1;
}

hipError_t launch_pass0_center(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int row, int64_t n,
                               int64_t m, float* shift, double* d0, double* mu, double* dres, hipStream_t st) {
  hipLaunchKernelGGL(pass0_center_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, nsplit,
                     split_stride, ldp, row, n, 1.0 / (double)m, shift, d0, mu, dres);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void pass0_mean_lp_kernel(const float* __restrict__ P, int nsplit,
                                                            int64_t split_stride, int64_t ldp, int row, int64_t n,
                                                            double inv_m, const float* __restrict__ cs,
                                                            double* __restrict__ mu) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  double v = 0.0;
  const float* p = P + (int64_t)row * ldp + c;
  v += sum_strided(p, nsplit, split_stride);
  if (cs != nullptr) v *= (double)cs[c];
  mu[c] = v * inv_m;
}

hipError_t launch_pass0_mean_lp(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int row, int64_t n,
                                int64_t m, const float* cs, double* mu, hipStream_t st) {
  hipLaunchKernelGGL(pass0_mean_lp_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, nsplit,
                     split_stride, ldp, row, n, 1.0 / (double)m, cs, mu);
  return hipGetLastError();
}

// X[r][c] -= corr[c] (float32, rows x cols)
__global__ void sub_cols_kernel(float* __restrict__ X, int64_t ldx, int64_t rows, int cols,
                                const float* __restrict__ corr) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  X[r * ldx + c] -= corr[c];
}

hipError_t launch_sub_cols(float* X, int64_t ldx, int64_t rows, int cols, const float* corr, hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(sub_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, ldx, rows, cols,
                     corr);
  return hipGetLastError();
}

// acc[r][c] += sum_s part[s][r][c] (float or double partials; rows x cols with leading dimension ld)
template <typename TP>
__global__ __launch_bounds__(256) void accumulate_parts_kernel(const TP* __restrict__ part, int nsplit,
                                                               int64_t split_stride, int64_t rows, int64_t cols,
                                                               int64_t ld, double* __restrict__ acc) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= cols || r >= rows) return;
  double v = 0.0;
  const TP* p = part + r * ld + c;
  v += sum_strided(p, nsplit, split_stride);
  acc[r * ld + c] += v;
}

hipError_t launch_accumulate_parts(bool f64, const void* part, int nsplit, int64_t split_stride, int64_t rows,
                                   int64_t cols, int64_t ld, double* acc, hipStream_t st) {
  dim3 grid((unsigned)((cols + 255) / 256), (unsigned)rows);
  if (f64)
    hipLaunchKernelGGL(accumulate_parts_kernel<double>, grid, dim3(256), 0, st, (const double*)part, nsplit,
                       split_stride, rows, cols, ld, acc);
  else
    hipLaunchKernelGGL(accumulate_parts_kernel<float>, grid, dim3(256), 0, st, (const float*)part, nsplit,
                       split_stride, rows, cols, ld, acc);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void check_finite_kernel(const float* __restrict__ X, int64_t rows,
                                                           int64_t cols, int64_t ld, int* __restrict__ flag) {
  const int64_t tot = rows * cols;
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / cols, c = e % cols;
    if (!isfinite(X[r * ld + c])) bad = 1;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_check_finite_f32(const float* X, int64_t rows, int64_t cols, int64_t ld, int* flag,
                                   hipStream_t st) {
  const int64_t tot = rows * cols;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, rows, cols, ld, flag);
  return hipGetLastError();
}

// out[r][c] = X[r][c] - colsum[c] * inv_rows in float64 (column means removed)
__global__ __launch_bounds__(256) void center_cols_kernel(const float* __restrict__ X, int64_t ldx, int64_t rows,
                                                          int64_t cols, const double* __restrict__ colsum,
                                                          double inv_rows, double* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e % cols;
  out[r * ldo + c] = (double)X[r * ldx + c] - colsum[c] * inv_rows;
}

hipError_t launch_center_cols(const float* X, int64_t ldx, int64_t rows, int64_t cols, const double* colsum,
                              double inv_rows, double* out, int64_t ldo, hipStream_t st) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(center_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, ldx, rows, cols,
                     colsum, inv_rows, out, ldo);
  return hipGetLastError();
}

__global__ void fill_f64_kernel(double* p, int64_t count, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

__global__ void fill_u32_kernel(unsigned* p, int64_t count, unsigned v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t st) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

}  // namespace rpca
