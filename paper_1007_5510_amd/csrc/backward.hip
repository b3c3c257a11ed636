// Small float64 kernels of the reverse-mode derivative of Steps 1-6 (G held
// fixed).  The passes over A reuse the forward panel kernels; these kernels
// carry the small-SVD adjoint of T, the QR adjoint of H = Q R, the reverse
// power sweep's bookkeeping, and the assembly of the low-rank factors of
// dL/dA = P Y^T:
//
//   small SVD (T = V~ S~ W^T, thin and complete, L <= n), F_ab = 1/(s_b^2 - s_a^2):
//     T_bar = V~ [ (F o (V~^T V_bar - V_bar^T V~)) S~ + diag(s_bar)
//                  + S~ (F o (W^T W_bar - W_bar^T W)) ] W^T + (I - V~ V~^T) V_bar S~^-1 W^T
//   with V~ = T W S~^-1, this is  T_bar = T B + V_bar S~^-1 W^T,
//     B = W S~^-1 N W^T,  N = M - (V~^T V_bar) S~^-1,  M = the bracket above;
//   QR (R_bar = 0):  H_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T,
//     copyltu(M) = tril(M) + tril(M, -1)^T.
#include "common.h"
#include "kernels.h"

namespace rpca {

// ---------------------------------------------------------------- X^T Y over a row split
// part[s][a][b] = sum_{r in split s} X[r][a] Y[r][b],  a < na, b < nb (64 x 64 tiles).  Rows are
// staged 16 at a time in LDS (two buffers); the next 16 rows are loaded to registers (from
// clamped addresses, zeroed when stored) while the current ones are multiplied.
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void xty_kernel(const TX* __restrict__ X, int64_t ldx, int na,
                                                  const TY* __restrict__ Y, int64_t ldy, int nb, int64_t rows,
                                                  int64_t rps, int tb, double* __restrict__ part) {
  __shared__ double XI[2][16][65];
  __shared__ double YJ[2][16][65];
  const int ti = blockIdx.x / tb, tj = blockIdx.x % tb;
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
  // staging: element q of this thread is row (tid + 256 q) / 64, column (tid + 256 q) % 64
  const int cc = threadIdx.x & 63, rq = threadIdx.x >> 6;
  const int xc = I0 + cc < na ? I0 + cc : na - 1, yc = J0 + cc < nb ? J0 + cc : nb - 1;
  TX px[4];
  TY py[4];
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + rq + 4 * q < re ? r0 + rq + 4 * q : re - 1;
      px[q] = X[r * ldx + xc];
      py[q] = Y[r * ldy + yc];
    }
  };
  auto store = [&](int buf, int64_t r0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool rok = r0 + rq + 4 * q < re;
      XI[buf][rq + 4 * q][cc] = (rok && I0 + cc < na) ? (double)px[q] : 0.0;
      YJ[buf][rq + 4 * q][cc] = (rok && J0 + cc < nb) ? (double)py[q] : 0.0;
    }
  };
  if (rb < re) {
    load(rb);
    store(0, rb);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t r0 = rb; r0 < re; r0 += 16) {
    const bool more = r0 + 16 < re;
    if (more) load(r0 + 16);
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
      double xi[4], yj[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xi[a] = XI[buf][rr][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) yj[b] = YJ[buf][rr][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xi[a], yj[b], acc[a][b]);
    }
    // the other buffer was last read before the previous barrier
    if (more) store(buf ^ 1, r0 + 16);
    __syncthreads();
    buf ^= 1;
  }
  double* out = part + (int64_t)s * na * nb;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = I0 + ty + 16 * a, j = J0 + tx + 16 * b;
      if (i < na && j < nb) out[(int64_t)i * nb + j] = acc[a][b];
    }
}

// out[a][b] = colscale[b] * sum_s part[s][a][b]: a block takes 16 entries, its 16 groups of 16
// threads sum every 16th split, and the group sums are combined in a fixed order
__global__ __launch_bounds__(256) void xty_reduce_kernel(const double* __restrict__ part, int nsplit, int na, int nb,
                                                         const double* __restrict__ colscale,
                                                         double* __restrict__ out) {
  __shared__ double sh[16][16];
  const int t = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t cnt = (int64_t)na * nb;
  const int64_t e = (int64_t)blockIdx.x * 16 + t;
  double v = 0.0;
  if (e < cnt)
    for (int s = grp; s < nsplit; s += 16) v += part[(int64_t)s * cnt + e];
  sh[grp][t] = v;
  __syncthreads();
  if (grp != 0 || e >= cnt) return;
  double tot = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) tot += sh[q][t];
  if (colscale != nullptr) tot *= colscale[e % nb];
  out[e] = tot;
}

hipError_t launch_xty(bool x64, const void* X, int64_t ldx, int na, bool y64, const void* Y, int64_t ldy, int nb,
                      int64_t rows, int64_t rows_per_split, int nsplit, const double* colscale, double* part,
                      double* out, hipStream_t st) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  const int ta = (na + 63) / 64, tb = (nb + 63) / 64;
  dim3 grid((unsigned)(ta * tb), (unsigned)nsplit);
  if (x64 && y64)
    hipLaunchKernelGGL((xty_kernel<double, double>), grid, dim3(256), 0, st, (const double*)X, ldx, na,
                       (const double*)Y, ldy, nb, rows, rows_per_split, tb, part);
  else if (x64 && !y64)
    hipLaunchKernelGGL((xty_kernel<double, float>), grid, dim3(256), 0, st, (const double*)X, ldx, na,
                       (const float*)Y, ldy, nb, rows, rows_per_split, tb, part);
  else if (!x64 && y64)
    hipLaunchKernelGGL((xty_kernel<float, double>), grid, dim3(256), 0, st, (const float*)X, ldx, na,
                       (const double*)Y, ldy, nb, rows, rows_per_split, tb, part);
  else
    hipLaunchKernelGGL((xty_kernel<float, float>), grid, dim3(256), 0, st, (const float*)X, ldx, na,
                       (const float*)Y, ldy, nb, rows, rows_per_split, tb, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cnt = (int64_t)na * nb;
  hipLaunchKernelGGL(xty_reduce_kernel, dim3((unsigned)((cnt + 15) / 16)), dim3(256), 0, st, part, nsplit, na, nb,
                     colscale, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small-SVD adjoint pieces
// A trailing S~_a (a >= k) at or below sqrt(u) S~_1 is rounding noise of the eigenvalues of T^T T:
// its direction of T has no defined singular vector.  In the adjoint such a direction only
// enters through the F-matrix term and the projector term, which cancel as S~_a -> 0, so it is
// treated as part of the complement (its column of W / S~ and its row of N are zero).
RPCA_DEV bool svd_dropped(const double* __restrict__ sig, int a, int k) {
  return a >= k && !(sig[a] > 1.4901161193847656e-08 * sig[0]);
}

// WT = W^T; Wsc[r][a] = W[r][a] / s_a (0 for a dropped direction); for a < k: Ck[a][c] = sgn_a W[c][a] / s_a,
// Bp[a][c] = sgn_a W[c][a]
__global__ void svdadj_prep_kernel(const double* __restrict__ W, const double* __restrict__ sig,
                                   const double* __restrict__ sgn, int L, int k, double* __restrict__ WT,
                                   double* __restrict__ Wsc, double* __restrict__ Ck, double* __restrict__ Bp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L * L) return;
  const int r = (int)(e / L), a = (int)(e % L);
  const double w = W[e];
  WT[(int64_t)a * L + r] = w;
  Wsc[e] = svd_dropped(sig, a, k) ? 0.0 : w / sig[a];
  if (a < k) {
    Ck[(int64_t)a * L + r] = sgn[a] * w / sig[a];
    Bp[(int64_t)a * L + r] = sgn[a] * w;
  }
}

// N = M - (V~^T V_bar) S~^-1 with M the bracket of the SVD adjoint;
// XV = W^T (T^T V_bar) (L x k, so (V~^T V_bar)[a][b] = XV[a][b] / s_a), YW = W^T W_bar (L x k).
// Entries with a, b >= k carry no cotangent (every factor is zero) and are skipped, so ties and
// zeros among the trailing S~ never meet a 0/0; a dropped trailing direction gives a zero row.
__global__ void svdadj_mid_kernel(const double* __restrict__ XV, const double* __restrict__ YW,
                                  const double* __restrict__ sig, const float* __restrict__ gS, int L, int k,
                                  double* __restrict__ N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L * L) return;
  const int a = (int)(e / L), b = (int)(e % L);
  if ((a >= k && b >= k) || svd_dropped(sig, a, k)) {
    N[e] = 0.0;
    return;
  }
  const double sa = sig[a], sb = sig[b];
  const double XVab = b < k ? XV[(int64_t)a * k + b] : 0.0;  // s_a (V~^T V_bar)[a][b]
  const double XVba = a < k ? XV[(int64_t)b * k + a] : 0.0;  // s_b (V~^T V_bar)[b][a]
  const double yab = b < k ? YW[(int64_t)a * k + b] : 0.0;
  const double yba = a < k ? YW[(int64_t)b * k + a] : 0.0;
  double m = 0.0;
  if (a != b) {
    // F_ab ((V~^T V_bar)_ab - (V~^T V_bar)_ba) s_b + s_a F_ab ((W^T W_bar)_ab - (W^T W_bar)_ba),
    // F_ab = 1 / (s_b^2 - s_a^2); no division by s_b (which may be a tiny trailing value)
    const double f = 1.0 / ((sb - sa) * (sb + sa));
    m = f * (XVab * (sb / sa) - XVba) + sa * f * (yab - yba);
  } else if (gS != nullptr && a < k) {
    m = (double)gS[a];
  }
  N[e] = b < k ? m - XVab / (sa * sb) : m;
}

hipError_t launch_svdadj_prep(const double* W, const double* sig, const double* sgn, int L, int k, double* WT,
                              double* Wsc, double* Ck, double* Bp, hipStream_t st) {
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(svdadj_prep_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st, W, sig, sgn, L, k, WT,
                     Wsc, Ck, Bp);
  return hipGetLastError();
}

hipError_t launch_svdadj_mid(const double* XV, const double* YW, const double* sig, const float* gS, int L, int k,
                             double* N, hipStream_t st) {
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(svdadj_mid_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st, XV, YW, sig, gS, L, k,
                     N);
  return hipGetLastError();
}

// ---------------------------------------------------------------- QR adjoint pieces
// S = copyltu(-M2): S[a][b] = -M2[max(a,b)][min(a,b)]
__global__ void copyltu_neg_kernel(const double* __restrict__ M2, int L, double* __restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L * L) return;
  const int a = (int)(e / L), b = (int)(e % L);
  const int hi = a > b ? a : b, lo = a > b ? b : a;
  S[e] = -M2[(int64_t)hi * L + lo];
}

// out = in^T (L x L), optionally keeping only the upper triangle of `in`
__global__ void transpose_sq_kernel(const double* __restrict__ in, int L, int upper_only, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L * L) return;
  const int a = (int)(e / L), b = (int)(e % L);
  out[(int64_t)b * L + a] = (upper_only && b < a) ? 0.0 : in[e];
}

hipError_t launch_copyltu_neg(const double* M2, int L, double* S, hipStream_t st) {
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(copyltu_neg_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st, M2, L, S);
  return hipGetLastError();
}

hipError_t launch_transpose_sq(const double* in, int L, bool upper_only, double* out, hipStream_t st) {
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(transpose_sq_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st, in, L,
                     upper_only ? 1 : 0, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- conversions
// out32[c][r] = (float) X[r][c] and out64[c][r] = X[r][c] (rows x cols -> cols x rows), either may be null
__global__ void transpose_out_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows, int cols,
                                     float* __restrict__ out32, double* __restrict__ out64, int64_t ldo) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  for (int c = blockIdx.y; c < cols; c += gridDim.y) {
    const double v = X[r * ldx + c];
    if (out32 != nullptr) out32[(int64_t)c * ldo + r] = (float)v;
    if (out64 != nullptr) out64[(int64_t)c * ldo + r] = v;
  }
}

hipError_t launch_transpose_out(const double* X, int64_t ldx, int64_t rows, int cols, float* out32, double* out64,
                                int64_t ldo, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)(cols < 65535 ? cols : 65535));
  hipLaunchKernelGGL(transpose_out_kernel, grid, dim3(256), 0, st, X, ldx, rows, cols, out32, out64, ldo);
  return hipGetLastError();
}

// Y64[c][r] = (double) X32[c][r] for c < rows_t (row-major copy of transposed float blocks)
__global__ void widen_kernel(const float* __restrict__ X, int64_t ldx, int nrows, int64_t cols,
                             double* __restrict__ Y, int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= cols) return;
  for (int c = blockIdx.y; c < nrows; c += gridDim.y) Y[(int64_t)c * ldy + r] = (double)X[(int64_t)c * ldx + r];
}

hipError_t launch_widen(const float* X, int64_t ldx, int nrows, int64_t ncols, double* Y, int64_t ldy,
                        hipStream_t st) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  dim3 grid((unsigned)((ncols + 255) / 256), (unsigned)(nrows < 65535 ? nrows : 65535));
  hipLaunchKernelGGL(widen_kernel, grid, dim3(256), 0, st, X, ldx, nrows, ncols, Y, ldy);
  return hipGetLastError();
}

// C[r][c] (+)= (double) Z[r][c]
__global__ void add_f32_kernel(const float* __restrict__ Z, int64_t ldz, int64_t rows, int cols,
                               double* __restrict__ C, int64_t ldc, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  const double z = (double)Z[r * ldz + c];
  C[r * ldc + c] = accumulate ? C[r * ldc + c] + z : z;
}

hipError_t launch_add_f32(const float* Z, int64_t ldz, int64_t rows, int cols, double* C, int64_t ldc,
                          bool accumulate, hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_f32_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Z, ldz, rows, cols, C,
                     ldc, accumulate ? 1 : 0);
  return hipGetLastError();
}

// t = alpha * (Hb[r][c] + (Zf ? Zf[r][c] : 0)):  out64[r][c] = t, out32[r][c] = (float) t
__global__ void combine_kernel(const double* __restrict__ Hb, int64_t ldh, const float* __restrict__ Zf,
                               int64_t ldz, int64_t rows, int cols, const double* __restrict__ alpha,
                               double* __restrict__ out64, int64_t ld64, float* __restrict__ out32, int64_t ld32) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  double t = Hb[r * ldh + c];
  if (Zf != nullptr) t += (double)Zf[r * ldz + c];
  if (alpha != nullptr) t *= *alpha;
  if (out64 != nullptr) out64[r * ld64 + c] = t;
  if (out32 != nullptr) out32[r * ld32 + c] = (float)t;
}

hipError_t launch_combine(const double* Hb, int64_t ldh, const float* Zf, int64_t ldz, int64_t rows, int cols,
                          const double* alpha, double* out64, int64_t ld64, float* out32, int64_t ld32,
                          hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Hb, ldh, Zf, ldz, rows,
                     cols, alpha, out64, ld64, out32, ld32);
  return hipGetLastError();
}

// copy a float or double block into double columns: out[r][c] = X[r][c]
template <typename T>
__global__ void copy_cols_kernel(const T* __restrict__ X, int64_t ldx, int64_t rows, int cols,
                                 double* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  out[r * ldo + c] = (double)X[r * ldx + c];
}

hipError_t launch_copy_cols(bool x64, const void* X, int64_t ldx, int64_t rows, int cols, double* out, int64_t ldo,
                            hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  if (x64)
    hipLaunchKernelGGL(copy_cols_kernel<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       (const double*)X, ldx, rows, cols, out, ldo);
  else
    hipLaunchKernelGGL(copy_cols_kernel<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       (const float*)X, ldx, rows, cols, out, ldo);
  return hipGetLastError();
}

// ---------------------------------------------------------------- column centring of a float64 matrix
__global__ __launch_bounds__(256) void colsum64_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                       int cols, int64_t rps, double* __restrict__ part) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (c >= cols) return;
  const int64_t r0 = (int64_t)s * rps;
  const int64_t r1 = r0 + rps < rows ? r0 + rps : rows;
  double a0 = 0.0, a1 = 0.0;
  int64_t r = r0;
  for (; r + 1 < r1; r += 2) {
    a0 += X[r * ldx + c];
    a1 += X[(r + 1) * ldx + c];
  }
  if (r < r1) a0 += X[r * ldx + c];
  part[(int64_t)s * cols + c] = a0 + a1;
}

__global__ void sub_colmean_kernel(double* __restrict__ X, int64_t ldx, int64_t rows, int cols,
                                   const double* __restrict__ part, int nsplit, double inv_rows) {
  __shared__ double mean[256];
  const int c0 = blockIdx.y * 256;
  const int c = c0 + threadIdx.x;
  if (c < cols) {
    const double s = sum_strided(part + c, nsplit, (int64_t)cols);
    mean[threadIdx.x] = s * inv_rows;
  }
  __syncthreads();
  const int64_t r = blockIdx.x;
  if (r >= rows || c >= cols) return;
  X[r * ldx + c] -= mean[threadIdx.x];
}

hipError_t launch_center_f64(double* X, int64_t ldx, int64_t rows, int cols, int64_t rows_per_split, int nsplit,
                             double* part, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(colsum64_kernel, dim3((unsigned)((cols + 255) / 256), (unsigned)nsplit), dim3(256), 0, st, X, ldx,
                     rows, cols, rows_per_split, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sub_colmean_kernel, dim3((unsigned)rows, (unsigned)((cols + 255) / 256)), dim3(256), 0, st, X,
                     ldx, rows, cols, part, nsplit, 1.0 / (double)rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------- residual estimator helpers
// out[r][c] = normal(seed, stream, r * cols + c) (float64)
__global__ void gen_normal64_kernel(uint64_t seed, uint32_t stream, int64_t rows, int cols, double* __restrict__ out,
                                    int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  out[r * ldo + c] = normal_elem(seed, stream, (uint64_t)e);
}

hipError_t launch_gen_normal64(uint64_t seed, uint32_t stream, int64_t rows, int cols, double* out, int64_t ldo,
                               hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(gen_normal64_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, seed, stream, rows,
                     cols, out, ldo);
  return hipGetLastError();
}

// C[a][b] = -s[a] * C[a][b]  (k x q)
__global__ void neg_rowscale_kernel(double* __restrict__ C, const float* __restrict__ s, int k, int q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * q) return;
  C[e] = -(double)s[e / q] * C[e];
}

hipError_t launch_neg_rowscale(double* C, const float* s, int k, int q, hipStream_t st) {
  if (k * q <= 0) return hipSuccess;
  hipLaunchKernelGGL(neg_rowscale_kernel, dim3((unsigned)((k * q + 255) / 256)), dim3(256), 0, st, C, s, k, q);
  return hipGetLastError();
}

// out = sqrt(max_c v[c]) (one workgroup)
__global__ __launch_bounds__(256) void sqrt_max_kernel(const double* __restrict__ v, int q, double* __restrict__ out) {
  __shared__ double sh[256];
  double best = 0.0;
  for (int c = threadIdx.x; c < q; c += 256) best = fmax(best, v[c]);
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(sh[0]);
}

hipError_t launch_sqrt_max(const double* v, int q, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sqrt_max_kernel, dim3(1), dim3(256), 0, st, v, q, out);
  return hipGetLastError();
}

}  // namespace rpca
