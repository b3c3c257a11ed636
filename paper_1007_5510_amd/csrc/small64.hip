// Float64 dense steps that touch only O((i+1) l (m+n)) entries (Section 4:
// Steps 2, 4, 5 and 6 run "in RAM"):
//   Step 2  H = Q R by Cholesky QR applied twice (Gram, Cholesky, Q = H R^-1),
//           with a shifted first round as the fallback for ill-conditioned H;
//   Step 4  the SVD of T through the symmetric eigenproblem of T^T T, solved
//           by a one-sided block Jacobi method (each workgroup orthogonalises
//           a pair of column blocks held in LDS);
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

hipError_t launch_gram(bool x_is_f64, const void* X, int64_t ldx, int64_t rows, int L, int64_t rows_per_split,
                       int nsplit, double* part, hipStream_t st) {
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

__global__ void gram_reduce_kernel(const double* __restrict__ part, int nsplit, int L, double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t LL = (int64_t)L * L;
  if (e >= LL) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * LL + e];
  W[e] = s;
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
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st, part, nsplit, L, W);
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
// Column j of the inverse of an upper triangular R depends only on R and on
// itself: X[j][j] = 1/R[j][j], X[i][j] = -(sum_{p=i+1..j} R[i][p] X[p][j]) / R[i][i].
// One thread per column; R read from LDS (packed) when it fits.
template <bool PACKED>
__global__ __launch_bounds__(1024) void triinv_kernel(const double* __restrict__ R, int L,
                                                      double* __restrict__ X) {
  extern __shared__ double smem[];
  TriAcc a{PACKED ? smem : const_cast<double*>(R), L, PACKED};
  if (PACKED) {
    for (int64_t e = threadIdx.x; e < (int64_t)L * L; e += blockDim.x) {
      const int i = (int)(e / L), j = (int)(e % L);
      if (j >= i) a.at(i, j) = R[e];
    }
    __syncthreads();
  }
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    for (int i = j + 1; i < L; ++i) X[(int64_t)i * L + j] = 0.0;
    X[(int64_t)j * L + j] = 1.0 / a.at(j, j);
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int p = i + 1; p <= j; ++p) s = fma(a.at(i, p), X[(int64_t)p * L + j], s);
      X[(int64_t)i * L + j] = -s / a.at(i, i);
    }
  }
}

hipError_t launch_triinv(const double* R, int L, double* Rinv, hipStream_t st) {
  const size_t bytes = (size_t)L * (L + 1) / 2 * sizeof(double);
  if (bytes <= g_max_lds) {
    hipLaunchKernelGGL(triinv_kernel<true>, dim3(1), dim3(1024), bytes, st, R, L, Rinv);
  } else {
    hipLaunchKernelGGL(triinv_kernel<false>, dim3(1), dim3(1024), 0, st, R, L, Rinv);
  }
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
// C[M x N] = A[M x K] B[K x N] (* colscale); 64 x 64 tiles, 4 x 4 per thread.
template <typename TA>
__global__ __launch_bounds__(256) void gemm64_kernel(const TA* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ B, int64_t ldb, int64_t M, int N,
                                                     int K, int b_upper, const double* __restrict__ colscale,
                                                     double* __restrict__ C, int64_t ldc, float* __restrict__ C32,
                                                     int64_t ldc32) {
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
      const double v = acc[a][b] * sc;
      if (C != nullptr) C[r * ldc + c] = v;
      if (C32 != nullptr) C32[r * ldc32 + c] = (float)v;
    }
  }
}

hipError_t launch_gemm64(bool a_is_f64, const void* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int N,
                         int K, bool b_upper, const double* colscale, double* C, int64_t ldc, float* C32,
                         int64_t ldc32, hipStream_t st) {
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  if (a_is_f64)
    hipLaunchKernelGGL(gemm64_kernel<double>, grid, dim3(256), 0, st, (const double*)A, lda, B, ldb, M, N, K,
                       b_upper ? 1 : 0, colscale, C, ldc, C32, ldc32);
  else
    hipLaunchKernelGGL(gemm64_kernel<float>, grid, dim3(256), 0, st, (const float*)A, lda, B, ldb, M, N, K,
                       b_upper ? 1 : 0, colscale, C, ldc, C32, ldc32);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Jacobi
// Round-robin ("circle") schedule: for an even count N, round r in [0, N-1)
// pairs t = 0 .. N/2-1 as (N-1, r) for t = 0 and ((r+t) mod (N-1),
// (r-t) mod (N-1)) otherwise; every pair meets exactly once per N-1 rounds.
RPCA_DEV void circle_pair(int r, int t, int N, int& a, int& b) {
  if (t == 0) {
    a = N - 1;
    b = r;
  } else {
    a = (r + t) % (N - 1);
    b = (r - t + (N - 1)) % (N - 1);
  }
}

JacobiPlan jacobi_plan(int L) {
  JacobiPlan jp;
  jp.L = L;
  int nb = 4608 / (L > 0 ? L : 1);  // 2 blocks x nb columns x L rows x (B, V) doubles <= 144 KiB
  if (nb > 32) nb = 32;
  if (nb < 1) nb = 1;
  if (2 * nb >= L) nb = (L + 1) / 2;  // one block pair covers every column
  jp.nb = nb;
  int nblk = (L + nb - 1) / nb;
  if (nblk < 2) nblk = 2;
  if (nblk & 1) ++nblk;
  jp.nblk = nblk;
  jp.lds_bytes = (size_t)2 * nb * L * 2 * sizeof(double);
  return jp;
}

__global__ void jacobi_init_kernel(const double* __restrict__ M, int L, double* __restrict__ B,
                                   double* __restrict__ V, int* __restrict__ rot_count, int max_sweeps) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t LL = (int64_t)L * L;
  if (e < LL) {
    const int c = (int)(e / L), r = (int)(e % L);  // column-major B, V
    B[e] = M[(int64_t)r * L + c];
    V[e] = (r == c) ? 1.0 : 0.0;
  }
  if (e < max_sweeps) rot_count[e] = 0;
}

hipError_t launch_jacobi_init(const double* M, int L, double* B, double* V, int* rot_count, int max_sweeps,
                              hipStream_t st) {
  int64_t tot = (int64_t)L * L;
  if (tot < max_sweeps) tot = max_sweeps;
  hipLaunchKernelGGL(jacobi_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, L, B, V,
                     rot_count, max_sweeps);
  return hipGetLastError();
}

// One round of the block schedule: workgroup w orthogonalises (one inner
// sweep over all column pairs) the union of its two column blocks, held in LDS.
__global__ __launch_bounds__(1024) void jacobi_round_kernel(double* __restrict__ B, double* __restrict__ V, int L,
                                                            int nb, int nblk, int sweep, int round,
                                                            int* __restrict__ rot_count, double tol) {
  if (sweep > 0 && rot_count[sweep - 1] == 0) return;  // previous sweep rotated nothing: converged
  extern __shared__ double smem[];
  int ba, bb;
  circle_pair(round, blockIdx.x, nblk, ba, bb);
  const int a0 = ba * nb, b0 = bb * nb;
  const int na = a0 < L ? (a0 + nb <= L ? nb : L - a0) : 0;
  const int nbb = b0 < L ? (b0 + nb <= L ? nb : L - b0) : 0;
  const int ncl = na + nbb;
  auto gcol = [&](int lc) { return lc < na ? a0 + lc : b0 + (lc - na); };
  if (ncl < 2) return;
  double* Bs = smem;                  // ncl columns of L
  double* Vs = smem + (int64_t)ncl * L;
  for (int64_t e = threadIdx.x; e < (int64_t)ncl * L; e += blockDim.x) {
    const int lc = (int)(e / L), r = (int)(e % L);
    Bs[e] = B[(int64_t)gcol(lc) * L + r];
    Vs[e] = V[(int64_t)gcol(lc) * L + r];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int NI = (ncl + 1) & ~1;
  int rotations = 0;
  for (int ir = 0; ir < NI - 1; ++ir) {
    for (int t = wave; t < NI / 2; t += nwave) {
      int p, q;
      circle_pair(ir, t, NI, p, q);
      if (p >= ncl || q >= ncl) continue;
      double* bp = Bs + (int64_t)p * L;
      double* bq = Bs + (int64_t)q * L;
      double al = 0.0, be = 0.0, ga = 0.0;
      for (int r = lane; r < L; r += 64) {
        const double x = bp[r], y = bq[r];
        al = fma(x, x, al);
        be = fma(y, y, be);
        ga = fma(x, y, ga);
      }
      al = wave_sum(al);
      be = wave_sum(be);
      ga = wave_sum(ga);
      if (!(fabs(ga) > tol * sqrt(al) * sqrt(be)) || al == 0.0 || be == 0.0) continue;
      const double zeta = (be - al) / (2.0 * ga);
      const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
      const double cs = 1.0 / sqrt(1.0 + tt * tt);
      const double sn = cs * tt;
      double* vp = Vs + (int64_t)p * L;
      double* vq = Vs + (int64_t)q * L;
      for (int r = lane; r < L; r += 64) {
        const double x = bp[r], y = bq[r];
        bp[r] = cs * x - sn * y;
        bq[r] = sn * x + cs * y;
        const double u = vp[r], w = vq[r];
        vp[r] = cs * u - sn * w;
        vq[r] = sn * u + cs * w;
      }
      ++rotations;
    }
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; e < (int64_t)ncl * L; e += blockDim.x) {
    const int lc = (int)(e / L), r = (int)(e % L);
    B[(int64_t)gcol(lc) * L + r] = Bs[e];
    V[(int64_t)gcol(lc) * L + r] = Vs[e];
  }
  if (lane == 0 && rotations > 0) atomicAdd(rot_count + sweep, rotations);
}

hipError_t launch_jacobi_round(const JacobiPlan& jp, double* B, double* V, int sweep, int round, int* rot_count,
                               double tol, hipStream_t st) {
  hipLaunchKernelGGL(jacobi_round_kernel, dim3((unsigned)(jp.nblk / 2)), dim3(1024), jp.lds_bytes, st, B, V, jp.L,
                     jp.nb, jp.nblk, sweep, round, rot_count, tol);
  return hipGetLastError();
}

// lam[j] = ||B[:, j]||; order sorts lam descending (ties by column index);
// Wsorted[i][r] = V[i][order[r]] row-major, sig_sorted[r] = sqrt(lam[order[r]]) (lam are
// eigenvalues of T^T T, so these are the singular values of T).
__global__ __launch_bounds__(1024) void jacobi_finish_kernel(const double* __restrict__ B,
                                                             const double* __restrict__ V, int L,
                                                             double* __restrict__ lam, int* __restrict__ order,
                                                             double* __restrict__ Wsorted,
                                                             double* __restrict__ sig_sorted) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int j = wave; j < L; j += nwave) {
    double s = 0.0;
    for (int r = lane; r < L; r += 64) {
      const double x = B[(int64_t)j * L + r];
      s = fma(x, x, s);
    }
    s = wave_sum(s);
    if (lane == 0) lam[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    const double v = lam[j];
    int rank = 0;
    for (int i = 0; i < L; ++i) {
      const double w = lam[i];
      rank += (w > v || (w == v && i < j)) ? 1 : 0;
    }
    order[rank] = j;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)L * L; e += blockDim.x) {
    const int i = (int)(e / L), r = (int)(e % L);
    Wsorted[e] = V[(int64_t)order[r] * L + i];
  }
  for (int r = threadIdx.x; r < L; r += blockDim.x) sig_sorted[r] = sqrt(lam[order[r]]);
}

hipError_t launch_jacobi_finish(const double* B, const double* V, int L, double* lam, int* order, double* Wsorted,
                                double* sig_sorted, hipStream_t st) {
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(1024), 0, st, B, V, L, lam, order, Wsorted, sig_sorted);
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
