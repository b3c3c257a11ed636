// Symmetric eigen-decomposition of the small Gram matrix M = T^T T (L x L,
// float64) that gives the SVD of T in Step 4 (eq. svd_small3): M = W S~^2 W^T.
// One workgroup does the whole job so that no grid-wide synchronisation or
// chain of launches is needed:
//
//   1. Householder reduction to tridiagonal form, M = H T_d H^T (lower
//      storage, reflectors kept in the zeroed part of M);
//   2. every eigenvalue of T_d by bisection on Sturm counts, a few threads
//      per eigenvalue evaluating several points per step;
//   3. eigenvectors of T_d for the wanted (largest) eigenvalues by inverse
//      iteration on the LU factors of T_d - lambda I with partial pivoting;
//      eigenvalues closer than 1e-7 ||T_d|| are treated as a cluster and
//      their vectors are orthogonalised against each other during the
//      iteration;
//   4. back-transformation W = H Y.
//
// The reduction is O(L^3) once, where a Jacobi method moves O(L^3) data per
// sweep, and it is backward stable, so the eigenvalues have absolute error
// O(u ||M||), the same bound as any method that starts from M.
#include "common.h"
#include "kernels.h"

namespace rpca {

namespace {

constexpr int EIG_THREADS = 1024;

// lower-triangular storage, column-major packed (column k holds rows k..L-1)
// when PACKED, full row-major otherwise
template <bool PACKED>
struct LowAcc {
  double* p;
  int L;
  RPCA_DEV double& at(int i, int k) const {  // requires i >= k
    return PACKED ? p[(int64_t)k * L - (int64_t)k * (k - 1) / 2 + (i - k)] : p[(int64_t)i * L + k];
  }
  RPCA_DEV double sym(int i, int k) const { return i >= k ? at(i, k) : at(k, i); }
};

RPCA_DEV double block_reduce_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int q = 0; q < nw; ++q) s += red[q];
  return s;  // every thread gets the same value
}

// number of eigenvalues of the tridiagonal (d, e2 = e^2) smaller than x
RPCA_DEV int sturm_count(const double* d, const double* e2, int L, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < L; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// deterministic start vector entry in (-1, 1)
RPCA_DEV double start_entry(int i, int r) {
  uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)r * 0x85EBCA77u + 0x165667B1u);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return ((double)(h >> 8) + 0.5) * (2.0 / 16777216.0) - 1.0;
}

}  // namespace

// work: global scratch of at least L*L + kk*6*L doubles (full-storage
// reduction area and per-vector inverse-iteration arrays).
template <bool PACKED>
__global__ __launch_bounds__(EIG_THREADS) void syev_small_kernel(const double* __restrict__ M, int L, int kk,
                                                                 double* __restrict__ work,
                                                                 double* __restrict__ lam_desc,
                                                                 double* __restrict__ sig_desc,
                                                                 double* __restrict__ W, int ldw) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x, nt = blockDim.x;
  double* red = smem;          // 32
  double* d = smem + 32;       // L
  double* e = d + L;           // L
  double* tau = e + L;         // L
  double* vw = tau + L;        // 2L: v (Householder vector) and p/w
  double* lstore = vw + 2 * L; // packed lower M when PACKED
  LowAcc<PACKED> a{PACKED ? lstore : work, L};
  double* Y = work + (PACKED ? 0 : (int64_t)L * L);  // L x kk column-major (vector c at Y + c*L)
  double* iw = Y + (int64_t)L * kk;                   // kk x 5L inverse-iteration work

  // load the lower triangle
  for (int64_t t = tid; t < (int64_t)L * L; t += nt) {
    const int i = (int)(t / L), k = (int)(t % L);
    if (i >= k) a.at(i, k) = M[t];
  }
  __syncthreads();

  // ---- 1. tridiagonalisation (Householder from the left and right, lower)
  double* v = vw;
  double* pw = vw + L;
  for (int j = 0; j + 2 < L; ++j) {
    const int r0 = j + 1;  // first row of the trailing block
    const int nr = L - r0;
    double xs = 0.0;
    for (int i = r0 + 1 + tid; i < L; i += nt) {
      const double x = a.at(i, j);
      xs = fma(x, x, xs);
    }
    const double xnorm2 = block_reduce_sum(xs, red);
    const double alpha = a.at(r0, j);
    if (xnorm2 == 0.0) {  // column already reduced: H_j = I
      if (tid == 0) {
        tau[j] = 0.0;
        e[j] = alpha;
      }
      __syncthreads();
      continue;
    }
    const double beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    const double tj = (beta - alpha) / beta;
    const double scal = 1.0 / (alpha - beta);
    for (int i = r0 + tid; i < L; i += nt) {
      const double vi = (i == r0) ? 1.0 : a.at(i, j) * scal;
      v[i] = vi;
      if (i > r0) a.at(i, j) = vi;  // reflector kept below the subdiagonal
    }
    if (tid == 0) {
      tau[j] = tj;
      e[j] = beta;
    }
    __syncthreads();
    // p = tau A22 v, several threads per row, partial sums combined in-wave
    int tpr = 1;
    while (tpr * 2 * nr <= nt && tpr < 64) tpr *= 2;
    {
      const int row = r0 + tid / tpr, part = tid % tpr;
      double s = 0.0;
      if (tid / tpr < nr) {
        for (int k = r0 + part; k < L; k += tpr) s = fma(a.sym(row, k), v[k], s);
      }
      for (int o = tpr / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (tid / tpr < nr && part == 0) pw[row] = tj * s;
    }
    __syncthreads();
    double ps = 0.0;
    for (int i = r0 + tid; i < L; i += nt) ps = fma(pw[i], v[i], ps);
    const double kdot = 0.5 * tj * block_reduce_sum(ps, red);
    for (int i = r0 + tid; i < L; i += nt) pw[i] -= kdot * v[i];
    __syncthreads();
    // A22 -= v w^T + w v^T (lower part)
    const int64_t tot = (int64_t)nr * nr;
    for (int64_t t = tid; t < tot; t += nt) {
      const int i = r0 + (int)(t / nr), k = r0 + (int)(t % nr);
      if (i >= k) a.at(i, k) -= v[i] * pw[k] + pw[i] * v[k];
    }
    __syncthreads();
  }
  for (int j = tid; j < L; j += nt) {
    d[j] = a.at(j, j);
    if (j + 2 >= L) tau[j] = 0.0;
  }
  if (tid == 0 && L >= 2) e[L - 2] = a.at(L - 1, L - 2);
  __syncthreads();

  // ---- 2. eigenvalues by multisection: G threads per eigenvalue
  double* e2 = pw;  // reuse: e^2
  for (int i = tid; i + 1 < L; i += nt) e2[i] = e[i] * e[i];
  double* lam = v;  // ascending eigenvalues
  __syncthreads();
  double gl = 0.0, gu = 0.0, emax2 = 0.0;
  for (int i = 0; i < L; ++i) {
    const double off = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < L ? fabs(e[i]) : 0.0);
    gl = i == 0 ? d[i] - off : fmin(gl, d[i] - off);
    gu = i == 0 ? d[i] + off : fmax(gu, d[i] + off);
    if (i + 1 < L) emax2 = fmax(emax2, e2[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  // the reduction is accurate to O(u ||T_d||) in absolute terms: bisect to that
  const double atol = 2.220446049250313e-16 * tnorm + 2.0 * pivmin;
  {
    int G = 1;
    while (G * 2 * L <= nt && G < 16) G *= 2;
    const int idx = tid / G, part = tid % G;
    // every eigenvalue index gets a group; bisection loop is uniform inside a group
    const bool active = idx < L;
    double lo = gl - 2.2e-16 * tnorm - atol, hi = gu + 2.2e-16 * tnorm + atol;
    for (int it = 0; it < 200; ++it) {
      const double width = hi - lo;
      const double tolr = 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + atol;
      // the group's lanes are consecutive in one wave; all take the same decision
      const bool done = !active || width <= tolr;
      const uint64_t ballot = __ballot(!done);
      if (ballot == 0) break;
      double x = lo + width * (double)(part + 1) / (double)(G + 1);
      int cnt = active ? sturm_count(d, e2, L, x, pivmin) : 0;
      // number of group points whose count is <= idx: the eigenvalue lies right of them
      int below = (cnt <= idx) ? 1 : 0;
      for (int o = G / 2; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
      if (!done) {
        const double nlo = lo + width * (double)below / (double)(G + 1);
        const double nhi = lo + width * (double)(below + 1) / (double)(G + 1);
        lo = below == 0 ? lo : nlo;
        hi = below == G ? hi : nhi;
      }
    }
    if (active && part == 0) lam[idx] = 0.5 * (lo + hi);
  }
  __syncthreads();
  for (int r = tid; r < L; r += nt) {
    lam_desc[r] = lam[L - 1 - r];
    sig_desc[r] = sqrt(fmax(lam[L - 1 - r], 0.0));
  }

  // ---- 3. inverse iteration for the kk largest eigenvalues (one thread each;
  // a cluster of close eigenvalues is handled by its first member, sequentially)
  const double ctol = 1e-7 * fmax(tnorm, 1e-300);
  for (int r = tid; r < kk; r += nt) {
    // skip if r belongs to a cluster that started at r-1
    const int ia = L - 1 - r;
    if (r > 0 && fabs(lam[ia + 1] - lam[ia]) <= ctol) continue;
    int cend = r;
    while (cend + 1 < kk && fabs(lam[L - 1 - cend] - lam[L - 2 - cend]) <= ctol) ++cend;
    for (int rr = r; rr <= cend; ++rr) {
      double* y = Y + (int64_t)rr * L;
      double* dl = iw + (int64_t)rr * 5 * L;  // sub-diagonal multipliers
      double* u0 = dl + L;                    // diagonal of U
      double* u1 = u0 + L;                    // first super-diagonal of U
      double* u2 = u1 + L;                    // second super-diagonal (fill-in)
      double* pv = u2 + L;                    // pivot flags
      // perturb inside a cluster so the shifted matrices differ
      const double lambda = lam[L - 1 - rr] + (double)(rr - r) * 4.0 * 2.220446049250313e-16 * tnorm;
      // LU of T_d - lambda I with partial pivoting (rows i, i+1)
      double diag = d[0] - lambda, sup = L > 1 ? e[0] : 0.0, sup2 = 0.0;
      for (int i = 0; i < L - 1; ++i) {
        const double sub = e[i];
        const double nd = d[i + 1] - lambda;
        const double nsup = (i + 2 < L) ? e[i + 1] : 0.0;
        if (fabs(diag) >= fabs(sub)) {  // no swap
          const double mlt = diag != 0.0 ? sub / diag : 0.0;
          dl[i] = mlt;
          pv[i] = 0.0;
          u0[i] = diag;
          u1[i] = sup;
          u2[i] = sup2;
          diag = nd - mlt * sup;
          sup = nsup;
          sup2 = 0.0;
        } else {  // swap rows i and i+1
          const double mlt = diag / sub;
          dl[i] = mlt;
          pv[i] = 1.0;
          u0[i] = sub;
          u1[i] = nd;
          u2[i] = nsup;
          diag = sup - mlt * nd;
          sup = -mlt * nsup;
          sup2 = 0.0;
        }
        if (u0[i] == 0.0) u0[i] = 2.220446049250313e-16 * tnorm + pivmin;
      }
      u0[L - 1] = diag != 0.0 ? diag : 2.220446049250313e-16 * tnorm + pivmin;
      u1[L - 1] = 0.0;
      u2[L - 1] = 0.0;
      if (L >= 2) u2[L - 2] = 0.0;
      for (int i = 0; i < L; ++i) y[i] = start_entry(i, rr);
      for (int iter = 0; iter < 3; ++iter) {
        // forward: apply the row swaps and multipliers
        for (int i = 0; i < L - 1; ++i) {
          if (pv[i] != 0.0) {
            const double t = y[i];
            y[i] = y[i + 1];
            y[i + 1] = t;
          }
          y[i + 1] -= dl[i] * y[i];
        }
        // backward substitution with U (three diagonals)
        for (int i = L - 1; i >= 0; --i) {
          double s = y[i];
          if (i + 1 < L) s -= u1[i] * y[i + 1];
          if (i + 2 < L) s -= u2[i] * y[i + 2];
          y[i] = s / u0[i];
        }
        // orthogonalise against the earlier members of the cluster
        for (int q = r; q < rr; ++q) {
          const double* yq = Y + (int64_t)q * L;
          double dot = 0.0;
          for (int i = 0; i < L; ++i) dot = fma(yq[i], y[i], dot);
          for (int i = 0; i < L; ++i) y[i] -= dot * yq[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < L; ++i) nrm = fma(y[i], y[i], nrm);
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = 0; i < L; ++i) y[i] *= inv;
      }
    }
  }
  __syncthreads();
  __threadfence_block();

  // ---- 4. back-transformation Y <- H_0 ... H_{L-3} Y (reflectors applied last-first)
  double* dots = pw;  // kk values
  for (int j = L - 3; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;  // uniform
    const int r0 = j + 1;
    // dots[c] = v^T Y[r0:, c]; a group of threads per column
    int tpc = 1;
    while (tpc * 2 * kk <= nt && tpc < 64) tpc *= 2;
    {
      const int c = tid / tpc, part = tid % tpc;
      double s = 0.0;
      if (c < kk) {
        const double* y = Y + (int64_t)c * L;
        for (int i = r0 + part; i < L; i += tpc) s = fma(i == r0 ? 1.0 : a.at(i, j), y[i], s);
      }
      for (int o = tpc / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (c < kk && part == 0) dots[c] = tj * s;
    }
    __syncthreads();
    const int nr = L - r0;
    for (int64_t t = tid; t < (int64_t)kk * nr; t += nt) {
      const int c = (int)(t / nr), i = r0 + (int)(t % nr);
      const double vi = i == r0 ? 1.0 : a.at(i, j);
      Y[(int64_t)c * L + i] -= dots[c] * vi;
    }
    __syncthreads();
  }
  // W row-major: W[i][c] = Y[c][i]
  for (int64_t t = tid; t < (int64_t)L * kk; t += nt) {
    const int i = (int)(t / kk), c = (int)(t % kk);
    W[(int64_t)i * ldw + c] = Y[(int64_t)c * L + i];
  }
}

size_t syev_small_lds(int L, bool packed) {
  size_t base = (32 + 5 * (size_t)L) * sizeof(double);
  if (packed) base += (size_t)L * (L + 1) / 2 * sizeof(double);
  return base;
}

size_t syev_small_work(int L, int kk) { return (size_t)L * L + (size_t)kk * 6 * L + 64; }

hipError_t launch_syev_small(const double* M, int L, int kk, double* work, double* lam_desc, double* sig_desc,
                             double* W, int ldw, size_t max_lds, hipStream_t st) {
  if (L < 1 || kk < 1 || kk > L) return hipErrorInvalidValue;
  const size_t packed = syev_small_lds(L, true);
  if (packed <= max_lds)
    hipLaunchKernelGGL(syev_small_kernel<true>, dim3(1), dim3(EIG_THREADS), packed, st, M, L, kk, work, lam_desc,
                       sig_desc, W, ldw);
  else
    hipLaunchKernelGGL(syev_small_kernel<false>, dim3(1), dim3(EIG_THREADS), syev_small_lds(L, false), st, M, L, kk,
                       work, lam_desc, sig_desc, W, ldw);
  return hipGetLastError();
}

}  // namespace rpca
