// Symmetric eigen-decomposition of the small Gram matrix M = T^T T (L x L,
// float64) that gives the SVD of T in Step 4 (eq. svd_small3): M = W S~^2 W^T.
// Four launches on one stream:
//
//   1. tridiag_kernel (one workgroup): Householder reduction to tridiagonal
//      form, M = H T_d H^T, on the packed lower triangle held in LDS (in
//      global memory when it does not fit).  Per step the symmetric product
//      p = tau A22 v takes 16 lanes per output entry, the rank-2 update one
//      wave per column; the wave that updates the first trailing column
//      builds the next reflector from its registers while the others finish
//      the update, so a step costs two workgroup barriers.  The reflectors
//      stay in the zeroed part of the packed matrix, which is written out.
//   2. bisect_kernel: every eigenvalue of T_d by multisection on Sturm
//      counts, one wave per eigenvalue evaluating 64 points per step.
//   3. inviter_kernel: eigenvectors of T_d for the wanted (largest)
//      eigenvalues by inverse iteration on the LU factors of T_d - lambda I
//      with partial pivoting, one thread per eigenvector with its arrays in
//      LDS; eigenvalues closer than 1e-7 ||T_d|| form a cluster whose vectors
//      the first member computes in turn, orthogonalising each against the
//      earlier ones.
//   4. backtrans_kernel: W = H Y, one wave per eigenvector, reflectors
//      staged in LDS when they fit.
//
// The reduction is O(L^3) once, where a Jacobi method moves O(L^3) data per
// sweep, and it is backward stable, so the eigenvalues have absolute error
// O(u ||M||), the same bound as any method that starts from M.
#include "common.h"
#include "kernels.h"

namespace rpca {

namespace {

constexpr int TRD_THREADS = 1024;
constexpr int TRD_WAVES = TRD_THREADS / 64;
constexpr int BT_WAVES = 8;  // eigenvectors per back-transformation workgroup
constexpr double EPS = 2.220446049250313e-16;

// start of packed column k (column k holds rows k .. L-1 contiguously)
RPCA_DEV int poff(int k, int L) { return k * L - (k * (k - 1)) / 2; }

template <int CTRL>
RPCA_DEV double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// sum over each group of 16 lanes (butterfly: xor 1, xor 2, half-row mirror,
// row mirror); every lane of the group ends with the same bits
RPCA_DEV double row_sum16(double x) {
  x += dpp_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f64<0x141>(x);  // row_half_mirror
  x += dpp_f64<0x140>(x);  // row_mirror
  return x;
}

// all 64 lanes; every lane ends with the same bits
RPCA_DEV double wave_sum64(double x) {
  x = row_sum16(x);
  x += __shfl_xor(x, 16, 64);
  x += __shfl_xor(x, 32, 64);
  return x;
}

// Reflector of column jj from x[q] = A(jj + lane + 64 q, jj) (wave-wide):
// H = I - tau v v^T with v(jj+1) = 1 maps the column below the diagonal to
// beta e_1.  v is written to vs[jj+1 ..] and below the subdiagonal of the
// packed column; tau to *tau_slot and taug[jj]; beta (or the unchanged
// subdiagonal when the column is already reduced, tau = 0) to eg[jj].
template <int NQ>
RPCA_DEV void make_reflector(const double (&x)[NQ], int jj, int L, double* P, double* vs, double* tau_slot,
                             double* __restrict__ eg, double* __restrict__ taug) {
  const int lane = threadIdx.x & 63;
  double xs = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = jj + lane + 64 * q;
    if (i >= jj + 2 && i < L) xs = fma(x[q], x[q], xs);
  }
  const double xnorm2 = wave_sum64(xs);
  const double alpha = __shfl(x[0], 1, 64);
  if (xnorm2 == 0.0) {  // uniform
    if (lane == 0) {
      *tau_slot = 0.0;
      taug[jj] = 0.0;
      eg[jj] = alpha;
    }
    return;
  }
  const double beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
  const double tj = (beta - alpha) / beta;
  const double scal = 1.0 / (alpha - beta);
  const int o = poff(jj, L) - jj;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = jj + lane + 64 * q;
    if (i == jj + 1) {
      vs[i] = 1.0;
    } else if (i >= jj + 2 && i < L) {
      const double vi = x[q] * scal;
      vs[i] = vi;
      P[o + i] = vi;
    }
  }
  if (lane == 0) {
    *tau_slot = tj;
    taug[jj] = tj;
    eg[jj] = beta;
  }
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

// Scratch layout (doubles): packed reflectors, d, e, tau, ascending
// eigenvalues, two scalars (||T_d||, pivmin), then the eigenvectors of T_d
// with entry i of vector r at [i * kk + r].
struct EigWork {
  double *P, *d, *e, *tau, *lam, *scal, *Y;
};

size_t packed_size(int L) { return ((size_t)L * (L + 1) / 2 + 7) / 8 * 8; }

EigWork eig_layout(double* work, int L, int kk) {
  EigWork w;
  w.P = work;
  w.d = work + packed_size(L);
  w.e = w.d + L;
  w.tau = w.e + L;
  w.lam = w.tau + L;
  w.scal = w.lam + L;
  w.Y = w.scal + 8;
  return w;
}

// ---- 1. Householder tridiagonalisation, one workgroup
// NQ >= ceil(L / 64) rows per lane for a whole column.  With COLMV (matrix in global memory)
// the symmetric product runs by columns: one wave per packed column, read once and
// contiguously, feeding both the column's dot product with v and its axpy into a
// wave-private partial p (TRD_WAVES x L doubles of LDS); the partials are then summed.
template <bool IN_LDS, int NQ, bool COLMV = false>
__global__ __launch_bounds__(TRD_THREADS) void tridiag_kernel(const double* __restrict__ M, int L,
                                                              double* __restrict__ gP, double* __restrict__ dg,
                                                              double* __restrict__ eg, double* __restrict__ taug) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* red = smem;        // per-wave partial sums
  double* tauS = smem + 16;  // tau of the pending reflector, by step parity
  double* vS = smem + 32;    // two reflector vectors, by step parity
  double* p = vS + 2 * L;    // tau A22 v
  double* P = IN_LDS ? p + L : gP;
  const int np = L * (L + 1) / 2;

  // packed lower triangle A(i, k), i >= k, read as row k of the symmetric M
  for (int k = wave; k < L; k += TRD_WAVES) {
    const int o = poff(k, L) - k;
    for (int i = k + lane; i < L; i += 64) P[o + i] = M[(int64_t)k * L + i];
  }
  __syncthreads();
  if (L >= 3 && wave == 0) {
    double x[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      x[q] = i < L ? P[i] : 0.0;
    }
    make_reflector<NQ>(x, 0, L, P, vS, tauS, eg, taug);
  }
  for (int j = 0; j + 2 < L; ++j) {
    __syncthreads();  // reflector j and the update of step j-1 are complete
    const int slot = j & 1;
    const double tj = tauS[slot];
    const double* v = vS + slot * L;
    const int r0 = j + 1, nr = L - r0;
    const bool next = j + 3 < L;  // reflector j+1 is still needed
    if (tj != 0.0) {
      double ptv = 0.0;
      if (COLMV) {
        // column c (rows c .. L-1 contiguous) adds A(i, c) v[c] to yw[i], i >= c, and its dot
        // with v below the diagonal to yw[c]; each wave owns its yw
        double* yw = p + L + wave * L;
        for (int i = r0 + lane; i < L; i += 64) yw[i] = 0.0;
        for (int c = r0 + wave; c < L; c += TRD_WAVES) {
          const int oc = poff(c, L) - c;
          const double vc = v[c];
          double d = 0.0;
          for (int i = c + lane; i < L; i += 64) {
            const double a = P[oc + i];
            yw[i] = fma(a, vc, yw[i]);
            if (i > c) d = fma(a, v[i], d);
          }
          d = wave_sum64(d);
          if (lane == 0) yw[c] += d;
        }
        __syncthreads();
        for (int t = r0 + tid; t < L; t += TRD_THREADS) {
          double s = 0.0;
#pragma unroll
          for (int w = 0; w < TRD_WAVES; ++w) s += p[L + w * L + t];
          const double pt = tj * s;
          p[t] = pt;
          ptv = fma(pt, v[t], ptv);
        }
      } else {
        // p[t] = tj sum_c A(t, c) v[c] over c >= r0; 16 lanes per t
        const int g = lane >> 4, u0 = lane & 15;
        for (int tb = r0 + 4 * wave; tb < L; tb += 4 * TRD_WAVES) {
          const int t = tb + g;
          double s = 0.0;
          if (t < L) {
            const int ot = poff(t, L) - t;
            for (int u = u0; u < nr; u += 16) {
              const int c = r0 + u;
              const double a = c <= t ? P[poff(c, L) + t - c] : P[ot + c];
              s = fma(a, v[c], s);
            }
          }
          s = row_sum16(s);
          if (u0 == 0 && t < L) {
            const double pt = tj * s;
            p[t] = pt;
            ptv = fma(pt, v[t], ptv);
          }
        }
      }
      ptv = wave_sum64(ptv);
      if (lane == 0) red[wave] = ptv;
      __syncthreads();
      double tot = 0.0;
#pragma unroll
      for (int q = 0; q < TRD_WAVES; ++q) tot += red[q];
      const double kdot = 0.5 * tj * tot;
      // A22 -= v w^T + w v^T with w = p - kdot v; one wave per column.  The wave that
      // builds reflector j+1 from column r0 takes no other column, so the reflector (on the
      // critical path of the next step) overlaps the other waves' column updates
      const int kfirst = next ? (wave == 0 ? r0 : r0 + wave) : r0 + wave;
      const int kstep = next ? (wave == 0 ? L : TRD_WAVES - 1) : TRD_WAVES;
      for (int k = kfirst; k < L; k += kstep) {
        const int ok = poff(k, L) - k;
        const double vk = v[k], wk = p[k] - kdot * vk;
        if (next && k == r0) {  // first trailing column: keep it and build reflector j+1
          double x[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int i = k + lane + 64 * q;
            x[q] = 0.0;
            if (i < L) {
              const double vi = v[i], wi = p[i] - kdot * vi;
              x[q] = P[ok + i] - (vi * wk + wi * vk);
              P[ok + i] = x[q];
            }
          }
          make_reflector<NQ>(x, r0, L, P, vS + (slot ^ 1) * L, tauS + (slot ^ 1), eg, taug);
        } else {
          for (int i = k + lane; i < L; i += 64) {
            const double vi = v[i], wi = p[i] - kdot * vi;
            P[ok + i] -= vi * wk + wi * vk;
          }
        }
      }
    } else if (next && wave == 0) {  // no update: reflector j+1 from the stored column
      double x[NQ];
      const int o = poff(r0, L) - r0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = r0 + lane + 64 * q;
        x[q] = i < L ? P[o + i] : 0.0;
      }
      make_reflector<NQ>(x, r0, L, P, vS + (slot ^ 1) * L, tauS + (slot ^ 1), eg, taug);
    }
  }
  __syncthreads();
  for (int i = tid; i < L; i += TRD_THREADS) dg[i] = P[poff(i, L)];
  if (tid == 0) {
    if (L >= 2) {
      eg[L - 2] = P[poff(L - 2, L) + 1];
      taug[L - 2] = 0.0;
    }
    eg[L - 1] = 0.0;
    taug[L - 1] = 0.0;
  }
  if (IN_LDS)
    for (int t = tid; t < np; t += TRD_THREADS) gP[t] = P[t];
}

// ---- 2. multisection, one wave per eigenvalue (ascending index idx)
__global__ __launch_bounds__(256) void bisect_kernel(const double* __restrict__ dg, const double* __restrict__ eg,
                                                     int L, double* __restrict__ lam, double* __restrict__ lam_desc,
                                                     double* __restrict__ sig_desc, double* __restrict__ scal) {
  extern __shared__ double smem[];
  double* d = smem;
  double* ea = smem + L;  // |e|, ea[L-1] = 0
  double* e2 = ea + L;    // e^2
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    d[i] = dg[i];
    const double ei = i + 1 < L ? eg[i] : 0.0;
    ea[i] = fabs(ei);
    e2[i] = ei * ei;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (idx >= L) return;
  // Gershgorin interval
  double gl = __builtin_inf(), gu = -__builtin_inf(), emax2 = 0.0;
  for (int i = lane; i < L; i += 64) {
    const double off = (i > 0 ? ea[i - 1] : 0.0) + ea[i];
    gl = fmin(gl, d[i] - off);
    gu = fmax(gu, d[i] + off);
    emax2 = fmax(emax2, e2[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  // the reduction is accurate to O(u ||T_d||) in absolute terms: bisect to that
  const double atol = EPS * tnorm + 2.0 * pivmin;
  double lo = gl - 2.2e-16 * tnorm - atol, hi = gu + 2.2e-16 * tnorm + atol;
  for (int it = 0; it < 200; ++it) {
    const double width = hi - lo;
    const double tolr = 2.0 * EPS * fmax(fabs(lo), fabs(hi)) + atol;
    if (width <= tolr) break;  // lo, hi are the same in every lane
    const double x = lo + width * (double)(lane + 1) / 65.0;
    const int cnt = sturm_count(d, e2, L, x, pivmin);
    // points with at most idx eigenvalues below them lie left of eigenvalue idx
    const int below = __popcll(__ballot(cnt <= idx));
    const double nlo = lo + width * (double)below / 65.0;
    const double nhi = lo + width * (double)(below + 1) / 65.0;
    lo = below == 0 ? lo : nlo;
    hi = below == 64 ? hi : nhi;
  }
  if (lane == 0) {
    const double lm = 0.5 * (lo + hi);
    lam[idx] = lm;
    lam_desc[L - 1 - idx] = lm;
    sig_desc[L - 1 - idx] = sqrt(fmax(lm, 0.0));
    if (idx == 0) {
      scal[0] = tnorm;
      scal[1] = pivmin;
    }
  }
}

// ---- 3. inverse iteration, one thread per wanted eigenvector r (descending).
// A workgroup of tpb threads keeps d, e and, per thread, the LU factors and
// the iterate in LDS (entry i of array a of thread t at [(a L + i) tpb + t]),
// so the sequential sweeps run at LDS latency.
__global__ __launch_bounds__(64) void inviter_kernel(const double* __restrict__ dg, const double* __restrict__ eg,
                                                     const double* __restrict__ lam, const double* __restrict__ scal,
                                                     int L, int kk, double* __restrict__ Y) {
  extern __shared__ double smem[];
  double* d = smem;
  double* e = smem + L;  // e[L-1] = 0
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    d[i] = dg[i];
    e[i] = eg[i];
  }
  __syncthreads();
  const int tpb = blockDim.x, t = threadIdx.x;
  const int r = blockIdx.x * tpb + t;
  if (r >= kk) return;
  const double tnorm = scal[0], pivmin = scal[1];
  const double ctol = 1e-7 * fmax(tnorm, 1e-300);
  const int ia = L - 1 - r;
  if (r > 0 && fabs(lam[ia + 1] - lam[ia]) <= ctol) return;  // computed by the cluster's first member
  int cend = r;
  while (cend + 1 < kk && fabs(lam[L - 1 - cend] - lam[L - 2 - cend]) <= ctol) ++cend;
  double* base = smem + 2 * L + t;
  const int64_t LT = (int64_t)L * tpb;
  double* dl = base;           // multipliers
  double* u1 = base + LT;      // first super-diagonal of U
  double* u2 = base + 2 * LT;  // second super-diagonal (fill-in)
  double* ru0 = base + 3 * LT; // 1 / diagonal of U
  double* pv = base + 4 * LT;  // pivot flags
  double* y = base + 5 * LT;   // iterate
  const double tiny = EPS * tnorm + pivmin;
  for (int rr = r; rr <= cend; ++rr) {
    // perturb inside a cluster so the shifted matrices differ
    const double lambda = lam[L - 1 - rr] + (double)(rr - r) * 4.0 * EPS * tnorm;
    // LU of T_d - lambda I with partial pivoting (rows i, i+1)
    double diag = d[0] - lambda, sup = L > 1 ? e[0] : 0.0;
    for (int i = 0; i < L - 1; ++i) {
      const double sub = e[i];
      const double nd = d[i + 1] - lambda;
      const double nsup = e[i + 1];
      double mlt, u0v, u1v, u2v, pvv;
      if (fabs(diag) >= fabs(sub)) {  // no swap
        mlt = diag != 0.0 ? sub / diag : 0.0;
        pvv = 0.0;
        u0v = diag;
        u1v = sup;
        u2v = 0.0;
        diag = nd - mlt * sup;
        sup = nsup;
      } else {  // swap rows i and i+1
        mlt = diag / sub;
        pvv = 1.0;
        u0v = sub;
        u1v = nd;
        u2v = nsup;
        diag = sup - mlt * nd;
        sup = -mlt * nsup;
      }
      if (u0v == 0.0) u0v = tiny;
      dl[i * tpb] = mlt;
      pv[i * tpb] = pvv;
      ru0[i * tpb] = 1.0 / u0v;
      u1[i * tpb] = u1v;
      u2[i * tpb] = u2v;
    }
    ru0[(L - 1) * tpb] = 1.0 / (diag != 0.0 ? diag : tiny);
    u1[(L - 1) * tpb] = 0.0;
    u2[(L - 1) * tpb] = 0.0;
    if (L >= 2) u2[(L - 2) * tpb] = 0.0;
    for (int i = 0; i < L; ++i) y[i * tpb] = start_entry(i, rr);
    for (int iter = 0; iter < 3; ++iter) {
      // forward: the row swaps and multipliers, the running entry in a register
      double cur = y[0];
#pragma unroll 4
      for (int i = 0; i < L - 1; ++i) {
        const double nxt = y[(i + 1) * tpb];
        const bool sw = pv[i * tpb] != 0.0;
        const double a = sw ? nxt : cur, b = sw ? cur : nxt;
        y[i * tpb] = a;
        cur = b - dl[i * tpb] * a;
      }
      y[(L - 1) * tpb] = cur;
      // backward substitution with U (three diagonals)
      double y1 = 0.0, y2 = 0.0;
#pragma unroll 4
      for (int i = L - 1; i >= 0; --i) {
        const double s = (y[i * tpb] - u1[i * tpb] * y1 - u2[i * tpb] * y2) * ru0[i * tpb];
        y[i * tpb] = s;
        y2 = y1;
        y1 = s;
      }
      // orthogonalise against the earlier members of the cluster (already in Y)
      for (int q = r; q < rr; ++q) {
        double dot = 0.0;
        for (int i = 0; i < L; ++i) dot = fma(Y[(int64_t)i * kk + q], y[i * tpb], dot);
        for (int i = 0; i < L; ++i) y[i * tpb] -= dot * Y[(int64_t)i * kk + q];
      }
      double nrm = 0.0;
      for (int i = 0; i < L; ++i) nrm = fma(y[i * tpb], y[i * tpb], nrm);
      const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = 0; i < L; ++i) y[i * tpb] *= inv;
    }
    for (int i = 0; i < L; ++i) Y[(int64_t)i * kk + rr] = y[i * tpb];
  }
}

// ---- 4. W[:, c] = H_0 ... H_{L-3} Y[:, c], one wave per eigenvector
template <bool IN_LDS, int NQ>
__global__ __launch_bounds__(64 * BT_WAVES) void backtrans_kernel(const double* __restrict__ gP,
                                                                  const double* __restrict__ taug, int L, int kk,
                                                                  const double* __restrict__ Y,
                                                                  double* __restrict__ W, int ldw) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * BT_WAVES + (threadIdx.x >> 6);
  if (IN_LDS) {
    const int np = L * (L + 1) / 2;
    for (int t = threadIdx.x; t < np; t += blockDim.x) smem[t] = gP[t];
    __syncthreads();
  }
  const double* P = IN_LDS ? smem : gP;
  if (c >= kk) return;
  double y[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    y[q] = i < L ? Y[(int64_t)i * kk + c] : 0.0;
  }
  for (int j = L - 3; j >= 0; --j) {
    const double tj = taug[j];
    if (tj == 0.0) continue;
    const int o = poff(j, L) - j;
    double vv[NQ];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      vv[q] = i == j + 1 ? 1.0 : ((i > j + 1 && i < L) ? P[o + i] : 0.0);
      s = fma(vv[q], y[q], s);
    }
    s = tj * wave_sum64(s);
#pragma unroll
    for (int q = 0; q < NQ; ++q) y[q] -= s * vv[q];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    if (i < L) W[(int64_t)i * ldw + c] = y[q];
  }
}

}  // namespace

size_t syev_small_work(int L, int kk) { return packed_size(L) + 4 * (size_t)L + 8 + (size_t)L * kk + 64; }

hipError_t launch_syev_small(const double* M, int L, int kk, double* work, double* lam_desc, double* sig_desc,
                             double* W, int ldw, size_t max_lds, hipStream_t st) {
  if (L < 1 || L > 1024 || kk < 1 || kk > L || ldw < kk) return hipErrorInvalidValue;
  const EigWork w = eig_layout(work, L, kk);
  const size_t np = (size_t)L * (L + 1) / 2;
  const size_t trd_lds = (32 + 3 * (size_t)L + np) * sizeof(double);
  if (L <= 256 && trd_lds <= max_lds)
    hipLaunchKernelGGL((tridiag_kernel<true, 4>), dim3(1), dim3(TRD_THREADS), trd_lds, st, M, L, w.P, w.d, w.e,
                       w.tau);
  else if ((32 + (3 + (size_t)TRD_WAVES) * L) * sizeof(double) <= max_lds)
    hipLaunchKernelGGL((tridiag_kernel<false, 16, true>), dim3(1), dim3(TRD_THREADS),
                       (32 + (3 + (size_t)TRD_WAVES) * L) * sizeof(double), st, M, L, w.P, w.d, w.e, w.tau);
  else
    hipLaunchKernelGGL((tridiag_kernel<false, 16>), dim3(1), dim3(TRD_THREADS), (32 + 3 * (size_t)L) * sizeof(double),
                       st, M, L, w.P, w.d, w.e, w.tau);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((L + 3) / 4)), dim3(256), 3 * (size_t)L * sizeof(double), st, w.d,
                     w.e, L, w.lam, lam_desc, sig_desc, w.scal);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // threads per inverse-iteration workgroup: as many as fit 6 L doubles each in LDS (at most 64)
  const int64_t tpb_fit = ((int64_t)(max_lds / sizeof(double)) - 2 * L) / (6 * (int64_t)L);
  if (tpb_fit < 1) return hipErrorInvalidValue;
  const int tpb = (int)(tpb_fit < 64 ? tpb_fit : 64);
  hipLaunchKernelGGL(inviter_kernel, dim3((unsigned)((kk + tpb - 1) / tpb)), dim3(tpb),
                     (2 * (size_t)L + 6 * (size_t)L * tpb) * sizeof(double), st, w.d, w.e, w.lam, w.scal, L, kk, w.Y);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 bt_grid((unsigned)((kk + BT_WAVES - 1) / BT_WAVES)), bt_block(64 * BT_WAVES);
  if (L <= 256 && np * sizeof(double) <= max_lds)
    hipLaunchKernelGGL((backtrans_kernel<true, 4>), bt_grid, bt_block, np * sizeof(double), st, w.P, w.tau, L, kk,
                       w.Y, W, ldw);
  else if (L <= 256)
    hipLaunchKernelGGL((backtrans_kernel<false, 4>), bt_grid, bt_block, 0, st, w.P, w.tau, L, kk, w.Y, W, ldw);
  else
    hipLaunchKernelGGL((backtrans_kernel<false, 16>), bt_grid, bt_block, 0, st, w.P, w.tau, L, kk, w.Y, W, ldw);
  return hipGetLastError();
}

}  // namespace rpca
