// Streaming products of the float32 data matrix with tall, skinny blocks on
// gfx950 FP32 matrix cores (v_mfma_f32_16x16x4_f32).  These are the passes
// over A of Steps 1 and 3 (eqs. first_prod .. last_prod and product_t3):
//
//   fwd:  Z = alpha * ((A - 1 s^T) X - 1 corr^T)        m x c   (contraction over n)
//   adj:  P_s = ((A_s - 1 s^T)^T Z_s)^T                 c x n   (contraction over the
//                                                                rows of split s)
//
// s is a per-column shift subtracted in registers before the product (the
// centring of the Introduction, applied without cancellation); corr and
// alpha are the rank-one correction and the positive block scale applied in
// the epilogue.  X is held transposed (Xt, c x n) and the adjoint writes its
// partial sums in the same transposed layout, so one pass's output is the
// next pass's input without a transpose.
//
// MFMA operand layout for 16x16x4 f32 (wave64):
//   A operand: lane = i + 16*kk holds A[i][kk]   (i: M index, kk: K index)
//   B operand: lane = j + 16*kk holds B[kk][j]
//   D:         lane = j + 16*g holds D[4g + v][j] in register v
// The forward kernel gives each lane a float4 along K of its own row, so four
// MFMAs consume one coalesced 16-byte load (the K order inside a 16-wide
// step is permuted identically for A and X, which leaves the sum unchanged).
//
// Accuracy: each float32 accumulation chain is limited to 64 MFMA K-steps and
// then folded into an outer accumulator (float64 in the forward product,
// a second float32 level in the adjoint, whose split partial sums are then
// reduced in float64), so the rounding of long sums (n = 20000 in the
// forward product, thousands of rows per split in the adjoint) grows with
// the square root of the number of folds rather than of the chain length.
//
// Out-of-range rows and columns are clamped to valid addresses instead of
// masked: their lanes compute values that the epilogue never stores, which
// keeps the main loops free of branches.  Only the K (or row) tail shorter
// than one register stage uses masked loads.
#include "common.h"
#include "kernels.h"

namespace rpca {

// unconditional 4-float load (vector when the address is 16-byte aligned)
template <bool VEC>
RPCA_DEV floatx4 ld4(const float* __restrict__ p) {
  if (VEC) return *reinterpret_cast<const floatx4*>(p);
  return floatx4{p[0], p[1], p[2], p[3]};
}

// p[k..k+3] with entries at or beyond n read as zero
RPCA_DEV floatx4 ld4_masked(const float* __restrict__ p, int64_t k, int64_t n) {
  floatx4 v = {0.f, 0.f, 0.f, 0.f};
  if (k < n) v.x = p[k];
  if (k + 1 < n) v.y = p[k + 1];
  if (k + 2 < n) v.z = p[k + 2];
  if (k + 3 < n) v.w = p[k + 3];
  return v;
}

RPCA_DEV floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// forward: each wave owns 16 rows x (16*NT) output columns; 4 waves per block.
// shift is always a valid n-vector (zeros when not centring).
// K is walked in steps of 16 (one float4 per lane), STAGE steps per register
// stage, with the next stage's loads issued before the current MFMAs.
// ---------------------------------------------------------------------------
template <int NT, bool VEC, int STAGE>
__global__ __launch_bounds__(256, 2) void fwd_f32_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const float* __restrict__ Xt, int64_t ldx, int ncols, const float* __restrict__ corr,
    const double* __restrict__ alpha_ptr, float* __restrict__ Z, int64_t ldz) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int ii = lane & 15;
  const int kk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int c0 = blockIdx.y * (16 * NT);
  const int64_t row = r0 + ii;
  const float* __restrict__ arow = A + (row < m ? row : m - 1) * lda;
  const float* __restrict__ xrow[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = c0 + 16 * t + ii;
    xrow[t] = Xt + (int64_t)(c < ncols ? c : ncols - 1) * ldx;
  }

  floatx4 acc[NT];
  double accd[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) accd[t][v] = 0.0;
  }
  auto fold = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[t][v] += (double)acc[t][v];
      acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto mma = [&](const floatx4& a, const floatx4 (&x)[NT]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma4(a[e], x[t][e], acc[t]);
    }
  };

  // main part: whole stages, unconditional loads, two register buffers
  // (the loads of one stage are in flight while the other stage's MFMAs run)
  constexpr int KS = 16 * STAGE;
  constexpr int FOLD = 8 / STAGE > 0 ? 8 / STAGE : 1;  // fold every ~64 MFMA K-steps
  const int64_t nmain = (n / (2 * KS)) * (2 * KS);
  const int koff = 4 * kk;
  struct Stage {
    floatx4 a[STAGE], s[STAGE], x[STAGE][NT];
  };
  auto load_stage = [&](Stage& b, int64_t kb) {
#pragma unroll
    for (int q = 0; q < STAGE; ++q) {
      const int64_t k = kb + 16 * q + koff;
      b.a[q] = ld4<VEC>(arow + k);
      b.s[q] = ld4<true>(shift + k);
#pragma unroll
      for (int t = 0; t < NT; ++t) b.x[q][t] = ld4<true>(xrow[t] + k);
    }
  };
  int it = 0;
  auto run_stage = [&](const Stage& b) {
#pragma unroll
    for (int q = 0; q < STAGE; ++q) mma(b.a[q] - b.s[q], b.x[q]);
    if (++it == 2 * FOLD) {
      it = 0;
      fold();
    }
  };
  // The loop body is straight-line (every load unconditional; the prefetch
  // after the last pair re-reads the current stage), so the wait counters
  // only ever wait for the stage about to be consumed.
  if (nmain > 0) {
    Stage b0, b1;
    load_stage(b0, 0);
    for (int64_t kb = 0; kb < nmain; kb += 2 * KS) {
      load_stage(b1, kb + KS);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      run_stage(b0);
      load_stage(b0, kb + 2 * KS < nmain ? kb + 2 * KS : kb);
      __builtin_amdgcn_sched_barrier(0);
      run_stage(b1);
    }
  }
  // tail: fewer than 2 KS columns, masked loads one 16-wide step at a time
  for (int64_t kb = nmain; kb < n; kb += 16) {
    const int64_t k = kb + koff;
    const floatx4 a = ld4_masked(arow, k, n) - ld4_masked(shift, k, n);
    floatx4 x[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) x[t] = ld4_masked(xrow[t], k, n);
    mma(a, x);
  }
  fold();

  const double alpha = alpha_ptr != nullptr ? *alpha_ptr : 1.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = c0 + 16 * t + ii;
    if (c >= ncols) continue;
    const double cr = corr != nullptr ? (double)corr[c] : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + 4 * kk + v;
      if (r < m) Z[r * ldz + c] = (float)(alpha * (accd[t][v] - cr));
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint: each wave owns 64 columns of A (a float4 per lane, 4 M-tiles) and
// 16*NT columns of Z; 4 waves per block cover 256 columns of A.  Rows of the
// split are walked 4 at a time.  Blocks are remapped so that consecutive
// logical blocks (same rows, neighbouring column tiles / Z tiles) share an
// XCD and therefore its L2.
// VEC: A 16-byte aligned, lda % 4 == 0 and n % 4 == 0 (every lane's float4 is
// either wholly inside the row or wholly past its end).
// ---------------------------------------------------------------------------
RPCA_DEV int64_t xcd_remap(int64_t b, int64_t total) {
  const int64_t q = total / 8, r = total % 8;
  const int64_t x = b % 8, local = b / 8;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

template <int NT, bool VEC, int STAGE>
__global__ __launch_bounds__(256, 2) void adj_f32_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const float* __restrict__ Z, int64_t ldz, int ncols, int64_t rows_per_split, int nsplit,
    int jtiles, int ctiles, float* __restrict__ P, int64_t ldp, int64_t split_stride) {
  const int64_t total = (int64_t)jtiles * ctiles * nsplit;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int jt = (int)(logical % jtiles);
  const int64_t rest = logical / jtiles;
  const int ct = (int)(rest % ctiles);
  const int sp = (int)(rest / ctiles);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int p = lane & 15;
  const int kk = lane >> 4;
  const int64_t c0 = (int64_t)ct * 256 + wave * 64;
  const int64_t cl = c0 + 4 * p;
  const int64_t clc = cl < n ? cl : 0;  // clamped column for the unmasked path
  const int j0 = jt * 16 * NT;
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;

  int zc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = j0 + 16 * t + p;
    zc[t] = c < ncols ? c : ncols - 1;
  }
  const floatx4 sh = VEC ? ld4<true>(shift + clc) : ld4_masked(shift, cl, n);

  // two float32 levels: acc takes 64 MFMA K-steps (256 rows), then is added
  // into acc2; the split partial sums are reduced in float64 afterwards
  floatx4 acc[4][NT], acc2[4][NT];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc2[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  auto fold = [&]() {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc2[v][t] += acc[v][t];
        acc[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
  };
  auto mma = [&](const floatx4& a, const float (&z)[NT]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[v][t] = mfma4(a[v], z[t], acc[v][t]);
    }
  };
  auto load_row = [&](int64_t r, floatx4& a, float (&z)[NT]) {
    const float* arow = A + r * lda;
    a = VEC ? ld4<true>(arow + clc) : ld4_masked(arow, cl, n);
#pragma unroll
    for (int t = 0; t < NT; ++t) z[t] = Z[r * ldz + zc[t]];
  };

  constexpr int RS = 4 * STAGE;
  constexpr int FOLD = 64 / STAGE;  // fold every ~64 MFMA K-steps (~256 rows)
  const int64_t nmain = rbeg + ((rend - rbeg) / (2 * RS)) * (2 * RS);
  struct Stage {
    floatx4 a[STAGE];
    float z[STAGE][NT];
  };
  auto load_stage = [&](Stage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < STAGE; ++q) load_row(rb + 4 * q + kk, b.a[q], b.z[q]);
  };
  int it = 0;
  auto run_stage = [&](const Stage& b) {
#pragma unroll
    for (int q = 0; q < STAGE; ++q) mma(b.a[q] - sh, b.z[q]);
    if (++it == FOLD) {
      it = 0;
      fold();
    }
  };
  // straight-line body as in the forward kernel
  if (nmain > rbeg) {
    Stage b0, b1;
    load_stage(b0, rbeg);
    for (int64_t rb = rbeg; rb < nmain; rb += 2 * RS) {
      load_stage(b1, rb + RS);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      run_stage(b0);
      load_stage(b0, rb + 2 * RS < nmain ? rb + 2 * RS : rb);
      __builtin_amdgcn_sched_barrier(0);
      run_stage(b1);
    }
  }
  // tail rows: fewer than 2 RS, masked by row
  for (int64_t rb = nmain; rb < rend; rb += 4) {
    const int64_t r = rb + kk;
    floatx4 a = {0.f, 0.f, 0.f, 0.f};
    float z[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) z[t] = 0.f;
    if (r < rend) {
      load_row(r, a, z);
      a -= sh;
    }
    mma(a, z);
  }
  fold();

  float* __restrict__ Ps = P + (int64_t)sp * split_stride;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + 16 * t + p;
    if (j >= ncols) continue;
    float* __restrict__ prow = Ps + (int64_t)j * ldp;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int64_t c = c0 + 16 * kk + 4 * w;
      const floatx4 o = floatx4{acc2[0][t][w], acc2[1][t][w], acc2[2][t][w], acc2[3][t][w]};
      if (c + 3 < n) {
        *reinterpret_cast<floatx4*>(prow + c) = o;
      } else {
        if (c < n) prow[c] = o.x;
        if (c + 1 < n) prow[c + 1] = o.y;
        if (c + 2 < n) prow[c + 2] = o.z;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int NT>
static hipError_t launch_fwd_nt(const FwdArgs& a, hipStream_t st) {
  dim3 grid((unsigned)((a.m + 63) / 64), (unsigned)((a.ncols + 16 * NT - 1) / (16 * NT)));
  if (a.vec)
    hipLaunchKernelGGL((fwd_f32_kernel<NT, true, 3>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                       a.shift, a.Xt, a.ldx, a.ncols, a.corr, a.alpha, a.Z, a.ldz);
  else
    hipLaunchKernelGGL((fwd_f32_kernel<NT, false, 3>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                       a.shift, a.Xt, a.ldx, a.ncols, a.corr, a.alpha, a.Z, a.ldz);
  return hipGetLastError();
}

hipError_t launch_fwd_f32(const FwdArgs& a, hipStream_t st) {
  if (a.m <= 0 || a.ncols <= 0) return hipSuccess;
  if (a.A == nullptr || a.shift == nullptr || a.Xt == nullptr || a.Z == nullptr) return hipErrorInvalidValue;
  if (a.ldx < a.n || a.lda < a.n) return hipErrorInvalidValue;
  const int tiles = (a.ncols + 15) / 16;
  if (tiles <= 1) return launch_fwd_nt<1>(a, st);
  if (tiles <= 2) return launch_fwd_nt<2>(a, st);
  if (tiles <= 3) return launch_fwd_nt<3>(a, st);
  return launch_fwd_nt<4>(a, st);
}

// rows / 4 per register stage of the adjoint kernel (two stages are in flight)
constexpr int ADJ_STAGE = 3;

int adj_nt_for(int ncols) {
  const int tiles = (ncols + 15) / 16;
  return tiles <= 1 ? 1 : tiles <= 2 ? 2 : tiles <= 3 ? 3 : 4;
}

template <int NT>
static hipError_t launch_adj_nt(const AdjArgs& a, hipStream_t st) {
  const int jtiles = (a.ncols + 16 * NT - 1) / (16 * NT);
  const int ctiles = (int)((a.n + 255) / 256);
  const int64_t total = (int64_t)jtiles * ctiles * a.nsplit;
  dim3 grid((unsigned)total);
  const bool vec = a.vec && (a.n % 4 == 0);
  if (vec)
    hipLaunchKernelGGL((adj_f32_kernel<NT, true, ADJ_STAGE>), grid, dim3(256), 0, st, (const float*)a.A, a.lda,
                       a.m, a.n, a.shift, a.Z, a.ldz, a.ncols, a.rows_per_split, a.nsplit, jtiles, ctiles, a.P,
                       a.ldp, a.split_stride);
  else
    hipLaunchKernelGGL((adj_f32_kernel<NT, false, ADJ_STAGE>), grid, dim3(256), 0, st, (const float*)a.A, a.lda,
                       a.m, a.n, a.shift, a.Z, a.ldz, a.ncols, a.rows_per_split, a.nsplit, jtiles, ctiles, a.P,
                       a.ldp, a.split_stride);
  return hipGetLastError();
}

hipError_t launch_adj_f32(const AdjArgs& a, hipStream_t st) {
  if (a.n <= 0 || a.ncols <= 0 || a.nsplit <= 0) return hipSuccess;
  if (a.A == nullptr || a.shift == nullptr || a.Z == nullptr || a.P == nullptr) return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldp < a.n || a.rows_per_split % 4 != 0) return hipErrorInvalidValue;
  if ((int64_t)a.nsplit * a.rows_per_split < a.m) return hipErrorInvalidValue;
  switch (adj_nt_for(a.ncols)) {
    case 1: return launch_adj_nt<1>(a, st);
    case 2: return launch_adj_nt<2>(a, st);
    case 3: return launch_adj_nt<3>(a, st);
    default: return launch_adj_nt<4>(a, st);
  }
}

}  // namespace rpca
