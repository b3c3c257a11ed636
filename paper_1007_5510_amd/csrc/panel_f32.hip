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
// MFMA operand layout for 16x16x4 f32 (wave64, adjoint kernel):
//   A operand: lane = i + 16*kk holds A[i][kk]   (i: M index, kk: K index)
//   B operand: lane = j + 16*kk holds B[kk][j]
//   D:         lane = j + 16*g holds D[4g + v][j] in register v
// Both kernels give each lane a float4 of A, so four MFMAs consume one
// 16-byte load; in the forward product the float4 runs along K and the K
// order inside a step is permuted identically for A and X, which leaves the
// sum unchanged.
//
// Accuracy: the long sums are split (over K in the forward product, over
// rows in the adjoint) and the split partial sums reduced in float64.  In the
// forward product each float32 chain is limited to 64 MFMA K-steps and folded
// into a second float32 level (a float outer level keeps the one-tile kernel
// within 128 registers, four workgroups per CU); the adjoint keeps one float32 chain
// per split (a few thousand rows), which frees the registers of a second
// level and measured about 5% faster.
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
// forward (v_mfma_f32_32x32x2_f32): each wave owns 32 rows x
// (32*NT2) columns, a block of 4 waves 128 rows.  X and the shift are staged
// once per block in LDS (32 columns of K per stage, double buffered, rows
// padded to 36 floats so the 32 lanes of a ds_read_b128 hit distinct banks);
// A goes straight to registers, one float4 along K per lane, two register
// stages in flight.  The K range is split over blockIdx.y so that the grid
// has enough blocks to fill every CU evenly; the split partial sums go to a
// buffer reduced in float64 by fwd_reduce_kernel (or straight to Z with the
// epilogue when there is a single split).
//   A operand: lane = i + 32*kk holds A[i][kk]; B operand: lane = j + 32*kk
//   holds B[kk][j]; D: lane l, register v holds D[8(v/4) + 4(l/32) + v%4][l%32].
// ---------------------------------------------------------------------------
RPCA_DEV floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

constexpr int F3_KST = 32;  // K per LDS stage of the launched configuration
// launched forward configurations, three workgroups per CU: two 32-column tiles
// with 32 K per stage (158 registers, no spills; 2.8% faster than four workgroups
// per CU at 128 registers with 19 spilled), one tile with 64 K per stage (161
// registers: twice the bytes of A in flight per wave for the narrow, read-bound
// products; 2-3% faster than 32 K at four workgroups per CU).  K chunks of the
// split are multiples of 64 so that every stage of either is whole.
template <int NT2>
constexpr int FWD32_MINB = 3;
template <int NT2>
constexpr int FWD32_KST = NT2 == 1 ? 64 : 32;
constexpr int F3_KCHUNK = 64;

// KST: K per LDS stage (32 or 64); NCH: independent accumulation chains per
// output tile (consecutive MFMAs of one tile alternate between them); OT:
// type of the outer accumulator (double, or float for fewer registers);
// MINB: workgroups per CU the register budget is sized for
template <int NT2, bool VEC, int KST = F3_KST, int NCH = 1, class OT = float, int MINB = 4>
__global__ __launch_bounds__(256, MINB) void fwd32_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const float* __restrict__ Xt, int64_t ldx, int ncols, int64_t kchunk, const float* __restrict__ corr,
    const double* __restrict__ alpha_ptr, float* __restrict__ Z, int64_t ldz, int64_t split_stride, int direct) {
  constexpr int XP = KST + 4;   // padded LDS row (floats)
  constexpr int XV = KST / 16;  // float4 of X per thread per stage
  constexpr int SV = KST / 4;   // float4 of the shift per stage
  __shared__ float Xs[2][64][XP];
  // shift of the stage: entries [0, KST) are read; every thread stores one entry of
  // its own (threads past KST store duplicates) so the store needs no branch
  __shared__ __attribute__((aligned(16))) float Ss[2][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, kh = lane >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const int sk = blockIdx.y;
  const int c0 = blockIdx.z * 64;
  const int64_t kbeg = (int64_t)sk * kchunk;
  const int64_t kend = kbeg + kchunk < n ? kbeg + kchunk : n;
  const int64_t row = r0 + li;
  const float* __restrict__ arow = A + (row < m ? row : m - 1) * lda;
  // cooperative stage loader: thread -> (X row xc, KST/4-float slice xq)
  const int xc = tid >> 2, xq = tid & 3;
  const float* __restrict__ xsrc = Xt + (int64_t)(c0 + xc < ncols ? c0 + xc : ncols - 1) * ldx;

  floatx16 acc[NCH][NT2];
  OT accd[NT2][16];
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) acc[ch][t][v] = 0.f;
      accd[t][v] = (OT)0;
    }
  }
  auto fold = [&]() {
#pragma unroll
    for (int t = 0; t < NT2; ++t) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          accd[t][v] += (OT)acc[ch][t][v];
          acc[ch][t][v] = 0.f;
        }
      }
    }
  };
  struct AStage {
    floatx4 a[KST / 8];
  };
  struct XStage {
    floatx4 x[XV];
    float s;
  };
  auto load_a = [&](AStage& b, int64_t kb) {
#pragma unroll
    for (int q = 0; q < KST / 8; ++q) b.a[q] = ld4<VEC>(arow + kb + 8 * q + 4 * kh);
  };
  auto load_x = [&](XStage& b, int64_t kb) {
#pragma unroll
    for (int v = 0; v < XV; ++v) b.x[v] = ld4<true>(xsrc + kb + (KST / 4) * xq + 4 * v);
    b.s = shift[kb + (tid & (KST - 1))];
  };
  auto store_x = [&](const XStage& b, int buf) {
#pragma unroll
    for (int v = 0; v < XV; ++v) *reinterpret_cast<floatx4*>(&Xs[buf][xc][(KST / 4) * xq + 4 * v]) = b.x[v];
    Ss[buf][tid] = b.s;
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int q = 0; q < KST / 8; ++q) {
      const floatx4 sv = *reinterpret_cast<const floatx4*>(&Ss[buf][8 * q + 4 * kh]);
      const floatx4 a = b.a[q] - sv;
      floatx4 x[NT2];
#pragma unroll
      for (int t = 0; t < NT2; ++t) x[t] = *reinterpret_cast<const floatx4*>(&Xs[buf][32 * t + li][8 * q + 4 * kh]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int t = 0; t < NT2; ++t) acc[e % NCH][t] = mfma32(a[e], x[t][e], acc[e % NCH][t]);
      }
    }
  };

  // whole stages on two register stages of A used alternately (no copy between
  // them, so a load has the whole next stage to arrive; the X loads of a stage
  // are issued before its A loads, so storing X waits for X only).  The
  // prologue's loads are waited for before the loop, so the loop header carries
  // no wait on loads issued inside the loop; past the last whole stage the
  // prefetch re-reads it.
  const int64_t nfull = (kend - kbeg) / KST;
  int it = 0;
  auto step_done = [&]() {
    if (++it == 128 / KST) {  // fold every 64 MFMA K-steps
      it = 0;
      fold();
    }
  };
  if (nfull > 0) {
    AStage a0, a1;
    XStage xr;
    load_x(xr, kbeg);
    load_a(a0, kbeg);
    store_x(xr, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int64_t st = 0;
    for (; st + 2 <= nfull; st += 2) {
      const int64_t k1 = kbeg + (st + 1) * KST;
      load_x(xr, k1);
      load_a(a1, k1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, 0);
      store_x(xr, 1);
      __syncthreads();
      step_done();
      const int64_t k2 = kbeg + (st + 2 < nfull ? st + 2 : st + 1) * KST;
      load_x(xr, k2);
      load_a(a0, k2);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, 1);
      store_x(xr, 0);
      __syncthreads();
      step_done();
    }
    if (st < nfull) {  // odd stage count: the last stage is in a0, X in buffer 0
      compute(a0, 0);
      __syncthreads();
      step_done();
    }
  }
  // tail stage (fewer than KST columns left): masked loads
  const int64_t kt = kbeg + nfull * KST;
  if (kt < kend) {
    AStage at;
#pragma unroll
    for (int q = 0; q < KST / 8; ++q) at.a[q] = ld4_masked(arow, kt + 8 * q + 4 * kh, kend);
    const int buf = (int)(nfull & 1);
#pragma unroll
    for (int v = 0; v < XV; ++v)
      *reinterpret_cast<floatx4*>(&Xs[buf][xc][(KST / 4) * xq + 4 * v]) =
          ld4_masked(xsrc, kt + (KST / 4) * xq + 4 * v, kend);
    const floatx4 sv = ld4_masked(shift, kt + 4 * (tid & (SV - 1)), kend);
    if (tid < SV) *reinterpret_cast<floatx4*>(&Ss[buf][4 * tid]) = sv;
    __syncthreads();
    compute(at, buf);
  }
  fold();

  const double alpha = (direct && alpha_ptr != nullptr) ? *alpha_ptr : 1.0;
  float* __restrict__ Zs = Z + (direct ? 0 : (int64_t)sk * split_stride);
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
    const int c = c0 + 32 * t + li;
    if (c >= ncols) continue;
    const double cr = (direct && corr != nullptr) ? (double)corr[c] : 0.0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t r = r0 + 8 * (v >> 2) + 4 * kh + (v & 3);
      if (r < m) Zs[r * ldz + c] = direct ? (float)(alpha * (accd[t][v] - cr)) : (float)accd[t][v];
    }
  }
}

// Z[r][c] = alpha (sum_s P[s][r][c] - corr[c]) in float64, s in split order
__global__ __launch_bounds__(256) void fwd_reduce_kernel(const float* __restrict__ P, int nsplit,
                                                         int64_t split_stride, int64_t ldp, int64_t m, int ncols,
                                                         const float* __restrict__ corr,
                                                         const double* __restrict__ alpha_ptr,
                                                         float* __restrict__ Z, int64_t ldz) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * ncols) return;
  const int64_t r = e / ncols;
  const int c = (int)(e % ncols);
  double v = 0.0;
  v += sum_strided(P + r * ldp + c, nsplit, split_stride);
  const double alpha = alpha_ptr != nullptr ? *alpha_ptr : 1.0;
  const double cr = corr != nullptr ? (double)corr[c] : 0.0;
  Z[r * ldz + c] = (float)(alpha * (v - cr));
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

constexpr int ADJ_RS = 16;  // rows of A per LDS stage of the launched configuration
constexpr int64_t ADJ_MAX_CHAIN = 8192;  // longest float32 accumulation chain (rows of one split)

// RS: rows of A per LDS stage (16 or 32); MINB: workgroups per CU the
// register budget is sized for; FOLD2: second float32 accumulation level
template <int NT, bool VEC, int RS = ADJ_RS, int MINB = 2, bool FOLD2 = false>
__global__ __launch_bounds__(256, MINB) void adj_f32_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const float* __restrict__ Z, int64_t ldz, int ncols, int64_t rows_per_split, int nsplit,
    int jtiles, int ctiles, float* __restrict__ P, int64_t ldp, int64_t split_stride, int ones) {
  // Z rows staged per block, interleaved so that lane (p, kk) finds its NT
  // B-operand values (columns p, 16+p, 32+p, 48+p) in one 16-byte word.
  constexpr int ZQ = RS / 4;  // Z elements per thread per stage
  __shared__ float Zs[2][RS][16][4];
  const int64_t total = (int64_t)jtiles * ctiles * nsplit;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int jt = (int)(logical % jtiles);
  const int64_t rest = logical / jtiles;
  const int ct = (int)(rest % ctiles);
  const int sp = (int)(rest / ctiles);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int p = lane & 15;
  const int kk = lane >> 4;
  const int64_t c0 = (int64_t)ct * 256 + wave * 64;
  const int64_t cl = c0 + 4 * p;
  const int64_t clc = cl < n ? cl : 0;  // clamped column for the unmasked path
  const int j0 = jt * 64;
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  const floatx4 sh = VEC ? ld4<true>(shift + clc) : ld4_masked(shift, cl, n);
  // cooperative Z loader: ZQ elements per thread per stage, element e = tid + 256 q
  // -> row e / 64, column e % 64 (clamped to the last real column)
  // with `ones`, column ncols of Z is an implicit column of ones (its product is the column sums)
  int zcol[ZQ], zrow[ZQ], zslot[ZQ];
  bool zone[ZQ];
#pragma unroll
  for (int q = 0; q < ZQ; ++q) {
    const int e = tid + 256 * q;
    const int cc = e & 63;
    zrow[q] = e >> 6;
    zcol[q] = j0 + cc < ncols ? j0 + cc : ncols - 1;
    zone[q] = ones && j0 + cc == ncols;
    zslot[q] = (cc & 15) * 4 + (cc >> 4);  // [p][t] with column 16 t + p
  }

  floatx4 acc[4][NT], acc2[4][FOLD2 ? NT : 1];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (FOLD2) acc2[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  auto fold = [&]() {
    if (!FOLD2) return;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc2[v][t] += acc[v][t];
        acc[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
  };
  struct AStage {
    floatx4 a[RS / 4];
  };
  struct ZStage {
    float z[ZQ];
  };
  auto load_a = [&](AStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const float* arow = A + (rb + 4 * q + kk) * lda;
      b.a[q] = VEC ? ld4<true>(arow + clc) : ld4_masked(arow, cl, n);
    }
  };
  // unconditional load (zcol is clamped, so the address is valid); the ones
  // column is substituted when the stage is stored to LDS, after the compute,
  // so that nothing waits on these loads before then
  auto load_z = [&](ZStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < ZQ; ++q) b.z[q] = Z[(rb + zrow[q]) * ldz + zcol[q]];
  };
  auto store_z = [&](const ZStage& b, int buf) {
    float* base = &Zs[buf][0][0][0];
#pragma unroll
    for (int q = 0; q < ZQ; ++q) base[zrow[q] * 64 + zslot[q]] = zone[q] ? 1.f : b.z[q];
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const floatx4 zz = *reinterpret_cast<const floatx4*>(&Zs[buf][4 * q + kk][p][0]);
      const floatx4 a = b.a[q] - sh;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[v][t] = mfma4(a[v], zz[t], acc[v][t]);
      }
    }
  };

  // Two register stages used alternately (no copy between them): stage st
  // computes from one while the loads of stage st + 1 land in the other, so a
  // load has a whole stage to arrive before its first use.  The prologue's
  // loads are waited for before the loop, so the loop header carries no wait
  // on loads issued inside the loop.
  const int64_t nfull = (rend - rbeg) / RS;
  int it = 0;
  auto step_done = [&]() {
    if (++it == 256 / RS) {  // fold every 64 MFMA K-steps (256 rows)
      it = 0;
      fold();
    }
  };
  if (nfull > 0) {
    AStage a0, a1;
    ZStage zr;
    load_z(zr, rbeg);
    load_a(a0, rbeg);
    store_z(zr, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int64_t st = 0;
    for (; st + 2 <= nfull; st += 2) {
      const int64_t r1 = rbeg + (st + 1) * RS;
      load_z(zr, r1);
      load_a(a1, r1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, 0);
      store_z(zr, 1);
      __syncthreads();
      step_done();
      // past the last whole stage the prefetch re-reads stage st + 1
      const int64_t r2 = rbeg + (st + 2 < nfull ? st + 2 : st + 1) * RS;
      load_z(zr, r2);
      load_a(a0, r2);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, 1);
      store_z(zr, 0);
      __syncthreads();
      step_done();
    }
    if (st < nfull) {  // odd stage count: the last stage is in a0, Z in buffer 0
      compute(a0, 0);
      __syncthreads();
      step_done();
    }
  }
  // tail rows (fewer than a stage): masked by row, zeros beyond rend
  const int64_t rt = rbeg + nfull * RS;
  if (rt < rend) {
    const int buf = (int)(nfull & 1);
    float* base = &Zs[buf][0][0][0];
#pragma unroll
    for (int q = 0; q < ZQ; ++q) {
      const int64_t r = rt + zrow[q];
      base[zrow[q] * 64 + zslot[q]] = r < rend ? (zone[q] ? 1.f : Z[r * ldz + zcol[q]]) : 0.f;
    }
    AStage at;
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const int64_t r = rt + 4 * q + kk;
      at.a[q] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (r < rend) {
        const float* arow = A + r * lda;
        at.a[q] = VEC ? ld4<true>(arow + clc) : ld4_masked(arow, cl, n);
      } else {
        at.a[q] = sh;  // (a - sh) = 0 for rows past the end
      }
    }
    __syncthreads();
    compute(at, buf);
  }
  fold();

  float* __restrict__ Ps = P + (int64_t)sp * split_stride;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + 16 * t + p;
    if (j > ncols || (j == ncols && !ones)) continue;
    float* __restrict__ prow = Ps + (int64_t)j * ldp;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int64_t c = c0 + 16 * kk + 4 * w;
      const floatx4 o = FOLD2 ? floatx4{acc2[0][t][w], acc2[1][t][w], acc2[2][t][w], acc2[3][t][w]}
                              : floatx4{acc[0][t][w], acc[1][t][w], acc[2][t][w], acc[3][t][w]};
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
// adjoint for a wide Z (the T pass): each wave owns 32 columns of A (a float2
// per lane feeds two M tiles) x 16 NT columns of Z (NT = 8 or 12 tiles), so
// one read of A serves every Z column of the block instead of one read per 64;
// 4 waves per block cover 128 columns of A.  The Z rows of a stage are staged
// in LDS as [row][p][t] (column 16 t + p), NT / 4 16-byte reads per lane per
// K step.  Each output is accumulated over the same rows in the same MFMA K
// grouping as adj_f32_kernel, so the two kernels give identical sums.  Lane
// (p, kk) ends with the A columns c0 + 8 kk .. + 7 of its Z column, written as
// two 16-byte vectors.
// VEC: A 8-byte aligned, lda and n even.  Z is read in 16-byte pieces: Z
// 16-byte aligned, ldz and ncols multiples of 4.
// ---------------------------------------------------------------------------
typedef float adjw_f2 __attribute__((ext_vector_type(2)));
constexpr int ADJW_ACOLS = 128;  // A columns per block

// Z tiles per block of the wide-Z adjoint for ncols columns (host side: launcher and split rule)
static inline int adjw_tiles(int ncols) { return ncols <= 96 ? 6 : (ncols <= 128 ? 8 : 12); }

template <int NT, bool VEC>
__global__ __launch_bounds__(256, 2) void adj_wide_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const float* __restrict__ Z, int64_t ldz, int ncols, int64_t rows_per_split, int nsplit, int jtiles,
    int ctiles, float* __restrict__ P, int64_t ldp, int64_t split_stride) {
  constexpr int RS = ADJ_RS;
  constexpr int ZCOLS = 16 * NT;            // Z columns per block
  constexpr int PW = NT % 4 == 0 ? 4 : 2;   // columns per Z piece (16 or 8 bytes)
  constexpr int ZH = NT / PW;               // Z pieces per thread per stage (16 threads per row)
  typedef float zpiece_t __attribute__((ext_vector_type(PW)));
  static_assert(NT % 2 == 0, "Z pieces of 2 or 4 columns");
  __shared__ __attribute__((aligned(16))) float Zs[2][RS][16][NT];
  const int64_t total = (int64_t)jtiles * ctiles * nsplit;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int jt = (int)(logical % jtiles);
  const int64_t rest = logical / jtiles;
  const int ct = (int)(rest % ctiles);
  const int sp = (int)(rest / ctiles);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int p = lane & 15;
  const int kk = lane >> 4;
  const int64_t c0 = (int64_t)ct * ADJW_ACOLS + wave * 32;
  const int64_t cl = c0 + 2 * p;
  const int64_t clc = cl < n ? cl : 0;  // clamped column for the unmasked path
  const int j0 = jt * ZCOLS;
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  auto ld2 = [&](const float* __restrict__ row) -> adjw_f2 {
    if (VEC) return *reinterpret_cast<const adjw_f2*>(row + clc);
    adjw_f2 v = {0.f, 0.f};
    if (cl < n) v.x = row[cl];
    if (cl + 1 < n) v.y = row[cl + 1];
    return v;
  };
  const adjw_f2 sh = ld2(shift);
  // cooperative Z loader: thread -> row zr of the stage, ZH PW-column pieces at columns
  // PW (ZH (tid % 16) + h); a piece past the last real column re-reads the last piece (its
  // products land in columns that are never stored; ncols is a multiple of 4, so no piece
  // straddles it).  Element cc of the stage row goes to LDS slot [zr][cc % 16][cc / 16].
  const int zr = tid >> 4;
  int zcol[ZH], zslot[ZH];
#pragma unroll
  for (int h = 0; h < ZH; ++h) {
    const int cc = PW * (ZH * (tid & 15) + h);
    zcol[h] = j0 + cc + PW <= ncols ? j0 + cc : ncols - PW;
    zslot[h] = zr * (16 * NT) + (cc & 15) * NT + (cc >> 4);
  }

  floatx4 acc[2][NT];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  struct AStage {
    adjw_f2 a[RS / 4];
  };
  struct ZStage {
    zpiece_t z[ZH];
  };
  auto load_a = [&](AStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) b.a[q] = ld2(A + (rb + 4 * q + kk) * lda);
  };
  auto load_z = [&](ZStage& b, int64_t rb) {
    const float* zrow = Z + (rb + zr) * ldz;
#pragma unroll
    for (int h = 0; h < ZH; ++h) b.z[h] = *reinterpret_cast<const zpiece_t*>(zrow + zcol[h]);
  };
  // columns cc .. cc + PW - 1 of a piece share the tile cc / 16 and take slots p = cc % 16 ..
  auto store_z = [&](const ZStage& b, int buf) {
    float* base = &Zs[buf][0][0][0];
#pragma unroll
    for (int h = 0; h < ZH; ++h)
#pragma unroll
      for (int e = 0; e < PW; ++e) base[zslot[h] + e * NT] = b.z[h][e];
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const zpiece_t* zp = reinterpret_cast<const zpiece_t*>(&Zs[buf][4 * q + kk][p][0]);
      zpiece_t z[ZH];
#pragma unroll
      for (int h = 0; h < ZH; ++h) z[h] = zp[h];
      const adjw_f2 a = b.a[q] - sh;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[v][t] = mfma4(a[v], z[t / PW][t % PW], acc[v][t]);
      }
    }
  };

  // two register stages used alternately, prologue drained (as in adj_f32_kernel)
  const int64_t nfull = (rend - rbeg) / RS;
  if (nfull > 0) {
    AStage a0, a1;
    ZStage zr;
    load_z(zr, rbeg);
    load_a(a0, rbeg);
    store_z(zr, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int64_t st = 0;
    for (; st + 2 <= nfull; st += 2) {
      const int64_t r1 = rbeg + (st + 1) * RS;
      load_z(zr, r1);
      load_a(a1, r1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, 0);
      store_z(zr, 1);
      __syncthreads();
      // past the last whole stage the prefetch re-reads stage st + 1
      const int64_t r2 = rbeg + (st + 2 < nfull ? st + 2 : st + 1) * RS;
      load_z(zr, r2);
      load_a(a0, r2);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, 1);
      store_z(zr, 0);
      __syncthreads();
    }
    if (st < nfull) {  // odd stage count: the last stage is in a0, Z in buffer 0
      compute(a0, 0);
      __syncthreads();
    }
  }
  // tail rows (fewer than a stage): Z zero past rend, A read as the shift there
  const int64_t rt = rbeg + nfull * RS;
  if (rt < rend) {
    const int buf = (int)(nfull & 1);
    ZStage zt;
    if (rt + zr < rend) {
      load_z(zt, rt);
    } else {
#pragma unroll
      for (int h = 0; h < ZH; ++h) zt.z[h] = zpiece_t(0.f);
    }
    store_z(zt, buf);
    AStage at;
#pragma unroll
    for (int q = 0; q < RS / 4; ++q) {
      const int64_t r = rt + 4 * q + kk;
      at.a[q] = r < rend ? ld2(A + r * lda) : sh;
    }
    __syncthreads();
    compute(at, buf);
  }

  // D of tile (v, t): lane (p, kk) register w holds A column c0 + 2 (4 kk + w) + v, Z column
  // j0 + 16 t + p; the eight values of a lane are A columns c0 + 8 kk .. + 7 in order
  float* __restrict__ Ps = P + (int64_t)sp * split_stride;
  const int64_t c = c0 + 8 * kk;
  const bool vst = (ldp & 3) == 0 && c + 7 < n;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + 16 * t + p;
    if (j >= ncols) continue;
    float* __restrict__ prow = Ps + (int64_t)j * ldp;
    const floatx4 o0 = {acc[0][t][0], acc[1][t][0], acc[0][t][1], acc[1][t][1]};
    const floatx4 o1 = {acc[0][t][2], acc[1][t][2], acc[0][t][3], acc[1][t][3]};
    if (vst) {
      *reinterpret_cast<floatx4*>(prow + c) = o0;
      *reinterpret_cast<floatx4*>(prow + c + 4) = o1;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (c + e < n) prow[c + e] = o0[e];
        if (c + 4 + e < n) prow[c + 4 + e] = o1[e];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int NT2>
static hipError_t launch_fwd32(const FwdArgs& a, hipStream_t st) {
  const int ctiles = (a.ncols + 63) / 64;
  const int ns = a.ksplit > 0 ? a.ksplit : 1;
  const int64_t kchunk = ns > 1 ? a.kchunk : a.n;
  dim3 grid((unsigned)((a.m + 127) / 128), (unsigned)ns, (unsigned)ctiles);
  const bool direct = ns == 1;
  float* out = direct ? a.Z : a.P;
  const int64_t ldo = direct ? a.ldz : a.ldp;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  if (a.vec)
    hipLaunchKernelGGL((fwd32_kernel<NT2, true, FWD32_KST<NT2>, 1, float, FWD32_MINB<NT2>>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n, a.shift,
                       a.Xt, a.ldx, a.ncols, kchunk, a.corr, a.alpha, out, ldo, a.split_stride, direct ? 1 : 0);
  else
    hipLaunchKernelGGL((fwd32_kernel<NT2, false, FWD32_KST<NT2>, 1, float, FWD32_MINB<NT2>>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                       a.shift, a.Xt, a.ldx, a.ncols, kchunk, a.corr, a.alpha, out, ldo, a.split_stride,
                       direct ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  if (e != hipSuccess || direct) return e;
  return launch_fwd_reduce(a, ns, st);
}

hipError_t launch_fwd_reduce(const FwdArgs& a, int ksplit, hipStream_t st) {
  const int64_t tot = a.m * a.ncols;
  hipLaunchKernelGGL(fwd_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a.P, ksplit,
                     a.split_stride, a.ldp, a.m, a.ncols, a.corr, a.alpha, a.Z, a.ldz);
  return hipGetLastError();
}

hipError_t launch_fwd_f32(const FwdArgs& a, hipStream_t st) {
  if (a.m <= 0 || a.ncols <= 0) return hipSuccess;
  if (a.A == nullptr || a.shift == nullptr || a.Xt == nullptr || a.Z == nullptr) return hipErrorInvalidValue;
  if (a.ldx < a.n || a.lda < a.n) return hipErrorInvalidValue;
  if (a.ksplit > 1) {
    if (a.P == nullptr || a.ldp < ((a.ncols + 63) / 64) * 64 || a.kchunk % F3_KST != 0 ||
        (int64_t)a.ksplit * a.kchunk < a.n || a.split_stride < a.m * a.ldp)
      return hipErrorInvalidValue;
  }
  if (a.ncols <= 32) return launch_fwd32<1>(a, st);
  return launch_fwd32<2>(a, st);
}

// K split of the forward product: the smallest split count (at most 8) whose
// grid of 128-row blocks fills `slots` concurrent blocks with < 6% idle in the
// last round; kchunk is a multiple of the LDS stage.
void fwd_split(int64_t m, int64_t n, int64_t slots, int* ksplit, int64_t* kchunk) {
  const int64_t rt = (m + 127) / 128;
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= 8; ++s) {
    const int64_t chunk = ((n + s - 1) / s + F3_KCHUNK - 1) / F3_KCHUNK * F3_KCHUNK;
    const int64_t ns = (n + chunk - 1) / chunk;
    const int64_t blocks = rt * ns;
    const int64_t rounds = (blocks + slots - 1) / slots;
    const double eff = (double)blocks / (double)(rounds * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = (int)ns;
    }
    if (eff >= 0.94) break;
  }
  const int64_t chunk = ((n + best - 1) / best + F3_KCHUNK - 1) / F3_KCHUNK * F3_KCHUNK;
  *ksplit = (int)((n + chunk - 1) / chunk);
  *kchunk = chunk;
}

// Row split of the adjoint product: among split counts giving at least two
// rounds of `slots` concurrent blocks and float32 chains of at most
// ADJ_MAX_CHAIN rows (up to twice the smallest such count), the one whose last
// round is fullest (ties to fewer splits, i.e. less partial-sum traffic); rows
// per split are a multiple of the LDS stage.
void adj_split(int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit, int64_t* rows_per_split) {
  // blocks per row split: 64 Z columns x 256 A columns, or for a wide Z (the kernel
  // launch_adj_f32 picks for more than 64 columns) 16 adjw_tiles Z columns x 128 A columns
  const int64_t wcols = 16 * adjw_tiles(ncols);
  const int64_t per = ncols > 64 ? (int64_t)((ncols + wcols - 1) / wcols) * ((n + ADJW_ACOLS - 1) / ADJW_ACOLS)
                                 : (int64_t)((ncols + 63) / 64) * ((n + 255) / 256);
  int64_t lo = (2 * slots + per - 1) / per;
  // every float32 chain (one split) within ADJ_MAX_CHAIN rows
  const int64_t lo_chain = (m + ADJ_MAX_CHAIN - 1) / ADJ_MAX_CHAIN;
  if (lo < lo_chain) lo = lo_chain;
  int64_t hi = lo * 2 > lo + 8 ? lo * 2 : lo + 8;
  const int64_t maxs = m / 64 > 0 ? m / 64 : 1;
  if (lo > maxs) lo = maxs;
  if (hi > maxs) hi = maxs;
  if (lo < 1) lo = 1;
  double best = -1.0;
  int64_t bs = 1, br = ((m + ADJ_RS - 1) / ADJ_RS) * ADJ_RS;
  for (int64_t s = lo; s <= hi; ++s) {
    const int64_t r = ((m + s - 1) / s + ADJ_RS - 1) / ADJ_RS * ADJ_RS;
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

hipError_t launch_adj_f32(const AdjArgs& a, hipStream_t st) {
  if (a.n <= 0 || a.ncols <= 0 || a.nsplit <= 0) return hipSuccess;
  if (a.A == nullptr || a.shift == nullptr || a.Z == nullptr || a.P == nullptr) return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldp < a.n || a.rows_per_split % 4 != 0) return hipErrorInvalidValue;
  if ((int64_t)a.nsplit * a.rows_per_split < a.m) return hipErrorInvalidValue;
  // a wide Z (the T pass) read in one pass over A when its layout allows 16-byte pieces
  const bool wide = a.ncols > 64 && !a.ones && a.vec && a.n % 2 == 0 && a.ncols % 4 == 0 && a.ldz % 4 == 0 &&
                    (reinterpret_cast<uintptr_t>(a.Z) & 15) == 0;
  if (wide) {
    const int nt = adjw_tiles(a.ncols);
    const int jt = (a.ncols + 16 * nt - 1) / (16 * nt);
    const int ct = (int)((a.n + ADJW_ACOLS - 1) / ADJW_ACOLS);
    const dim3 grid((unsigned)((int64_t)jt * ct * a.nsplit));
    if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
    if (nt == 6)
      hipLaunchKernelGGL((adj_wide_kernel<6, true>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                         a.shift, a.Z, a.ldz, a.ncols, a.rows_per_split, a.nsplit, jt, ct, a.P, a.ldp, a.split_stride);
    else if (nt == 8)
      hipLaunchKernelGGL((adj_wide_kernel<8, true>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                         a.shift, a.Z, a.ldz, a.ncols, a.rows_per_split, a.nsplit, jt, ct, a.P, a.ldp, a.split_stride);
    else
      hipLaunchKernelGGL((adj_wide_kernel<12, true>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                         a.shift, a.Z, a.ldz, a.ncols, a.rows_per_split, a.nsplit, jt, ct, a.P, a.ldp, a.split_stride);
    hipError_t e = hipGetLastError();
    if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
    return e;
  }
  const int jtiles = (a.ncols + (a.ones ? 1 : 0) + 63) / 64;
  const int ctiles = (int)((a.n + 255) / 256);
  const int64_t total = (int64_t)jtiles * ctiles * a.nsplit;
  dim3 grid((unsigned)total);
  const bool vec = a.vec && (a.n % 4 == 0);
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  // up to 32 output columns (with the ones column): two 16-column tiles per wave instead of four,
  // half the matrix-core work of the padded 64 (the narrow blocks of a small l are bound by the
  // read of A, not by the matrix cores); identical sums, since every output column has its own chain
  const bool narrow = a.ncols + (a.ones ? 1 : 0) <= 32;
#define RPCA_ADJ(NT_, VEC_)                                                                               \
  hipLaunchKernelGGL((adj_f32_kernel<NT_, VEC_, ADJ_RS, NT_ == 2 ? 3 : 2>), grid, dim3(256), 0, st,      \
                     (const float*)a.A, a.lda, a.m, a.n, a.shift, a.Z, a.ldz, a.ncols, a.rows_per_split,  \
                     a.nsplit, jtiles, ctiles, a.P, a.ldp, a.split_stride, a.ones ? 1 : 0)
  if (narrow) {
    if (vec)
      RPCA_ADJ(2, true);
    else
      RPCA_ADJ(2, false);
  } else {
    if (vec)
      RPCA_ADJ(4, true);
    else
      RPCA_ADJ(4, false);
  }
#undef RPCA_ADJ
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  return e;
}

}  // namespace rpca
