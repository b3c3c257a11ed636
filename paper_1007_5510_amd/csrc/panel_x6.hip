// Float32 streaming products of Steps 1 and 3 (eqs. first_prod .. last_prod,
// product_t3) on gfx950 bfloat16 matrix cores with float32 accuracy:
//
//   fwd:  Z = alpha * ((A - 1 s^T) X - 1 corr^T)       (as fwd32_kernel)
//   adj:  P_s = ((A_s - 1 s^T)^T Z_s)^T                 (as adj_f32_kernel)
//
// Every float32 operand value x (after the shift) is split by round-to-nearest
// into three bfloat16 parts, x = x0 + x1 + x2 + e with |x1| <= 2^-8 |x|,
// |x2| <= 2^-16 |x| and |e| <= 2^-24 |x|.  A product a x is formed as the six
// terms a_i x_j with i + j <= 2, each exact in float32, accumulated by
// v_mfma_f32_32x32x16_bf16 in float32; the dropped terms a1 x2, a2 x1, a2 x2
// and the split residuals together stay below 2^-22 |a x| per product, the
// rounding level of a float32 product.  The matrix-core rate for bfloat16 is
// 16 times the float32 one, so the six products cost less than a third of the
// float32 MFMA time and the passes become bound by the read of A.
//
// The other operand (X, or Z in the adjoint) is split once per pass into three
// bfloat16 planes (split3_x_kernel, split3_zt_kernel); A is split in registers
// right after it is loaded and shifted.
//
// MFMA 32x32x16 bf16 (wave64): A operand lane i + 32 g holds row i, K entries
// 8 g .. 8 g + 7; B operand lane j + 32 g holds column j for the same K
// entries; D: lane l, register v holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
// In the adjoint the roles are swapped (A operand = Z^T, B operand = A), so the
// output lanes run along the columns of A and its partial-sum rows are written
// with consecutive lanes at consecutive addresses.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace rpca {

typedef __bf16 x6_bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 x6_bf16x2 __attribute__((ext_vector_type(2)));
typedef float x6_floatx2 __attribute__((ext_vector_type(2)));
typedef uint32_t x6_u32x4 __attribute__((ext_vector_type(4)));

RPCA_DEV uint32_t x6_cvt(float a, float b) {  // RNE bfloat16 pair, a in the low half
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((x6_floatx2){a, b}, x6_bf16x2));
}

// (a, b) -> three packed bfloat16 pairs: x = hi + mid + lo (+ <= 2^-24 |x|)
struct X6Parts {
  uint32_t h, m, l;
};
RPCA_DEV X6Parts x6_split(float a, float b) {
  X6Parts p;
  p.h = x6_cvt(a, b);
  const float ra = a - __uint_as_float(p.h << 16), rb = b - __uint_as_float(p.h & 0xFFFF0000u);
  p.m = x6_cvt(ra, rb);
  const float sa = ra - __uint_as_float(p.m << 16), sb = rb - __uint_as_float(p.m & 0xFFFF0000u);
  p.l = x6_cvt(sa, sb);
  return p;
}

RPCA_DEV floatx16 x6_mfma(x6_u32x4 a, x6_u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(x6_bf16x8, a), __builtin_bit_cast(x6_bf16x8, b), c,
                                                 0, 0, 0);
}

// acc += sum of the six products with i + j <= 2 (small terms first)
RPCA_DEV floatx16 x6_six(const x6_u32x4 (&a)[3], const x6_u32x4 (&b)[3], floatx16 acc) {
  acc = x6_mfma(a[2], b[0], acc);
  acc = x6_mfma(a[1], b[1], acc);
  acc = x6_mfma(a[0], b[2], acc);
  acc = x6_mfma(a[1], b[0], acc);
  acc = x6_mfma(a[0], b[1], acc);
  return x6_mfma(a[0], b[0], acc);
}

// the same sums for two tiles (za with acc0, zb with acc1) with the two chains interleaved
RPCA_DEV void x6_six2(const x6_u32x4 (&za)[3], const x6_u32x4 (&zb)[3], const x6_u32x4 (&b)[3], floatx16& acc0,
                      floatx16& acc1) {
  acc0 = x6_mfma(za[2], b[0], acc0);
  acc1 = x6_mfma(zb[2], b[0], acc1);
  acc0 = x6_mfma(za[1], b[1], acc0);
  acc1 = x6_mfma(zb[1], b[1], acc1);
  acc0 = x6_mfma(za[0], b[2], acc0);
  acc1 = x6_mfma(zb[0], b[2], acc1);
  acc0 = x6_mfma(za[1], b[0], acc0);
  acc1 = x6_mfma(zb[1], b[0], acc1);
  acc0 = x6_mfma(za[0], b[1], acc0);
  acc1 = x6_mfma(zb[0], b[1], acc1);
  acc0 = x6_mfma(za[0], b[0], acc0);
  acc1 = x6_mfma(zb[0], b[0], acc1);
}

// ---------------------------------------------------------------------------
// operand planes
// ---------------------------------------------------------------------------
// Xp[p][c][k] (p = 0, 1, 2) = part p of Xt[c][k] for c < ncols, k < n; zero for
// c < cpad, k < ldxs otherwise.
__global__ __launch_bounds__(256) void split3_x_kernel(const float* __restrict__ Xt, int64_t ldx, int64_t n,
                                                       int ncols, int cpad, int64_t ldxs,
                                                       uint16_t* __restrict__ Xp, int64_t plane) {
  const int64_t k2 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  const int c = blockIdx.y;
  if (k2 >= ldxs || c >= cpad) return;
  float a = 0.f, b = 0.f;
  if (c < ncols) {
    if (k2 < n) a = Xt[(int64_t)c * ldx + k2];
    if (k2 + 1 < n) b = Xt[(int64_t)c * ldx + k2 + 1];
  }
  const X6Parts q = x6_split(a, b);
  uint32_t* o = reinterpret_cast<uint32_t*>(Xp + (int64_t)c * ldxs + k2);
  o[0] = q.h;
  o[plane / 2] = q.m;
  o[plane] = q.l;
}

// Zp[p][j][r] = part p of Z[r][j] (transposed) for r < m, j < ncols; with
// `ones`, column ncols is 1 (the column sums of A_s - 1 s^T come out as row
// ncols of the adjoint's partials); zero elsewhere (j < cpad, r < ldzs).
// 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void split3_zt_kernel(const float* __restrict__ Z, int64_t ldz, int64_t m,
                                                        int ncols, int ones, int cpad, int64_t ldzs,
                                                        uint16_t* __restrict__ Zp, int64_t plane) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y;
    const int j = j0 + tx;
    float v = 0.f;
    if (r < m) v = j < ncols ? Z[r * ldz + j] : ((ones && j == ncols) ? 1.f : 0.f);
    tile[y][tx] = v;
  }
  __syncthreads();
  // thread -> output column j0 + jy, rows r0 + 2 rx, r0 + 2 rx + 1
  const int rx = threadIdx.x & 31, jy0 = threadIdx.x >> 5;
  for (int jy = jy0; jy < 64; jy += 8) {
    const int j = j0 + jy;
    const int64_t r = r0 + 2 * rx;
    if (j >= cpad || r >= ldzs) continue;
    const X6Parts q = x6_split(tile[2 * rx][jy], tile[2 * rx + 1][jy]);
    uint32_t* o = reinterpret_cast<uint32_t*>(Zp + (int64_t)j * ldzs + r);
    o[0] = q.h;
    o[plane / 2] = q.m;
    o[plane] = q.l;
  }
}

// ---------------------------------------------------------------------------
// forward: each wave owns 32 rows x 64 columns (two 32-column tiles), a block
// of 4 waves 128 rows.  The three X planes and the shift are staged per block
// in LDS (32 K per stage, double buffered, rows padded to 40 bfloat16); A goes
// to registers one stage ahead and is shifted and split there.  K is split
// over blockIdx.y as in fwd32_kernel, partial sums reduced in float64.
// ---------------------------------------------------------------------------
constexpr int X6_KST = 64;  // K per LDS stage of the launched configuration

// KST: K per LDS stage (32 or 64); MINB: workgroups per CU the register budget is sized for
template <bool VEC, int KST = X6_KST, int MINB = 3>
__global__ __launch_bounds__(256, MINB) void fwd_x6_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const uint16_t* __restrict__ Xp, int64_t ldxs, int64_t xplane, int ncols, int64_t kchunk,
    const float* __restrict__ corr, const double* __restrict__ alpha_ptr, float* __restrict__ Z, int64_t ldz,
    int64_t split_stride, int direct) {
  constexpr int XP = KST + 8;  // padded LDS row (bfloat16)
  constexpr int NS = KST / 16;  // MFMA K-steps per stage
  constexpr int XQ = KST / 32;  // 16-byte X chunks per thread per plane
  __shared__ uint16_t Xs[2][3][64][XP];
  // shift of the stage: entries [0, KST) are read; every thread stores one entry of
  // its own (threads past KST store duplicates) so the store needs no branch
  __shared__ __attribute__((aligned(16))) float Ss[2][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, g = lane >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const int sk = blockIdx.y;
  const int c0 = blockIdx.z * 64;
  const int64_t kbeg = (int64_t)sk * kchunk;
  const int64_t kend = kbeg + kchunk < n ? kbeg + kchunk : n;
  const int64_t row = r0 + li;
  const float* __restrict__ arow = A + (row < m ? row : m - 1) * lda;
  // cooperative X loader: plane q, column (tid >> 2), K offsets (KST / 4) (tid & 3) + 8 h
  const int xc = tid >> 2, xk = (tid & 3) * (KST / 4);
  const uint16_t* __restrict__ xsrc = Xp + (int64_t)(c0 + xc) * ldxs + xk;

  floatx16 acc[2], acc2[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc[t][v] = 0.f;
      acc2[t][v] = 0.f;
    }
  auto fold = [&]() {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      acc2[t] += acc[t];
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
    }
  };
  struct AStage {
    floatx4 a[2 * NS];  // K-step s: a[2 s], a[2 s + 1] = K 16 s + 8 g .. + 8
  };
  struct XStage {
    x6_u32x4 x[3][XQ];
    float s;
  };
  auto load_a = [&](AStage& b, int64_t kb) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const float* p = arow + kb + 16 * s + 8 * g;
      b.a[2 * s] = VEC ? *reinterpret_cast<const floatx4*>(p) : floatx4{p[0], p[1], p[2], p[3]};
      b.a[2 * s + 1] = VEC ? *reinterpret_cast<const floatx4*>(p + 4) : floatx4{p[4], p[5], p[6], p[7]};
    }
  };
  auto load_x = [&](XStage& b, int64_t kb) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int h = 0; h < XQ; ++h) b.x[q][h] = *reinterpret_cast<const x6_u32x4*>(xsrc + q * xplane + kb + 8 * h);
    b.s = shift[kb + (tid & (KST - 1))];
  };
  auto store_x = [&](const XStage& b, int buf) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int h = 0; h < XQ; ++h) *reinterpret_cast<x6_u32x4*>(&Xs[buf][q][xc][xk + 8 * h]) = b.x[q][h];
    Ss[buf][tid] = b.s;
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const floatx4 s0 = *reinterpret_cast<const floatx4*>(&Ss[buf][16 * s + 8 * g]);
      const floatx4 s1 = *reinterpret_cast<const floatx4*>(&Ss[buf][16 * s + 8 * g + 4]);
      const floatx4 x0 = b.a[2 * s] - s0, x1 = b.a[2 * s + 1] - s1;
      const X6Parts p0 = x6_split(x0[0], x0[1]), p1 = x6_split(x0[2], x0[3]);
      const X6Parts p2 = x6_split(x1[0], x1[1]), p3 = x6_split(x1[2], x1[3]);
      const x6_u32x4 ap[3] = {x6_u32x4{p0.h, p1.h, p2.h, p3.h}, x6_u32x4{p0.m, p1.m, p2.m, p3.m},
                              x6_u32x4{p0.l, p1.l, p2.l, p3.l}};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        x6_u32x4 bp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) bp[q] = *reinterpret_cast<const x6_u32x4*>(&Xs[buf][q][32 * t + li][16 * s + 8 * g]);
        acc[t] = x6_six(ap, bp, acc[t]);
      }
    }
  };

  // whole stages on two register stages used alternately (no copy between
  // them, so a load has a whole stage to arrive); the prologue's loads are
  // waited for before the loop, so its header carries no wait on loads issued
  // inside it
  const int64_t nfull = (kend - kbeg) / KST;
  int it = 0;
  auto step_done = [&]() {
    if (++it == 1024 / KST) {  // fold every 1024 K
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
      // past the last whole stage the prefetch re-reads stage st + 1
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
  // tail stage (fewer than KST columns left): A and the shift read as zero beyond kend
  const int64_t kt = kbeg + nfull * KST;
  if (kt < kend) {
    AStage at;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t k = kt + 16 * s + 8 * g + 4 * h;
        floatx4 v = {0.f, 0.f, 0.f, 0.f};
        if (k < kend) v.x = arow[k];
        if (k + 1 < kend) v.y = arow[k + 1];
        if (k + 2 < kend) v.z = arow[k + 2];
        if (k + 3 < kend) v.w = arow[k + 3];
        at.a[2 * s + h] = v;
      }
    const int buf = (int)(nfull & 1);
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int h = 0; h < XQ; ++h)
        *reinterpret_cast<x6_u32x4*>(&Xs[buf][q][xc][xk + 8 * h]) =
            *reinterpret_cast<const x6_u32x4*>(xsrc + q * xplane + kt + 8 * h);
    if (tid < KST / 4) {
      floatx4 sv = {0.f, 0.f, 0.f, 0.f};
      const int64_t k = kt + 4 * tid;
      if (k < kend) sv.x = shift[k];
      if (k + 1 < kend) sv.y = shift[k + 1];
      if (k + 2 < kend) sv.z = shift[k + 2];
      if (k + 3 < kend) sv.w = shift[k + 3];
      *reinterpret_cast<floatx4*>(&Ss[buf][4 * tid]) = sv;
    }
    __syncthreads();
    compute(at, buf);
  }
  fold();

  const double alpha = (direct && alpha_ptr != nullptr) ? *alpha_ptr : 1.0;
  float* __restrict__ Zs = Z + (direct ? 0 : (int64_t)sk * split_stride);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = c0 + 32 * t + li;
    if (c >= ncols) continue;
    const double cr = (direct && corr != nullptr) ? (double)corr[c] : 0.0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t r = r0 + 8 * (v >> 2) + 4 * g + (v & 3);
      if (r < m) Zs[r * ldz + c] = direct ? (float)(alpha * ((double)acc2[t][v] - cr)) : acc2[t][v];
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint: each wave owns 64 columns of A (lane i: columns c0 + 2 i, c0 + 2 i
// + 1, one float2 per row) x 64 columns of Z (two 32-column tiles); 4 waves
// per block cover 256 columns of A.  Rows of the split are walked 32 at a time
// (two K-steps of 16); the three transposed Z planes of a stage are staged in
// LDS.  Blocks are remapped so that logical neighbours share an XCD.
// Requires A 8-byte aligned with lda and n even (a float2 is wholly inside a
// row or wholly past its end).
// ---------------------------------------------------------------------------
constexpr int X6_RS = 32;
constexpr int X6_ZP = X6_RS + 8;

RPCA_DEV int64_t x6_xcd_remap(int64_t b, int64_t total) {
  const int64_t q = total / 8, r = total % 8;
  const int64_t x = b % 8, local = b / 8;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

__global__ __launch_bounds__(256, 2) void adj_x6_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const uint16_t* __restrict__ Zp, int64_t ldzs, int64_t zplane, int nout, int64_t rows_per_split, int nsplit,
    int jtiles, int ctiles, float* __restrict__ P, int64_t ldp, int64_t split_stride) {
  __shared__ uint16_t Zs[2][3][64][X6_ZP];
  const int64_t total = (int64_t)jtiles * ctiles * nsplit;
  const int64_t logical = x6_xcd_remap(blockIdx.x, total);
  const int jt = (int)(logical % jtiles);
  const int64_t rest = logical / jtiles;
  const int ct = (int)(rest % ctiles);
  const int sp = (int)(rest / ctiles);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, g = lane >> 5;
  const int64_t c0 = (int64_t)ct * 256 + wave * 64;
  const int64_t cl = c0 + 2 * li;
  const int64_t clc = cl < n ? cl : n - 2;  // clamped (n even)
  const int j0 = jt * 64;
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  const x6_floatx2 sh = *reinterpret_cast<const x6_floatx2*>(shift + clc);
  // cooperative Z loader: chunk tid + 256 q -> plane q, Z column (tid >> 2), rows 8 (tid & 3)
  const int zc = tid >> 2, zr = (tid & 3) * 8;
  const uint16_t* __restrict__ zsrc = Zp + (int64_t)(j0 + zc) * ldzs + zr;

  floatx16 acc[2][2];  // [A-column half v][Z tile t]
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[v][t][e] = 0.f;
  struct AStage {
    x6_floatx2 a[16];  // row 16 s + 8 g + u at a[8 s + u]
  };
  struct ZStage {
    x6_u32x4 z[3];
  };
  auto load_a = [&](AStage& b, int64_t rb) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        b.a[8 * s + u] = *reinterpret_cast<const x6_floatx2*>(A + (rb + 16 * s + 8 * g + u) * lda + clc);
  };
  auto load_z = [&](ZStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < 3; ++q) b.z[q] = *reinterpret_cast<const x6_u32x4*>(zsrc + q * zplane + rb);
  };
  auto store_z = [&](const ZStage& b, int buf) {
#pragma unroll
    for (int q = 0; q < 3; ++q) *reinterpret_cast<x6_u32x4*>(&Zs[buf][q][zc][zr]) = b.z[q];
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // B operands (A, shifted and split): column half v, rows 16 s + 8 g .. + 8
      x6_u32x4 bp[2][3];
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        X6Parts pu[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          pu[u] = x6_split(b.a[8 * s + 2 * u][v] - sh[v], b.a[8 * s + 2 * u + 1][v] - sh[v]);
        bp[v][0] = x6_u32x4{pu[0].h, pu[1].h, pu[2].h, pu[3].h};
        bp[v][1] = x6_u32x4{pu[0].m, pu[1].m, pu[2].m, pu[3].m};
        bp[v][2] = x6_u32x4{pu[0].l, pu[1].l, pu[2].l, pu[3].l};
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        x6_u32x4 zp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) zp[q] = *reinterpret_cast<const x6_u32x4*>(&Zs[buf][q][32 * t + li][16 * s + 8 * g]);
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[v][t] = x6_six(zp, bp[v], acc[v][t]);
      }
    }
  };

  // two register stages used alternately, prologue drained (as in the forward kernel)
  const int64_t nfull = (rend - rbeg) / X6_RS;
  if (nfull > 0) {
    AStage a0, a1;
    ZStage zs;
    load_z(zs, rbeg);
    load_a(a0, rbeg);
    store_z(zs, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int64_t st = 0;
    for (; st + 2 <= nfull; st += 2) {
      const int64_t r1 = rbeg + (st + 1) * X6_RS;
      load_z(zs, r1);
      load_a(a1, r1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, 0);
      store_z(zs, 1);
      __syncthreads();
      // past the last whole stage the prefetch re-reads stage st + 1
      const int64_t r2 = rbeg + (st + 2 < nfull ? st + 2 : st + 1) * X6_RS;
      load_z(zs, r2);
      load_a(a0, r2);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, 1);
      store_z(zs, 0);
      __syncthreads();
    }
    if (st < nfull) {  // odd stage count: the last stage is in a0, Z in buffer 0
      compute(a0, 0);
      __syncthreads();
    }
  }
  // tail rows (fewer than a stage): rows at or past rend read as the shift (zero after shifting)
  const int64_t rt = rbeg + nfull * X6_RS;
  if (rt < rend) {
    const int buf = (int)(nfull & 1);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      *reinterpret_cast<x6_u32x4*>(&Zs[buf][q][zc][zr]) = *reinterpret_cast<const x6_u32x4*>(zsrc + q * zplane + rt);
    AStage at;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t r = rt + 16 * s + 8 * g + u;
        at.a[8 * s + u] = r < rend ? *reinterpret_cast<const x6_floatx2*>(A + r * lda + clc) : sh;
      }
    __syncthreads();
    compute(at, buf);
  }

  // D[Z column][A column]: register e of tile (v, t) holds Z column
  // j0 + 32 t + 8 (e / 4) + 4 g + e % 4 and A column c0 + 2 li + v
  float* __restrict__ Ps = P + (int64_t)sp * split_stride;
  if (cl >= n) return;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = j0 + 32 * t + 8 * (e >> 2) + 4 * g + (e & 3);
      if (j < nout) *reinterpret_cast<x6_floatx2*>(Ps + (int64_t)j * ldp + cl) = x6_floatx2{acc[0][t][e], acc[1][t][e]};
    }
}

// ---------------------------------------------------------------------------
// wide adjoint for the T pass: one read of A for up to 32 NT columns of Z.
// Each wave owns 32 columns of A (lane i: column c0 + i, one float per row) x
// 32 NT columns of Z (NT tiles of 32); 8 waves per block cover 256 columns of A
// and share the Z planes of a stage in LDS.  Two tiles are computed at a time so
// that two accumulation chains are in flight.  Every output element sees the same
// rows, K-steps, splits and six-term order as in adj_x6_kernel, so the partial
// sums are the same.  Six bfloat16 products over up to 192 columns make the pass
// bound by the matrix cores rather than by the read of A.  Requires
// rows_per_split % 32 == 0 (a stage of Z rows stays inside the zero-padded planes)
// and 32 NT <= the planes' columns.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(512, 1) void adj_x6w_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const uint16_t* __restrict__ Zp, int64_t ldzs, int64_t zplane, int nout, int64_t rows_per_split, int nsplit,
    int ctiles, float* __restrict__ P, int64_t ldp, int64_t split_stride) {
  constexpr int ZC = 32 * NT;            // Z columns of the block
  constexpr int NCH = 3 * ZC * 4;        // 16-byte chunks per stage: 3 planes x ZC columns x 4 row groups
  constexpr int ZQ = (NCH + 511) / 512;  // chunks per thread
  static_assert(ZQ * 512 - NCH <= 3 * ZC, "spare chunks need a padding slot each");
  __shared__ __attribute__((aligned(16))) uint16_t Zs[2][3][ZC][X6_ZP];
  const int64_t total = (int64_t)ctiles * nsplit;
  const int64_t logical = x6_xcd_remap(blockIdx.x, total);
  const int ct = (int)(logical % ctiles);
  const int sp = (int)(logical / ctiles);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, g = lane >> 5;
  const int64_t c = (int64_t)ct * 256 + wave * 32 + li;
  const int64_t cc = c < n ? c : n - 1;  // clamped column
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  const float sh = shift[cc];
  const float* __restrict__ acol = A + cc;
  // cooperative Z loader: chunk e = tid + 512 q -> plane e / (4 ZC), column (e / 4) % ZC,
  // rows 8 (e % 4) .. + 8 of the stage.  Chunks past NCH load chunk e - NCH again and
  // store it into the unused padding of a row (columns 32 .. 39), so no store needs a branch.
  int64_t zoff[ZQ];
  int ldsoff[ZQ];
#pragma unroll
  for (int q = 0; q < ZQ; ++q) {
    const int e = tid + 512 * q;
    const int es = e < NCH ? e : e - NCH;
    const int pl = es / (4 * ZC), col = (es / 4) % ZC, rg = es % 4;
    zoff[q] = (int64_t)pl * zplane + (int64_t)col * ldzs + 8 * rg;
    ldsoff[q] = e < NCH ? (pl * ZC + col) * X6_ZP + 8 * rg : es * X6_ZP + 32;
  }

  floatx16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[t][e] = 0.f;
  struct AStage {
    float a[16];  // row 16 s + 8 g + u at a[8 s + u]
  };
  struct ZStage {
    x6_u32x4 z[ZQ];
  };
  auto load_a = [&](AStage& b, int64_t rb) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < 8; ++u) b.a[8 * s + u] = acol[(rb + 16 * s + 8 * g + u) * lda];
  };
  auto load_z = [&](ZStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < ZQ; ++q) b.z[q] = *reinterpret_cast<const x6_u32x4*>(Zp + zoff[q] + rb);
  };
  auto store_z = [&](const ZStage& b, int buf) {
    uint16_t* base = &Zs[buf][0][0][0];
#pragma unroll
    for (int q = 0; q < ZQ; ++q) *reinterpret_cast<x6_u32x4*>(base + ldsoff[q]) = b.z[q];
  };
  auto compute = [&](const AStage& b, int buf) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // B operand (A, shifted and split): rows 16 s + 8 g .. + 8 of column c
      X6Parts pu[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pu[u] = x6_split(b.a[8 * s + 2 * u] - sh, b.a[8 * s + 2 * u + 1] - sh);
      const x6_u32x4 bp[3] = {x6_u32x4{pu[0].h, pu[1].h, pu[2].h, pu[3].h},
                              x6_u32x4{pu[0].m, pu[1].m, pu[2].m, pu[3].m},
                              x6_u32x4{pu[0].l, pu[1].l, pu[2].l, pu[3].l}};
      // two tiles at a time: two independent accumulation chains
#pragma unroll
      for (int t = 0; t < NT; t += 2) {
        x6_u32x4 za[3], zb[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          za[q] = *reinterpret_cast<const x6_u32x4*>(&Zs[buf][q][32 * t + li][16 * s + 8 * g]);
          zb[q] = *reinterpret_cast<const x6_u32x4*>(&Zs[buf][q][32 * t + 32 + li][16 * s + 8 * g]);
        }
        x6_six2(za, zb, bp, acc[t], acc[t + 1]);
      }
    }
  };

  // two register stages used alternately, prologue drained (as in adj_x6_kernel)
  const int64_t nfull = (rend - rbeg) / X6_RS;
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
      const int64_t r1 = rbeg + (st + 1) * X6_RS;
      load_z(zr, r1);
      load_a(a1, r1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, 0);
      store_z(zr, 1);
      __syncthreads();
      // past the last whole stage the prefetch re-reads stage st + 1
      const int64_t r2 = rbeg + (st + 2 < nfull ? st + 2 : st + 1) * X6_RS;
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
  // tail rows (fewer than a stage): rows at or past rend read as the shift (zero after shifting)
  const int64_t rt = rbeg + nfull * X6_RS;
  if (rt < rend) {
    const int buf = (int)(nfull & 1);
    ZStage zt;
    load_z(zt, rt);
    store_z(zt, buf);
    AStage at;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t r = rt + 16 * s + 8 * g + u;
        at.a[8 * s + u] = r < rend ? acol[r * lda] : sh;
      }
    __syncthreads();
    compute(at, buf);
  }

  // D[Z column][A column]: register e of tile t holds Z column 32 t + 8 (e / 4) + 4 g + e % 4
  float* __restrict__ Ps = P + (int64_t)sp * split_stride + c;
  if (c >= n) return;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = 32 * t + 8 * (e >> 2) + 4 * g + (e & 3);
      if (j < nout) Ps[(int64_t)j * ldp] = acc[t][e];
    }
}

// ---------------------------------------------------------------------------
// rank-K product with a wide output, O = P Y^T (the dense derivative of the
// reverse sweep): O[r][c] = sum over k < kp of P[r][k] Y[c][k], from the three
// bfloat16 parts of P and of Y, each held K-step-major: the 16 entries of K-step
// s, part q of row r are contiguous at ((3 s + q) rows_pad + r) 16, so the rows of
// a tile for one K-step and part are one contiguous run.  Both are padded with
// zeros to whole 256-row tiles and to kp, a multiple of 32.  A block of 8 waves
// computes 256 x 256 tiles of O, a wave 64 x 128 (two by four 32 x 32 tiles, six
// products each per K-step of 16).  The parts of a K-step go from global memory
// straight into LDS (no registers) through a ring of three stages, so two
// K-steps are in flight while one is multiplied.  The blocks are persistent,
// one per compute unit: each XCD takes one eighth of the column tiles and its
// blocks walk them row tile by row tile, so its slice of Y stays in its L2 while
// P streams through, and the copies of a block's next tile overlap the last
// K-steps and the stores of the one before.  O is written with non-temporal
// stores, and any non-finite entry sets the flag.
// ---------------------------------------------------------------------------
constexpr int OX_T = 256;  // tile rows and columns

// Xp in the K-step-major layout above: part q of X[r][k] for r < rows, k < cols; zero for
// r < rows_pad, k < kp otherwise.  Thread: one pair of entries (row r, K-step s, pair j).
__global__ __launch_bounds__(256) void split3_rows_kernel(const float* __restrict__ X, int64_t ldx, int64_t rows,
                                                          int cols, int64_t rows_pad, int kp,
                                                          uint16_t* __restrict__ Xp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = (int)(e & 7);
  const int64_t sr = e >> 3;  // s * rows_pad + r
  const int64_t s = sr / rows_pad, r = sr - s * rows_pad;
  if (s >= kp / 16) return;
  const int k = 16 * (int)s + 2 * j;
  float a = 0.f, b = 0.f;
  if (r < rows) {
    const float* __restrict__ x = X + r * ldx;
    if (k < cols) a = x[k];
    if (k + 1 < cols) b = x[k + 1];
  }
  const X6Parts q = x6_split(a, b);
  const int64_t panel = rows_pad * 16;
  uint32_t* o = reinterpret_cast<uint32_t*>(Xp + 3 * s * panel + r * 16 + 2 * j);
  o[0] = q.h;
  o[panel / 2] = q.m;
  o[panel] = q.l;
}

typedef __attribute__((address_space(3))) void* ox_lds_ptr_t;
typedef const __attribute__((address_space(1))) void* ox_gbl_ptr_t;

// s_waitcnt immediate (gfx9 encoding): vmcnt <= vm, lgkmcnt and expcnt not waited
constexpr int ox_vmcnt(int vm) { return (vm & 15) | ((vm >> 4) << 14) | (7 << 4) | (15 << 8); }

constexpr int OX_CHUNK = 8192;             // one K-step, one part of a 256-row tile (bytes)
constexpr int OX_STAGE = 6 * OX_CHUNK;     // P parts 0..2, then Y parts 0..2
constexpr int OX_DX = 3;                   // ring stages (two K-steps in flight)
constexpr int OX_BPX = 32;                 // persistent blocks per XCD (one per compute unit)

// LDS slot of the 16-byte half h of tile row r (32-byte rows): the halves of rows r and
// r + 4 (which share banks modulo 128 bytes) and of rows r and r + 8 (modulo 256 bytes)
// are swapped relative to each other, so the 16-byte reads of 8 or 16 consecutive rows
// by consecutive lanes hit distinct banks
RPCA_DEV int ox_slot(int r, int h) { return 2 * r + (h ^ (((r >> 2) ^ (r >> 3)) & 1)); }

__global__ __launch_bounds__(512, 1) void outer_x6_kernel(const uint16_t* __restrict__ Pp, int64_t mpad,
                                                          const uint16_t* __restrict__ Yp, int64_t npad, int kp,
                                                          int64_t m, int64_t n, int nbr, int nbc, int cg,
                                                          float* __restrict__ O, int64_t ldo,
                                                          int* __restrict__ nonfinite) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[OX_DX * OX_STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, g = lane >> 5;
  // tiles of this block: XCD x owns the column tiles [x cg, x cg + cnt) of every row tile,
  // numbered row-major; the B blocks on it take every B-th of them
  const int x = (int)(blockIdx.x & 7), lb = (int)(blockIdx.x >> 3), B = (int)(gridDim.x >> 3);
  const int cnt = nbc - x * cg < cg ? nbc - x * cg : cg;
  if (cnt <= 0 || (int64_t)lb >= (int64_t)nbr * cnt) return;
  const int nmine = (int)(((int64_t)nbr * cnt - lb + B - 1) / B);
  const int nst = kp / 16;
  const int F = nmine * nst;  // K-steps of all this block's tiles, in order
  auto origin = [&](int j, int64_t& r0, int64_t& c0) {
    const int64_t idx = lb + (int64_t)j * B;
    r0 = (idx / cnt) * OX_T;
    c0 = ((int64_t)x * cg + idx % cnt) * OX_T;
  };
  // global -> LDS copies (global_load_lds_dwordx4: lane l's 16 bytes land at the wave's
  // base + 16 l): thread tid fills slot tid of each chunk, i.e. row dr, half dh
  const int dr = tid >> 1, dh = (tid & 1) ^ (((dr >> 2) ^ (dr >> 3)) & 1);
  const unsigned char* __restrict__ pbase = reinterpret_cast<const unsigned char*>(Pp + dr * 16 + 8 * dh);
  const unsigned char* __restrict__ ybase = reinterpret_cast<const unsigned char*>(Yp + dr * 16 + 8 * dh);
  const int64_t pkb = mpad * 32, ykb = npad * 32;  // bytes per K-step and part
  auto issue = [&](int f) {
    f = f < F ? f : F - 1;  // past the last K-step: re-read it into a slot no longer read
    const int j = f / nst, ks = f - j * nst;
    int64_t r0, c0;
    origin(j, r0, c0);
    const unsigned char* ps = pbase + r0 * 32 + (int64_t)(3 * ks) * pkb;
    const unsigned char* ys = ybase + c0 * 32 + (int64_t)(3 * ks) * ykb;
    unsigned char* st = lds + (f % OX_DX) * OX_STAGE + wave * 1024;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      __builtin_amdgcn_global_load_lds((ox_gbl_ptr_t)(ps + q * pkb), (ox_lds_ptr_t)(st + q * OX_CHUNK), 16, 0, 0);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      __builtin_amdgcn_global_load_lds((ox_gbl_ptr_t)(ys + q * ykb), (ox_lds_ptr_t)(st + (3 + q) * OX_CHUNK), 16, 0,
                                       0);
  };
  // wave w: rows 64 (w >> 1) .. + 63 (two 32-row tiles) x columns 128 (w & 1) .. + 127 (four)
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 128;
  const int ao0 = 16 * ox_slot(wr + li, g), ao1 = 16 * ox_slot(wr + 32 + li, g);
  floatx16 acc[2][4];
  auto zero = [&]() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;
  };
  zero();
  auto compute = [&](const unsigned char* st) {
    x6_u32x4 a0[3], a1[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a0[q] = *reinterpret_cast<const x6_u32x4*>(st + q * OX_CHUNK + ao0);
      a1[q] = *reinterpret_cast<const x6_u32x4*>(st + q * OX_CHUNK + ao1);
    }
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
      const int bo = (3 * OX_CHUNK) + 16 * ox_slot(wc + 32 * tc + li, g);
      x6_u32x4 b[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) b[q] = *reinterpret_cast<const x6_u32x4*>(st + q * OX_CHUNK + bo);
      // the six products of order <= 2, small terms first, the two row tiles interleaved
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int i = e < 3 ? 2 - e : (e < 5 ? 4 - e : 0), k = e < 3 ? e : (e < 5 ? e - 3 : 0);
        acc[0][tc] = x6_mfma(a0[i], b[k], acc[0][tc]);
        acc[1][tc] = x6_mfma(a1[i], b[k], acc[1][tc]);
      }
    }
  };
  bool bad = false;
  auto put = [&](int j) {
    int64_t r0, c0;
    origin(j, r0, c0);
    auto body = [&](auto checked) {
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) {
        const int64_t c = c0 + wc + 32 * tc + li;
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int64_t r = r0 + wr + 32 * tr + 8 * (v >> 2) + 4 * g + (v & 3);
            const float o = acc[tr][tc][v];
            if (!decltype(checked)::value || (r < m && c < n)) {
              __builtin_nontemporal_store(o, O + r * ldo + c);
              bad = bad || !isfinite(o);
            }
          }
      }
    };
    if (r0 + OX_T <= m && c0 + OX_T <= n)
      body(std::false_type{});
    else
      body(std::true_type{});
  };

  // ring of OX_DX stages over the block's K-steps f = 0 .. F - 1: K-step f is multiplied
  // from slot f % OX_DX while K-steps f + 1 .. f + OX_DX - 1 are in flight.  Every iteration
  // issues exactly 6 copies per wave, so "K-step f has landed" is a counted wait (the
  // stores of a finished tile are issued before the copies of that iteration, so they are
  // older than every copy the wait may leave in flight); the barrier after the wait makes
  // every wave's copies visible and tells that every wave is done with the slot the next
  // copies overwrite.  No __syncthreads (its fence would wait for every copy in flight).
#pragma unroll
  for (int v = 0; v < OX_DX - 1; ++v) issue(v);
  int ks = 0, j = 0;
  for (int f = 0; f < F; ++f) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(ox_vmcnt(6 * (OX_DX - 2)));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if (ks == nst) {  // tile j is complete: write it, start tile j + 1
      put(j);
      zero();
      ks = 0;
      ++j;
    }
    __builtin_amdgcn_sched_barrier(0);
    issue(f + OX_DX - 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(lds + (f % OX_DX) * OX_STAGE);
    ++ks;
  }
  put(j);
  __builtin_amdgcn_s_waitcnt(ox_vmcnt(0));  // no copy in flight at exit
  if (bad) atomicOr(nonfinite, 1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_split3_x(const float* Xt, int64_t ldx, int64_t n, int ncols, int cpad, uint16_t* Xp, int64_t ldxs,
                           int64_t plane, hipStream_t st) {
  if (ldxs % 8 != 0 || plane % 8 != 0 || cpad < ncols || ldxs < n) return hipErrorInvalidValue;
  dim3 grid((unsigned)((ldxs / 2 + 255) / 256), (unsigned)cpad);
  hipLaunchKernelGGL(split3_x_kernel, grid, dim3(256), 0, st, Xt, ldx, n, ncols, cpad, ldxs, Xp, plane);
  return hipGetLastError();
}

hipError_t launch_split3_zt(const float* Z, int64_t ldz, int64_t m, int ncols, bool ones, int cpad, uint16_t* Zp,
                            int64_t ldzs, int64_t plane, hipStream_t st) {
  if (ldzs % 64 != 0 || plane % 8 != 0 || cpad % 64 != 0 || cpad < ncols + (ones ? 1 : 0) || ldzs < m)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)(ldzs / 64), (unsigned)(cpad / 64));
  hipLaunchKernelGGL(split3_zt_kernel, grid, dim3(256), 0, st, Z, ldz, m, ncols, ones ? 1 : 0, cpad, ldzs, Zp, plane);
  return hipGetLastError();
}

hipError_t launch_fwd_x6(const FwdArgs& a, hipStream_t st) {
  if (a.m <= 0 || a.ncols <= 0) return hipSuccess;
  if (a.A == nullptr || a.shift == nullptr || a.X3 == nullptr || a.Z == nullptr) return hipErrorInvalidValue;
  if (a.ldxs3 % 32 != 0 || a.xplane3 % 8 != 0 || a.ldxs3 < a.n) return hipErrorInvalidValue;
  const int ns = a.ksplit > 0 ? a.ksplit : 1;
  const int64_t kchunk = ns > 1 ? a.kchunk : a.n;
  if (ns > 1 && (a.P == nullptr || a.kchunk % 32 != 0 || (int64_t)ns * a.kchunk < a.n)) return hipErrorInvalidValue;
  if (a.ldxs3 < a.n + 64) return hipErrorInvalidValue;  // a tail stage of up to 64 K stays inside the planes
  const int ctiles = (a.ncols + 63) / 64;
  dim3 grid((unsigned)((a.m + 127) / 128), (unsigned)ns, (unsigned)ctiles);
  const bool direct = ns == 1;
  float* out = direct ? a.Z : a.P;
  const int64_t ldo = direct ? a.ldz : a.ldp;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  if (a.vec)
    hipLaunchKernelGGL((fwd_x6_kernel<true>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n, a.shift, a.X3,
                       a.ldxs3, a.xplane3, a.ncols, kchunk, a.corr, a.alpha, out, ldo, a.split_stride, direct ? 1 : 0);
  else
    hipLaunchKernelGGL((fwd_x6_kernel<false>), grid, dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n, a.shift,
                       a.X3, a.ldxs3, a.xplane3, a.ncols, kchunk, a.corr, a.alpha, out, ldo, a.split_stride,
                       direct ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  if (e != hipSuccess || direct) return e;
  return launch_fwd_reduce(a, ns, st);
}

hipError_t launch_adj_x6(const AdjArgs& a, hipStream_t st) {
  if (a.n <= 0 || a.ncols <= 0 || a.nsplit <= 0) return hipSuccess;
  if (a.A == nullptr || a.shift == nullptr || a.Z3 == nullptr || a.P == nullptr) return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldp < a.n || a.lda % 2 != 0 || a.n % 2 != 0 || a.ldp % 2 != 0) return hipErrorInvalidValue;
  if (a.ldzs3 % 64 != 0 || a.zplane3 % 8 != 0 || a.ldzs3 < a.m) return hipErrorInvalidValue;
  if ((int64_t)a.nsplit * a.rows_per_split < a.m || a.rows_per_split % 8 != 0) return hipErrorInvalidValue;
  const int nout = a.ncols + (a.ones ? 1 : 0);
  // the T pass (more than 64 columns, up to 192): one read of A in the wide kernel
  const int64_t zcols = a.zplane3 / a.ldzs3;
  const int wnt = nout <= 128 ? 4 : 6;
  if (nout > 64 && nout <= 192 && 32 * wnt <= zcols && a.rows_per_split % X6_RS == 0) {
    const int wct = (int)((a.n + 255) / 256);
    const int64_t wtotal = (int64_t)wct * a.nsplit;
    if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
    if (wnt == 4)
      hipLaunchKernelGGL(adj_x6w_kernel<4>, dim3((unsigned)wtotal), dim3(512), 0, st, (const float*)a.A, a.lda, a.m,
                         a.n, a.shift, a.Z3, a.ldzs3, a.zplane3, nout, a.rows_per_split, a.nsplit, wct, a.P, a.ldp,
                         a.split_stride);
    else
      hipLaunchKernelGGL(adj_x6w_kernel<6>, dim3((unsigned)wtotal), dim3(512), 0, st, (const float*)a.A, a.lda, a.m,
                         a.n, a.shift, a.Z3, a.ldzs3, a.zplane3, nout, a.rows_per_split, a.nsplit, wct, a.P, a.ldp,
                         a.split_stride);
    hipError_t e = hipGetLastError();
    if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
    return e;
  }
  const int jtiles = (nout + 63) / 64;
  const int ctiles = (int)((a.n + 255) / 256);
  const int64_t total = (int64_t)jtiles * ctiles * a.nsplit;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  hipLaunchKernelGGL(adj_x6_kernel, dim3((unsigned)total), dim3(256), 0, st, (const float*)a.A, a.lda, a.m, a.n,
                     a.shift, a.Z3, a.ldzs3, a.zplane3, nout, a.rows_per_split, a.nsplit, jtiles, ctiles, a.P, a.ldp,
                     a.split_stride);
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  return e;
}

hipError_t launch_split3_rows(const float* X, int64_t ldx, int64_t rows, int cols, int64_t rows_pad, int kp,
                              uint16_t* Xp, hipStream_t st) {
  if (rows_pad <= 0) return hipSuccess;
  if (X == nullptr || Xp == nullptr || kp <= 0 || kp % 16 != 0 || cols > kp || ldx < cols || rows > rows_pad)
    return hipErrorInvalidValue;
  const int64_t blocks = (rows_pad * (kp / 16) * 8 + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split3_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, ldx, rows, cols, rows_pad, kp,
                     Xp);
  return hipGetLastError();
}

hipError_t launch_outer_x6(const uint16_t* Pp, int64_t mpad, const uint16_t* Yp, int64_t npad, int kp, int64_t m,
                           int64_t n, float* O, int64_t ldo, int* nonfinite, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (Pp == nullptr || Yp == nullptr || O == nullptr || nonfinite == nullptr || kp < 32 || kp % 32 != 0 || ldo < n)
    return hipErrorInvalidValue;
  const int64_t nbr = (m + OX_T - 1) / OX_T, nbc = (n + OX_T - 1) / OX_T;
  if (mpad != nbr * OX_T || npad < nbc * OX_T) return hipErrorInvalidValue;
  const int64_t cg = (nbc + 7) / 8;
  if (nbr * cg * (kp / 16) > 0x7fffffff) return hipErrorInvalidValue;
  // persistent blocks, one per compute unit (eight XCDs of 32), each walking its XCD's tiles
  hipLaunchKernelGGL(outer_x6_kernel, dim3(8 * OX_BPX), dim3(512), 0, st, Pp, mpad, Yp, npad, kp, m, n, (int)nbr,
                     (int)nbc, (int)cg, O, ldo, nonfinite);
  return hipGetLastError();
}

}  // namespace rpca
