// Streaming products with A stored in a low-precision format (bfloat16,
// OCP FP8 e4m3 with per-column float scales, or a bfloat16 hi + lo pair) on
// gfx950 bfloat16 matrix cores (v_mfma_f32_32x32x16_bf16, float accumulation).
// The products are those of Steps 1 and 3, with the stored matrix as A:
//
//   fwd:  Z = alpha * (A (c o X) - 1 corr^T)     (c: column scales, FP8 only)
//   adj:  P_s = (A_s^T Z_s)^T                     (scales applied by the reduction)
//
// Every stored value is exact in bfloat16 (e4m3 is a subset of bfloat16), so
// A enters the MFMA unrounded.  The float32 operand (X, or Z in the adjoint)
// is split once per pass into bfloat16 hi = bf16(x), lo = bf16(x - hi) and
// both parts are multiplied, which keeps 16 significant bits of the operand
// (relative representation error <= 2^-17); a hi + lo stored matrix adds the
// lo(A) hi(X) term.  No shift is applied in registers: centring uses the
// exact rank-one correction with the full column mean.
//
// MFMA 32x32x16 bf16 (wave64): A operand lane i + 32 g holds row i, 8
// consecutive K entries of group g; B operand lane j + 32 g holds column j
// for the same K entries; D: lane l, register v holds D[8(v/4) + 4(l/32) +
// v%4][l%32].  Only the pairing of A and B entries by (g, element) matters
// for the contraction, so the K order inside a step is free as long as both
// operands use it.
//
// Adjoint: the contraction runs over rows of A, which are strided in memory.
// A 32 x 32 tile is loaded row-wise (16 consecutive columns per lane) and
// transposed by two MFMAs against 0/1 routing matrices, D = T1 E1 + T2 E2,
// each D entry being one stored value times 1 (exact); the D layout holds a
// column of the tile per lane, which is the A-operand layout the adjoint
// product needs.  The Z operand is pre-split into bfloat16 planes, transposed
// and with rows permuted within groups of 32 to match that layout.
#include "common.h"
#include "kernels.h"
#include "storage.h"

namespace rpca {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

RPCA_DEV floatx16 mfma_bf16(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// round-to-nearest-even float -> bfloat16 bits
RPCA_DEV uint32_t bf16_rne(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// two floats that are exact in bfloat16 -> one packed dword (lo in bits 0..15)
RPCA_DEV uint32_t pack_bf16(float lo, float hi) {
  return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}

// eight e4m3 bytes -> eight bfloat16 (exact), element e from byte e
RPCA_DEV u32x4 fp8x8_to_bf16(uint32_t w0, uint32_t w1) {
  u32x4 r;
  floatx2 f = __builtin_amdgcn_cvt_pk_f32_fp8((int)w0, false);
  r.x = pack_bf16(f.x, f.y);
  f = __builtin_amdgcn_cvt_pk_f32_fp8((int)w0, true);
  r.y = pack_bf16(f.x, f.y);
  f = __builtin_amdgcn_cvt_pk_f32_fp8((int)w1, false);
  r.z = pack_bf16(f.x, f.y);
  f = __builtin_amdgcn_cvt_pk_f32_fp8((int)w1, true);
  r.w = pack_bf16(f.x, f.y);
  return r;
}

RPCA_DEV u32x4 ld16(const void* p) { return *reinterpret_cast<const u32x4*>(p); }

// keep the first `valid` 16-bit elements of a bf16x8 (0 <= valid <= 8)
RPCA_DEV u32x4 keep_bf16(u32x4 v, int valid) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int e = 2 * d;
    const uint32_t mk = (e + 1 < valid) ? 0xFFFFFFFFu : (e < valid ? 0x0000FFFFu : 0u);
    v[d] &= mk;
  }
  return v;
}

// keep the first `valid` bytes of 16 (0 <= valid <= 16)
RPCA_DEV u32x4 keep_u8(u32x4 v, int valid) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int e = 4 * d;
    const int k = valid - e;
    const uint32_t mk = k >= 4 ? 0xFFFFFFFFu : (k <= 0 ? 0u : (0xFFFFFFFFu >> (32 - 8 * k)));
    v[d] &= mk;
  }
  return v;
}

RPCA_DEV int64_t xcd_remap_lp(int64_t b, int64_t total) {
  const int64_t q = total / 8, r = total % 8;
  const int64_t x = b % 8, local = b / 8;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// ---------------------------------------------------------------------------
// operand preparation
// ---------------------------------------------------------------------------
// Xh/Xl[c][k] = hi/lo of (cs[k] * Xt[c][k]) for c < ncols, k < n; 0 elsewhere
// (c < cpad, k < ldxs).
__global__ __launch_bounds__(256) void split_x_kernel(const float* __restrict__ Xt, int64_t ldx, int64_t n,
                                                      int ncols, const float* __restrict__ cs,
                                                      uint16_t* __restrict__ Xh, uint16_t* __restrict__ Xl,
                                                      int64_t ldxs) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= ldxs) return;
  float x = 0.f;
  if (c < ncols && k < n) {
    x = Xt[(int64_t)c * ldx + k];
    if (cs != nullptr) x *= cs[k];
  }
  const uint32_t h = bf16_rne(x);
  const float r = x - __uint_as_float(h << 16);
  Xh[(int64_t)c * ldxs + k] = (uint16_t)h;
  Xl[(int64_t)c * ldxs + k] = (uint16_t)bf16_rne(r);
}

// Row permutation inside a group of 32 rows used by the adjoint: position
// p = 8 u + e (chunk u = 2 s + g, element e) holds row 16 s + 8 (e/4) + 4 g + e%4.
RPCA_DEV int zperm_row(int p) {
  const int u = p >> 3, e = p & 7;
  return 16 * (u >> 1) + 8 * (e >> 2) + 4 * (u & 1) + (e & 3);
}

// Zh/Zl[j][32 b + p] = hi/lo of Z[32 b + zperm_row(p)][j] (0 outside m x ncols)
__global__ __launch_bounds__(256) void split_zt_kernel(const float* __restrict__ Z, int64_t ldz, int64_t m,
                                                       int ncols, uint16_t* __restrict__ Zh,
                                                       uint16_t* __restrict__ Zl, int64_t ldzs) {
  __shared__ float tile[32][65];
  const int tid = threadIdx.x;
  const int64_t rb = (int64_t)blockIdx.x * 32;
  const int j0 = blockIdx.y * 64;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = tid + 256 * q;
    const int r = e >> 6, c = e & 63;
    float v = 0.f;
    if (rb + r < m && j0 + c < ncols) v = Z[(rb + r) * ldz + j0 + c];
    tile[r][c] = v;
  }
  __syncthreads();
  const int j = tid >> 2, u = tid & 3;
  u32x4 hv, lv;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    uint32_t hw = 0, lw = 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float x = tile[zperm_row(8 * u + 2 * d + t)][j];
      const uint32_t h = bf16_rne(x);
      const uint32_t lo = bf16_rne(x - __uint_as_float(h << 16));
      hw |= h << (16 * t);
      lw |= lo << (16 * t);
    }
    hv[d] = hw;
    lv[d] = lw;
  }
  const int64_t off = (int64_t)(j0 + j) * ldzs + rb + 8 * u;
  *reinterpret_cast<u32x4*>(Zh + off) = hv;
  *reinterpret_cast<u32x4*>(Zl + off) = lv;
}

// ---------------------------------------------------------------------------
// forward: a wave owns 64 rows (two 32-row tiles) x 64 columns (two tiles);
// a block of 4 waves 256 rows.  X hi/lo is staged per block in LDS, 64 K per
// stage, double buffered; A goes to registers, 16 bytes per lane per load.
// K offsets within a stage of the 8-entry group of MFMA step s, lane group g:
//   bf16 / hi+lo: 16 s + 8 g;   fp8: 32 (s/2) + 16 g + 8 (s%2)  (16-byte loads)
// ---------------------------------------------------------------------------
constexpr int LP_KST = 64;
constexpr int LP_XP = LP_KST + 8;  // LDS row of 72 bf16 (144 B)

template <int ST>
RPCA_DEV int lp_koff(int s, int g) {
  return ST == ST_FP8 ? 32 * (s >> 1) + 16 * g + 8 * (s & 1) : 16 * s + 8 * g;
}

template <int ST>
struct FwdStage {
  static constexpr int NL = ST == ST_FP8 ? 2 : (ST == ST_HILO ? 8 : 4);  // 16-byte loads per row tile
  u32x4 a[2][NL];
};

template <int ST>
__global__ __launch_bounds__(256, ST == ST_HILO ? 1 : 2) void fwd_lp_kernel(
    const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n, int64_t plane,
    const uint16_t* __restrict__ Xh, const uint16_t* __restrict__ Xl, int64_t ldxs, int ncols, int64_t kchunk,
    const float* __restrict__ corr, const double* __restrict__ alpha_ptr, float* __restrict__ Z, int64_t ldz,
    int64_t split_stride, int direct) {
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][2][64][LP_XP];  // [buffer][hi, lo][column][k]
  constexpr int ES = ST == ST_FP8 ? 1 : 2;  // bytes per stored element
  constexpr int NL = FwdStage<ST>::NL;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, g = lane >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 256 + wave * 64;
  const int sk = blockIdx.y;
  const int c0 = blockIdx.z * 64;
  const int64_t kbeg = (int64_t)sk * kchunk;
  const int64_t kend = kbeg + kchunk < n ? kbeg + kchunk : n;
  const unsigned char* __restrict__ arow[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int64_t r = r0 + 32 * rt + li;
    arow[rt] = reinterpret_cast<const unsigned char*>(Av) + (r < m ? r : m - 1) * lda * ES;
  }
  const int64_t plane_bytes = plane * ES;
  // cooperative X loader: chunk e = tid + 256 q -> plane e/512, column (e/8)%64, k 8 (e%8)
  const uint16_t* xsrc[4];
  int xdst[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    const int pl = e >> 9, col = (e >> 3) & 63, kq = e & 7;
    xsrc[q] = (pl ? Xl : Xh) + (int64_t)(c0 + col) * ldxs + 8 * kq;
    xdst[q] = ((pl * 64 + col) * LP_XP) + 8 * kq;
  }

  floatx16 acc[2][2], acc2[2][2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[rt][ct][v] = 0.f;
        acc2[rt][ct][v] = 0.f;
      }
  auto fold = [&]() {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        acc2[rt][ct] += acc[rt][ct];
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[rt][ct][v] = 0.f;
      }
  };
  // byte offset (within a row) of 16-byte load q of a stage at K position kb
  auto aoff = [&](int q, int64_t kb) -> int64_t {
    if (ST == ST_FP8) return kb + 32 * q + 16 * g;
    if (ST == ST_HILO) return (q & 4 ? plane_bytes : 0) + 2 * (kb + 16 * (q & 3) + 8 * g);
    return 2 * (kb + 16 * q + 8 * g);
  };
  // element index of the first entry of load q (for tail masking) and its length
  auto aelem = [&](int q, int64_t kb) -> int64_t {
    if (ST == ST_FP8) return kb + 32 * q + 16 * g;
    return kb + 16 * (q & 3) + 8 * g;
  };
  auto load_a = [&](FwdStage<ST>& b, int64_t kb) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = 0; q < NL; ++q) b.a[rt][q] = ld16(arow[rt] + aoff(q, kb));
  };
  auto load_a_tail = [&](FwdStage<ST>& b, int64_t kb) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int64_t e0 = aelem(q, kb);
        const int64_t valid = kend - e0;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (valid > 0) {
          v = ld16(arow[rt] + aoff(q, kb));
          if (ST == ST_FP8)
            v = keep_u8(v, valid < 16 ? (int)valid : 16);
          else
            v = keep_bf16(v, valid < 8 ? (int)valid : 8);
        }
        b.a[rt][q] = v;
      }
  };
  struct XStage {
    u32x4 x[4];
  };
  auto load_x = [&](XStage& b, int64_t kb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) b.x[q] = ld16(xsrc[q] + kb);
  };
  auto store_x = [&](const XStage& b, int buf) {
    uint16_t* base = &Xs[buf][0][0][0];
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<u32x4*>(base + xdst[q]) = b.x[q];
  };
  // A operand (bf16 bits) of row tile rt, MFMA step s; lo plane when LO
  auto a_op = [&](const FwdStage<ST>& b, int rt, int s, bool lo) -> u32x4 {
    if (ST == ST_FP8) {
      const u32x4 w = b.a[rt][s >> 1];
      return (s & 1) ? fp8x8_to_bf16(w.z, w.w) : fp8x8_to_bf16(w.x, w.y);
    }
    if (ST == ST_HILO) return b.a[rt][s + (lo ? 4 : 0)];
    return b.a[rt][s];
  };
  // One stage of MFMAs.  With REFILL, the registers of each A load are
  // reloaded from the next stage (K position kn) right after their last use,
  // so one register stage gives one stage of prefetch distance.
  auto compute = [&](FwdStage<ST>& b, int buf, bool refill, int64_t kn) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int ko = lp_koff<ST>(s, g);
      u32x4 xo[2][2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) xo[ct][hl] = ld16(&Xs[buf][hl][32 * ct + li][ko]);
      u32x4 a[2], al[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        a[rt] = a_op(b, rt, s, false);
        if (ST == ST_HILO) al[rt] = a_op(b, rt, s, true);
      }
      // hi parts for the four accumulators, then lo parts (independent chains back to back)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = mfma_bf16(a[rt], xo[ct][0], acc[rt][ct]);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = mfma_bf16(a[rt], xo[ct][1], acc[rt][ct]);
      if (ST == ST_HILO) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = mfma_bf16(al[rt], xo[ct][0], acc[rt][ct]);
      }
      if (refill) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          if (ST == ST_FP8) {
            if (s & 1) b.a[rt][s >> 1] = ld16(arow[rt] + aoff(s >> 1, kn));
          } else {
            b.a[rt][s] = ld16(arow[rt] + aoff(s, kn));
            if (ST == ST_HILO) b.a[rt][s + 4] = ld16(arow[rt] + aoff(s + 4, kn));
          }
        }
      }
    }
  };

  const int64_t nfull = (kend - kbeg) / LP_KST;
  int it = 0;
  FwdStage<ST> ac;
  if (nfull > 0) {
    XStage xr;
    load_x(xr, kbeg);
    load_a(ac, kbeg);
    store_x(xr, 0);
    __syncthreads();
    for (int64_t st = 0; st < nfull; ++st) {
      const int64_t kn = kbeg + (st + 1 < nfull ? st + 1 : st) * LP_KST;
      load_x(xr, kn);
      compute(ac, (int)(st & 1), true, kn);
      store_x(xr, (int)((st + 1) & 1));
      __syncthreads();
      if (++it == 2) {  // fold every 2 stages (128 K, 256 products per chain with hi + lo)
        it = 0;
        fold();
      }
    }
  }
  const int64_t kt = kbeg + nfull * LP_KST;
  if (kt < kend) {  // tail stage: X is zero-padded to a whole stage, A masked by column
    XStage xt;
    load_x(xt, kt);
    load_a_tail(ac, kt);
    store_x(xt, (int)(nfull & 1));
    __syncthreads();
    compute(ac, (int)(nfull & 1), false, kt);
  }
  fold();

  const double alpha = (direct && alpha_ptr != nullptr) ? *alpha_ptr : 1.0;
  float* __restrict__ Zs = Z + (direct ? 0 : (int64_t)sk * split_stride);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int c = c0 + 32 * ct + li;
    if (c >= ncols) continue;
    const double cr = (direct && corr != nullptr) ? (double)corr[c] : 0.0;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = r0 + 32 * rt + 8 * (v >> 2) + 4 * g + (v & 3);
        if (r < m) Zs[r * ldz + c] = direct ? (float)(alpha * ((double)acc2[rt][ct][v] - cr)) : acc2[rt][ct][v];
      }
  }
}

// Z[r][c] = alpha (sum_s P[s][r][c] - corr[c]) in float64, s in split order
__global__ __launch_bounds__(256) void fwd_lp_reduce_kernel(const float* __restrict__ P, int nsplit,
                                                            int64_t split_stride, int64_t ldp, int64_t m,
                                                            int ncols, const float* __restrict__ corr,
                                                            const double* __restrict__ alpha_ptr,
                                                            float* __restrict__ Z, int64_t ldz) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * ncols) return;
  const int64_t r = e / ncols;
  const int c = (int)(e % ncols);
  double v = 0.0;
  for (int s = 0; s < nsplit; ++s) v += (double)P[(int64_t)s * split_stride + r * ldp + c];
  const double alpha = alpha_ptr != nullptr ? *alpha_ptr : 1.0;
  const double cr = corr != nullptr ? (double)corr[c] : 0.0;
  Z[r * ldz + c] = (float)(alpha * (v - cr));
}

// ---------------------------------------------------------------------------
// adjoint: a wave owns 64 columns of A (two 32-column tiles) and 64 columns
// of Z (two tiles); a block of 4 waves 256 columns of A.  Rows of the split
// are walked 32 at a time; Z hi/lo for the stage is staged in LDS.
// Lane i + 32 g loads columns 16 g .. 16 g + 15 of its row within a tile;
// after the transposing MFMAs lane j + 32 h holds tile column
//   cmap(j) = 16 ((j % 16) / 8) + 8 (j / 16) + j % 8
// at rows 8 (v/4) + 4 h + v%4 (register v).
// ---------------------------------------------------------------------------
constexpr int LA_RS = 32;
constexpr int LA_ZP = LA_RS + 8;  // LDS row of 40 bf16 (80 B)

template <int ST>
struct AdjStage {
  static constexpr int NL = ST == ST_FP8 ? 1 : (ST == ST_HILO ? 4 : 2);  // 16-byte loads per tile
  u32x4 a[2][NL];
};

template <int ST>
__global__ __launch_bounds__(256, ST == ST_HILO ? 1 : 2) void adj_lp_kernel(
    const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n, int64_t plane,
    const uint16_t* __restrict__ Zh, const uint16_t* __restrict__ Zl, int64_t ldzs, int ncols,
    int64_t rows_per_split, int jtiles, int ctiles, int nsplit, float* __restrict__ P, int64_t ldp,
    int64_t split_stride) {
  __shared__ __attribute__((aligned(16))) uint16_t Zs[2][2][64][LA_ZP];  // [buffer][hi, lo][Z column][permuted row]
  constexpr int ES = ST == ST_FP8 ? 1 : 2;
  constexpr int NL = AdjStage<ST>::NL;
  const int64_t total = (int64_t)jtiles * ctiles * nsplit;
  const int64_t logical = xcd_remap_lp(blockIdx.x, total);
  const int jt = (int)(logical % jtiles);
  const int64_t rest = logical / jtiles;
  const int ct = (int)(rest % ctiles);
  const int sp = (int)(rest / ctiles);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, g = lane >> 5;
  const int64_t cw = (int64_t)ct * 256 + wave * 64;
  const int j0 = jt * 64;
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  const int64_t plane_bytes = plane * ES;

  // this lane's 16 columns of each tile: address (clamped to column 0 past n) and valid count
  int64_t coff[2];
  int cvalid[2];
#pragma unroll
  for (int at = 0; at < 2; ++at) {
    const int64_t c = cw + 32 * at + 16 * g;
    const int64_t v = n - c;
    cvalid[at] = v <= 0 ? 0 : (v >= 16 ? 16 : (int)v);
    coff[at] = (c < n ? c : 0) * ES;
  }
  // routing matrices of the transpose (bf16 1.0 = 0x3F80)
  u32x4 E1 = {0u, 0u, 0u, 0u}, E2 = {0u, 0u, 0u, 0u};
  {
    const int jj = li & 15, e = jj & 7;
    if ((jj >> 3) == g) {
      const uint32_t one = 0x3F80u << (16 * (e & 1));
      if (li < 16)
        E1[e >> 1] = one;
      else
        E2[e >> 1] = one;
    }
  }
  // cooperative Z loader: chunk e = tid + 256 q -> plane e/256, column (e/4)%64, rows 8 (e%4)
  const uint16_t* zsrc[2];
  int zdst[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + 256 * q;
    const int pl = e >> 8, col = (e >> 2) & 63, rq = e & 3;
    zsrc[q] = (pl ? Zl : Zh) + (int64_t)(j0 + col) * ldzs + 8 * rq;
    zdst[q] = (pl * 64 + col) * LA_ZP + 8 * rq;
  }

  floatx16 acc[2][2], acc2[2][2];
#pragma unroll
  for (int at = 0; at < 2; ++at)
#pragma unroll
    for (int zt = 0; zt < 2; ++zt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[at][zt][v] = 0.f;
        acc2[at][zt][v] = 0.f;
      }
  auto fold = [&]() {
#pragma unroll
    for (int at = 0; at < 2; ++at)
#pragma unroll
      for (int zt = 0; zt < 2; ++zt) {
        acc2[at][zt] += acc[at][zt];
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[at][zt][v] = 0.f;
      }
  };
  auto load_a = [&](AdjStage<ST>& b, int64_t rb) {
    const int64_t r = rb + li < m ? rb + li : m - 1;
    const unsigned char* base = reinterpret_cast<const unsigned char*>(Av) + r * lda * ES;
#pragma unroll
    for (int at = 0; at < 2; ++at) {
      const unsigned char* p = base + coff[at];
      if (ST == ST_FP8) {
        b.a[at][0] = ld16(p);
      } else {
        b.a[at][0] = ld16(p);
        b.a[at][1] = ld16(p + 16);
        if (ST == ST_HILO) {
          b.a[at][2] = ld16(p + plane_bytes);
          b.a[at][3] = ld16(p + plane_bytes + 16);
        }
      }
    }
  };
  struct ZStage {
    u32x4 z[2];
  };
  auto load_z = [&](ZStage& b, int64_t rb) {
#pragma unroll
    for (int q = 0; q < 2; ++q) b.z[q] = ld16(zsrc[q] + rb);
  };
  auto store_z = [&](const ZStage& b, int buf) {
    uint16_t* base = &Zs[buf][0][0][0];
#pragma unroll
    for (int q = 0; q < 2; ++q) *reinterpret_cast<u32x4*>(base + zdst[q]) = b.z[q];
  };
  // transposed operands (alpha: tile rows 0..15, beta: rows 16..31) of tile `at`
  auto transpose = [&](u32x4 t1, u32x4 t2, int valid, u32x4& oa, u32x4& ob) {
    t1 = keep_bf16(t1, valid < 8 ? valid : 8);
    t2 = keep_bf16(t2, valid > 8 ? valid - 8 : 0);
    floatx16 d;
#pragma unroll
    for (int v = 0; v < 16; ++v) d[v] = 0.f;
    d = mfma_bf16(t1, E1, d);
    d = mfma_bf16(t2, E2, d);
    oa = u32x4{pack_bf16(d[0], d[1]), pack_bf16(d[2], d[3]), pack_bf16(d[4], d[5]), pack_bf16(d[6], d[7])};
    ob = u32x4{pack_bf16(d[8], d[9]), pack_bf16(d[10], d[11]), pack_bf16(d[12], d[13]), pack_bf16(d[14], d[15])};
  };
  auto compute = [&](const AdjStage<ST>& b, int buf) {
    u32x4 oa[2], ob[2], la[2], lb[2];
#pragma unroll
    for (int at = 0; at < 2; ++at) {
      if (ST == ST_FP8) {
        const u32x4 w = b.a[at][0];
        transpose(fp8x8_to_bf16(w.x, w.y), fp8x8_to_bf16(w.z, w.w), cvalid[at], oa[at], ob[at]);
      } else {
        transpose(b.a[at][0], b.a[at][1], cvalid[at], oa[at], ob[at]);
        if (ST == ST_HILO) transpose(b.a[at][2], b.a[at][3], cvalid[at], la[at], lb[at]);
      }
    }
#pragma unroll
    for (int zt = 0; zt < 2; ++zt) {
      const u32x4 zah = ld16(&Zs[buf][0][32 * zt + li][8 * g]);
      const u32x4 zbh = ld16(&Zs[buf][0][32 * zt + li][16 + 8 * g]);
      const u32x4 zal = ld16(&Zs[buf][1][32 * zt + li][8 * g]);
      const u32x4 zbl = ld16(&Zs[buf][1][32 * zt + li][16 + 8 * g]);
#pragma unroll
      for (int at = 0; at < 2; ++at) {
        acc[at][zt] = mfma_bf16(oa[at], zah, acc[at][zt]);
        acc[at][zt] = mfma_bf16(oa[at], zal, acc[at][zt]);
        acc[at][zt] = mfma_bf16(ob[at], zbh, acc[at][zt]);
        acc[at][zt] = mfma_bf16(ob[at], zbl, acc[at][zt]);
        if (ST == ST_HILO) {
          acc[at][zt] = mfma_bf16(la[at], zah, acc[at][zt]);
          acc[at][zt] = mfma_bf16(lb[at], zbh, acc[at][zt]);
        }
      }
    }
  };

  // rows past m read row m-1 (finite) against zero Z rows
  const int64_t nst = (rend - rbeg + LA_RS - 1) / LA_RS;
  int it = 0;
  if (nst > 0) {
    AdjStage<ST> ac, an;
    ZStage zr;
    load_z(zr, rbeg);
    load_a(ac, rbeg);
    store_z(zr, 0);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
      const int64_t rn = rbeg + (st + 1 < nst ? st + 1 : st) * LA_RS;
      load_z(zr, rn);
      load_a(an, rn);
      __builtin_amdgcn_sched_barrier(0);
      compute(ac, (int)(st & 1));
      store_z(zr, (int)((st + 1) & 1));
      __syncthreads();
      ac = an;
      if (++it == 4) {  // fold every 4 stages (128 rows)
        it = 0;
        fold();
      }
    }
  }
  fold();

  float* __restrict__ Ps = P + (int64_t)sp * split_stride;
#pragma unroll
  for (int zt = 0; zt < 2; ++zt) {
    const int j = j0 + 32 * zt + li;
    if (j >= ncols) continue;
    float* __restrict__ prow = Ps + (int64_t)j * ldp;
#pragma unroll
    for (int at = 0; at < 2; ++at)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t c = cw + 32 * at + 16 * (q & 1) + 8 * (q >> 1) + 4 * g;
        const floatx4 o = {acc2[at][zt][4 * q], acc2[at][zt][4 * q + 1], acc2[at][zt][4 * q + 2],
                           acc2[at][zt][4 * q + 3]};
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
static bool lp_layout_ok(const void* A, int64_t lda) {
  return A != nullptr && (reinterpret_cast<uintptr_t>(A) & 15) == 0 && lda % 16 == 0;
}

hipError_t launch_split_x(const float* Xt, int64_t ldx, int64_t n, int ncols, const float* col_scale,
                          uint16_t* Xh, uint16_t* Xl, int64_t ldxs, int cpad, hipStream_t st) {
  if (ldxs % LP_KST != 0 || ldxs < n || cpad % 64 != 0 || cpad < ncols) return hipErrorInvalidValue;
  dim3 grid((unsigned)((ldxs + 255) / 256), (unsigned)cpad);
  hipLaunchKernelGGL(split_x_kernel, grid, dim3(256), 0, st, Xt, ldx, n, ncols, col_scale, Xh, Xl, ldxs);
  return hipGetLastError();
}

hipError_t launch_split_zt(const float* Z, int64_t ldz, int64_t m, int ncols, uint16_t* Zh, uint16_t* Zl,
                           int64_t ldzs, int cpad, hipStream_t st) {
  if (ldzs % LA_RS != 0 || ldzs < m || cpad % 64 != 0 || cpad < ncols) return hipErrorInvalidValue;
  dim3 grid((unsigned)(ldzs / 32), (unsigned)(cpad / 64));
  hipLaunchKernelGGL(split_zt_kernel, grid, dim3(256), 0, st, Z, ldz, m, ncols, Zh, Zl, ldzs);
  return hipGetLastError();
}

template <int ST>
static void launch_fwd_lp_t(const FwdArgs& a, dim3 grid, float* out, int64_t ldo, int64_t kchunk, bool direct,
                            hipStream_t st) {
  hipLaunchKernelGGL((fwd_lp_kernel<ST>), grid, dim3(256), 0, st, a.A, a.lda, a.m, a.n, a.plane, a.Xh, a.Xl,
                     a.ldxs, a.ncols, kchunk, a.corr, a.alpha, out, ldo, a.split_stride, direct ? 1 : 0);
}

hipError_t launch_fwd_lowp(int storage, const FwdArgs& a, hipStream_t st) {
  if (a.m <= 0 || a.ncols <= 0) return hipSuccess;
  if (!lp_layout_ok(a.A, a.lda) || a.Xh == nullptr || a.Xl == nullptr || a.Z == nullptr) return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldxs < a.n || a.ldxs % LP_KST != 0) return hipErrorInvalidValue;
  if (storage == ST_HILO && a.plane < a.m * a.lda) return hipErrorInvalidValue;
  const int ns = a.ksplit > 0 ? a.ksplit : 1;
  const int64_t kchunk = ns > 1 ? a.kchunk : a.n;
  if (ns > 1 && (a.P == nullptr || a.ldp < ((a.ncols + 63) / 64) * 64 || a.kchunk % LP_KST != 0 ||
                 (int64_t)ns * a.kchunk < a.n || a.split_stride < a.m * a.ldp))
    return hipErrorInvalidValue;
  const int ctiles = (a.ncols + 63) / 64;
  dim3 grid((unsigned)((a.m + 255) / 256), (unsigned)ns, (unsigned)ctiles);
  const bool direct = ns == 1;
  float* out = direct ? a.Z : a.P;
  const int64_t ldo = direct ? a.ldz : a.ldp;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  switch (storage) {
    case ST_BF16: launch_fwd_lp_t<ST_BF16>(a, grid, out, ldo, kchunk, direct, st); break;
    case ST_FP8: launch_fwd_lp_t<ST_FP8>(a, grid, out, ldo, kchunk, direct, st); break;
    case ST_HILO: launch_fwd_lp_t<ST_HILO>(a, grid, out, ldo, kchunk, direct, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  if (e != hipSuccess || direct) return e;
  const int64_t tot = a.m * a.ncols;
  hipLaunchKernelGGL(fwd_lp_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a.P, ns,
                     a.split_stride, a.ldp, a.m, a.ncols, a.corr, a.alpha, a.Z, a.ldz);
  return hipGetLastError();
}

template <int ST>
static void launch_adj_lp_t(const AdjArgs& a, int jtiles, int ctiles, hipStream_t st) {
  const int64_t total = (int64_t)jtiles * ctiles * a.nsplit;
  hipLaunchKernelGGL((adj_lp_kernel<ST>), dim3((unsigned)total), dim3(256), 0, st, a.A, a.lda, a.m, a.n, a.plane,
                     a.Zh, a.Zl, a.ldzs, a.ncols, a.rows_per_split, jtiles, ctiles, a.nsplit, a.P, a.ldp,
                     a.split_stride);
}

hipError_t launch_adj_lowp(int storage, const AdjArgs& a, hipStream_t st) {
  if (a.n <= 0 || a.ncols <= 0 || a.nsplit <= 0) return hipSuccess;
  if (!lp_layout_ok(a.A, a.lda) || a.Zh == nullptr || a.Zl == nullptr || a.P == nullptr)
    return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldp < a.n || a.rows_per_split % LA_RS != 0) return hipErrorInvalidValue;
  if ((int64_t)a.nsplit * a.rows_per_split < a.m || a.ldzs % LA_RS != 0 || a.ldzs < a.m)
    return hipErrorInvalidValue;
  if (storage == ST_HILO && a.plane < a.m * a.lda) return hipErrorInvalidValue;
  const int jtiles = (a.ncols + 63) / 64;
  const int ctiles = (int)((a.n + 255) / 256);
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  switch (storage) {
    case ST_BF16: launch_adj_lp_t<ST_BF16>(a, jtiles, ctiles, st); break;
    case ST_FP8: launch_adj_lp_t<ST_FP8>(a, jtiles, ctiles, st); break;
    case ST_HILO: launch_adj_lp_t<ST_HILO>(a, jtiles, ctiles, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  return e;
}

// K split for the low-precision forward product (256-row blocks, 64-K stages)
void fwd_split_lp(int64_t m, int64_t n, int64_t slots, int* ksplit, int64_t* kchunk) {
  const int64_t rt = (m + 255) / 256;
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= 8; ++s) {
    const int64_t chunk = ((n + s - 1) / s + LP_KST - 1) / LP_KST * LP_KST;
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
  const int64_t chunk = ((n + best - 1) / best + LP_KST - 1) / LP_KST * LP_KST;
  *ksplit = (int)((n + chunk - 1) / chunk);
  *kchunk = chunk;
}

// Row split of the low-precision adjoint (rows per split a multiple of 32)
void adj_split_lp(int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit, int64_t* rows_per_split) {
  const int64_t per = (int64_t)((ncols + 63) / 64) * ((n + 255) / 256);
  int64_t lo = (2 * slots + per - 1) / per;
  int64_t hi = lo * 4 + 8;
  const int64_t maxs = m / 128 > 0 ? m / 128 : 1;
  if (lo > maxs) lo = maxs;
  if (hi > maxs) hi = maxs;
  if (lo < 1) lo = 1;
  double best = -1.0;
  int64_t bs = 1, br = ((m + LA_RS - 1) / LA_RS) * LA_RS;
  for (int64_t s = lo; s <= hi; ++s) {
    const int64_t r = ((m + s - 1) / s + LA_RS - 1) / LA_RS * LA_RS;
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

}  // namespace rpca
