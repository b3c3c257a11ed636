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

// Zh/Zl[j][32 b + p] = hi/lo of Z[32 b + zperm_row(p)][j] (0 outside m x ncols);
// with `ones`, column ncols is an implicit column of ones (its product gives the
// column sums of A)
__global__ __launch_bounds__(256) void split_zt_kernel(const float* __restrict__ Z, int64_t ldz, int64_t m,
                                                       int ncols, int ones, uint16_t* __restrict__ Zh,
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
    if (rb + r < m && ones && j0 + c == ncols) v = 1.f;
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
// Pipelining (both kernels).  The A data a wave multiplies is its own: it
// goes from global memory straight into VGPRs (buffer loads whose range ends
// with the matrix) through a ring of DA stages held in registers, so DA - 1
// stages are in flight per wave without LDS traffic.  The float operand (X,
// or Z hi/lo in the adjoint) is shared by the workgroup: it goes from global
// memory into LDS (global_load_lds_dwordx4: lane l's 16 bytes land at
// M0 + 16 l) through a ring of DX stages, stored with the 16-byte chunk index
// XOR-swizzled by the column (chunk c of column j at position c ^ (j & 7)),
// which makes the column-strided 16-byte operand reads conflict-free.  Every
// wave issues, per stage, its shared-operand loads and then its A loads (the
// order pinned by scheduling barriers, every address clamped into range), so
// a counted s_waitcnt vmcnt means "this wave's shared-operand loads of the
// stage have landed"; a plain s_barrier after it makes all waves' loads
// visible.  The loads are issued without branches (a branch around loads
// makes the compiler wait for all of them where the paths join), and the
// split sizes are whole rings, so only the last split has a partial ring.
// No __syncthreads (its fence would wait for every load).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef const __attribute__((address_space(1))) void* gbl_ptr_t;

RPCA_DEV void dma16(const void* g, void* lds) {
  __builtin_amdgcn_global_load_lds((gbl_ptr_t)g, (lds_ptr_t)lds, 16, 0, 0);
}

// s_waitcnt immediate (gfx9 encoding): vmcnt <= vm, lgkmcnt <= lgkm, expcnt not waited
constexpr int waitcnt_imm(int vm, int lgkm) {
  return (vm & 15) | ((vm >> 4) << 14) | (7 << 4) | ((lgkm & 15) << 8);
}

// swizzled byte offset of 16-byte chunk c of column j (128-byte rows)
RPCA_DEV int swz(int j, int c) { return j * 128 + 16 * (c ^ (j & 7)); }

// ---------------------------------------------------------------------------
// forward: stage = 64 K = 4 MFMA steps.
// K offsets within a stage of the 8-entry group of MFMA step s, lane group g:
//   bf16 / hi+lo: 16 s + 8 g;   fp8: 32 (s/2) + 16 g + 8 (s%2)  (16-byte loads)
// ---------------------------------------------------------------------------
constexpr int LP_KST = 64;

template <int ST>
RPCA_DEV int lp_koff(int s, int g) {
  return ST == ST_FP8 ? 32 * (s >> 1) + 16 * g + 8 * (s & 1) : 16 * s + 8 * g;
}

// forward: a wave owns RT x 32 rows x 64 columns (RT row tiles share every X operand read);
// a workgroup of W waves 32 RT W rows shares one X stage, so X traffic per byte of A falls
// with RT.  A goes global -> VGPRs through a ring of DA stages (buffer loads, branch-free);
// X goes global -> LDS (global_load_lds) through a ring of DX stages.  Per stage every wave
// issues its XQ X loads and then its A loads, in that order (scheduling barriers pin it), so
// "X of stage t has landed" is a counted wait.
template <int ST>
struct LpFwdCfg {
  static constexpr int ES = ST == ST_FP8 ? 1 : 2;
  static constexpr int W = 8;
  static constexpr int RT = ST == ST_HILO ? 1 : 2;
  static constexpr int AQ1 = ST == ST_FP8 ? 2 : (ST == ST_HILO ? 8 : 4);  // 16-byte A loads per lane per row tile
  static constexpr int AQ = RT * AQ1;
  static constexpr int DA = ST == ST_FP8 ? 4 : (ST == ST_HILO ? 3 : 2);
  static constexpr int DX = 3 < DA ? 3 : DA;
  static constexpr int XQ = 16 / W;
  static constexpr int P = AQ + XQ;
  static constexpr int SX = 16384;
  static constexpr int LDS = DX * SX;
  static constexpr int ROWS = 32 * RT * W;
  static constexpr int XWAIT = AQ + (DX - 2) * P;  // loads younger than X of the stage being computed
  static_assert(XWAIT < 64, "vmcnt range");
  static_assert(DA >= DX && DX >= 2, "the prologue issues X of stage 0 only when DA >= DX");
};

template <int ST>
__global__ __launch_bounds__(512, 1) void fwd_lp_kernel(
    const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n, int64_t plane,
    const uint16_t* __restrict__ Xh, const uint16_t* __restrict__ Xl, int64_t ldxs, int ncols, int64_t kchunk,
    const float* __restrict__ corr, const double* __restrict__ alpha_ptr, float* __restrict__ Z, int64_t ldz,
    int64_t split_stride, int direct) {
  using C = LpFwdCfg<ST>;
  constexpr int ES = C::ES, W = C::W, RT = C::RT, AQ1 = C::AQ1, AQ = C::AQ, DA = C::DA, DX = C::DX, XQ = C::XQ,
                SX = C::SX;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 31, g = lane >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * C::ROWS + wave * (32 * RT);
  const int sk = blockIdx.y;
  const int c0 = blockIdx.z * 64;
  const int64_t kbeg = (int64_t)sk * kchunk;
  const int64_t kend = kbeg + kchunk < n ? kbeg + kchunk : n;
  const int64_t plane_bytes = plane * ES;
  // A through buffer loads: the wave's first row (clamped) is the base; lane offsets hold the
  // row (clamped to m - 1) and 16 g bytes; the stage's K offset is a scalar.  The range ends
  // with the matrix, so loads past it return zeros.
  const int64_t rb = r0 < m ? r0 : m - 1;
  const unsigned char* abase = reinterpret_cast<const unsigned char*>(Av) + rb * lda * ES;
  const int64_t arange = (m - rb) * lda * ES;
  const int nrec = arange < 0x7FFFFFFF ? (int)arange : 0x7FFFFFFF;
  const __amdgpu_buffer_rsrc_t rs_hi = __builtin_amdgcn_make_buffer_rsrc((void*)abase, (short)0, nrec, 0x00020000);
  const __amdgpu_buffer_rsrc_t rs_lo =
      __builtin_amdgcn_make_buffer_rsrc((void*)(abase + plane_bytes), (short)0, nrec, 0x00020000);
  int voff[RT];
  const unsigned char* arow[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = r0 + 32 * rt + li;
    const int64_t rc = row < m ? row : m - 1;
    voff[rt] = (int)((rc - rb) * lda * ES) + 16 * g;
    arow[rt] = reinterpret_cast<const unsigned char*>(Av) + rc * lda * ES;
  }

  const uint16_t* xsrc[XQ];
#pragma unroll
  for (int q = 0; q < XQ; ++q) {
    const int j = wave * XQ + q;
    const int col = 8 * (j & 7) + (lane >> 3);
    const int c = (lane & 7) ^ (col & 7);
    xsrc[q] = ((j >> 3) ? Xl : Xh) + (int64_t)(c0 + col) * ldxs + 8 * c;
  }
  auto aoff = [&](int q, int64_t kb) -> int64_t {
    if (ST == ST_FP8) return kb + 32 * q + 16 * g;
    if (ST == ST_HILO) return (q & 4 ? plane_bytes : 0) + 2 * (kb + 16 * (q & 3) + 8 * g);
    return 2 * (kb + 16 * q + 8 * g);
  };
  auto aelem = [&](int q, int64_t kb) -> int64_t {
    if (ST == ST_FP8) return kb + 32 * q + 16 * g;
    return kb + 16 * (q & 3) + 8 * g;
  };

  const int64_t nfull = (kend - kbeg) / LP_KST;
  const int64_t kt = kbeg + nfull * LP_KST;
  const bool tail = kt < kend;
  const int64_t nst = nfull + (tail ? 1 : 0);
  auto issue_x = [&](int64_t t) {
    if (t < 0) return;
    const int64_t tx = t < nst ? t : nst - 1;
    unsigned char* xs = lds + (int)(t % DX) * SX;
    const int64_t kbx = kbeg + tx * LP_KST;
#pragma unroll
    for (int q = 0; q < XQ; ++q) dma16(xsrc[q] + kbx, xs + 1024 * (wave * XQ + q));
  };
  // branch-free (a branch around loads makes the compiler wait for every load at the join);
  // with no full stage the loads read the split's first 64 K of the rows (never used)
  auto issue_a = [&](int64_t t, u32x4 (&dst)[AQ]) {
    const int64_t ta = t < nfull ? t : nfull - 1;
    const int kbs = (int)((kbeg + (ta > 0 ? ta : 0) * LP_KST) * ES);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < AQ1; ++q)
        dst[rt * AQ1 + q] = __builtin_bit_cast(
            u32x4, __builtin_amdgcn_raw_buffer_load_b128((q & 4) && ST == ST_HILO ? rs_lo : rs_hi, voff[rt],
                                                         kbs + 32 * (q & 3), 0));
  };

  // one float32 chain per output over the split (the MFMA sums 16 exact products per step)
  floatx16 acc[RT][2];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[rt][ct][v] = 0.f;
  auto read_x = [&](u32x4 (&xo)[2][2], const unsigned char* xs, int s) {
    const int c = lp_koff<ST>(s, g) >> 3;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int hl = 0; hl < 2; ++hl) xo[ct][hl] = ld16(xs + hl * 8192 + swz(32 * ct + li, c));
  };
  // A operands (hi, lo) of row tile rt, step s; `masked` keeps only entries with K < kend
  auto a_op = [&](const u32x4 (&ar)[AQ], int rt, int s, int64_t kb, bool masked, u32x4& ah, u32x4& al) {
    if (ST == ST_FP8) {
      u32x4 w = ar[rt * AQ1 + (s >> 1)];
      if (masked) {
        const int64_t valid = kend - aelem(s >> 1, kb);
        w = keep_u8(w, valid <= 0 ? 0 : (valid >= 16 ? 16 : (int)valid));
      }
      ah = (s & 1) ? fp8x8_to_bf16(w.z, w.w) : fp8x8_to_bf16(w.x, w.y);
    } else {
      ah = ar[rt * AQ1 + s];
      if (ST == ST_HILO) al = ar[rt * AQ1 + s + 4];
      if (masked) {
        const int64_t valid = kend - aelem(s, kb);
        const int v = valid <= 0 ? 0 : (valid >= 8 ? 8 : (int)valid);
        ah = keep_bf16(ah, v);
        if (ST == ST_HILO) al = keep_bf16(al, v);
      }
    }
  };
  auto compute = [&](const unsigned char* xs, const u32x4 (&ar)[AQ], int64_t kb, bool masked) {
    u32x4 xo[2][2], xn[2][2];
    read_x(xo, xs, 0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < 3) read_x(xn, xs, s + 1);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        u32x4 ah, al;
        a_op(ar, rt, s, kb, masked, ah, al);
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = mfma_bf16(ah, xo[ct][hl], acc[rt][ct]);
        if (ST == ST_HILO) {
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = mfma_bf16(al, xo[ct][0], acc[rt][ct]);
        }
      }
      if (s < 3) {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int hl = 0; hl < 2; ++hl) xo[ct][hl] = xn[ct][hl];
      }
    }
  };
  auto stage_sync = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(C::XWAIT, 0));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };
  auto issue = [&](int64_t t_x, int64_t t_a, u32x4 (&dst)[AQ]) {
    issue_x(t_x);
    __builtin_amdgcn_sched_barrier(0);
    issue_a(t_a, dst);
    __builtin_amdgcn_sched_barrier(0);
  };

  u32x4 ar[DA][AQ];
  // prologue: virtual iterations v = -(DA-1) .. -1 issue X(v + DX - 1) (when >= 0) and A(v + DA - 1)
  if (nst > 0) {
#pragma unroll
    for (int v = -(DA - 1); v < 0; ++v) issue(v + DX - 1, v + DA - 1, ar[v + DA - 1]);
  }
  int64_t t = 0;
  for (; t + DA <= nfull; t += DA) {
#pragma unroll
    for (int u = 0; u < DA; ++u) {
      stage_sync();
      issue(t + u + DX - 1, t + u + DA - 1, ar[(u + DA - 1) % DA]);
      compute(lds + (int)((t + u) % DX) * SX, ar[u], 0, false);
    }
  }
#pragma unroll
  for (int u = 0; u < DA; ++u) {
    if (t + u < nfull) {
      stage_sync();
      issue(t + u + DX - 1, t + u + DA - 1, ar[(u + DA - 1) % DA]);
      compute(lds + (int)((t + u) % DX) * SX, ar[u], 0, false);
    }
  }
  __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));
  if (tail) {
    __builtin_amdgcn_s_barrier();
    u32x4 at[AQ];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < AQ1; ++q) {
        const int64_t valid = kend - aelem(q, kt);
        u32x4 v = {0u, 0u, 0u, 0u};
        if (valid > 0) v = ld16(arow[rt] + aoff(q, kt));
        at[rt * AQ1 + q] = v;
      }
    compute(lds + (int)(nfull % DX) * SX, at, kt, true);
  }

  const double alpha = (direct && alpha_ptr != nullptr) ? *alpha_ptr : 1.0;
  float* __restrict__ Zs = Z + (direct ? 0 : (int64_t)sk * split_stride);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int c = c0 + 32 * ct + li;
      if (c >= ncols) continue;
      const double cr = (direct && corr != nullptr) ? (double)corr[c] : 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = r0 + 32 * rt + 8 * (v >> 2) + 4 * g + (v & 3);
        const float a2 = acc[rt][ct][v];
        if (r < m) Zs[r * ldz + c] = direct ? (float)(alpha * ((double)a2 - cr)) : a2;
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
  v += sum_strided(P + r * ldp + c, nsplit, split_stride);
  const double alpha = alpha_ptr != nullptr ? *alpha_ptr : 1.0;
  const double cr = corr != nullptr ? (double)corr[c] : 0.0;
  Z[r * ldz + c] = (float)(alpha * (v - cr));
}

// ---------------------------------------------------------------------------
// adjoint: a wave owns 32 CT columns of A (CT tiles: 2 for the power steps,
// where the two tiles share every Z operand read, 1 for a wide Z) and 32 ZT
// columns of Z (ZT tiles: 2 for the power steps, 6 for a wide Z such as the T
// pass, so that A is read once for up to 192 Z columns); a workgroup of W
// waves 32 CT W columns of A.  Stage = 64 rows (two 32-row halves).  Lane
// i + 32 g loads columns 16 g .. 16 g + 15 of row i of a half and tile;
// after the transposing MFMAs lane j + 32 h holds tile column
//   cmap(j) = 16 ((j % 16) / 8) + 8 (j / 16) + j % 8
// at rows 8 (v/4) + 4 h + v%4 (register v) of the half.  The Z planes hold
// rows permuted within 32-row groups so that the 8-row chunk 4 h + 2 s + g of
// a stage is the B operand of half h, step s (alpha 0, beta 1), lane group g.
// ---------------------------------------------------------------------------
constexpr int LA_RS = 64;

// Z tiles per wave for a product with ncols columns of Z
constexpr int lp_zt(int ncols) { return ncols > 64 ? 6 : 2; }
template <int ST, int ZT>
struct LpAdjCfg {
  static constexpr int ES = ST == ST_FP8 ? 1 : 2;
  static constexpr int W = 8;
  static constexpr int CT = ZT == 2 && ST != ST_HILO ? 2 : 1;   // 32-column tiles of A per wave
  static constexpr int HQ = ST == ST_FP8 ? 1 : (ST == ST_HILO ? 4 : 2);  // A loads per lane per 32-row half and tile
  static constexpr int AQ = 2 * CT * HQ;
  static constexpr int COLS = 32 * CT * W;
  static constexpr int DA = ZT == 2 ? (ST == ST_HILO ? 2 : (ST == ST_FP8 ? 3 : 2))
                                    : (ST == ST_HILO ? 2 : 4);
  static constexpr int DZ0 = ZT == 2 ? 4 : 3;
  static constexpr int DZ = DZ0 < DA ? DZ0 : DA;
  static constexpr int SX = ZT * 8192;              // Z bytes per stage (2 planes x 32 ZT x 64 rows)
  static constexpr int XQ = 8 * ZT / W;             // Z loads per lane per stage
  static constexpr int P = AQ + XQ;
  static constexpr int LDS = DZ * SX;
  static constexpr int XWAIT = AQ + (DZ - 2) * P;
  static_assert((8 * ZT) % W == 0, "Z loads must divide evenly over the waves");
  static_assert(LDS <= 163840, "ring exceeds the LDS of a workgroup");
  static_assert(DZ >= 2 && XWAIT < 64, "ring depth");
};

template <int ST, int ZT>
__global__ __launch_bounds__(512, 1) void adj_lp_kernel(
    const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n, int64_t plane,
    const uint16_t* __restrict__ Zh, const uint16_t* __restrict__ Zl, int64_t ldzs, int ncols,
    int64_t rows_per_split, int jtiles, int ctiles, int nsplit, float* __restrict__ P, int64_t ldp,
    int64_t split_stride) {
  using D = LpAdjCfg<ST, ZT>;
  constexpr int ES = D::ES, W = D::W, CT = D::CT, HQ = D::HQ, AQ = D::AQ, DA = D::DA, DZ = D::DZ, XQ = D::XQ, SX = D::SX;
  constexpr int ZPL = SX / 2;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int64_t total = (int64_t)jtiles * ctiles * nsplit;
  const int64_t logical = xcd_remap_lp(blockIdx.x, total);
  const int jt = (int)(logical % jtiles);
  const int64_t rest = logical / jtiles;
  const int ct = (int)(rest % ctiles);
  const int sp = (int)(rest / ctiles);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 31, g = lane >> 5;
  const int64_t cw = (int64_t)ct * D::COLS + wave * (32 * CT);
  const int j0 = jt * 32 * ZT;
  const int64_t rbeg = (int64_t)sp * rows_per_split;
  const int64_t rend = rbeg + rows_per_split < m ? rbeg + rows_per_split : m;
  const int64_t plane_bytes = plane * ES;

  int cvalid[CT], coff[CT];
#pragma unroll
  for (int c2 = 0; c2 < CT; ++c2) {
    const int64_t cA = cw + 32 * c2 + 16 * g;
    cvalid[c2] = n - cA <= 0 ? 0 : (n - cA >= 16 ? 16 : (int)(n - cA));
    coff[c2] = (int)((cA < n ? cA : 0) * ES);
  }
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
  const uint16_t* zsrc[XQ];
#pragma unroll
  for (int q = 0; q < XQ; ++q) {
    const int j = wave * XQ + q;
    const int col = 8 * (j % (4 * ZT)) + (lane >> 3);
    const int c = (lane & 7) ^ (col & 7);
    zsrc[q] = ((j / (4 * ZT)) ? Zl : Zh) + (int64_t)(j0 + col) * ldzs + 8 * c;
  }
  const int64_t nfull = rend > rbeg ? (rend - rbeg + LA_RS - 1) / LA_RS : 0;
  auto issue_z = [&](int64_t t) {
    if (t < 0) return;
    const int64_t tc = t < nfull ? t : nfull - 1;
    const int64_t rb = rbeg + tc * LA_RS;
    unsigned char* zs = lds + (int)(t % DZ) * SX;
#pragma unroll
    for (int q = 0; q < XQ; ++q) dma16(zsrc[q] + rb, zs + 1024 * (wave * XQ + q));
  };
  // rows past m read row m - 1 (finite) against zero Z rows
  auto issue_a = [&](int64_t t, u32x4 (&dst)[AQ]) {
    const int64_t tc = t < nfull ? t : nfull - 1;
    const int64_t rb = rbeg + tc * LA_RS;
    const unsigned char* base = reinterpret_cast<const unsigned char*>(Av) + rb * lda * ES;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7FFFFFFF, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsl =
        __builtin_amdgcn_make_buffer_rsrc((void*)(base + plane_bytes), (short)0, 0x7FFFFFFF, 0x00020000);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r = rb + 32 * h + li;
      const int vr = (int)(((r < m ? r : m - 1) - rb) * lda * ES);
#pragma unroll
      for (int c2 = 0; c2 < CT; ++c2)
#pragma unroll
        for (int e = 0; e < HQ; ++e)
          dst[(h * CT + c2) * HQ + e] = __builtin_bit_cast(
              u32x4, __builtin_amdgcn_raw_buffer_load_b128(ST == ST_HILO && e >= 2 ? rsl : rs, vr + coff[c2],
                                                           16 * (e & 1), 0));
    }
  };

  // one float32 chain per output over the row split
  floatx16 acc[CT][ZT];
#pragma unroll
  for (int c2 = 0; c2 < CT; ++c2)
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[c2][zt][v] = 0.f;
  auto transpose = [&](u32x4 t1, u32x4 t2, int cv, u32x4& oa, u32x4& ob) {
    t1 = keep_bf16(t1, cv < 8 ? cv : 8);
    t2 = keep_bf16(t2, cv > 8 ? cv - 8 : 0);
    floatx16 d;
#pragma unroll
    for (int v = 0; v < 16; ++v) d[v] = 0.f;
    d = mfma_bf16(t1, E1, d);
    d = mfma_bf16(t2, E2, d);
    oa = u32x4{pack_bf16(d[0], d[1]), pack_bf16(d[2], d[3]), pack_bf16(d[4], d[5]), pack_bf16(d[6], d[7])};
    ob = u32x4{pack_bf16(d[8], d[9]), pack_bf16(d[10], d[11]), pack_bf16(d[12], d[13]), pack_bf16(d[14], d[15])};
  };
  auto tr_half = [&](const u32x4 (&ar)[AQ], int h, int c2, u32x4& oa, u32x4& ob, u32x4& la, u32x4& lb) {
    const int b = (h * CT + c2) * HQ;
    if (ST == ST_FP8) {
      const u32x4 w = ar[b];
      transpose(fp8x8_to_bf16(w.x, w.y), fp8x8_to_bf16(w.z, w.w), cvalid[c2], oa, ob);
    } else {
      transpose(ar[b], ar[b + 1], cvalid[c2], oa, ob);
      if (ST == ST_HILO) transpose(ar[b + 2], ar[b + 3], cvalid[c2], la, lb);
    }
  };
  auto compute = [&](const unsigned char* zs, const u32x4 (&ar)[AQ]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4 oa[CT], ob[CT], la[CT], lb[CT];
#pragma unroll
      for (int c2 = 0; c2 < CT; ++c2) tr_half(ar, h, c2, oa[c2], ob[c2], la[c2], lb[c2]);
#pragma unroll
      for (int zt = 0; zt < ZT; ++zt) {
        const int col = 32 * zt + li;
        const u32x4 zah = ld16(zs + swz(col, 4 * h + g));
        const u32x4 zbh = ld16(zs + swz(col, 4 * h + 2 + g));
        const u32x4 zal = ld16(zs + ZPL + swz(col, 4 * h + g));
        const u32x4 zbl = ld16(zs + ZPL + swz(col, 4 * h + 2 + g));
#pragma unroll
        for (int c2 = 0; c2 < CT; ++c2) {
          acc[c2][zt] = mfma_bf16(oa[c2], zah, acc[c2][zt]);
          acc[c2][zt] = mfma_bf16(ob[c2], zbh, acc[c2][zt]);
          acc[c2][zt] = mfma_bf16(oa[c2], zal, acc[c2][zt]);
          acc[c2][zt] = mfma_bf16(ob[c2], zbl, acc[c2][zt]);
          if (ST == ST_HILO) {
            acc[c2][zt] = mfma_bf16(la[c2], zah, acc[c2][zt]);
            acc[c2][zt] = mfma_bf16(lb[c2], zbh, acc[c2][zt]);
          }
        }
      }
    }
  };
  auto stage_sync = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(D::XWAIT, 0));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };
  auto issue = [&](int64_t tz, int64_t ta, u32x4 (&dst)[AQ]) {
    issue_z(tz);
    __builtin_amdgcn_sched_barrier(0);
    issue_a(ta, dst);
    __builtin_amdgcn_sched_barrier(0);
  };

  u32x4 ar[DA][AQ];
  if (nfull > 0) {
#pragma unroll
    for (int v = -(DA - 1); v < 0; ++v) issue(v + DZ - 1, v + DA - 1, ar[v + DA - 1]);
  }
  int64_t t = 0;
  for (; t + DA <= nfull; t += DA) {
#pragma unroll
    for (int u = 0; u < DA; ++u) {
      stage_sync();
      issue(t + u + DZ - 1, t + u + DA - 1, ar[(u + DA - 1) % DA]);
      compute(lds + (int)((t + u) % DZ) * SX, ar[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < DA; ++u) {
    if (t + u < nfull) {
      stage_sync();
      issue(t + u + DZ - 1, t + u + DA - 1, ar[(u + DA - 1) % DA]);
      compute(lds + (int)((t + u) % DZ) * SX, ar[u]);
    }
  }
  __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));  // no load in flight at exit

  float* __restrict__ Ps = P + (int64_t)sp * split_stride;
#pragma unroll
  for (int c2 = 0; c2 < CT; ++c2)
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) {
    const int j = j0 + 32 * zt + li;
    if (j >= ncols) continue;
    float* __restrict__ prow = Ps + (int64_t)j * ldp;
    const floatx16& r = acc[c2][zt];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t c = cw + 32 * c2 + 16 * (q & 1) + 8 * (q >> 1) + 4 * g;
      const floatx4 o = {r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]};
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
                           int64_t ldzs, int cpad, hipStream_t st, bool ones) {
  if (ldzs % 32 != 0 || ldzs < m || cpad % 64 != 0 || cpad < ncols + (ones ? 1 : 0)) return hipErrorInvalidValue;
  dim3 grid((unsigned)(ldzs / 32), (unsigned)(cpad / 64));
  hipLaunchKernelGGL(split_zt_kernel, grid, dim3(256), 0, st, Z, ldz, m, ncols, ones ? 1 : 0, Zh, Zl, ldzs);
  return hipGetLastError();
}

template <int ST>
static void launch_fwd_lp_t(const FwdArgs& a, int ns, int ctiles, float* out, int64_t ldo, int64_t kchunk,
                            bool direct, hipStream_t st) {
  using C = LpFwdCfg<ST>;
  dim3 grid((unsigned)((a.m + C::ROWS - 1) / C::ROWS), (unsigned)ns, (unsigned)ctiles);
  hipLaunchKernelGGL((fwd_lp_kernel<ST>), grid, dim3(64 * C::W), C::LDS, st, a.A, a.lda, a.m, a.n, a.plane, a.Xh,
                     a.Xl, a.ldxs, a.ncols, kchunk, a.corr, a.alpha, out, ldo, a.split_stride, direct ? 1 : 0);
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
  const bool direct = ns == 1;
  float* out = direct ? a.Z : a.P;
  const int64_t ldo = direct ? a.ldz : a.ldp;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  switch (storage) {
    case ST_BF16: launch_fwd_lp_t<ST_BF16>(a, ns, ctiles, out, ldo, kchunk, direct, st); break;
    case ST_FP8: launch_fwd_lp_t<ST_FP8>(a, ns, ctiles, out, ldo, kchunk, direct, st); break;
    case ST_HILO: launch_fwd_lp_t<ST_HILO>(a, ns, ctiles, out, ldo, kchunk, direct, st); break;
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

template <int ST, int ZT>
static void launch_adj_lp_t(const AdjArgs& a, int jtiles, hipStream_t st) {
  using D = LpAdjCfg<ST, ZT>;
  const int ctiles = (int)((a.n + D::COLS - 1) / D::COLS);
  const int64_t total = (int64_t)jtiles * ctiles * a.nsplit;
  constexpr size_t lds = D::LDS;
  hipLaunchKernelGGL((adj_lp_kernel<ST, ZT>), dim3((unsigned)total), dim3(64 * D::W), lds, st,
                     a.A, a.lda, a.m, a.n, a.plane, a.Zh, a.Zl, a.ldzs, a.ncols, a.rows_per_split, jtiles, ctiles,
                     a.nsplit, a.P, a.ldp, a.split_stride);
}

hipError_t launch_adj_lowp(int storage, const AdjArgs& a, hipStream_t st) {
  if (a.n <= 0 || a.ncols <= 0 || a.nsplit <= 0) return hipSuccess;
  if (!lp_layout_ok(a.A, a.lda) || a.Zh == nullptr || a.Zl == nullptr || a.P == nullptr)
    return hipErrorInvalidValue;
  if (a.lda < a.n || a.ldp < a.n || a.rows_per_split % LA_RS != 0) return hipErrorInvalidValue;
  if ((int64_t)a.nsplit * a.rows_per_split < a.m || a.ldzs % LA_RS != 0 || a.ldzs < a.m)
    return hipErrorInvalidValue;
  if (storage == ST_HILO && a.plane < a.m * a.lda) return hipErrorInvalidValue;
  const int zt = lp_zt(a.ncols);
  const int jtiles = (a.ncols + 32 * zt - 1) / (32 * zt);
  // the Z planes must hold every column the tiles read
  if (a.cpad_z < jtiles * 32 * zt) return hipErrorInvalidValue;
  if (a.ev_begin != nullptr) (void)hipEventRecord(a.ev_begin, st);
  switch (storage * 8 + zt) {
    case ST_BF16 * 8 + 2: launch_adj_lp_t<ST_BF16, 2>(a, jtiles, st); break;
    case ST_BF16 * 8 + 6: launch_adj_lp_t<ST_BF16, 6>(a, jtiles, st); break;
    case ST_FP8 * 8 + 2: launch_adj_lp_t<ST_FP8, 2>(a, jtiles, st); break;
    case ST_FP8 * 8 + 6: launch_adj_lp_t<ST_FP8, 6>(a, jtiles, st); break;
    case ST_HILO * 8 + 2: launch_adj_lp_t<ST_HILO, 2>(a, jtiles, st); break;
    case ST_HILO * 8 + 6: launch_adj_lp_t<ST_HILO, 6>(a, jtiles, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (a.ev_end != nullptr) (void)hipEventRecord(a.ev_end, st);
  return e;
}


// K split for the low-precision forward product (32 W-row workgroups, 64-K stages;
// slots = workgroups resident at once, one per CU)
static int64_t fwd_gran(int storage) {
  const int da = storage == ST_FP8 ? LpFwdCfg<ST_FP8>::DA : (storage == ST_HILO ? LpFwdCfg<ST_HILO>::DA : LpFwdCfg<ST_BF16>::DA);
  return (int64_t)LP_KST * da;
}

void fwd_split_lp(int storage, int64_t m, int64_t n, int64_t slots, int* ksplit, int64_t* kchunk) {
  const int64_t rows = storage == ST_FP8 ? LpFwdCfg<ST_FP8>::ROWS : (storage == ST_HILO ? LpFwdCfg<ST_HILO>::ROWS : LpFwdCfg<ST_BF16>::ROWS);
  const int64_t rt = (m + rows - 1) / rows;
  const int64_t gran = fwd_gran(storage);  // whole register rings per split
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= 8; ++s) {
    const int64_t chunk = ((n + s - 1) / s + gran - 1) / gran * gran;
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
  const int64_t chunk = ((n + best - 1) / best + gran - 1) / gran * gran;
  *ksplit = (int)((n + chunk - 1) / chunk);
  *kchunk = chunk;
}

// Row split of the low-precision adjoint (rows per split a multiple of 64)
void adj_split_lp(int storage, int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit,
                  int64_t* rows_per_split) {
  const int ztc = 32 * lp_zt(ncols);
  const int64_t cols = lp_zt(ncols) == 2 ? (storage == ST_FP8 ? LpAdjCfg<ST_FP8, 2>::COLS : (storage == ST_HILO ? LpAdjCfg<ST_HILO, 2>::COLS : LpAdjCfg<ST_BF16, 2>::COLS))
                                         : (storage == ST_FP8 ? LpAdjCfg<ST_FP8, 6>::COLS : (storage == ST_HILO ? LpAdjCfg<ST_HILO, 6>::COLS : LpAdjCfg<ST_BF16, 6>::COLS));
  const int64_t per = (int64_t)((ncols + ztc - 1) / ztc) * ((n + cols - 1) / cols);
  int64_t lo = (2 * slots + per - 1) / per;
  int64_t hi = lo * 4 + 8;
  const int64_t maxs = m / 128 > 0 ? m / 128 : 1;
  if (lo > maxs) lo = maxs;
  if (hi > maxs) hi = maxs;
  if (lo < 1) lo = 1;
  double best = -1.0;
  const int zt = lp_zt(ncols);
  const int da = zt == 2 ? (storage == ST_FP8 ? LpAdjCfg<ST_FP8, 2>::DA : (storage == ST_HILO ? LpAdjCfg<ST_HILO, 2>::DA : LpAdjCfg<ST_BF16, 2>::DA))
                         : (storage == ST_FP8 ? LpAdjCfg<ST_FP8, 6>::DA : (storage == ST_HILO ? LpAdjCfg<ST_HILO, 6>::DA : LpAdjCfg<ST_BF16, 6>::DA));
  const int64_t gran = (int64_t)LA_RS * da;  // whole register rings per split
  int64_t bs = 1, br = ((m + gran - 1) / gran) * gran;
  for (int64_t s = lo; s <= hi; ++s) {
    const int64_t r = ((m + s - 1) / s + gran - 1) / gran * gran;
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
