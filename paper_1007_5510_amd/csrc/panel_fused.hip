// One power step of Step 1 (eqs. second_prod .. last_prod) on a single read of
// the float32 data matrix:
//
//   Z   = alpha ((A - 1 s^T) X - 1 corr^T)          (the block H^(j), m x c)
//   P_q = rows of (A - 1 s^T)^T Z over row segment q (the adjoint partial sums;
//         with `ones`, row c of P_q holds the column sums of A - 1 s^T)
//
// Section 4.1 asks that every contribution of a row of A be made while that row
// is at hand.  Here a row block A_b (16 rows) is read from HBM once: its
// forward product Z_b = A_b X needs all n columns, so the columns are split over
// the 32 compute units of one XCD (each holds its column slice of X and of the
// adjoint accumulator Y in registers for the whole launch), the per-CU partial
// sums of Z_b are combined through the XCD's L2, and each CU then applies
// A_b^T Z_b to its own slice of A_b, kept in LDS since the forward product.
//
// Launch: cooperative, one workgroup of four waves per CU.  Each workgroup reads
// its XCD id from the hardware register, registers as the next member of that
// XCD's group, and after a one-time grid barrier knows its group (row range),
// member index (column range) and the group size.  Group g takes rows
// [g R_g, (g+1) R_g) in blocks of 16; member c takes 16-column tiles
// [c T / G, (c+1) T / G) of the T = ceil(n/16) tiles, wave w ten of them.
//
// Per row block b, software pipelined two blocks deep (iteration t does the
// forward product of block t and the adjoint of block t-2):
//   forward   Zp = X_c^T (A_b,c - s)^T on v_mfma_f32_16x16x4_f32 (X^T as the A
//             operand, four consecutive columns of a row of A per lane as the B
//             operand), the four waves' sums added in LDS, the member's partial
//             (64 x 16 floats) stored to the group's exchange buffer; the shifted
//             A slice is stored transposed in LDS for the adjoint;
//   barrier 1 (all partials of block b stored);
//   reduce    member c sums its 1/G share of the 1024 entries over the G
//             partials in float64 (fixed order), applies alpha and corr, writes
//             those entries of Z to H and to the group's reduced buffer;
//   barrier 2 (all shares of block b written);
//   adjoint   every member loads the reduced Z_b (plus a ones column in pass 0),
//             Y_c += (A_b,c - s)^T Z_b from LDS on the same MFMA.
// A counter per barrier kind and slot (b mod 4) counts arrivals; arrivals are
// L2 atomics of the XCD and the spins are bounded (a timeout sets an error flag
// and every later wait gives up, so the launch always drains).  Y_c leaves the
// registers as the partial sums P_q of a row segment (at most 8192 rows, one
// float32 chain each), reduced afterwards in float64 in a fixed order with the
// other groups' segments, as the two-launch path does with its row splits.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace rpca {

namespace {

constexpr int FU_R = 16;        // rows per block
constexpr int FU_WAVES = 4;     // waves per workgroup (one per SIMD)
constexpr int FU_TILES = 5;     // 16-column tiles per wave (80 columns)
constexpr int FU_SKEW_RS = 2;   // block reduced in iteration t: t - 2
constexpr int FU_SKEW_ADJ = 4;  // block whose adjoint runs in iteration t: t - 4
constexpr int FU_SLOTS = FU_SKEW_ADJ + 1;  // LDS slots of transposed A
constexpr int FU_D = 8;         // exchange-buffer and counter slots
constexpr int FU_BLK = 1024;    // entries of one block's Z (64 x 16)
constexpr int FU_ZP = 20;       // LDS row pitch of Z^T (floats)
constexpr unsigned FU_SPIN = 1u << 24;

typedef float floatx4_t __attribute__((ext_vector_type(4)));

RPCA_DEV floatx4_t mfma4x4(float a, float b, floatx4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

RPCA_DEV float pick4(const floatx4_t& v, int q) {
  const float a = (q & 1) ? v.y : v.x;
  const float b = (q & 1) ? v.w : v.z;
  return (q & 2) ? b : a;
}

// ----------------------------------------------------------------- exchange primitives
// Everything shared between workgroups (partials, reduced Z, counters) is
// accessed only through agent-scope atomics, which the device keeps coherent
// (they bypass the CU's L1 and are served at the device coherence level).  A
// writer's stores are complete (s_waitcnt) and the workgroup has met at a
// barrier before one thread counts the arrival; a reader issues its loads only
// after the count was seen and the workgroup has met again.

RPCA_DEV void xstore4(float* p, floatx4_t v) {
  __hip_atomic_store(p + 0, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 2, v.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 3, v.w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

RPCA_DEV void xstore1(float* p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

RPCA_DEV floatx4_t xload4(const float* p) {
  floatx4_t v;
  v.x = __hip_atomic_load(p + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.z = __hip_atomic_load(p + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.w = __hip_atomic_load(p + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

RPCA_DEV float xload1(const float* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

RPCA_DEV void xarrive(unsigned* ctr) { __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// spin (bounded) until *ctr >= target; returns false after a timeout or when
// another workgroup has flagged one
RPCA_DEV bool xwait(unsigned* ctr, unsigned target, unsigned* err) {
  unsigned it = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    if (++it > FU_SPIN) {
      __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// barrier of the whole grid (agent scope), used once for the group set-up
RPCA_DEV void grid_barrier_once(unsigned* ctr, unsigned target, unsigned* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned it = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it > FU_SPIN) {
        __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

}  // namespace

// ws layout (unsigned words): [0, 16*16) registration counters per XCD (stride 16),
// [256] grid barrier, [257] error flag, [258], [259] groups and group size seen
// (diagnostics), [512 + (g*2 + kind)*FU_D*16 + slot*16] barrier counters of group g.
// xpart: [16 groups][FU_D][gsize][1024] floats; xred: [16][FU_D][1024] floats.
template <bool VEC>
__global__ __launch_bounds__(256, 1) void fused_power_f32_kernel(
    const float* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ shift,
    const float* __restrict__ Xt, int64_t ldx, int ncols, int ones, const float* __restrict__ corr,
    const double* __restrict__ alpha_ptr, float* __restrict__ Z, int64_t ldz, float* __restrict__ P, int64_t ldp,
    int64_t split_stride, int ngroups_expect, int xcc_per_group, int cu_per_xcc, int64_t rows_per_group, int nseg,
    int64_t seg_rows, unsigned* ws, float* xpart, float* xred) {
  __shared__ __attribute__((aligned(16))) float s_at[FU_SLOTS][FU_WAVES][FU_TILES * 16 * FU_R];
  __shared__ __attribute__((aligned(16))) float s_red[FU_WAVES][FU_BLK];
  __shared__ __attribute__((aligned(16))) float s_zt[64 * FU_ZP];
  __shared__ __attribute__((aligned(16))) float s_sh[FU_WAVES][FU_TILES * 16];
  __shared__ unsigned s_info[4];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int j16 = lane & 15, kk = lane >> 4;
  unsigned* err = ws + 257;

  // ---- group set-up: XCD id from the hardware register, member index by registration
  if (tid == 0) {
    const unsigned x = __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & 15u;
    const unsigned idx = __hip_atomic_fetch_add(ws + x * 16, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_info[0] = x;
    s_info[1] = idx;
  }
  grid_barrier_once(ws + 256, gridDim.x, err);
  if (tid == 0) {
    const unsigned x = s_info[0];
    int nx = 0, rank = 0;
    bool ok = s_info[1] < (unsigned)cu_per_xcc;
    for (unsigned q = 0; q < 16; ++q) {
      const unsigned c = __hip_atomic_load(ws + q * 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c == 0) continue;
      if ((int)c != cu_per_xcc) ok = false;
      if (q < x) ++rank;
      ++nx;
    }
    if (nx != ngroups_expect * xcc_per_group) ok = false;
    if (!ok) __hip_atomic_fetch_or(err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_info[2] = (unsigned)(rank / xcc_per_group);                                       // group
    s_info[1] = (unsigned)((rank % xcc_per_group) * cu_per_xcc) + s_info[1];           // member
    s_info[3] = ok ? 1u : 0u;
    if (blockIdx.x == 0) {
      ws[258] = (unsigned)nx;
      ws[259] = __hip_atomic_load(ws + x * 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  if (s_info[3] == 0u) return;
  const int G = xcc_per_group * cu_per_xcc;
  const int member = (int)s_info[1];
  const int grp = (int)s_info[2];

  // rows of the group, columns of the member and of this wave
  const int64_t g_r0 = (int64_t)grp * rows_per_group;
  const int64_t g_r1 = g_r0 + rows_per_group < m ? g_r0 + rows_per_group : m;
  const int64_t g_rows = g_r1 > g_r0 ? g_r1 - g_r0 : 0;
  const int nblk = (int)((g_rows + FU_R - 1) / FU_R);
  const int64_t ntile = (n + 15) / 16;
  const int64_t tb = (int64_t)member * ntile / G, te = (int64_t)(member + 1) * ntile / G;
  const int64_t wt0 = tb + (int64_t)wave * FU_TILES;
  const int64_t col0 = wt0 * 16;  // first column of this wave's slice

  unsigned* ctr1 = ws + 512 + (grp * 2 + 0) * FU_D * 16;
  unsigned* ctr2 = ws + 512 + (grp * 2 + 1) * FU_D * 16;
  float* xp_g = xpart + (size_t)grp * FU_D * G * FU_BLK;
  float* xr_g = xred + (size_t)grp * FU_D * FU_BLK;

  // ---- stationary operands: X^T slice (A operand of the forward MFMA) and the shift
  // xr[mt][kt] holds X^T[16 mt + j16][col0 + 16 kt + 4 kk + 0..3]
  floatx4_t xr[4][FU_TILES];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int lr = mt * 16 + j16;
#pragma unroll
    for (int kt = 0; kt < FU_TILES; ++kt) {
      floatx4_t v = {0.f, 0.f, 0.f, 0.f};
      const int64_t c = col0 + kt * 16 + kk * 4;
      if (lr < ncols && wt0 + kt < te) {
        const float* p = Xt + (int64_t)lr * ldx;
        if (c < n) v.x = p[c];
        if (c + 1 < n) v.y = p[c + 1];
        if (c + 2 < n) v.z = p[c + 2];
        if (c + 3 < n) v.w = p[c + 3];
      }
      xr[mt][kt] = v;
    }
  }
  for (int q = lane; q < FU_TILES * 16; q += 64) {
    const int64_t c = col0 + q;
    s_sh[wave][q] = (shift != nullptr && c < n && wt0 + q / 16 < te) ? shift[c] : 0.f;
  }

  floatx4_t yacc[FU_TILES][4];
#pragma unroll
  for (int nt = 0; nt < FU_TILES; ++nt)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) yacc[nt][mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};

  // A loads of one block: lane (j16, kk) gets row r0 + j16, columns col0 + 16 kt + 4 kk + 0..3
  floatx4_t acur[FU_TILES];
  auto load_block = [&](int b) {
    const int64_t row = g_r0 + (int64_t)b * FU_R + j16;
    const bool rin = row < g_r1;
    const float* __restrict__ ar = A + (rin ? row : g_r0) * lda;
#pragma unroll
    for (int kt = 0; kt < FU_TILES; ++kt) {
      const int64_t c = col0 + kt * 16 + kk * 4;
      floatx4_t v = {0.f, 0.f, 0.f, 0.f};
      if (rin && wt0 + kt < te) {
        if (VEC && c + 3 < n) {
          v = __builtin_nontemporal_load(reinterpret_cast<const floatx4_t*>(ar + c));
        } else {
          if (c < n) v.x = ar[c];
          if (c + 1 < n) v.y = ar[c + 1];
          if (c + 2 < n) v.z = ar[c + 2];
          if (c + 3 < n) v.w = ar[c + 3];
        }
      }
      acur[kt] = v;
    }
  };

  auto target = [&](int b) { return (unsigned)G * (unsigned)(b / FU_D + 1); };

  // Y^T of a finished row segment -> P[grp * nseg + sg] (rows ncols (+1), this wave's columns)
  const int nrows_p = ncols + (ones ? 1 : 0);
  auto flush = [&](int sg) {
    // lane (j16, kk) holds Y^T[16 mt + 4 kk + v][16 nt + j16] in yacc[nt][mt][v]
    float* __restrict__ dst = P + (int64_t)(grp * nseg + sg) * split_stride + (int64_t)(4 * kk) * ldp + col0 + j16;
    const int ldp32 = (int)ldp;
    const int rows_here = nrows_p - 4 * kk;
    const int64_t cend = (te - wt0) * 16 < n - col0 ? (te - wt0) * 16 : n - col0;
    const int cols_here = (int)cend - j16;
#pragma unroll
    for (int nt = 0; nt < FU_TILES; ++nt) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (nt * 16 < cols_here && mt * 16 + v < rows_here) dst[(mt * 16 + v) * ldp32 + nt * 16] = yacc[nt][mt][v];
        }
        yacc[nt][mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
      }
    }
  };

  if (nblk > 0) load_block(0);
  int cur_seg = 0;
  bool alive = true;

  // reduce-scatter share of a member: entries [member*E, member*E + E), E = 1024 / G;
  // thread -> (entry tid / TPE, partial subset tid % TPE), TPE = 256 / E threads per entry
  const int E = FU_BLK / G;
  const int TPE = 256 / E;
  const int PPT = G / TPE;  // partials per thread (4 for G = 32 or 64)
  const int rs_entry = member * E + tid / TPE;
  const int rs_sub = tid % TPE;

  for (int it = 0; it < nblk + FU_SKEW_ADJ; ++it) {
    const int bf = it, brs = it - FU_SKEW_RS, bg = it - FU_SKEW_ADJ;
    const bool do_f = bf < nblk, do_rs = brs >= 0 && brs < nblk, do_g = bg >= 0 && bg < nblk;

    // ---- (1) forward product of block bf, first half of the tiles
    floatx4_t zacc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) zacc[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    auto fwd_tiles = [&](auto k0c, auto k1c) {
      constexpr int k0 = decltype(k0c)::value, k1 = decltype(k1c)::value;
      const int64_t row = g_r0 + (int64_t)bf * FU_R + j16;
#pragma unroll
      for (int kt = k0; kt < k1; ++kt) {
        const floatx4_t s4 = *reinterpret_cast<const floatx4_t*>(&s_sh[wave][kt * 16 + kk * 4]);
        floatx4_t a = acur[kt] - s4;
        if (row >= g_r1) a = floatx4_t{0.f, 0.f, 0.f, 0.f};
        acur[kt] = a;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) zacc[mt] = mfma4x4(xr[mt][kt][t], a[t], zacc[mt]);
      }
    };
    if (do_f) fwd_tiles(std::integral_constant<int, 0>{}, std::integral_constant<int, FU_TILES / 2>{});

    // ---- (2) waits for the partials of block brs and the reduced Z of block bg; loads issued
    if (tid == 0 && alive) {
      if (do_rs) alive = xwait(ctr1 + (brs % FU_D) * 16, target(brs), err);
      if (alive && do_g) alive = xwait(ctr2 + (bg % FU_D) * 16, target(bg), err);
    }
    __syncthreads();
    float rsv[4] = {0.f, 0.f, 0.f, 0.f};
    floatx4_t zg = {0.f, 0.f, 0.f, 0.f};
    if (do_rs) {
      const float* src = xp_g + (size_t)(brs % FU_D) * G * FU_BLK;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < PPT) rsv[q] = xload1(src + (size_t)(rs_sub * PPT + q) * FU_BLK + rs_entry);
    }
    if (do_g) zg = xload4(xr_g + (size_t)(bg % FU_D) * FU_BLK + tid * 4);

    // ---- (3) forward product, second half
    if (do_f) fwd_tiles(std::integral_constant<int, FU_TILES / 2>{}, std::integral_constant<int, FU_TILES>{});

    // ---- (4) forward partial to LDS, shifted A transposed into its slot, next block's A in flight
    if (do_f) {
      *reinterpret_cast<floatx4_t*>(&s_red[wave][lane * 16 + 0]) = zacc[0];
      *reinterpret_cast<floatx4_t*>(&s_red[wave][lane * 16 + 4]) = zacc[1];
      *reinterpret_cast<floatx4_t*>(&s_red[wave][lane * 16 + 8]) = zacc[2];
      *reinterpret_cast<floatx4_t*>(&s_red[wave][lane * 16 + 12]) = zacc[3];
      float* at = s_at[bf % FU_SLOTS][wave];
      // element (column c = 16 kt + 4 kk + t, row j16) at c*16 + ((j16/4) ^ kk)*4 + j16%4;
      // write instruction tw stores t = (tw + kk) % 4 so the four lane groups hit different banks
#pragma unroll
      for (int kt = 0; kt < FU_TILES; ++kt) {
#pragma unroll
        for (int tw = 0; tw < 4; ++tw) {
          const int t = (tw + kk) & 3;
          const int c = kt * 16 + kk * 4 + t;
          at[c * 16 + (((j16 >> 2) ^ kk) << 2) + (j16 & 3)] = pick4(acur[kt], t);
        }
      }
      if (bf + 1 < nblk) load_block(bf + 1);
    }
    // ---- (5) reduce-scatter of block brs: float64 sum of the G partials of the member's entries
    if (do_rs) {
      double rs_sum = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < PPT) rs_sum += (double)rsv[q];
      // the TPE threads of an entry are consecutive lanes of one wave (TPE a power of two <= 16)
      for (int off = 1; off < TPE; off <<= 1) rs_sum += __shfl_xor(rs_sum, off, 64);
      if (rs_sub == 0) {
        // entry e = lane' * 16 + mt * 4 + v of the wave-lane layout: Z^T[16 mt + 4 (lane'/16) + v][lane' % 16]
        const int e = rs_entry;
        const int ln = e >> 4, mt = (e >> 2) & 3, v = e & 3;
        const int lrow = mt * 16 + 4 * (ln >> 4) + v;
        const int r = ln & 15;
        const int64_t row = g_r0 + (int64_t)brs * FU_R + r;
        float zval = 0.f;
        if (row < g_r1) {
          if (lrow < ncols) {
            const double alpha = alpha_ptr != nullptr ? *alpha_ptr : 1.0;
            const double cr = corr != nullptr ? (double)corr[lrow] : 0.0;
            zval = (float)(alpha * (rs_sum - cr));
            Z[row * ldz + lrow] = zval;
          } else if (ones && lrow == ncols) {
            zval = 1.f;
          }
        }
        xstore1(xr_g + (size_t)(brs % FU_D) * FU_BLK + e, zval);
      }
    }
    // gathered Z of block bg into LDS as Z^T[lrow][row] (pitch FU_ZP)
    if (do_g) {
      const int ln = tid >> 2, mt = tid & 3;
      const int r = ln & 15, lr0 = mt * 16 + 4 * (ln >> 4);
      s_zt[(lr0 + 0) * FU_ZP + r] = zg.x;
      s_zt[(lr0 + 1) * FU_ZP + r] = zg.y;
      s_zt[(lr0 + 2) * FU_ZP + r] = zg.z;
      s_zt[(lr0 + 3) * FU_ZP + r] = zg.w;
    }
    __syncthreads();
    // ---- (6) member partial of block bf: the four waves' sums in fixed order
    if (do_f) {
      floatx4_t s = *reinterpret_cast<const floatx4_t*>(&s_red[0][tid * 4]);
#pragma unroll
      for (int w = 1; w < FU_WAVES; ++w) s += *reinterpret_cast<const floatx4_t*>(&s_red[w][tid * 4]);
      xstore4(xp_g + ((size_t)(bf % FU_D) * G + member) * FU_BLK + tid * 4, s);
    }

    // ---- (7) adjoint of block bg: Y^T += Z_b^T (A_b - s) on the slice of this wave
    if (do_g) {
      const int seg = (int)(((int64_t)bg * FU_R) / seg_rows);
      while (cur_seg < seg) flush(cur_seg++);
      floatx4_t zf[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) zf[mt] = *reinterpret_cast<const floatx4_t*>(&s_zt[(mt * 16 + j16) * FU_ZP + kk * 4]);
      const float* at = s_at[bg % FU_SLOTS][wave];
#pragma unroll
      for (int nt = 0; nt < FU_TILES; ++nt) {
        const int c = nt * 16 + j16;
        const floatx4_t bv = *reinterpret_cast<const floatx4_t*>(&at[c * 16 + ((kk ^ ((c >> 2) & 3)) << 2)]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) yacc[nt][mt] = mfma4x4(zf[mt][t], bv[t], yacc[nt][mt]);
      }
    }

    // ---- (8) stores complete, arrivals counted
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      if (do_f) xarrive(ctr1 + (bf % FU_D) * 16);
      if (do_rs) xarrive(ctr2 + (brs % FU_D) * 16);
    }
  }
  while (cur_seg < nseg) flush(cur_seg++);
}

// Workspace words of the exchange (counters) and floats of the exchange buffers.
size_t fused_ws_words() { return 512 + 16 * 2 * FU_D * 16; }
size_t fused_xpart_floats(int gsize) { return (size_t)16 * FU_D * gsize * FU_BLK; }
size_t fused_xred_floats() { return (size_t)16 * FU_D * FU_BLK; }
int fused_max_tiles_per_member() { return FU_WAVES * FU_TILES; }

// Can the fused power step take this problem on a device of `ngroups` XCDs with
// `gsize` compute units each?  (Columns: at most 40 tiles of 16 per member.)
bool fused_fits(int64_t n, int ncols, bool ones, int ngroups, int gsize) {
  if (gsize != 32 && gsize != 64) return false;
  if (ngroups < 1 || ngroups > 16) return false;
  if (ncols + (ones ? 1 : 0) > 64) return false;
  const int64_t ntile = (n + 15) / 16;
  return (ntile + gsize - 1) / gsize <= FU_WAVES * FU_TILES && n >= 16 * gsize;
}

hipError_t launch_fused_f32(const FusedArgs& a, hipStream_t st) {
  if (a.xcc_per_group * a.cu_per_xcc != a.gsize ||
      !fused_fits(a.n, a.ncols, a.ones, a.ngroups, a.gsize) || a.ws == nullptr || a.xpart == nullptr ||
      a.xred == nullptr || a.nseg < 1 || a.seg_rows < FU_R || a.seg_rows % FU_R != 0)
    return hipErrorInvalidValue;
  const int64_t rpg = a.rows_per_group;
  if (rpg % FU_R != 0 || rpg * a.ngroups < a.m || (int64_t)a.nseg * a.seg_rows < rpg) return hipErrorInvalidValue;
  hipError_t e = launch_fill_u32(a.ws, (int64_t)fused_ws_words(), 0u, st);
  if (e != hipSuccess) return e;
  const float* A = static_cast<const float*>(a.A);
  int64_t lda = a.lda, m = a.m, n = a.n, ldx = a.ldx, ldz = a.ldz, ldp = a.ldp, ss = a.split_stride;
  int64_t seg_rows = a.seg_rows;
  const float* shift = a.shift;
  const float* Xt = a.Xt;
  int ncols = a.ncols, ones = a.ones ? 1 : 0, nge = a.ngroups, xpg = a.xcc_per_group, cpx = a.cu_per_xcc,
      nseg = a.nseg;
  const float* corr = a.corr;
  const double* alpha = a.alpha;
  float* Z = a.Z;
  float* P = a.P;
  unsigned* ws = a.ws;
  float* xpart = a.xpart;
  float* xred = a.xred;
  void* args[] = {&A, &lda, &m, &n, &shift, &Xt, &ldx, &ncols, &ones, &corr, &alpha, &Z, &ldz, &P, &ldp, &ss,
                  &nge, &xpg, &cpx, const_cast<int64_t*>(&rpg), &nseg, &seg_rows, &ws, &xpart, &xred};
  if (a.ev_begin != nullptr) {
    e = hipEventRecord(a.ev_begin, st);
    if (e != hipSuccess) return e;
  }
  const void* fn = a.vec ? reinterpret_cast<const void*>(&fused_power_f32_kernel<true>)
                         : reinterpret_cast<const void*>(&fused_power_f32_kernel<false>);
  e = hipLaunchCooperativeKernel(fn, dim3((unsigned)(a.ngroups * a.gsize)), dim3(256), args, 0, st);
  if (e != hipSuccess) return e;
  if (a.ev_end != nullptr) e = hipEventRecord(a.ev_end, st);
  return e;
}

}  // namespace rpca
