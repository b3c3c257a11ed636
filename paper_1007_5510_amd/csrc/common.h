// Shared device helpers for the gfx950 kernels of the PCA library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

#define RPCA_DEV __device__ __forceinline__

namespace rpca {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds over a 4-word counter with
// a 2-word key that is bumped by the two Weyl increments between rounds.
// The library uses it only to draw the Gaussian test matrix G of Step 1 when
// the caller does not pass one.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

RPCA_DEV U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 o;
    o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    o.y = (uint32_t)p1;
    o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    o.w = (uint32_t)p0;
    c = o;
  }
  return c;
}

// 53-bit uniform strictly inside (0,1) from two words: (k + 1/2) 2^-53.
RPCA_DEV double u53(uint32_t hi, uint32_t lo) {
  const uint64_t k = (uint64_t)(hi >> 5) * 67108864ull + (uint64_t)(lo >> 6);
  return ((double)k + 0.5) * 1.1102230246251565e-16;
}

// Standard normal for element e of `stream`: block e>>1, Box-Muller in double.
RPCA_DEV double normal_elem(uint64_t seed, uint32_t stream, uint64_t e) {
  const uint64_t b = e >> 1;
  U4 c{(uint32_t)b, (uint32_t)(b >> 32), stream, 0u};
  const U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = u53(x.x, x.y);
  const double u2 = u53(x.z, x.w);
  const double r = sqrt(-2.0 * log(u1));
  const double t = 6.283185307179586 * u2;
  return (e & 1) ? r * sin(t) : r * cos(t);
}

// ---------------------------------------------------------------------------
// wave64 reductions (DPP/permute via __shfl_xor)
// ---------------------------------------------------------------------------
// sum_{s < ns} p[s * stride] in float64, in order of s; the loads go out eight at a time
// (a plain loop waits for each load before the next add)
template <typename T>
RPCA_DEV double sum_strided(const T* __restrict__ p, int ns, int64_t stride) {
  double v = 0.0;
  for (int s = 0; s < ns; s += 8) {
    // the last batch re-reads entry ns - 1 in its unused slots (no branch around the
    // loads, which would make them wait one by one) and adds only the real entries
    T x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = p[(int64_t)(s + u < ns ? s + u : ns - 1) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s + u < ns) v += (double)x[u];
  }
  return v;
}

RPCA_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

RPCA_DEV float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

RPCA_DEV int lane_id() { return threadIdx.x & 63; }

}  // namespace rpca
