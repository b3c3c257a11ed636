// Element decoding for the stored formats of A (rpca_storage).
#pragma once

#include "common.h"

namespace rpca {

enum { ST_F32 = 0, ST_BF16 = 1, ST_FP8 = 2, ST_HILO = 3 };

RPCA_DEV float bf16_bits_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// OCP FP8 E4M3: sign, 4 exponent bits (bias 7), 3 mantissa bits, no
// infinities, S.1111.111 is NaN.  Every e4m3 value is exact in bfloat16/float.
RPCA_DEV float e4m3_to_f32(uint8_t q) {
  const uint32_t s = (q >> 7) & 1u, e = (q >> 3) & 15u, mt = q & 7u;
  float v;
  if (e == 0u)
    v = (float)mt * 0.001953125f;  // mt/8 * 2^-6
  else if (e == 15u && mt == 7u)
    v = __uint_as_float(0x7fc00000u);
  else
    v = __uint_as_float(((e + 120u) << 23) | (mt << 20));  // (1 + mt/8) 2^(e-7)
  return s ? -v : v;
}

template <int ST>
RPCA_DEV float load_elem(const void* __restrict__ X, int64_t idx, int64_t plane) {
  if (ST == ST_F32) return reinterpret_cast<const float*>(X)[idx];
  if (ST == ST_BF16) return bf16_bits_to_f32(reinterpret_cast<const uint16_t*>(X)[idx]);
  if (ST == ST_FP8) return e4m3_to_f32(reinterpret_cast<const uint8_t*>(X)[idx]);
  const uint16_t* h = reinterpret_cast<const uint16_t*>(X);
  return bf16_bits_to_f32(h[idx]) + bf16_bits_to_f32(h[idx + plane]);
}

}  // namespace rpca
