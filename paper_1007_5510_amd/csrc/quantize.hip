// Conversion of a float32 matrix into the stored formats of A:
//   bfloat16: round to nearest, ties to even;
//   hi + lo:  hi = bf16(a), lo = bf16(a - hi) (a - hi is exact in float32);
//   FP8 e4m3 (OCP: bias 7, subnormals, no infinities, max 448): per-column
//            scale c = max |a| / 448 (1 for a zero column), code = e4m3(a / c)
//            rounded to nearest, ties to even, saturated at +-448.
// An optional per-column shift s is subtracted first (float32), so that data
// with large column means keeps its spread in the stored bits; the centred
// factorisation of the stored matrix is then that of the centred data.
#include "common.h"
#include "kernels.h"
#include "storage.h"

namespace rpca {

RPCA_DEV uint32_t q_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

RPCA_DEV uint32_t q_e4m3(float x) {
  const float a = fminf(fabsf(x), 448.f);
  uint32_t code;
  if (a < 0.015625f) {  // below 2^-6: subnormal grid of step 2^-9 (8 = first normal)
    code = (uint32_t)rintf(a * 512.f);
  } else {
    const int e = (int)((__float_as_uint(a) >> 23) & 255u) - 127;  // -6 .. 8
    const uint32_t mq = (uint32_t)rintf(ldexpf(a, 3 - e));          // 8 .. 16 (16 carries)
    code = ((uint32_t)(e + 7) << 3) + (mq - 8u);
  }
  if (x < 0.f && code != 0u) code |= 0x80u;
  return code;
}

// part[s][c] = max over rows of split s of |A[r][c] - shift[c]|
__global__ __launch_bounds__(256) void colmax_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                     const float* __restrict__ shift, int64_t rps,
                                                     float* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (c >= n) return;
  const float sh = shift != nullptr ? shift[c] : 0.f;
  const int64_t r0 = (int64_t)s * rps;
  const int64_t r1 = r0 + rps < m ? r0 + rps : m;
  float mx = 0.f;
  for (int64_t r = r0; r < r1; ++r) mx = fmaxf(mx, fabsf(A[r * lda + c] - sh));
  part[(int64_t)s * n + c] = mx;
}

__global__ __launch_bounds__(256) void colscale_kernel(const float* __restrict__ part, int nsplit, int64_t n,
                                                       float* __restrict__ cs) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  float mx = 0.f;
  for (int s = 0; s < nsplit; ++s) mx = fmaxf(mx, part[(int64_t)s * n + c]);
  cs[c] = mx > 0.f ? mx / 448.f : 1.f;
}

// 16 rows per thread at one column; columns n .. ldo-1 are written as zero
template <int ST>
__global__ __launch_bounds__(256) void quantize_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                       const float* __restrict__ shift, void* __restrict__ out,
                                                       int64_t ldo, const float* __restrict__ cs) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= ldo) return;
  const bool in = c < n;
  const float sh = (in && shift != nullptr) ? shift[c] : 0.f;
  const float sc = (ST == ST_FP8 && in) ? cs[c] : 1.f;
  for (int64_t rb = (int64_t)blockIdx.y * 16; rb < m; rb += (int64_t)gridDim.y * 16) {
    const int64_t re = rb + 16 < m ? rb + 16 : m;
    for (int64_t r = rb; r < re; ++r) {
      const float v = in ? A[r * lda + c] - sh : 0.f;
      if (ST == ST_FP8) {
        reinterpret_cast<uint8_t*>(out)[r * ldo + c] = (uint8_t)q_e4m3(v / sc);
      } else {
        const uint32_t h = q_bf16(v);
        reinterpret_cast<uint16_t*>(out)[r * ldo + c] = (uint16_t)h;
        if (ST == ST_HILO)
          reinterpret_cast<uint16_t*>(out)[m * ldo + r * ldo + c] = (uint16_t)q_bf16(v - __uint_as_float(h << 16));
      }
    }
  }
}

hipError_t launch_quantize(int storage, int64_t m, int64_t n, const float* A, int64_t lda, const float* shift,
                           void* out, int64_t ldo, float* col_scale, float* amax_part, int nsplit,
                           int64_t rows_per_split, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (storage == ST_FP8) {
    if (col_scale == nullptr || amax_part == nullptr || nsplit <= 0 || (int64_t)nsplit * rows_per_split < m)
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nsplit), dim3(256), 0, st, A, lda,
                       m, n, shift, rows_per_split, amax_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colscale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, amax_part, nsplit, n,
                       col_scale);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t rgroups = (m + 15) / 16;
  dim3 grid((unsigned)((ldo + 255) / 256), (unsigned)(rgroups < 65535 ? rgroups : 65535));
  switch (storage) {
    case ST_BF16:
      hipLaunchKernelGGL(quantize_kernel<ST_BF16>, grid, dim3(256), 0, st, A, lda, m, n, shift, out, ldo, col_scale);
      break;
    case ST_FP8:
      hipLaunchKernelGGL(quantize_kernel<ST_FP8>, grid, dim3(256), 0, st, A, lda, m, n, shift, out, ldo, col_scale);
      break;
    case ST_HILO:
      hipLaunchKernelGGL(quantize_kernel<ST_HILO>, grid, dim3(256), 0, st, A, lda, m, n, shift, out, ldo, col_scale);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rpca
