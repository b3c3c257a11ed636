// GPU twin of synth/philox.py and synth/fixtures.py: builds the large seeded
// inputs directly in HBM.  Element addressing and arithmetic order follow the
// Python module so that the two agree to the last bit except where the device
// and host libm round log/sin/cos differently.  Holds no PCA arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct W4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ W4 philox4x32_10(W4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    W4 o;
    o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    o.y = (uint32_t)p1;
    o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    o.w = (uint32_t)p0;
    c = o;
  }
  return c;
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  const uint64_t k = (uint64_t)(hi >> 5) * 67108864ull + (uint64_t)(lo >> 6);
  return ((double)k + 0.5) * 1.1102230246251565e-16;
}

__device__ __forceinline__ double gauss(uint64_t seed, uint32_t stream, uint64_t e) {
  const uint64_t b = e >> 1;
  const W4 x = philox4x32_10(W4{(uint32_t)b, (uint32_t)(b >> 32), stream, 0u}, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  const double u1 = unit53(x.x, x.y), u2 = unit53(x.z, x.w);
  const double r = sqrt(-2.0 * log(u1));
  const double t = 2.0 * 3.141592653589793 * u2;
  return (e & 1) ? r * sin(t) : r * cos(t);
}

// A[r][c] = fl32( sum_j (Ur[r][j] * sigma[j]) * Vr[c][j]  + noise * N(row0+r, c) + off[c] )
// with the low-rank sum taken in the order j = 0..rank-1, multiply then add.
__global__ __launch_bounds__(256) void lowrank_noise_kernel(float* __restrict__ A, int64_t lda, int64_t rows,
                                                            int64_t n, int64_t row0,
                                                            const double* __restrict__ Ur, int rank,
                                                            const double* __restrict__ sigma,
                                                            const double* __restrict__ Vr, double noise,
                                                            const double* __restrict__ off, uint64_t seed,
                                                            uint32_t noise_stream) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = blockIdx.y + (int64_t)blockIdx.z * 65535;
  if (c >= n || r >= rows) return;
  const double* u = Ur + (row0 + r) * rank;
  const double* v = Vr + c * rank;
  double acc = 0.0;
  for (int j = 0; j < rank; ++j) acc = __dadd_rn(acc, __dmul_rn(__dmul_rn(u[j], sigma[j]), v[j]));
  acc = __dadd_rn(acc, __dmul_rn(noise, gauss(seed, noise_stream, (uint64_t)(row0 + r) * (uint64_t)n + c)));
  if (off != nullptr) acc = __dadd_rn(acc, off[c]);
  A[r * lda + c] = (float)acc;
}

__global__ void normals_kernel(double* __restrict__ out, uint64_t seed, uint32_t stream, uint64_t start,
                               int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = gauss(seed, stream, start + (uint64_t)e);
}

// dst[r][c] = src[r][c] for r < rows, c < n
__global__ __launch_bounds__(256) void copy_rows_kernel(float* __restrict__ dst, int64_t ldd,
                                                        const float* __restrict__ src, int64_t lds, int64_t rows,
                                                        int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = blockIdx.y + (int64_t)blockIdx.z * 65535;
  if (c >= n || r >= rows) return;
  dst[r * ldd + c] = src[r * lds + c];
}

}  // namespace

extern "C" int synth_copy_rows(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows, int64_t n,
                               void* stream) {
  if (rows <= 0 || n <= 0) return 0;
  const int64_t gy = rows < 65535 ? rows : 65535;
  const int64_t gz = (rows + 65534) / 65535;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)gy, (unsigned)gz);
  hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, (hipStream_t)stream, dst, ldd, src, lds, rows, n);
  return (int)hipGetLastError();
}

extern "C" int synth_lowrank_noise(float* A, int64_t lda, int64_t rows, int64_t n, int64_t row0, const double* Ur,
                                   int rank, const double* sigma, const double* Vr, double noise, const double* off,
                                   uint64_t seed, uint32_t noise_stream, void* stream) {
  if (rows <= 0 || n <= 0) return 0;
  const int64_t gy = rows < 65535 ? rows : 65535;
  const int64_t gz = (rows + 65534) / 65535;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)gy, (unsigned)gz);
  hipLaunchKernelGGL(lowrank_noise_kernel, grid, dim3(256), 0, (hipStream_t)stream, A, lda, rows, n, row0, Ur, rank,
                     sigma, Vr, noise, off, seed, noise_stream);
  return (int)hipGetLastError();
}

extern "C" int synth_normals(double* out, uint64_t seed, uint32_t stream_id, uint64_t start, int64_t count,
                             void* stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(normals_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, out,
                     seed, stream_id, start, count);
  return (int)hipGetLastError();
}
