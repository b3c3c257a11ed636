// rpca_quantize_noalloc: the stored-format conversion of rpca_quantize without
// any device allocation.  Its scratch (per-split float64 column sums, the float64
// column means and per-split float32 column maxima, sized and split exactly as
// rpca_quantize sizes and splits them, so both produce identical bits) lives in
// one file-scope device array.  Host code never passes the array's name to a
// kernel: each device's address of it is taken once with hipGetSymbolAddress,
// with that device current, and kept per device.
#include <mutex>

#include "../../include/rpca.h"
#include "common.h"
#include "kernels.h"

namespace rpca {
namespace {

constexpr size_t kNoAllocScratchBytes = RPCA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array (first call on a device looks it up).
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace rpca

extern "C" rpca_status rpca_quantize_noalloc(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda,
                                             void* out, int64_t ldo, float* col_scale, float* shift,
                                             int32_t shift_mode, void* hip_stream) {
  using namespace rpca;
  const int vs = quantize_check(storage, m, n, A, lda, out, ldo, col_scale, shift, shift_mode);
  if (vs != RPCA_OK) return static_cast<rpca_status>(vs);
  int ns = 1;
  int64_t rps = 0;
  const size_t nbytes = quantize_scratch(m, n, &ns, &rps);
  if (nbytes > kNoAllocScratchBytes) return RPCA_ERR_SCRATCH_LIMIT;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  void* ptr = nullptr;
  if (e == hipSuccess) e = scratch_address(dev, &ptr);
  if (e == hipSuccess)
    e = quantize_run(storage, m, n, A, lda, out, ldo, col_scale, shift, shift_mode, ptr, ns, rps,
                     reinterpret_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return RPCA_ERR_HIP;
  }
  return RPCA_OK;
}
