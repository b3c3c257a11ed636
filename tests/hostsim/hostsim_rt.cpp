// Host-only HIP stand-in: device memory is zero-filled host memory, every stream
// operation runs at once in issue order, events hold a running counter.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>

#include "hostsim.h"

struct ihipStream_t {
  int id;
};
struct ihipEvent_t {
  double t;
};

namespace hostsim {

static Faults g_faults;
static Record g_record;
static std::set<void*> g_device, g_host;
static double g_clock = 0.0;
static hipError_t g_last = hipSuccess;

Faults& faults() { return g_faults; }
Record& record() { return g_record; }

void reset() {
  g_faults = Faults();
  const long live = g_record.live_device;
  g_record = Record();
  g_record.live_device = live;
}

int launch(const char* name) {
  long& n = g_record.launches[name];
  const long idx = n++;
  if (!g_faults.launch_fail_name.empty() && g_faults.launch_fail_name == name && g_faults.launch_fail_at == idx) {
    g_last = hipErrorLaunchFailure;
    return hipErrorLaunchFailure;
  }
  return hipSuccess;
}

static hipError_t copy_fault() {
  const long idx = g_record.copies++;
  if (g_faults.copy_fail_at >= 0 && idx == g_faults.copy_fail_at) return hipErrorLaunchFailure;
  return hipSuccess;
}

}  // namespace hostsim

using namespace hostsim;

hipError_t hipMalloc(void** ptr, size_t bytes) {
  if (ptr == nullptr) return hipErrorInvalidValue;
  const long idx = g_record.mallocs++;
  if (g_faults.malloc_fail_at >= 0 && idx == g_faults.malloc_fail_at) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  *ptr = std::calloc(bytes ? bytes : 1, 1);
  if (*ptr == nullptr) return hipErrorOutOfMemory;
  g_device.insert(*ptr);
  ++g_record.live_device;
  return hipSuccess;
}

hipError_t hipFree(void* ptr) {
  if (ptr == nullptr) return hipSuccess;
  if (g_device.erase(ptr) == 0) {
    std::fprintf(stderr, "hostsim: hipFree of a pointer that is not a live device allocation\n");
    std::abort();
  }
  ++g_record.frees;
  --g_record.live_device;
  std::free(ptr);
  return hipSuccess;
}

hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned) {
  *ptr = std::calloc(bytes ? bytes : 1, 1);
  if (*ptr == nullptr) return hipErrorOutOfMemory;
  g_host.insert(*ptr);
  ++g_record.host_mallocs;
  return hipSuccess;
}

hipError_t hipHostFree(void* ptr) {
  if (ptr == nullptr) return hipSuccess;
  if (g_host.erase(ptr) == 0) {
    std::fprintf(stderr, "hostsim: hipHostFree of a pointer that is not a live pinned allocation\n");
    std::abort();
  }
  ++g_record.host_frees;
  std::free(ptr);
  return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  return hipMemcpyAsync(dst, src, bytes, kind, nullptr);
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t) {
  const hipError_t e = copy_fault();
  if (e != hipSuccess) return e;
  if (bytes) std::memmove(dst, src, bytes);
  if (kind == hipMemcpyHostToDevice) g_record.h2d_bytes += bytes;
  return hipSuccess;
}

hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t) {
  const hipError_t e = copy_fault();
  if (e != hipSuccess) return e;
  if (width > dpitch || width > spitch) return hipErrorInvalidValue;
  for (size_t r = 0; r < height; ++r)
    std::memmove(static_cast<char*>(dst) + r * dpitch, static_cast<const char*>(src) + r * spitch, width);
  if (kind == hipMemcpyHostToDevice) g_record.h2d_bytes += width * height;
  return hipSuccess;
}

hipError_t hipMemset(void* dst, int value, size_t bytes) {
  if (bytes) std::memset(dst, value, bytes);
  return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t) { return hipMemset(dst, value, bytes); }

hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned) {
  static int next = 1;
  *st = new ihipStream_t{next++};
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t st) {
  delete st;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }

hipError_t hipEventCreate(hipEvent_t* ev) {
  *ev = new ihipEvent_t{0.0};
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* ev, unsigned) { return hipEventCreate(ev); }

hipError_t hipEventDestroy(hipEvent_t ev) {
  delete ev;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t ev, hipStream_t) {
  if (ev == nullptr) return hipErrorInvalidValue;
  g_clock += 0.001;
  ev->t = g_clock;
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(b->t - a->t);
  return hipSuccess;
}

hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}

hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }

hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}

hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int dev) {
  if (dev != 0) return hipErrorInvalidValue;
  std::memset(prop, 0, sizeof(*prop));
  std::strcpy(prop->name, "hostsim");
  prop->totalGlobalMem = (size_t)288 << 30;
  prop->sharedMemPerBlock = 160 * 1024;
  prop->multiProcessorCount = 256;
  prop->cooperativeLaunch = 1;
  prop->warpSize = 64;
  prop->maxThreadsPerBlock = 1024;
  return hipSuccess;
}

hipError_t hipDeviceSynchronize() { return hipSuccess; }

hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hostsim error"; }
