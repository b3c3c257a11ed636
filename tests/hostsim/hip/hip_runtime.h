// Host-only stand-in for the HIP runtime, used to build the library's plan/scheduler code
// (plan.cpp) on the CPU for tests: device memory is host memory, streams run every
// operation at once in issue order, events record a counter.  Failures can be injected
// (see hostsim.h).  Device-side helpers the shared headers define are given host bodies.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __shared__

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
  hipErrorLaunchTimeOut = 702,
  hipErrorLaunchFailure = 719,
  hipErrorUnknown = 999
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

struct ihipStream_t;
struct ihipEvent_t;
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef struct hipDeviceProp_t {
  char name[256];
  size_t totalGlobalMem;
  size_t sharedMemPerBlock;
  int multiProcessorCount;
  int cooperativeLaunch;
  int warpSize;
  int maxThreadsPerBlock;
} hipDeviceProp_t;

#define hipStreamNonBlocking 0x01
#define hipEventDefault 0x0
#define hipEventDisableTiming 0x2
#define hipHostMallocDefault 0x0

hipError_t hipMalloc(void** ptr, size_t bytes);
template <class T>
hipError_t hipMalloc(T** ptr, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(ptr), bytes);
}
hipError_t hipFree(void* ptr);
hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned flags = 0);
template <class T>
hipError_t hipHostMalloc(T** ptr, size_t bytes, unsigned flags = 0) {
  return hipHostMalloc(reinterpret_cast<void**>(ptr), bytes, flags);
}
hipError_t hipHostFree(void* ptr);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t st = nullptr);
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t st = nullptr);
hipError_t hipMemset(void* dst, int value, size_t bytes);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t st = nullptr);
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t st);
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t ev, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* ev);
hipError_t hipEventCreateWithFlags(hipEvent_t* ev, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t ev);
hipError_t hipEventRecord(hipEvent_t ev, hipStream_t st = nullptr);
hipError_t hipEventSynchronize(hipEvent_t ev);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetDevice(int* dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int dev);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);

// host bodies of device helpers used in the shared headers
struct hostsim_dim3_idx {
  unsigned x, y, z;
};
static const hostsim_dim3_idx threadIdx = {0, 0, 0};
template <class T>
inline T __shfl_xor(T v, int, int = 64) {
  return v;
}
inline float __uint_as_float(uint32_t u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
inline uint32_t __float_as_uint(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}
using std::cos;
using std::log;
using std::sin;
using std::sqrt;
