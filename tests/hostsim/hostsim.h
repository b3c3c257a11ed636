// Controls and records of the host-only HIP stand-in (hip/hip_runtime.h in this folder).
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace hostsim {

struct Faults {
  long malloc_fail_at = -1;       // the n-th hipMalloc (0-based, counted from reset) returns OutOfMemory
  std::string launch_fail_name;   // a launcher of this name returns LaunchFailure ...
  long launch_fail_at = 0;        // ... on its n-th call (0-based)
  long copy_fail_at = -1;         // the n-th hipMemcpy*Async returns LaunchFailure
};

struct Record {
  long mallocs = 0, frees = 0, host_mallocs = 0, host_frees = 0;
  long live_device = 0;           // device allocations not yet freed
  long copies = 0;
  uint64_t h2d_bytes = 0;
  std::map<std::string, long> launches;
};

Faults& faults();
Record& record();
void reset();  // clears faults and records (live allocations are kept)

// launcher stubs call this: records the call and returns the injected error or success
int launch(const char* name);

}  // namespace hostsim
