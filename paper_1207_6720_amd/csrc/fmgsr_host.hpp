// fmgsr_host.hpp -- host-side pieces shared by the library's entry points:
// per-launch event timing (fmgsr_profile_*), the device-pointer check and
// the device's LDS limit.
#pragma once

#include <hip/hip_runtime.h>

namespace fmgsr {

struct ProfRecord {
  const char* name;
  hipEvent_t start, stop;
  double bytes;
};

// Brackets the launches issued during its lifetime with two events on `s`
// when profiling is enabled and `name` passes the filter.
struct ProfScope {
  ProfRecord rec{};
  bool on = false;
  hipStream_t st;
  ProfScope(const char* name, double bytes, hipStream_t s);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;
};

// True for device (or managed) memory; host pointers are rejected.
bool is_device_ptr(const void* ptr);

// Largest LDS one workgroup may use on the current device after opting in
// (hipDeviceAttributeSharedMemPerBlockOptin), queried once per device.
hipError_t device_lds_limit(size_t* bytes);

}  // namespace fmgsr
