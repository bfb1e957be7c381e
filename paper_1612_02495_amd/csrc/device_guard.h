// Makes a plan's device current for the duration of one entry-point call and
// restores the caller's device afterwards.  Plans remember the device that
// was current when they were created; their buffers and streams belong to it.
#pragma once

#include <hip/hip_runtime.h>

namespace swept {

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev) {
      err = hipSetDevice(dev);
      ok = err == hipSuccess;
    }
  }
  ~DeviceGuard() {
    int cur = -1;
    if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
};

}  // namespace swept
