// util.h — host helpers shared by the libphos translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phos.h"

namespace phos {
// Record a thread-local error message and return s.
phos_status fail(phos_status s, const char *fmt, ...);
// Unsigned environment override, or dflt.
uint32_t env_u32(const char *name, uint32_t dflt);

// Make `dev` current for the lifetime of the guard.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  DeviceGuard(const DeviceGuard &) = delete;
  DeviceGuard &operator=(const DeviceGuard &) = delete;

 private:
  int prev_ = -1;
};
}  // namespace phos
