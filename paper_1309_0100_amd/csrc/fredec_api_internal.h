// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "fredec.h"

namespace fredec {

// Makes `dev` current for the lifetime of the guard and restores the
// caller's device afterwards.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;

 private:
  int prev_ = -1;
};

int upload(fredec_ctx* ctx, hipStream_t st, void* dst, const void* src, size_t bytes);

// Records a pair of HIP events on `st` around the dominant kernel launches of
// a call when the context has profiling enabled.
class ProfScope {
 public:
  ProfScope(fredec_ctx* ctx, hipStream_t st);
  ~ProfScope();

 private:
  fredec_ctx* ctx_;
  hipStream_t st_;
  long idx_ = -1;
};
size_t align_up(size_t v);

}  // namespace fredec
