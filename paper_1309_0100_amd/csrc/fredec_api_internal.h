// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <utility>
#include <vector>

#include "fredec.h"

// Library context: device, staging buffer for descriptor uploads, tile
// settings and the optional timing events.
struct fredec_ctx {
  int device = 0;
  int n_cu = 0;
  void* staging = nullptr;  // pinned host buffer for descriptor uploads
  size_t staging_bytes = 0;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;
  int f16x3_ft[5] = {0, 0, 0, 0, 0};  // split-float16 scan: 16-frequency tiles per wave, by column tiles (0 = default)
  int f32_form = FREDEC_F32_FORM_AUTO;   // kernel family of the reduced-precision scan (FREDEC_F32_FORM_*)
  int tuple_lanes[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // lane-group tuple kernels: lanes per tuple, by size (0 = default)
  int f32_auto_valu_max_kp = 6;      // automatic form: VALU kernel up to this KP = 2m + 2 (m <= 2)
  // side streams (default priority) for launches of independent kernel
  // groups, joined back to the caller's stream with events
  static constexpr int NSIDE = 3;
  hipStream_t side[NSIDE] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[NSIDE] = {};
  // optional timing of the dominant kernel of each call (HIP events)
  bool profiling = false;
  struct ProfEvent {
    hipEvent_t begin, end;
    int kind;  // FREDEC_PROF_*
  };
  std::vector<ProfEvent> prof_events;
  size_t prof_used = 0;
  // device address of this device's copy of the static scratch array of
  // fredec_scan_static (resolved when the context is created)
  void* static_scratch = nullptr;
};

// A prepared call (fredec_*_plan): the host-side launch schedule of a batch
// whose device descriptors already sit in the caller's workspace, so that a
// launch only enqueues kernels.
struct fredec_plan {
  enum Kind { SCAN = 1, TUPLES = 2, ASCENT = 3 };
  explicit fredec_plan(int k) : kind(k) {}
  virtual ~fredec_plan() = default;
  int kind;
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
};

namespace fredec {

// Makes `dev` current for the lifetime of the guard and restores the
// caller's device afterwards (no device call at all when `dev` is current).
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
// Waits until every upload enqueued so far has reached the device.
int upload_wait(fredec_ctx* ctx);

// Records a pair of HIP events on `st` around a group of kernel launches of
// one kind (FREDEC_PROF_*) when the context has profiling enabled (nothing
// for a null context).
class ProfScope {
 public:
  ProfScope(fredec_ctx* ctx, hipStream_t st, int kind = FREDEC_PROF_SCAN);
  ~ProfScope();

 private:
  fredec_ctx* ctx_;
  hipStream_t st_;
  long idx_ = -1;
};
size_t align_up(size_t v);

}  // namespace fredec
