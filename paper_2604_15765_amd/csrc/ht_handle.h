// The handle behind the C ABI and helpers shared by the API sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "hermtile.h"
#include "ht_internal.h"

// Record an error message for ht_last_error() and return st.
ht_status ht_fail(ht_status st, const char* fmt, ...);

#define HT_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return ht_fail(HT_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

struct ht_pending_event {
  int cls;
  hipEvent_t a, b;
  double bytes;
};

struct ht_herm {
  int n = 0, m_req = 0, m = 0;
  int dtype = 0;
  uint64_t nelems = 0;
  size_t bytes = 0;
  void* buf = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cu = 256;
  // device scratch
  double* coef_dev = nullptr;   // 512 doubles: two-qubit transfer matrices
  double* out_dev = nullptr;    // 8 doubles: reduction results
  double out_host[8] = {};      // host copy of a reduction result
  double* red = nullptr;        // reduction partial sums
  size_t red_cap = 0;           // doubles
  void* tmp = nullptr;          // term tables and other per-call uploads
  size_t tmp_cap = 0;           // bytes
  // profiling
  bool prof = false;
  std::vector<ht_pending_event> pending;
  std::vector<hipEvent_t> pool;
  int64_t prof_launches[2 * ht::kClassesPerDtype] = {};
  double prof_ms[2 * ht::kClassesPerDtype] = {};
  double prof_bytes[2 * ht::kClassesPerDtype] = {};
};

// Upload the coefficients of a prepared op and enqueue its pass on h's
// stream (profiled when h's profiling is on).
ht_status ht_launch_prepared(ht_herm* h, const ht::PreparedOp& op);

// Switch to a device for the lifetime of the guard, if it is not current.
struct ht_device_guard {
  int prev = -1;
  explicit ht_device_guard(int dev) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != dev) {
      prev = cur;
      (void)hipSetDevice(dev);
    }
  }
  ~ht_device_guard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};
