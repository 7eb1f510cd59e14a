// Host side of one persistent batch launch: builds the device tables for a
// set of operators (each with its op sequence) and enqueues the launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "ht_internal.h"

namespace ht {

// One operator and the ops to apply to it in this launch.
struct BatchItem {
  void* buf;
  size_t bytes;
  int n, m, dtype;
  const BatchOp* ops;  // coef_off relative to coefs
  uint32_t nops;
  const double* coefs;
  uint32_t ncoefs;
};

struct BatchSchedule {
  int threads = 256;         // threads per workgroup
  int wg_per_cu = 2;         // workgroups per compute unit
  size_t lds_max = 65536;    // operators up to this many bytes run in LDS
};

// Owns pinned staging and device tables; one run may be in flight at a time
// (run() waits for the previous one before reusing the staging buffer).
class BatchRunner {
 public:
  BatchRunner() = default;
  BatchRunner(const BatchRunner&) = delete;
  BatchRunner& operator=(const BatchRunner&) = delete;
  ~BatchRunner();

  // Enqueue the launch(es) on s: one per storage type present, operators
  // ordered largest work first.  Returns the first HIP error.
  hipError_t run(const std::vector<BatchItem>& items, const BatchSchedule& sched, int num_cu,
                 hipStream_t s);
  // Event recorded after the last run (nullptr before the first).
  hipEvent_t done() const { return done_; }
  // Wait for the last run.
  hipError_t wait();

 private:
  void* stage_ = nullptr;
  size_t stage_cap_ = 0;
  void* dev_ = nullptr;
  size_t dev_cap_ = 0;
  unsigned* counters_ = nullptr;
  size_t lds_set_[2] = {0, 0};
  hipEvent_t done_ = nullptr;
  bool pending_ = false;
};

}  // namespace ht
