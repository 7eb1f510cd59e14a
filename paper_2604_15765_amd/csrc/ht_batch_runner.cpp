#include "ht_batch_runner.h"

#include <algorithm>
#include <cstring>

namespace ht {

namespace {
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
}  // namespace

BatchRunner::~BatchRunner() {
  if (done_) {
    (void)hipEventSynchronize(done_);
    (void)hipEventDestroy(done_);
  }
  if (dev_) (void)hipFree(dev_);
  if (counters_) (void)hipFree(counters_);
  if (stage_) (void)hipHostFree(stage_);
}

hipError_t BatchRunner::wait() {
  if (!pending_) return hipSuccess;
  pending_ = false;
  return hipEventSynchronize(done_);
}

hipError_t BatchRunner::run(const std::vector<BatchItem>& items, const BatchSchedule& sched,
                            int num_cu, hipStream_t s) {
  if (items.empty()) return hipSuccess;
  hipError_t e = wait();  // the staging buffer may still feed the previous copy
  if (e != hipSuccess) return e;
  // per storage type, largest work first (longest-processing-time-first queue)
  std::vector<size_t> order[2];
  for (size_t i = 0; i < items.size(); ++i) order[items[i].dtype].push_back(i);
  for (auto& o : order)
    std::stable_sort(o.begin(), o.end(), [&](size_t x, size_t y) {
      return (double)items[x].bytes * items[x].nops > (double)items[y].bytes * items[y].nops;
    });
  size_t nopers[2] = {order[0].size(), order[1].size()}, nops[2] = {0, 0}, ncoef[2] = {0, 0};
  for (int d = 0; d < 2; ++d)
    for (size_t i : order[d]) {
      nops[d] += items[i].nops;
      ncoef[d] += items[i].ncoefs;
    }
  size_t off_opers[2], off_ops[2], off_coef[2], total = 0;
  for (int d = 0; d < 2; ++d) {
    off_opers[d] = total;
    total = align_up(total + nopers[d] * sizeof(BatchOperator), 256);
    off_ops[d] = total;
    total = align_up(total + nops[d] * sizeof(BatchOp), 256);
    off_coef[d] = total;
    total = align_up(total + ncoef[d] * sizeof(double), 256);
  }
  if (stage_cap_ < total) {
    if (stage_) (void)hipHostFree(stage_);
    stage_ = nullptr;
    stage_cap_ = 0;
    if ((e = hipHostMalloc(&stage_, total, hipHostMallocDefault)) != hipSuccess) return e;
    stage_cap_ = total;
  }
  if (dev_cap_ < total) {
    if (dev_) (void)hipFree(dev_);
    dev_ = nullptr;
    dev_cap_ = 0;
    if ((e = hipMalloc(&dev_, total)) != hipSuccess) return e;
    dev_cap_ = total;
  }
  if (!counters_ && (e = hipMalloc(&counters_, 2 * sizeof(unsigned))) != hipSuccess) return e;
  if (!done_ && (e = hipEventCreateWithFlags(&done_, hipEventDisableTiming)) != hipSuccess) return e;

  char* st = reinterpret_cast<char*>(stage_);
  size_t lds_need[2] = {0, 0};
  for (int d = 0; d < 2; ++d) {
    auto* opers = reinterpret_cast<BatchOperator*>(st + off_opers[d]);
    auto* ops = reinterpret_cast<BatchOp*>(st + off_ops[d]);
    auto* coefs = reinterpret_cast<double*>(st + off_coef[d]);
    uint32_t op_pos = 0, coef_pos = 0;
    for (size_t r = 0; r < order[d].size(); ++r) {
      const BatchItem& it = items[order[d][r]];
      BatchOperator o{};
      o.buf = it.buf;
      o.bytes = it.bytes;
      o.n = it.n;
      o.m = it.m;
      o.op_begin = op_pos;
      o.op_end = op_pos + it.nops;
      o.in_lds = it.bytes <= sched.lds_max ? 1 : 0;
      if (o.in_lds) lds_need[d] = std::max(lds_need[d], it.bytes);
      opers[r] = o;
      for (uint32_t k = 0; k < it.nops; ++k) {
        BatchOp x = it.ops[k];
        x.coef_off += coef_pos;
        ops[op_pos++] = x;
      }
      std::memcpy(coefs + coef_pos, it.coefs, (size_t)it.ncoefs * sizeof(double));
      coef_pos += it.ncoefs;
    }
  }
  if ((e = hipMemcpyAsync(dev_, stage_, total, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  char* dv = reinterpret_cast<char*>(dev_);
  for (int d = 0; d < 2; ++d) {
    if (nopers[d] == 0) continue;
    if (lds_need[d] > lds_set_[d]) {
      if ((e = set_batch_lds_limit(d, lds_need[d])) != hipSuccess) return e;
      lds_set_[d] = lds_need[d];
    }
    int grid = num_cu * sched.wg_per_cu;
    if ((size_t)grid > nopers[d]) grid = (int)nopers[d];
    e = launch_batch(d, reinterpret_cast<const BatchOperator*>(dv + off_opers[d]),
                     (unsigned)nopers[d], reinterpret_cast<const BatchOp*>(dv + off_ops[d]),
                     reinterpret_cast<const double*>(dv + off_coef[d]), counters_ + d,
                     sched.threads, grid, lds_need[d], s);
    if (e != hipSuccess) return e;
  }
  if ((e = hipEventRecord(done_, s)) != hipSuccess) return e;
  pending_ = true;
  return hipSuccess;
}

}  // namespace ht
