// Autotuner of batched launches: picks a tile edge per qubit count and the
// persistent launch's shape by timing candidates on a sample of the batch.
//
// The sample is stratified by qubit count and storage type, so that it is a
// miniature of the batch.  Scratch copies of the sampled operators are
// zero-initialised (the run time of a pass does not depend on the values)
// and evolved by the sampled operators' own ops, prepared again for each
// candidate tile edge.  Search, by coordinate descent:
//   1. per qubit count n, every tile edge 2^m, 2 <= m <= min(n, 7), plus the
//      operators' own, timed on that n's operators alone (LDS staging on, so
//      that edges which let an operator fit in LDS show their gain);
//   2. with those edges, every launch shape threads x wg_per_cu
//      (<= 2048 threads per compute unit) x LDS limit in {0, 64 KiB, max}
//      on the whole sample;
//   3. step 1 again at the shape of step 2; its edges are kept if the whole
//      sample then runs faster.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <vector>

#include "hermtile.h"
#include "ht_batch_state.h"
#include "ht_handle.h"
#include "ht_internal.h"
#include "ht_prep.h"

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t storage_bytes(int n, int m, int dtype) {
  return ht_storage_bytes(n, m, dtype == 0 ? HT_C128 : HT_C64);
}

// Timing context: a private stream, two events, the runner of the batch.
struct Timer {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Timer() {
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  }
};

// One sampled operator: its batch entry and its tile exponent in a trial.
struct Trial {
  const ht_batch::Entry* e;
  int m_req;
  std::vector<ht::BatchOp> ops;
  std::vector<double> coefs;
};

class Tuner {
 public:
  Tuner(ht_batch* b, Timer* t) : b_(b), t_(t) {}
  ~Tuner() {
    if (scratch_) {
      (void)hipStreamSynchronize(t_->s);
      (void)hipFree(scratch_);
    }
  }

  // Prepare the ops of each trial for its tile edge.  Fails only on a
  // preparation error (which add_op already excluded).
  ht_status prepare(std::vector<Trial>& trials) {
    char msg[256];
    for (auto& tr : trials) {
      const int n = tr.e->h->n;
      if (ht::entry_ops(*tr.e, std::min(n, tr.m_req), b_->fuse_q, tr.ops, tr.coefs, msg, sizeof msg) != 0)
        return ht_fail(HT_EINVAL, "autotune: %s", msg);
    }
    return HT_OK;
  }

  // Time the trials as one batch at schedule sc: one untimed run, then the
  // best of reps timed runs (seconds).
  ht_status time(std::vector<Trial>& trials, const ht::BatchSchedule& sc, int reps, double* sec) {
    ht_status st = prepare(trials);
    if (st != HT_OK) return st;
    size_t total = 0;
    for (const auto& tr : trials)
      total += align256(storage_bytes(tr.e->h->n, std::min(tr.e->h->n, tr.m_req), tr.e->h->dtype));
    if (total > scratch_cap_) {
      if (scratch_) {
        HT_HIP(hipStreamSynchronize(t_->s));
        HT_HIP(hipFree(scratch_));
        scratch_ = nullptr;
        scratch_cap_ = 0;
      }
      size_t free_b = 0, total_b = 0;
      HT_HIP(hipMemGetInfo(&free_b, &total_b));
      if (total > free_b / 2)
        return ht_fail(HT_ENOMEM, "autotune: the sample needs %zu bytes of scratch, %zu free", total,
                       free_b);
      if (hipMalloc(&scratch_, total) != hipSuccess) {
        scratch_ = nullptr;
        return ht_fail(HT_ENOMEM, "autotune: could not allocate %zu bytes of scratch", total);
      }
      scratch_cap_ = total;
    }
    std::vector<ht::BatchItem> items;
    items.reserve(trials.size());
    char* p = reinterpret_cast<char*>(scratch_);
    for (const auto& tr : trials) {
      const int n = tr.e->h->n, m = std::min(n, tr.m_req);
      const size_t bytes = storage_bytes(n, m, tr.e->h->dtype);
      items.push_back(ht::BatchItem{p, bytes, n, m, tr.e->h->dtype, tr.ops.data(),
                                    (uint32_t)tr.ops.size(), tr.coefs.data(),
                                    (uint32_t)tr.coefs.size()});
      p += align256(bytes);
    }
    HT_HIP(ht::launch_fill_zero(scratch_, total, t_->s));
    double best = 1e300;
    for (int i = 0; i <= reps; ++i) {
      HT_HIP(hipEventRecord(t_->e0, t_->s));
      HT_HIP(b_->runner.run(items, sc, b_->num_cu, t_->s));
      HT_HIP(hipEventRecord(t_->e1, t_->s));
      HT_HIP(hipEventSynchronize(t_->e1));
      float ms = 0.f;
      HT_HIP(hipEventElapsedTime(&ms, t_->e0, t_->e1));
      if (i > 0) best = std::min(best, (double)ms * 1e-3);
    }
    ++timed_;
    *sec = best;
    return HT_OK;
  }

  int timed() const { return timed_; }

 private:
  ht_batch* b_;
  Timer* t_;
  void* scratch_ = nullptr;
  size_t scratch_cap_ = 0;
  int timed_ = 0;
};

// Tile exponents worth trying for n qubits.
std::vector<int> edge_candidates(int n, int own) {
  std::vector<int> c;
  const int hi = std::min(n, 7);
  for (int m = std::min(2, n); m <= hi; ++m) c.push_back(m);
  const int o = std::min(n, own);
  if (std::find(c.begin(), c.end(), o) == c.end()) c.push_back(o);
  std::sort(c.begin(), c.end());
  return c;
}

}  // namespace

extern "C" ht_status ht_batch_autotune(ht_batch* b, int sample_operators, ht_batch_tuning* out) {
  if (!b || !out) return ht_fail(HT_EINVAL, "batch or out is NULL");
  if (sample_operators < 0) return ht_fail(HT_EINVAL, "sample_operators must be >= 0");
  if (b->entries.empty()) return ht_fail(HT_EINVAL, "autotune: the batch is empty");
  const auto t_start = std::chrono::steady_clock::now();
  std::memset(out, 0, sizeof *out);
  const int want = sample_operators == 0 ? 512 : sample_operators;
  ht_device_guard dg(b->device);
  HT_HIP(b->runner.wait());

  // stratified sample: per (n, dtype), a share proportional to its count,
  // at least one, spread evenly over the stratum's entries
  std::map<std::pair<int, int>, std::vector<const ht_batch::Entry*>> strata;
  for (const auto& e : b->entries) strata[{e.h->n, e.h->dtype}].push_back(&e);
  const double frac = std::min(1.0, (double)want / (double)b->entries.size());
  std::vector<Trial> sample;
  for (auto& kv : strata) {
    const auto& v = kv.second;
    const size_t take = std::max<size_t>(1, (size_t)(frac * (double)v.size() + 0.5));
    for (size_t i = 0; i < take; ++i)
      sample.push_back(Trial{v[i * v.size() / take], v[i * v.size() / take]->h->m_req, {}, {}});
  }

  Timer tm;
  HT_HIP(hipStreamCreateWithFlags(&tm.s, hipStreamNonBlocking));
  HT_HIP(hipEventCreate(&tm.e0));
  HT_HIP(hipEventCreate(&tm.e1));
  Tuner tuner(b, &tm);
  const int reps = 2;
  ht_status st;

  double before = 0.0;
  if ((st = tuner.time(sample, b->sched, reps, &before)) != HT_OK) return st;

  std::map<int, int> edge;  // n -> chosen tile exponent
  auto tune_edges = [&](const ht::BatchSchedule& sc) -> ht_status {
    std::map<int, std::vector<size_t>> by_n;
    for (size_t i = 0; i < sample.size(); ++i) by_n[sample[i].e->h->n].push_back(i);
    for (auto& kv : by_n) {
      const int n = kv.first;
      std::vector<Trial> sub;
      for (size_t i : kv.second) sub.push_back(sample[i]);
      double best = 1e300;
      int best_m = std::min(n, sub[0].m_req);
      for (int m : edge_candidates(n, sub[0].e->h->m_req)) {
        for (auto& tr : sub) tr.m_req = m;
        double sec = 0.0;
        ht_status s2 = tuner.time(sub, sc, reps, &sec);
        if (s2 != HT_OK) return s2;
        if (sec < best * 0.99) {  // a new edge must win by 1 %
          best = sec;
          best_m = m;
        }
      }
      edge[n] = best_m;
    }
    for (auto& tr : sample) tr.m_req = edge[tr.e->h->n];
    return HT_OK;
  };

  // 1. tile edges at the batch's shape with LDS staging allowed
  ht::BatchSchedule sc = b->sched;
  sc.lds_max = (size_t)kBatchLdsMax;
  if ((st = tune_edges(sc)) != HT_OK) return st;

  // 2. launch shape
  const int thread_opts[] = {256, 512, 1024};
  const int wg_opts[] = {1, 2, 4, 8};
  const size_t lds_opts[] = {0, 65536, (size_t)kBatchLdsMax};
  double best = 1e300;
  ht::BatchSchedule best_sc = b->sched;
  std::vector<size_t> seen_lds_sets;
  for (size_t lds : lds_opts) {
    // an LDS limit that stages exactly the same operators as a smaller one
    // is the same schedule
    size_t staged = 0;
    for (const auto& tr : sample)
      if (storage_bytes(tr.e->h->n, std::min(tr.e->h->n, tr.m_req), tr.e->h->dtype) <= lds) ++staged;
    if (lds > 0 && staged == 0) continue;
    if (std::find(seen_lds_sets.begin(), seen_lds_sets.end(), staged) != seen_lds_sets.end()) continue;
    seen_lds_sets.push_back(staged);
    for (int th : thread_opts)
      for (int wg : wg_opts) {
        if (th * wg > 2048) continue;
        ht::BatchSchedule c;
        c.threads = th;
        c.wg_per_cu = wg;
        c.lds_max = lds;
        double sec = 0.0;
        if ((st = tuner.time(sample, c, reps, &sec)) != HT_OK) return st;
        if (sec < best) {
          best = sec;
          best_sc = c;
        }
      }
  }

  // 3. edges again at the chosen shape; keep them if the sample gains
  {
    const std::map<int, int> prev = edge;
    if ((st = tune_edges(best_sc)) != HT_OK) return st;
    if (edge != prev) {
      double sec = 0.0;
      if ((st = tuner.time(sample, best_sc, reps, &sec)) != HT_OK) return st;
      if (sec < best) {
        best = sec;
      } else {
        edge = prev;
        for (auto& tr : sample) tr.m_req = edge[tr.e->h->n];
      }
    }
  }

  b->sched = best_sc;
  for (const auto& kv : edge) out->tile_log2[kv.first] = kv.second;
  out->threads = best_sc.threads;
  out->wg_per_cu = best_sc.wg_per_cu;
  out->lds_max_bytes = (int64_t)best_sc.lds_max;
  out->sample_operators = (int)sample.size();
  out->configs_timed = tuner.timed();
  out->sample_seconds_before = before;
  out->sample_seconds_after = best;
  out->tuning_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return HT_OK;
}
