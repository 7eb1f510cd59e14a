// Request server with continuous batching.
//
// A scheduler thread owns every GPU resource of the server.  Requests (an
// initial state G G^dagger / tr, a sequence of k-local ops, a readout) are
// admitted first-come first-served as soon as a slot and enough of the HBM
// budget are free; their operators stay resident until the readout is done.
// Small operators (n <= batch_max_qubits) advance in rounds: every round is
// one persistent batch launch that takes up to chunk_ops ops of every small
// request that is ready, so requests join and leave the running batch round
// by round.  Large operators run on their own streams in chunks of
// large_chunk_ops plain grid-wide passes, overlapping with the rounds.
// Readouts (trace or Pauli-sum expectation, FP64) are enqueued behind each
// request's last op and detected with event queries, so the scheduler never
// blocks on the device.  With fifo = 1 the same machinery serves one request
// at a time with plain launches: the baseline the batching is compared to.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hermtile.h"
#include "ht_batch_runner.h"
#include "ht_handle.h"
#include "ht_batch_state.h"
#include "ht_fuse.h"
#include "ht_internal.h"
#include "ht_prep.h"

namespace {

enum ReqState { QUEUED, INIT, RUN, READOUT, DONE };

struct Req {
  int64_t id = 0;
  int n = 0, m = 0, dtype = 0;
  size_t bytes = 0;
  std::vector<ht::BatchOp> ops;
  std::vector<double> coefs;
  std::vector<double> G;
  int rank = 0;
  std::vector<ht::PauliTerm> terms;
  double t_submit = 0, t_admit = 0, t_done = 0;
  double value = 0;
  int status = HT_OK;
  // runtime
  ReqState state = QUEUED;
  int slot = -1;
  void* buf = nullptr;
  size_t next = 0;  // first op not yet enqueued
  void* gbuf = nullptr;  // device copy of G, released after the initial state is built
  size_t gbytes = 0;
  int lane = 0;          // 0: batched rounds, 1: medium, 2: large (plain passes)
  bool large = false;    // lane > 0: runs plain passes on its slot's stream
  int chunks_in_flight = 0;  // large path: chunks enqueued and not yet seen complete (<= 2)
  int chunk_ev = 0;          // event slot the next chunk records
  bool failed = false;       // its batch round could not be enqueued
};

// Per-slot resources, allocated once at server creation at their largest size
// (growing them later would need hipFree, which waits for the whole device).
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev_init = nullptr, ev_chunk[2] = {nullptr, nullptr}, ev_done = nullptr;
  double* red = nullptr;             // reduction partial sums
  ht::PauliTerm* terms_dev = nullptr;  // kMaxTerms terms
  double* coef_dev = nullptr;        // 512 doubles
  double* out_dev = nullptr;         // 8 doubles
  Req* req = nullptr;
};

constexpr int kMaxTerms = 4096;

size_t storage_bytes_of(int n, int m, int dtype) {
  const uint64_t N = 1ull << n, M = 1ull << m;
  return (size_t)(N * (N + M) / 2) * (dtype == 0 ? 16 : 8);
}


}  // namespace

struct ht_server {
  ht_server_config cfg;
  int device = 0;
  int num_cu = 256;
  std::chrono::steady_clock::time_point t0;

  // shared with callers
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::unique_ptr<Req>> inbox;
  std::deque<std::unique_ptr<Req>> outbox;
  int64_t next_id = 1;
  int64_t in_flight = 0;  // submitted and not yet in the outbox
  std::string error;
  std::atomic<bool> stop{false};

  // scheduler thread only
  std::deque<std::unique_ptr<Req>> pending[3];  // per lane, arrival order
  std::vector<std::unique_ptr<Req>> active;
  std::vector<Slot> slots;
  std::vector<int> free_slots;
  std::multimap<size_t, void*> pool;  // free operator buffers by size
  size_t allocated = 0;               // bytes of operator buffers (in use + pooled)
  hipStream_t batch_stream = nullptr;
  ht::BatchRunner runners[2];
  int next_runner = 0;
  ht::BatchSchedule sched;
  std::thread worker;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void set_error(ht_server* s, const std::string& msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error.empty()) s->error = msg;
}

// Outcome of asking for an operator buffer.
enum class Take { kOk, kWait, kNoMemory };

// An operator buffer of exactly `bytes` within the budget: kWait when the
// budget is taken (memory frees up as requests finish), kNoMemory when the
// device itself cannot provide it even after the pool is given back.
Take take_buffer(ht_server* s, size_t bytes, void** out) {
  *out = nullptr;
  auto it = s->pool.find(bytes);
  if (it != s->pool.end()) {
    *out = it->second;
    s->pool.erase(it);
    return Take::kOk;
  }
  while (s->allocated + bytes > s->cfg.budget_bytes && !s->pool.empty()) {
    auto big = std::prev(s->pool.end());  // release the largest pooled buffer
    (void)hipFree(big->second);
    s->allocated -= big->first;
    s->pool.erase(big);
  }
  if (s->allocated + bytes > s->cfg.budget_bytes) return Take::kWait;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();  // clear the allocation error
    for (auto& kv : s->pool) {
      (void)hipFree(kv.second);
      s->allocated -= kv.first;
    }
    s->pool.clear();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return Take::kNoMemory;
    }
  }
  s->allocated += bytes;
  *out = p;
  return Take::kOk;
}

void give_buffer(ht_server* s, void* p, size_t bytes) { s->pool.emplace(bytes, p); }

// Enqueue a request's readout on stream st behind its last op.
hipError_t enqueue_readout(Req* r, Slot& sl, hipStream_t st) {
  hipError_t e;
  if (r->terms.empty())
    e = ht::launch_trace(r->dtype, r->buf, r->n, r->m, sl.red, sl.out_dev, st);
  else
    e = ht::launch_pauli_expect(r->dtype, r->buf, r->n, r->m, sl.terms_dev, (int)r->terms.size(),
                                sl.red, sl.out_dev, st);
  if (e != hipSuccess) return e;
  return hipEventRecord(sl.ev_done, st);
}

// Admission: G upload, G G^dagger, division by the trace, Pauli table upload.
hipError_t start_request(Req* r, Slot& sl) {
  hipError_t e;
  if (!r->terms.empty() &&
      (e = hipMemcpyAsync(sl.terms_dev, r->terms.data(), r->terms.size() * sizeof(ht::PauliTerm),
                          hipMemcpyHostToDevice, sl.stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(r->gbuf, r->G.data(), r->G.size() * sizeof(double), hipMemcpyHostToDevice,
                          sl.stream)) != hipSuccess)
    return e;
  if ((e = ht::launch_lowrank(r->dtype, r->buf, r->n, r->m, reinterpret_cast<const double*>(r->gbuf),
                              r->rank, sl.stream)) != hipSuccess)
    return e;
  if ((e = ht::launch_trace(r->dtype, r->buf, r->n, r->m, sl.red, sl.out_dev, sl.stream)) !=
      hipSuccess)
    return e;
  const uint64_t nel = r->bytes / (r->dtype == 0 ? 16 : 8);
  if ((e = ht::launch_scale_inv(r->dtype, r->buf, nel, sl.out_dev, sl.stream)) != hipSuccess) return e;
  return hipEventRecord(sl.ev_init, sl.stream);
}

// Plain grid-wide passes for the next chunk of a large request.
hipError_t enqueue_chunk(ht_server* s, Req* r, Slot& sl, size_t count) {
  hipError_t e = hipSuccess;
  for (size_t c = 0; c < count && r->next < r->ops.size(); ++c, ++r->next) {
    const ht::BatchOp& b = r->ops[r->next];
    ht::PreparedOp op{};
    op.k = b.k;
    op.ncross = b.ncross;
    op.form = b.form;
    op.sorted[0] = b.sorted[0];
    op.sorted[1] = b.sorted[1];
    for (int u = 0; u < 4; ++u) op.perm[u] = b.perm[u];
    op.active = b.active;
    const int nd = ht::op_coef_doubles(b.k, b.form);
    std::memcpy(op.coef, r->coefs.data() + b.coef_off, nd * sizeof(double));
    if (((op.k == 2 && op.form == 1) || op.form == 2) &&
        (e = ht::launch_upload(sl.coef_dev, op.coef, op.form == 2 ? nd : 512, sl.stream)) != hipSuccess)
      return e;
    e = op.form == 2
            ? ht::launch_native(r->dtype, r->buf, r->n, r->m, op, sl.coef_dev, s->num_cu, sl.stream)
            : ht::launch_conj(r->dtype, r->buf, r->n, r->m, op, sl.coef_dev, s->num_cu, sl.stream);
    if (e != hipSuccess) return e;
  }
  if ((e = hipEventRecord(sl.ev_chunk[r->chunk_ev], sl.stream)) != hipSuccess) return e;
  r->chunk_ev ^= 1;
  ++r->chunks_in_flight;
  return hipSuccess;
}

void finish(ht_server* s, std::unique_ptr<Req>& rp) {
  Req* r = rp.get();
  if (r->slot >= 0) {
    s->slots[r->slot].req = nullptr;
    s->free_slots.push_back(r->slot);
    r->slot = -1;
  }
  if (r->buf) {
    give_buffer(s, r->buf, r->bytes);
    r->buf = nullptr;
  }
  if (r->gbuf) {
    give_buffer(s, r->gbuf, r->gbytes);
    r->gbuf = nullptr;
  }
  r->t_done = s->now();
  r->state = DONE;
  r->G.clear();
  r->G.shrink_to_fit();
  std::lock_guard<std::mutex> lk(s->mu);
  s->outbox.push_back(std::move(rp));
  --s->in_flight;
  s->cv.notify_all();
}

// Fail a request after its enqueued work has drained (its buffers go back to
// the pool and may be handed to the next request at once).
void fail_request(ht_server* s, std::unique_ptr<Req>& rp, hipError_t e) {
  rp->status = HT_EDEVICE;
  set_error(s, std::string("request failed: ") + hipGetErrorString(e));
  if (rp->slot >= 0) (void)hipStreamSynchronize(s->slots[rp->slot].stream);
  if (rp->lane == 0) (void)hipStreamSynchronize(s->batch_stream);
  finish(s, rp);
}

// Admit the request at the front of `pending` if a slot and its memory are
// available (false: it has to wait).  A request whose initialisation cannot
// be enqueued fails and is reported; the call still returns true.  A request
// whose buffers the device cannot allocate fails with HT_ENOMEM unless the
// memory of the resident requests, once they finish, would make room.
bool admit_front(ht_server* s, std::deque<std::unique_ptr<Req>>& pending) {
  if (s->free_slots.empty()) return false;
  Req* r = pending.front().get();
  void* buf = nullptr;
  void* gbuf = nullptr;
  Take t = take_buffer(s, r->bytes, &buf);
  if (t == Take::kOk) {
    t = take_buffer(s, r->gbytes, &gbuf);
    if (t != Take::kOk) give_buffer(s, buf, r->bytes);
  }
  if (t == Take::kWait) return false;
  if (t == Take::kNoMemory) {
    // Wait while the resident requests could free enough; fail otherwise.
    size_t held = 0, free_b = 0, total_b = 0;
    for (const auto& a : s->active) held += a->bytes + a->gbytes;
    if (!s->active.empty() && hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
        free_b + held >= r->bytes + r->gbytes)
      return false;
    std::unique_ptr<Req> rp = std::move(pending.front());
    pending.pop_front();
    rp->t_admit = s->now();
    rp->status = HT_ENOMEM;
    set_error(s, "request failed: the device cannot hold its operator");
    finish(s, rp);
    return true;
  }
  std::unique_ptr<Req> rp = std::move(pending.front());
  pending.pop_front();
  r->buf = buf;
  r->gbuf = gbuf;
  r->slot = s->free_slots.back();
  s->free_slots.pop_back();
  Slot& sl = s->slots[r->slot];
  sl.req = r;
  r->t_admit = s->now();
  hipError_t e = start_request(r, sl);
  if (e != hipSuccess) {
    fail_request(s, rp, e);
    return true;
  }
  r->state = INIT;
  s->active.push_back(std::move(rp));
  return true;
}

void scheduler(ht_server* s) {
  (void)hipSetDevice(s->device);
  const bool fifo = s->cfg.fifo != 0;
  while (true) {
    bool progressed = false;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      while (!s->inbox.empty()) {
        std::unique_ptr<Req>& q = s->inbox.front();
        q->lane = fifo ? 2 : q->n <= s->cfg.batch_max_qubits ? 0 : q->n <= s->cfg.medium_max_qubits ? 1 : 2;
        q->large = q->lane > 0;
        s->pending[q->lane].push_back(std::move(q));
        s->inbox.pop_front();
        progressed = true;
      }
    }
    if (s->stop.load() && s->pending[0].empty() && s->pending[1].empty() && s->pending[2].empty() &&
        s->active.empty())
      break;
    const int lane_limit[3] = {s->cfg.max_active, s->cfg.max_medium_active, s->cfg.max_large_active};

    // admission: first come first served within each lane.  The plain-pass
    // lanes admit up to their concurrency limit plus one request that builds
    // its initial state ahead.
    int admitted[3] = {0, 0, 0};
    for (const auto& a : s->active) ++admitted[a->lane];
    for (int lane = 0; lane < 3; ++lane) {
      const int cap = lane == 0 ? s->cfg.max_active : lane_limit[lane] + 1;
      while (!s->pending[lane].empty() && admitted[lane] < cap && admit_front(s, s->pending[lane])) {
        ++admitted[lane];
        progressed = true;
      }
    }

    // per-request progress: init done, chunks, readouts.  `active` is in
    // admission order; in each plain-pass lane only the oldest requests up to
    // the lane's concurrency limit that still have ops to run enqueue chunks.
    std::vector<Req*> batch_ready;
    int lane_rank[3] = {0, 0, 0};
    for (size_t i = 0; i < s->active.size();) {
      Req* r = s->active[i].get();
      Slot& sl = s->slots[r->slot];
      hipError_t e = hipSuccess;
      bool finished = false;
      bool may_run = true;
      if (r->large && (r->state == INIT || r->state == RUN)) {
        may_run = lane_rank[r->lane] < lane_limit[r->lane];
        ++lane_rank[r->lane];
      }
      if (r->state == INIT) {
        hipError_t q = hipEventQuery(sl.ev_init);
        if (q == hipSuccess) {
          give_buffer(s, r->gbuf, r->gbytes);  // G is no longer needed
          r->gbuf = nullptr;
          r->state = RUN;
          progressed = true;
        } else if (q != hipErrorNotReady) {
          e = q;
        }
      }
      if (e == hipSuccess && r->state == RUN && r->large) {
        // retire the oldest chunk if it has finished
        if (r->chunks_in_flight > 0) {
          const int oldest = (r->chunk_ev - r->chunks_in_flight) & 1;
          hipError_t q = hipEventQuery(sl.ev_chunk[oldest]);
          if (q == hipSuccess) {
            --r->chunks_in_flight;
            progressed = true;
          } else if (q != hipErrorNotReady) {
            e = q;
          }
        }
        // keep up to two chunks queued; the readout follows the last one
        if (e == hipSuccess && may_run && r->chunks_in_flight < 2 && r->next < r->ops.size()) {
          e = enqueue_chunk(s, r, sl, (size_t)s->cfg.large_chunk_ops);
          if (e == hipSuccess && r->next >= r->ops.size()) {
            e = enqueue_readout(r, sl, sl.stream);
            r->state = READOUT;
          }
          progressed = true;
        } else if (e == hipSuccess && may_run && r->ops.empty()) {
          e = enqueue_readout(r, sl, sl.stream);
          r->state = READOUT;
          progressed = true;
        }
      } else if (e == hipSuccess && r->state == RUN) {
        batch_ready.push_back(r);
      }
      if (e == hipSuccess && r->state == READOUT) {
        hipError_t q = hipEventQuery(sl.ev_done);
        if (q == hipSuccess) {
          e = hipMemcpyAsync(&r->value, sl.out_dev, sizeof(double), hipMemcpyDeviceToHost, sl.stream);
          if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
          finished = e == hipSuccess;
        } else if (q != hipErrorNotReady) {
          e = q;
        }
      }
      if (e != hipSuccess) {
        fail_request(s, s->active[i], e);
        s->active.erase(s->active.begin() + i);
        progressed = true;
        continue;
      }
      if (finished) {
        finish(s, s->active[i]);
        s->active.erase(s->active.begin() + i);
        progressed = true;
        continue;
      }
      ++i;
    }

    // one batch round over the ready small requests, if a runner is free
    if (!batch_ready.empty()) {
      ht::BatchRunner& run = s->runners[s->next_runner];
      const bool free = run.done() == nullptr || hipEventQuery(run.done()) == hipSuccess;
      if (free) {
        std::vector<ht::BatchItem> items;
        std::vector<std::vector<ht::BatchOp>> chunks(batch_ready.size());
        for (size_t i = 0; i < batch_ready.size(); ++i) {
          Req* r = batch_ready[i];
          const size_t cnt = std::min((size_t)s->cfg.chunk_ops, r->ops.size() - r->next);
          if (cnt > 0) {
            // ops keep their coefficients in op order: pass only this chunk's range
            const uint32_t c0 = r->ops[r->next].coef_off;
            const uint32_t c1 = r->next + cnt < r->ops.size() ? r->ops[r->next + cnt].coef_off
                                                              : (uint32_t)r->coefs.size();
            chunks[i].assign(r->ops.begin() + r->next, r->ops.begin() + r->next + cnt);
            for (auto& op : chunks[i]) op.coef_off -= c0;
            items.push_back(ht::BatchItem{r->buf, r->bytes, r->n, r->m, r->dtype, chunks[i].data(),
                                          (uint32_t)cnt, r->coefs.data() + c0, c1 - c0});
            r->next += cnt;
          }
        }
        hipError_t e = run.run(items, s->sched, s->num_cu, s->batch_stream);
        for (Req* r : batch_ready) {
          if (e == hipSuccess && r->next >= r->ops.size()) {
            e = enqueue_readout(r, s->slots[r->slot], s->batch_stream);
            r->state = READOUT;
          }
        }
        if (e != hipSuccess) {
          // the round's ops may not have run: every request in it fails
          set_error(s, std::string("batch round failed: ") + hipGetErrorString(e));
          for (Req* r : batch_ready) r->failed = true;
          for (size_t i = 0; i < s->active.size();) {
            if (s->active[i]->failed) {
              fail_request(s, s->active[i], e);
              s->active.erase(s->active.begin() + i);
            } else {
              ++i;
            }
          }
        }
        s->next_runner ^= 1;
        progressed = true;
      }
    }

    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  (void)hipDeviceSynchronize();
}

}  // namespace

extern "C" {

void ht_server_config_default(ht_server_config* c) {
  if (!c) return;
  c->budget_bytes = (size_t)200 << 30;
  c->max_active = 32;
  c->chunk_ops = 64;
  c->large_chunk_ops = 4;
  c->tile_log2 = 5;
  c->fifo = 0;
  c->batch_threads = 256;
  c->batch_wg_per_cu = 2;
  c->lds_max_bytes = 65536;
  c->max_large_active = 1;
  c->batch_max_qubits = 8;
  c->medium_max_qubits = 12;
  c->max_medium_active = 4;
  c->fuse_qubits = 0;
}

ht_status ht_server_create(const ht_server_config* cfg, ht_server** out) {
  if (!cfg || !out) return ht_fail(HT_EINVAL, "config or out is NULL");
  *out = nullptr;
  if (cfg->max_active < 1 || cfg->max_active > 256)
    return ht_fail(HT_EINVAL, "max_active must be in [1, 256]");
  if (cfg->chunk_ops < 1 || cfg->large_chunk_ops < 1)
    return ht_fail(HT_EINVAL, "chunk sizes must be positive");
  if (cfg->tile_log2 < HT_MIN_TILE_LOG2 || cfg->tile_log2 > HT_MAX_TILE_LOG2)
    return ht_fail(HT_EINVAL, "tile_log2 out of range");
  if (cfg->max_large_active < 1 || cfg->max_medium_active < 1)
    return ht_fail(HT_EINVAL, "lane concurrency limits must be positive");
  if (cfg->fuse_qubits < 0 || cfg->fuse_qubits > 2)
    return ht_fail(HT_EINVAL, "fuse_qubits must be 0, 1 or 2");
  ht_server* s = new ht_server();
  s->cfg = *cfg;
  if (s->cfg.fifo) s->cfg.max_active = 1;
  s->sched.threads = cfg->batch_threads;
  s->sched.wg_per_cu = cfg->batch_wg_per_cu;
  s->sched.lds_max = cfg->lds_max_bytes;
  s->t0 = std::chrono::steady_clock::now();
  auto fail_create = [&](hipError_t e, const char* what) {
    ht_server_destroy(s);
    return ht_fail(HT_EDEVICE, "server creation (%s): %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&s->device)) != hipSuccess) return fail_create(e, "device");
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) == hipSuccess &&
      cus > 0)
    s->num_cu = cus;
  if ((e = hipStreamCreateWithFlags(&s->batch_stream, hipStreamNonBlocking)) != hipSuccess)
    return fail_create(e, "stream");
  s->slots.resize(s->cfg.max_active);
  const size_t red_doubles = ht::reduce_scratch_doubles(0, 0, kMaxTerms);
  for (int i = 0; i < s->cfg.max_active; ++i) {
    Slot& sl = s->slots[i];
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.ev_init, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.ev_chunk[0], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.ev_chunk[1], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.ev_done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc(&sl.red, red_doubles * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&sl.terms_dev, kMaxTerms * sizeof(ht::PauliTerm))) != hipSuccess ||
        (e = hipMalloc(&sl.coef_dev, 512 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&sl.out_dev, 8 * sizeof(double))) != hipSuccess)
      return fail_create(e, "slot resources");
    s->free_slots.push_back(s->cfg.max_active - 1 - i);
  }
  s->worker = std::thread(scheduler, s);
  *out = s;
  return HT_OK;
}

ht_status ht_server_submit(ht_server* s, const ht_request* q, int64_t* id) {
  if (!s || !q) return ht_fail(HT_EINVAL, "server or request is NULL");
  if (q->n < 1 || q->n > HT_MAX_QUBITS) return ht_fail(HT_EINVAL, "n out of range");
  if (q->dtype != HT_C128 && q->dtype != HT_C64) return ht_fail(HT_EINVAL, "unknown dtype");
  if (q->rank < 1 || q->rank > 4096 || !q->G) return ht_fail(HT_EINVAL, "bad initial factor");
  if (q->nops < 0 || (q->nops > 0 && (!q->op_k || !q->op_targets || !q->op_r || !q->op_mats)))
    return ht_fail(HT_EINVAL, "bad op arrays");
  if (q->nterms < 0 || q->nterms > kMaxTerms || (q->nterms > 0 && (!q->codes || !q->coeffs)))
    return ht_fail(HT_EINVAL, "bad Pauli sum");
  if (q->picture != HT_SCHRODINGER && q->picture != HT_HEISENBERG)
    return ht_fail(HT_EINVAL, "unknown picture");
  auto r = std::make_unique<Req>();
  r->n = q->n;
  r->dtype = q->dtype;
  r->m = std::min(q->n, s->cfg.tile_log2);
  r->bytes = storage_bytes_of(r->n, r->m, r->dtype);
  if (r->bytes > s->cfg.budget_bytes)
    return ht_fail(HT_EINVAL, "request needs %zu bytes, more than the budget", r->bytes);
  r->rank = q->rank;
  r->G.assign(q->G, q->G + (size_t)2 * ((size_t)1 << q->n) * (size_t)q->rank);
  r->gbytes = (r->G.size() * sizeof(double) + 255) / 256 * 256;
  if (r->bytes + r->gbytes > s->cfg.budget_bytes)
    return ht_fail(HT_EINVAL, "request needs %zu bytes, more than the budget", r->bytes + r->gbytes);
  size_t mat_off = 0;
  std::vector<ht::FuseOp> fops(q->nops);
  for (int i = 0; i < q->nops; ++i) {
    const int k = q->op_k[i];
    if (k != 1 && k != 2) return ht_fail(HT_EINVAL, "op %d: k must be 1 or 2 in a request", i);
    ht::PreparedOp op;
    char msg[256];
    if (ht::prepare_op(r->n, r->m, k, q->op_targets + 2 * i, q->op_r[i], q->op_mats + mat_off,
                       q->picture == HT_HEISENBERG, &op, msg, sizeof msg, ht::native_policy(r->bytes)) != 0)
      return ht_fail(HT_EINVAL, "op %d: %s", i, msg);
    ht::FuseOp& f = fops[i];
    f.k = k;
    f.targets[0] = q->op_targets[2 * i];
    f.targets[1] = k > 1 ? q->op_targets[2 * i + 1] : -1;
    f.targets[2] = -1;
    f.r = q->op_r[i];
    f.adj = q->picture == HT_HEISENBERG ? 1 : 0;
    f.mats = q->op_mats + mat_off;
    mat_off += (size_t)2 * q->op_r[i] * (1u << (2 * k));
    if (s->cfg.fuse_qubits == 0) ht::append_batch_op(op, r->ops, r->coefs);
  }
  if (s->cfg.fuse_qubits > 0) {
    std::vector<const ht::FuseOp*> seq(fops.size());
    for (size_t i = 0; i < fops.size(); ++i) seq[i] = &fops[i];
    std::vector<ht::PreparedOp> prepared;
    char msg[256];
    if (ht::fuse_ops(seq, s->cfg.fuse_qubits, r->n, r->m, ht::native_policy(r->bytes), &prepared, msg,
                     sizeof msg) != 0)
      return ht_fail(HT_EINVAL, "fusing the request's ops: %s", msg);
    for (const ht::PreparedOp& op : prepared) ht::append_batch_op(op, r->ops, r->coefs);
  }
  for (int t = 0; t < q->nterms; ++t) {
    uint32_t x = 0, z = 0;
    int ny = 0;
    for (int qb = 0; qb < q->n; ++qb) {
      const uint8_t c = q->codes[(size_t)t * q->n + qb];
      if (c > 3) return ht_fail(HT_EINVAL, "Pauli code %d is not in 0..3", c);
      if (c == 1 || c == 2) x |= 1u << qb;
      if (c == 2 || c == 3) z |= 1u << qb;
      if (c == 2) ++ny;
    }
    r->terms.push_back(ht::PauliTerm{x, z, ny & 3, 0, q->coeffs[t]});
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->t_submit = s->now();
  if (id) *id = r->id;
  ++s->in_flight;
  s->inbox.push_back(std::move(r));
  return HT_OK;
}

ht_status ht_server_wait_idle(ht_server* s, double timeout_s) {
  if (!s) return ht_fail(HT_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                 [&] { return s->in_flight == 0; });
  if (!ok) return ht_fail(HT_EDEVICE, "server still busy after %.1f s", timeout_s);
  return HT_OK;
}

ht_status ht_server_poll(ht_server* s, int64_t max, int64_t* ids, int* status, double* values,
                         double* t_submit, double* t_admit, double* t_done, int64_t* count) {
  if (!s || !count) return ht_fail(HT_EINVAL, "server or count is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  int64_t c = 0;
  while (c < max && !s->outbox.empty()) {
    std::unique_ptr<Req> r = std::move(s->outbox.front());
    s->outbox.pop_front();
    if (ids) ids[c] = r->id;
    if (status) status[c] = r->status;
    if (values) values[c] = r->value;
    if (t_submit) t_submit[c] = r->t_submit;
    if (t_admit) t_admit[c] = r->t_admit;
    if (t_done) t_done[c] = r->t_done;
    ++c;
  }
  *count = c;
  return HT_OK;
}

ht_status ht_server_now(const ht_server* s, double* t) {
  if (!s || !t) return ht_fail(HT_EINVAL, "server or t is NULL");
  *t = s->now();
  return HT_OK;
}

ht_status ht_server_last_error(ht_server* s, char* buf, size_t len) {
  if (!s || !buf || !len) return ht_fail(HT_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  std::snprintf(buf, len, "%s", s->error.c_str());
  return HT_OK;
}

ht_status ht_server_destroy(ht_server* s) {
  if (!s) return HT_OK;
  s->stop.store(true);
  if (s->worker.joinable()) s->worker.join();
  ht_device_guard dg(s->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : s->pool) (void)hipFree(kv.second);
  for (auto& sl : s->slots) {
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ev_init) (void)hipEventDestroy(sl.ev_init);
    if (sl.ev_chunk[0]) (void)hipEventDestroy(sl.ev_chunk[0]);
    if (sl.ev_chunk[1]) (void)hipEventDestroy(sl.ev_chunk[1]);
    if (sl.ev_done) (void)hipEventDestroy(sl.ev_done);
    if (sl.red) (void)hipFree(sl.red);
    if (sl.terms_dev) (void)hipFree(sl.terms_dev);
    if (sl.coef_dev) (void)hipFree(sl.coef_dev);
    if (sl.out_dev) (void)hipFree(sl.out_dev);
  }
  if (s->batch_stream) (void)hipStreamDestroy(s->batch_stream);
  delete s;
  return HT_OK;
}

}  // extern "C"
