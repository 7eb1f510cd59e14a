// C-ABI of batched execution and of captured op sequences (HIP graphs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "hermtile.h"
#include "ht_handle.h"
#include "ht_internal.h"
#include "ht_prep.h"

struct ht_batch {
  struct Entry {
    ht_herm* h;
    std::vector<ht::BatchOp> ops;
    std::vector<double> coefs;
  };
  std::vector<Entry> entries;
  std::unordered_map<ht_herm*, size_t> index;
  int device = 0;
  int num_cu = 256;
  int threads = 256;
  int wg_per_cu = 2;
  size_t lds_max = 64 * 1024;
  size_t lds_set[2] = {0, 0};
  // device tables, per dtype: [opers | ops | coefs], and two queue counters
  void* dev = nullptr;
  size_t dev_cap = 0;
  unsigned* counters = nullptr;
  void* stage = nullptr;  // pinned host staging of the tables
  size_t stage_cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

struct ht_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

ht_status add_op(ht_batch* b, ht_herm* h, int k, const int* targets, int r, const double* mats,
                 ht_picture picture) {
  if (!b || !h) return ht_fail(HT_EINVAL, "batch or handle is NULL");
  if (picture != HT_SCHRODINGER && picture != HT_HEISENBERG)
    return ht_fail(HT_EINVAL, "unknown picture %d", (int)picture);
  if (!b->entries.empty() && h->device != b->device)
    return ht_fail(HT_EINVAL, "all operators of a batch must live on one device");
  ht::PreparedOp op;
  char msg[256];
  if (ht::prepare_op(h->n, h->m, k, targets, r, mats, picture == HT_HEISENBERG, &op, msg,
                     sizeof msg) != 0)
    return ht_fail(HT_EINVAL, "%s", msg);
  auto it = b->index.find(h);
  size_t e;
  if (it == b->index.end()) {
    if (b->entries.empty()) {
      b->device = h->device;
      b->num_cu = h->num_cu;
    }
    e = b->entries.size();
    b->entries.push_back({h, {}, {}});
    b->index[h] = e;
  } else {
    e = it->second;
  }
  auto& en = b->entries[e];
  ht::BatchOp bo{};
  bo.k = op.k;
  bo.ncross = op.ncross;
  bo.form = op.form;
  bo.sorted[0] = op.sorted[0];
  bo.sorted[1] = op.k > 1 ? op.sorted[1] : 0;
  bo.coef_off = (uint32_t)en.coefs.size();
  const int D = 1 << op.k;
  const int nd = 2 * (op.form == 0 ? D * D : D * D * D * D);
  en.coefs.insert(en.coefs.end(), op.coef, op.coef + nd);
  en.ops.push_back(bo);
  return HT_OK;
}

}  // namespace

extern "C" {

ht_status ht_batch_create(ht_batch** out) {
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  *out = new ht_batch();
  return HT_OK;
}

ht_status ht_batch_destroy(ht_batch* b) {
  if (!b) return HT_OK;
  ht_device_guard dg(b->device);
  if (b->done) {
    (void)hipEventSynchronize(b->done);
    (void)hipEventDestroy(b->done);
  }
  if (b->dev) (void)hipFree(b->dev);
  if (b->counters) (void)hipFree(b->counters);
  if (b->stage) (void)hipHostFree(b->stage);
  delete b;
  return HT_OK;
}

ht_status ht_batch_set_param(ht_batch* b, const char* name, int64_t value) {
  if (!b || !name) return ht_fail(HT_EINVAL, "batch or name is NULL");
  const std::string k(name);
  if (k == "threads") {
    if (value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
      return ht_fail(HT_EINVAL, "threads must be 64, 128, 256, 512 or 1024");
    b->threads = (int)value;
  } else if (k == "wg_per_cu") {
    if (value < 1 || value > 32) return ht_fail(HT_EINVAL, "wg_per_cu must be in [1, 32]");
    b->wg_per_cu = (int)value;
  } else if (k == "lds_max_bytes") {
    if (value < 0 || value > 160 * 1024) return ht_fail(HT_EINVAL, "lds_max_bytes must be in [0, 163840]");
    b->lds_max = (size_t)value;
  } else {
    return ht_fail(HT_EINVAL, "unknown batch parameter '%s'", name);
  }
  return HT_OK;
}

ht_status ht_batch_add_unitary(ht_batch* b, ht_herm* h, int k, const int* targets, const double* U,
                               ht_picture picture) {
  return add_op(b, h, k, targets, 1, U, picture);
}

ht_status ht_batch_add_channel(ht_batch* b, ht_herm* h, int k, const int* targets, int r,
                               const double* kraus, ht_picture picture) {
  return add_op(b, h, k, targets, r, kraus, picture);
}

ht_status ht_batch_clear(ht_batch* b) {
  if (!b) return ht_fail(HT_EINVAL, "batch is NULL");
  b->entries.clear();
  b->index.clear();
  return HT_OK;
}

ht_status ht_batch_size(const ht_batch* b, int64_t* noperators, int64_t* nops) {
  if (!b) return ht_fail(HT_EINVAL, "batch is NULL");
  int64_t t = 0;
  for (const auto& e : b->entries) t += (int64_t)e.ops.size();
  if (noperators) *noperators = (int64_t)b->entries.size();
  if (nops) *nops = t;
  return HT_OK;
}

ht_status ht_batch_run(ht_batch* b, void* hip_stream) {
  if (!b) return ht_fail(HT_EINVAL, "batch is NULL");
  if (b->entries.empty()) return HT_OK;
  ht_device_guard dg(b->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  // the staging buffer may still feed the previous run's copies
  if (b->pending) {
    HT_HIP(hipEventSynchronize(b->done));
    b->pending = false;
  }
  // earlier work on the operators' own streams must be complete
  std::vector<hipStream_t> seen;
  for (const auto& e : b->entries)
    if (e.h->stream != s && std::find(seen.begin(), seen.end(), e.h->stream) == seen.end()) {
      seen.push_back(e.h->stream);
      HT_HIP(hipStreamSynchronize(e.h->stream));
    }
  // order: per dtype, largest work first (longest-processing-time-first queue)
  std::vector<size_t> order[2];
  for (size_t i = 0; i < b->entries.size(); ++i) order[b->entries[i].h->dtype].push_back(i);
  for (auto& o : order)
    std::stable_sort(o.begin(), o.end(), [&](size_t x, size_t y) {
      const auto& a = b->entries[x];
      const auto& c = b->entries[y];
      return (double)a.h->bytes * a.ops.size() > (double)c.h->bytes * c.ops.size();
    });
  size_t nopers[2] = {order[0].size(), order[1].size()}, nops[2] = {0, 0}, ncoef[2] = {0, 0};
  for (int d = 0; d < 2; ++d)
    for (size_t i : order[d]) {
      nops[d] += b->entries[i].ops.size();
      ncoef[d] += b->entries[i].coefs.size();
    }
  // layout of the tables (identical in the staging buffer and on the device)
  size_t off_opers[2], off_ops[2], off_coef[2], total = 0;
  for (int d = 0; d < 2; ++d) {
    off_opers[d] = total;
    total = align_up(total + nopers[d] * sizeof(ht::BatchOperator), 256);
    off_ops[d] = total;
    total = align_up(total + nops[d] * sizeof(ht::BatchOp), 256);
    off_coef[d] = total;
    total = align_up(total + ncoef[d] * sizeof(double), 256);
  }
  if (b->stage_cap < total) {
    if (b->stage) HT_HIP(hipHostFree(b->stage));
    b->stage = nullptr;
    b->stage_cap = 0;
    if (hipHostMalloc(&b->stage, total, hipHostMallocDefault) != hipSuccess)
      return ht_fail(HT_ENOMEM, "could not allocate %zu bytes of pinned staging", total);
    b->stage_cap = total;
  }
  if (b->dev_cap < total) {
    if (b->dev) HT_HIP(hipFree(b->dev));
    b->dev = nullptr;
    b->dev_cap = 0;
    if (hipMalloc(&b->dev, total) != hipSuccess)
      return ht_fail(HT_ENOMEM, "could not allocate %zu bytes of batch tables", total);
    b->dev_cap = total;
  }
  if (!b->counters && hipMalloc(&b->counters, 2 * sizeof(unsigned)) != hipSuccess) {
    b->counters = nullptr;
    return ht_fail(HT_ENOMEM, "could not allocate the batch queue counters");
  }
  if (!b->done) HT_HIP(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
  char* st = reinterpret_cast<char*>(b->stage);
  size_t lds_need[2] = {0, 0};
  for (int d = 0; d < 2; ++d) {
    auto* opers = reinterpret_cast<ht::BatchOperator*>(st + off_opers[d]);
    auto* ops = reinterpret_cast<ht::BatchOp*>(st + off_ops[d]);
    auto* coefs = reinterpret_cast<double*>(st + off_coef[d]);
    uint32_t op_pos = 0;
    uint32_t coef_pos = 0;
    for (size_t r = 0; r < order[d].size(); ++r) {
      const auto& e = b->entries[order[d][r]];
      ht::BatchOperator o{};
      o.buf = e.h->buf;
      o.bytes = e.h->bytes;
      o.n = e.h->n;
      o.m = e.h->m;
      o.op_begin = op_pos;
      o.op_end = op_pos + (uint32_t)e.ops.size();
      o.in_lds = e.h->bytes <= b->lds_max ? 1 : 0;
      if (o.in_lds) lds_need[d] = std::max(lds_need[d], (size_t)e.h->bytes);
      opers[r] = o;
      for (const auto& op : e.ops) {
        ht::BatchOp x = op;
        x.coef_off += coef_pos;
        ops[op_pos++] = x;
      }
      std::memcpy(coefs + coef_pos, e.coefs.data(), e.coefs.size() * sizeof(double));
      coef_pos += (uint32_t)e.coefs.size();
    }
  }
  HT_HIP(hipMemcpyAsync(b->dev, b->stage, total, hipMemcpyHostToDevice, s));
  char* dv = reinterpret_cast<char*>(b->dev);
  for (int d = 0; d < 2; ++d) {
    if (nopers[d] == 0) continue;
    if (lds_need[d] > b->lds_set[d]) {
      HT_HIP(ht::set_batch_lds_limit(d, lds_need[d]));
      b->lds_set[d] = lds_need[d];
    }
    int grid = b->num_cu * b->wg_per_cu;
    if ((size_t)grid > nopers[d]) grid = (int)nopers[d];
    HT_HIP(ht::launch_batch(d, reinterpret_cast<const ht::BatchOperator*>(dv + off_opers[d]),
                            (unsigned)nopers[d], reinterpret_cast<const ht::BatchOp*>(dv + off_ops[d]),
                            reinterpret_cast<const double*>(dv + off_coef[d]), b->counters + d,
                            b->threads, grid, lds_need[d], s));
  }
  HT_HIP(hipEventRecord(b->done, s));
  b->pending = true;
  return HT_OK;
}

ht_status ht_capture_begin(void* hip_stream) {
  if (!hip_stream) return ht_fail(HT_EINVAL, "capture needs a non-null stream");
  HT_HIP(hipStreamBeginCapture(reinterpret_cast<hipStream_t>(hip_stream),
                               hipStreamCaptureModeThreadLocal));
  return HT_OK;
}

ht_status ht_capture_end(void* hip_stream, ht_graph** out) {
  if (!hip_stream || !out) return ht_fail(HT_EINVAL, "stream or out is NULL");
  *out = nullptr;
  hipGraph_t g = nullptr;
  HT_HIP(hipStreamEndCapture(reinterpret_cast<hipStream_t>(hip_stream), &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return ht_fail(HT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  ht_graph* r = new ht_graph();
  r->graph = g;
  r->exec = ex;
  *out = r;
  return HT_OK;
}

ht_status ht_graph_launch(ht_graph* g, void* hip_stream) {
  if (!g) return ht_fail(HT_EINVAL, "graph is NULL");
  HT_HIP(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(hip_stream)));
  return HT_OK;
}

ht_status ht_graph_destroy(ht_graph* g) {
  if (!g) return HT_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return HT_OK;
}

}  // extern "C"
