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
#include "ht_batch_runner.h"
#include "ht_batch_state.h"
#include "ht_fuse.h"
#include "ht_prep.h"

struct ht_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace ht {

int entry_ops(const ht_batch::Entry& e, int m_eff, int fuse_q, std::vector<BatchOp>& ops,
              std::vector<double>& coefs, char* err, size_t errlen) {
  ops.clear();
  coefs.clear();
  std::vector<FuseOp> fops(e.raw.size());
  std::vector<const FuseOp*> seq(e.raw.size());
  for (size_t i = 0; i < e.raw.size(); ++i) {
    const ht_batch::RawOp& r = e.raw[i];
    FuseOp& f = fops[i];
    f.k = r.k;
    f.targets[0] = r.targets[0];
    f.targets[1] = r.targets[1];
    f.targets[2] = -1;
    f.r = r.r;
    f.adj = r.heisenberg;
    f.mats = e.mats.data() + r.mat_off;
    seq[i] = &f;
  }
  std::vector<PreparedOp> prepared;
  const size_t bytes = ht_storage_bytes(e.h->n, m_eff, e.h->dtype == 0 ? HT_C128 : HT_C64);
  if (fuse_ops(seq, fuse_q, e.h->n, m_eff, native_policy(bytes), &prepared, err, errlen) != 0) return 1;
  for (const PreparedOp& op : prepared) append_batch_op(op, ops, coefs);
  return 0;
}

}  // namespace ht

namespace {

ht_status add_op(ht_batch* b, ht_herm* h, int k, const int* targets, int r, const double* mats,
                 ht_picture picture) {
  if (!b || !h) return ht_fail(HT_EINVAL, "batch or handle is NULL");
  if (picture != HT_SCHRODINGER && picture != HT_HEISENBERG)
    return ht_fail(HT_EINVAL, "unknown picture %d", (int)picture);
  if (!b->entries.empty() && h->device != b->device)
    return ht_fail(HT_EINVAL, "all operators of a batch must live on one device");
  if (k != 1 && k != 2) return ht_fail(HT_EINVAL, "batches take ops with k = 1 or 2");
  ht::PreparedOp op;
  char msg[256];
  if (ht::prepare_op(h->n, h->m, k, targets, r, mats, picture == HT_HEISENBERG, &op, msg,
                     sizeof msg, ht::native_policy(h->bytes)) != 0)
    return ht_fail(HT_EINVAL, "%s", msg);
  auto it = b->index.find(h);
  size_t e;
  if (it == b->index.end()) {
    if (b->entries.empty()) {
      b->device = h->device;
      b->num_cu = h->num_cu;
    }
    e = b->entries.size();
    b->entries.emplace_back();
    b->entries.back().h = h;
    b->index[h] = e;
  } else {
    e = it->second;
  }
  auto& en = b->entries[e];
  ht::append_batch_op(op, en.ops, en.coefs);
  en.fused_q = -1;  // the fused list is stale
  const int D = 1 << k;
  ht_batch::RawOp raw{};
  raw.k = k;
  raw.targets[0] = targets[0];
  raw.targets[1] = k > 1 ? targets[1] : 0;
  raw.r = r;
  raw.heisenberg = picture == HT_HEISENBERG ? 1 : 0;
  raw.mat_off = en.mats.size();
  en.mats.insert(en.mats.end(), mats, mats + (size_t)2 * r * D * D);
  en.raw.push_back(raw);
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
  delete b;  // the runner waits for its last launch and frees its tables
  return HT_OK;
}

ht_status ht_batch_set_param(ht_batch* b, const char* name, int64_t value) {
  if (!b || !name) return ht_fail(HT_EINVAL, "batch or name is NULL");
  const std::string k(name);
  if (k == "threads") {
    if (value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
      return ht_fail(HT_EINVAL, "threads must be 64, 128, 256, 512 or 1024");
    b->sched.threads = (int)value;
  } else if (k == "wg_per_cu") {
    if (value < 1 || value > 32) return ht_fail(HT_EINVAL, "wg_per_cu must be in [1, 32]");
    b->sched.wg_per_cu = (int)value;
  } else if (k == "fuse_qubits") {
    if (value < 0 || value > 2) return ht_fail(HT_EINVAL, "fuse_qubits must be 0, 1 or 2");
    b->fuse_q = (int)value;
  } else if (k == "lds_max_bytes") {
    if (value < 0 || value > kBatchLdsMax)
      return ht_fail(HT_EINVAL, "lds_max_bytes must be in [0, %lld]", (long long)kBatchLdsMax);
    b->sched.lds_max = (size_t)value;
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
  // earlier work on the operators' own streams must be complete
  std::vector<hipStream_t> seen;
  for (const auto& e : b->entries)
    if (e.h->stream != s && std::find(seen.begin(), seen.end(), e.h->stream) == seen.end()) {
      seen.push_back(e.h->stream);
      HT_HIP(hipStreamSynchronize(e.h->stream));
    }
  std::vector<ht::BatchItem> items;
  items.reserve(b->entries.size());
  char msg[256];
  for (auto& e : b->entries) {
    const std::vector<ht::BatchOp>* ops = &e.ops;
    const std::vector<double>* coefs = &e.coefs;
    if (b->fuse_q > 0) {
      if (e.fused_q != b->fuse_q) {
        if (ht::entry_ops(e, e.h->m, b->fuse_q, e.fused_ops, e.fused_coefs, msg, sizeof msg) != 0)
          return ht_fail(HT_EINVAL, "fusing the ops of an operator: %s", msg);
        e.fused_q = b->fuse_q;
      }
      ops = &e.fused_ops;
      coefs = &e.fused_coefs;
    }
    items.push_back(ht::BatchItem{e.h->buf, e.h->bytes, e.h->n, e.h->m, e.h->dtype, ops->data(),
                                  (uint32_t)ops->size(), coefs->data(), (uint32_t)coefs->size()});
  }
  HT_HIP(b->runner.run(items, b->sched, b->num_cu, s));
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
