// Circuits: op sequences applied with fusion of neighbouring ops (the
// planner and composer live in ht_fuse.cpp).  The C ABI keeps the ops,
// plans them for a picture and a pass size, reports the passes and applies
// them to an operator.
#include <hip/hip_runtime.h>

#include <vector>

#include "hermtile.h"
#include "ht_fuse.h"
#include "ht_handle.h"
#include "ht_internal.h"

namespace {

struct COp {
  ht::FuseOp view;
  std::vector<double> mats;
};

}  // namespace

struct ht_circuit {
  std::vector<COp> ops;
  // last plan
  int picture = -1;
  std::vector<const ht::FuseOp*> seq;
  std::vector<ht::FusePass> passes;
  bool planned = false;
};

namespace {

ht_status add(ht_circuit* c, int k, const int* targets, int r, const double* mats) {
  if (!c || !targets || !mats) return ht_fail(HT_EINVAL, "NULL argument");
  if (k < 1 || k > 3) return ht_fail(HT_EINVAL, "k must be 1, 2 or 3");
  const int D = 1 << k;
  if (r < 1 || r > D * D) return ht_fail(HT_EINVAL, "Kraus rank r must satisfy 1 <= r <= 4^k");
  for (int l = 0; l < k; ++l) {
    if (targets[l] < 0 || targets[l] >= HT_MAX_QUBITS)
      return ht_fail(HT_EINVAL, "target qubit out of range");
    for (int l2 = 0; l2 < l; ++l2)
      if (targets[l] == targets[l2]) return ht_fail(HT_EINVAL, "targets must be distinct");
  }
  c->ops.emplace_back();
  COp& o = c->ops.back();
  o.mats.assign(mats, mats + (size_t)2 * r * D * D);
  o.view.k = k;
  for (int l = 0; l < 3; ++l) o.view.targets[l] = l < k ? targets[l] : -1;
  o.view.r = r;
  o.view.adj = 0;
  o.view.mats = o.mats.data();  // stays valid: moving a vector keeps its buffer
  c->planned = false;
  return HT_OK;
}

}  // namespace

extern "C" {

ht_status ht_circuit_create(ht_circuit** out) {
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  *out = new ht_circuit();
  return HT_OK;
}

ht_status ht_circuit_destroy(ht_circuit* c) {
  delete c;  // NULL is fine
  return HT_OK;
}

ht_status ht_circuit_add_unitary(ht_circuit* c, int k, const int* targets, const double* U) {
  return add(c, k, targets, 1, U);
}

ht_status ht_circuit_add_channel(ht_circuit* c, int k, const int* targets, int r, const double* kraus) {
  return add(c, k, targets, r, kraus);
}

ht_status ht_circuit_size(const ht_circuit* c, int64_t* nops) {
  if (!c || !nops) return ht_fail(HT_EINVAL, "NULL argument");
  *nops = (int64_t)c->ops.size();
  return HT_OK;
}

ht_status ht_circuit_plan(ht_circuit* c, ht_picture picture, int max_qubits, int64_t* npasses) {
  if (!c) return ht_fail(HT_EINVAL, "circuit is NULL");
  if (picture != HT_SCHRODINGER && picture != HT_HEISENBERG)
    return ht_fail(HT_EINVAL, "unknown picture %d", (int)picture);
  if (max_qubits < 0 || max_qubits > 2) return ht_fail(HT_EINVAL, "max_qubits must be 0, 1 or 2");
  const bool adj = picture == HT_HEISENBERG;
  c->seq.clear();
  for (size_t i = 0; i < c->ops.size(); ++i) {
    COp& o = c->ops[adj ? c->ops.size() - 1 - i : i];
    o.view.adj = adj ? 1 : 0;
    c->seq.push_back(&o.view);
  }
  c->passes = ht::fuse_plan(c->seq, max_qubits);
  for (auto& p : c->passes)
    if (p.ops.size() > 1) ht::fuse_compose(p, c->seq, false);
  c->picture = picture;
  c->planned = true;
  if (npasses) *npasses = (int64_t)c->passes.size();
  return HT_OK;
}

ht_status ht_circuit_pass_info(const ht_circuit* c, int64_t i, int* k, int* targets, int64_t* nops,
                               int64_t* op_indices, double* transfer) {
  if (!c || !c->planned) return ht_fail(HT_EINVAL, "circuit is NULL or not planned");
  if (i < 0 || i >= (int64_t)c->passes.size()) return ht_fail(HT_EINVAL, "pass index out of range");
  const ht::FusePass& p = c->passes[i];
  const bool adj = c->picture == HT_HEISENBERG;  // the plan ran over the reversed ops
  const int64_t total = (int64_t)c->ops.size();
  if (k) *k = p.k;
  if (targets)
    for (int l = 0; l < p.k; ++l) targets[l] = p.sorted[l];
  if (nops) *nops = (int64_t)p.ops.size();
  if (op_indices)  // indices into the circuit as added
    for (size_t j = 0; j < p.ops.size(); ++j) op_indices[j] = adj ? total - 1 - p.ops[j] : p.ops[j];
  if (transfer) {
    if (p.k > 2) return ht_fail(HT_EUNSUPPORTED, "pass %lld acts on 3 qubits", (long long)i);
    // transfer matrix of the pass (row-major block vector, ascending bits)
    ht::FusePass q = p;
    ht::fuse_compose(q, c->seq, true);
    const int DD = 1 << (2 * p.k);
    for (int e = 0; e < DD * DD; ++e) {
      transfer[2 * e] = q.mat[e].real();
      transfer[2 * e + 1] = q.mat[e].imag();
    }
  }
  return HT_OK;
}

ht_status ht_circuit_apply(ht_circuit* c, ht_herm* h) {
  if (!c || !h) return ht_fail(HT_EINVAL, "circuit or handle is NULL");
  if (!c->planned) return ht_fail(HT_EINVAL, "plan the circuit first (ht_circuit_plan)");
  // prepare every pass before enqueueing any, so a bad op leaves h untouched
  std::vector<ht::PreparedOp> prepared(c->passes.size());
  char msg[256];
  for (size_t i = 0; i < c->passes.size(); ++i) {
    const ht::FusePass& p = c->passes[i];
    for (int l = 0; l < p.k; ++l)
      if (p.sorted[l] >= h->n) return ht_fail(HT_EINVAL, "pass %zu: qubit %d >= n", i, p.sorted[l]);
    if (ht::fuse_prepare(p, c->seq, h->n, h->m, ht::native_policy(h->bytes), &prepared[i], msg,
                         sizeof msg) != 0)
      return ht_fail(HT_EINVAL, "pass %zu: %s", i, msg);
  }
  for (const ht::PreparedOp& op : prepared) {
    const ht_status st = ht_launch_prepared(h, op);
    if (st != HT_OK) return st;
  }
  return HT_OK;
}

}  // extern "C"
