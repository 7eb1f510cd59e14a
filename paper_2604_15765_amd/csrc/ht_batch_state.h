// State behind the ht_batch handle, shared by the batch API and its autotuner.
#pragma once

#include <cstddef>
#include <unordered_map>
#include <vector>

#include "ht_batch_runner.h"
#include "ht_handle.h"
#include "ht_internal.h"

// Largest LDS stage of one operator: the 160 KiB of a compute unit minus
// room for the batch kernel's own static LDS.
constexpr int64_t kBatchLdsMax = 160 * 1024 - 256;

struct ht_batch {
  // An op as the caller gave it, kept so that it can be prepared again for
  // another tile edge (the autotuner does).
  struct RawOp {
    int k, targets[2], r, heisenberg;
    size_t mat_off;  // offset (doubles) into Entry::mats
  };
  struct Entry {
    ht_herm* h;
    std::vector<ht::BatchOp> ops;
    std::vector<double> coefs;
    std::vector<RawOp> raw;
    std::vector<double> mats;
    // fused op list (ops and coefficients) for fuse_q, rebuilt when stale
    int fused_q = -1;
    std::vector<ht::BatchOp> fused_ops;
    std::vector<double> fused_coefs;
  };
  std::vector<Entry> entries;
  std::unordered_map<ht_herm*, size_t> index;
  int device = 0;
  int num_cu = 256;
  ht::BatchSchedule sched;
  int fuse_q = 0;  // 0: one pass per op; 1, 2: fused passes on at most that many qubits
  ht::BatchRunner runner;
};

namespace ht {

// Append a prepared op (k <= 2) to an op list and its coefficients to coefs.
inline void append_batch_op(const PreparedOp& op, std::vector<BatchOp>& ops,
                            std::vector<double>& coefs) {
  BatchOp bo{};
  bo.k = op.k;
  bo.ncross = op.ncross;
  bo.form = op.form;
  bo.sorted[0] = op.sorted[0];
  bo.sorted[1] = op.k > 1 ? op.sorted[1] : 0;
  bo.coef_off = (uint32_t)coefs.size();
  for (int u = 0; u < 4; ++u) bo.perm[u] = u < (1 << op.k) ? op.perm[u] : u;
  bo.active = (uint32_t)op.active;
  coefs.insert(coefs.end(), op.coef, op.coef + op_coef_doubles(op.k, op.form));
  ops.push_back(bo);
}

// The op list of entry e for tile exponent m_eff (the operator's own or a
// candidate's) with fusion on at most fuse_q qubits (0: the ops as queued,
// prepared again).  Returns 0 or nonzero with a message.
int entry_ops(const ht_batch::Entry& e, int m_eff, int fuse_q, std::vector<BatchOp>& ops,
              std::vector<double>& coefs, char* err, size_t errlen);

}  // namespace ht
