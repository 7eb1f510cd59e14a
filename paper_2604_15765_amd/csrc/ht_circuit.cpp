// Circuits: op sequences applied with fusion of neighbouring ops.
//
// Each conjugation pass streams the whole operator through HBM (Section
// III-C), so a sequence of L ops costs L passes.  Ops that together act on at
// most two qubits compose into one 2-qubit map (its transfer matrix is the
// product of theirs, Eq. (3)), which one pass applies.  The planner groups
// ops greedily: starting from the earliest op not yet applied, it absorbs
// later ops whose qubits keep the group within max_qubits, as long as no
// skipped op in between shares a qubit with them (ops on disjoint qubits
// commute, so moving an absorbed op ahead of skipped ones does not change
// the map).  A group grows towards the qubits of the next op that couples it
// to other qubits, so a 1-qubit op joins the partner of its next 2-qubit
// gate.  A group of one op runs exactly as ht_apply_* would run it.
//
// The Heisenberg picture applies the adjoint maps in reverse order; the
// planner works on that sequence with the adjoint Kraus operators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstring>
#include <vector>

#include "hermtile.h"
#include "ht_handle.h"
#include "ht_internal.h"
#include "ht_prep.h"

using cplx = std::complex<double>;

namespace {

struct COp {
  int k;
  int targets[3];
  int r;                    // 1: unitary (mats holds U)
  std::vector<double> mats; // r x 2^k x 2^k interleaved complex, caller's order
};

struct CPass {
  std::vector<int> ops;     // indices into the effective sequence, in order
  int k;                    // qubits of the pass
  int sorted[3];            // ascending qubits
  bool unitary;             // every op a unitary
  std::vector<cplx> mat;    // composed map: U (D x D) or S (D^2 x D^2), ascending local bits
};

// Kraus operator a of op o as a 2^k x 2^k complex matrix in the effective
// (Schroedinger) sequence: adjoined for the Heisenberg picture.
cplx kraus_at(const COp& o, int a, int row, int col, bool adj) {
  const int D = 1 << o.k;
  const double* L = o.mats.data() + (size_t)2 * D * D * a;
  if (adj) return std::conj(cplx(L[2 * (col * D + row)], L[2 * (col * D + row) + 1]));
  return cplx(L[2 * (row * D + col)], L[2 * (row * D + col) + 1]);
}

// Lift Kraus operator a of op o to the pass qubits q[0..kq) (ascending):
// L_Q[u][v] = L[a(u)][a(v)] when u and v agree on the pass bits the op does
// not act on, else 0; a(u) collects u's bits at the op's targets.
void lift(const COp& o, int a, bool adj, const int* q, int kq, cplx* out) {
  const int DQ = 1 << kq;
  int pos[3];
  int opmask = 0;
  for (int l = 0; l < o.k; ++l) {
    for (int j = 0; j < kq; ++j)
      if (q[j] == o.targets[l]) pos[l] = j;
    opmask |= 1 << pos[l];
  }
  for (int u = 0; u < DQ; ++u)
    for (int v = 0; v < DQ; ++v) {
      if ((u & ~opmask) != (v & ~opmask)) {
        out[u * DQ + v] = 0.0;
        continue;
      }
      int au = 0, av = 0;
      for (int l = 0; l < o.k; ++l) {
        au |= ((u >> pos[l]) & 1) << l;
        av |= ((v >> pos[l]) & 1) << l;
      }
      out[u * DQ + v] = kraus_at(o, a, au, av, adj);
    }
}

uint32_t mask_of(const COp& o) {
  uint32_t m = 0;
  for (int l = 0; l < o.k; ++l) m |= 1u << o.targets[l];
  return m;
}

// Greedy grouping of the effective sequence (see the file comment).
std::vector<CPass> plan(const std::vector<const COp*>& seq, int max_q) {
  const size_t n = seq.size();
  std::vector<char> done(n, 0);
  std::vector<CPass> passes;
  size_t first = 0;
  constexpr size_t kWindow = 4096;  // ops scanned beyond the group's first
  while (first < n) {
    while (first < n && done[first]) ++first;
    if (first >= n) break;
    CPass p;
    p.ops.push_back((int)first);
    done[first] = 1;
    uint32_t Q = mask_of(*seq[first]);
    if (seq[first]->k <= max_q) {
      // The qubits to grow into: those of the next op that couples the
      // group's qubits to others within the size bound (so that a 1-qubit op
      // is grouped with the partner of its next 2-qubit gate); without such
      // an op, any qubits within the bound.
      uint32_t allow = 0;
      if (__builtin_popcount(Q) < max_q)
        for (size_t o = first + 1; o < n && o <= first + kWindow; ++o) {
          if (done[o]) continue;
          const uint32_t T = mask_of(*seq[o]);
          if (!(T & Q)) continue;
          if ((T & ~Q) && seq[o]->k <= max_q && __builtin_popcount(Q | T) <= max_q) allow = Q | T;
          if (T & ~Q) break;  // the first op that reaches beyond the group decides
        }
      uint32_t blocked = 0;
      for (size_t o = first + 1; o < n && o <= first + kWindow; ++o) {
        if (done[o]) continue;
        const uint32_t T = mask_of(*seq[o]);
        const bool fits = allow ? (T & ~allow) == 0 : __builtin_popcount(Q | T) <= max_q;
        if (!(T & blocked) && seq[o]->k <= max_q && fits) {
          Q |= T;
          p.ops.push_back((int)o);
          done[o] = 1;
        } else {
          blocked |= T;
        }
        if (__builtin_popcount(Q) == max_q && (Q & ~blocked) == 0) break;  // nothing more can join
        if (allow && (allow & ~blocked) == 0) break;
      }
    }
    p.k = 0;
    for (int b = 0; b < 32; ++b)
      if ((Q >> b) & 1) p.sorted[p.k++] = b;
    p.unitary = true;
    for (int i : p.ops) p.unitary = p.unitary && seq[i]->r == 1;
    passes.push_back(std::move(p));
  }
  return passes;
}

// Compose the ops of a pass of two or more ops (effective Schroedinger
// order): U = U_last ... U_first, or S = S_last ... S_first with
// S_op = sum_a L_a (x) conj(L_a) on the row-major block vector.
void compose(CPass& p, const std::vector<const COp*>& seq, bool adj) {
  const int DQ = 1 << p.k, DD = DQ * DQ;
  std::vector<cplx> L(DQ * DQ);
  if (p.unitary) {
    std::vector<cplx> U(DQ * DQ, 0.0), T(DQ * DQ);
    for (int u = 0; u < DQ; ++u) U[u * DQ + u] = 1.0;
    for (int i : p.ops) {
      lift(*seq[i], 0, adj, p.sorted, p.k, L.data());
      for (int u = 0; u < DQ; ++u)
        for (int v = 0; v < DQ; ++v) {
          cplx s = 0.0;
          for (int w = 0; w < DQ; ++w) s += L[u * DQ + w] * U[w * DQ + v];
          T[u * DQ + v] = s;
        }
      U.swap(T);
    }
    p.mat = std::move(U);
    return;
  }
  std::vector<cplx> S(DD * DD, 0.0), So(DD * DD), T(DD * DD);
  for (int e = 0; e < DD; ++e) S[e * DD + e] = 1.0;
  for (int i : p.ops) {
    const COp& o = *seq[i];
    std::fill(So.begin(), So.end(), cplx(0.0));
    for (int a = 0; a < o.r; ++a) {
      lift(o, a, adj, p.sorted, p.k, L.data());
      for (int u = 0; u < DQ; ++u)
        for (int v = 0; v < DQ; ++v)
          for (int u2 = 0; u2 < DQ; ++u2)
            for (int v2 = 0; v2 < DQ; ++v2)
              So[(u * DQ + v) * DD + (u2 * DQ + v2)] += L[u * DQ + u2] * std::conj(L[v * DQ + v2]);
    }
    for (int e = 0; e < DD; ++e)
      for (int f = 0; f < DD; ++f) {
        cplx s = 0.0;
        for (int g = 0; g < DD; ++g) s += So[e * DD + g] * S[g * DD + f];
        T[e * DD + f] = s;
      }
    S.swap(T);
  }
  p.mat = std::move(S);
}

}  // namespace

struct ht_circuit {
  std::vector<COp> ops;
  // last plan
  int picture = -1, max_q = -1;
  std::vector<const COp*> seq;
  std::vector<CPass> passes;
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
  COp o;
  o.k = k;
  for (int l = 0; l < 3; ++l) o.targets[l] = l < k ? targets[l] : -1;
  o.r = r;
  o.mats.assign(mats, mats + (size_t)2 * r * D * D);
  c->ops.push_back(std::move(o));
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
  for (size_t i = 0; i < c->ops.size(); ++i)
    c->seq.push_back(&c->ops[adj ? c->ops.size() - 1 - i : i]);
  c->passes = plan(c->seq, max_qubits == 0 ? 0 : max_qubits);
  for (auto& p : c->passes)
    if (p.ops.size() > 1) compose(p, c->seq, adj);
  c->picture = picture;
  c->max_q = max_qubits;
  c->planned = true;
  if (npasses) *npasses = (int64_t)c->passes.size();
  return HT_OK;
}

ht_status ht_circuit_pass_info(const ht_circuit* c, int64_t i, int* k, int* targets, int64_t* nops,
                               int64_t* op_indices, double* transfer) {
  if (!c || !c->planned) return ht_fail(HT_EINVAL, "circuit is NULL or not planned");
  if (i < 0 || i >= (int64_t)c->passes.size()) return ht_fail(HT_EINVAL, "pass index out of range");
  const CPass& p = c->passes[i];
  const bool adj = c->picture == HT_HEISENBERG;
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
    CPass q = p;
    q.unitary = false;
    compose(q, c->seq, adj);
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
    const CPass& p = c->passes[i];
    ht::PreparedOp& op = prepared[i];
    for (int l = 0; l < p.k; ++l)
      if (p.sorted[l] >= h->n) return ht_fail(HT_EINVAL, "pass %zu: qubit %d >= n", i, p.sorted[l]);
    int st;
    if (p.ops.size() == 1) {
      const COp& o = *c->seq[p.ops[0]];
      st = ht::prepare_op(h->n, h->m, o.k, o.targets, o.r, o.mats.data(),
                          c->picture == HT_HEISENBERG, &op, msg, sizeof msg, ht::tuning().native);
    } else if (p.unitary) {
      std::vector<double> U(2 * p.mat.size());
      for (size_t e = 0; e < p.mat.size(); ++e) {
        U[2 * e] = p.mat[e].real();
        U[2 * e + 1] = p.mat[e].imag();
      }
      st = ht::prepare_op(h->n, h->m, p.k, p.sorted, 1, U.data(), 0, &op, msg, sizeof msg,
                          ht::tuning().native);
    } else {
      std::vector<double> S(2 * p.mat.size());
      for (size_t e = 0; e < p.mat.size(); ++e) {
        S[2 * e] = p.mat[e].real();
        S[2 * e + 1] = p.mat[e].imag();
      }
      st = ht::prepare_transfer(h->n, h->m, p.k, p.sorted, S.data(), ht::tuning().native, &op, msg,
                                sizeof msg);
    }
    if (st != 0) return ht_fail(HT_EINVAL, "pass %zu: %s", i, msg);
  }
  for (const ht::PreparedOp& op : prepared) {
    const ht_status st = ht_launch_prepared(h, op);
    if (st != HT_OK) return st;
  }
  return HT_OK;
}

}  // extern "C"
