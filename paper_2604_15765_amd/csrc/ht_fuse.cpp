// Fusion of neighbouring ops into passes on at most two qubits.
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
// Each op may be an adjoint map (sum_a L_a^dagger H L_a); a circuit in the
// Heisenberg picture is its ops' adjoint maps in reverse order.
#include "ht_fuse.h"

#include <algorithm>
#include <cstdint>

namespace ht {

using cplx = std::complex<double>;

// Entry (row, col) of the operator A_a that op o applies as A H A^dagger:
// L_a, or L_a^dagger for an adjoint op.
static cplx kraus_at(const FuseOp& o, int a, int row, int col) {
  const int D = 1 << o.k;
  const double* L = o.mats + (size_t)2 * D * D * a;
  if (o.adj) return std::conj(cplx(L[2 * (col * D + row)], L[2 * (col * D + row) + 1]));
  return cplx(L[2 * (row * D + col)], L[2 * (row * D + col) + 1]);
}

// Lift Kraus operator a of op o to the pass qubits q[0..kq) (ascending):
// L_Q[u][v] = L[a(u)][a(v)] when u and v agree on the pass bits the op does
// not act on, else 0; a(u) collects u's bits at the op's targets.
static void lift(const FuseOp& o, int a, const int* q, int kq, cplx* out) {
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
      out[u * DQ + v] = kraus_at(o, a, au, av);
    }
}

static uint32_t mask_of(const FuseOp& o) {
  uint32_t m = 0;
  for (int l = 0; l < o.k; ++l) m |= 1u << o.targets[l];
  return m;
}

// Greedy grouping of the effective sequence (see the file comment).
std::vector<FusePass> fuse_plan(const std::vector<const FuseOp*>& seq, int max_q) {
  const size_t n = seq.size();
  std::vector<char> done(n, 0);
  std::vector<FusePass> passes;
  size_t first = 0;
  constexpr size_t kWindow = 4096;  // ops scanned beyond the group's first
  while (first < n) {
    while (first < n && done[first]) ++first;
    if (first >= n) break;
    FusePass p;
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

void fuse_compose(FusePass& p, const std::vector<const FuseOp*>& seq, bool as_transfer) {
  const int DQ = 1 << p.k, DD = DQ * DQ;
  std::vector<cplx> L(DQ * DQ);
  if (p.unitary && !as_transfer) {
    std::vector<cplx> U(DQ * DQ, 0.0), T(DQ * DQ);
    for (int u = 0; u < DQ; ++u) U[u * DQ + u] = 1.0;
    for (int i : p.ops) {
      lift(*seq[i], 0, p.sorted, p.k, L.data());
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
    const FuseOp& o = *seq[i];
    std::fill(So.begin(), So.end(), cplx(0.0));
    for (int a = 0; a < o.r; ++a) {
      lift(o, a, p.sorted, p.k, L.data());
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


int fuse_prepare(const FusePass& p, const std::vector<const FuseOp*>& seq, int n, int m,
                 int allow_native, PreparedOp* out, char* err, size_t errlen) {
  if (p.ops.size() == 1) {
    const FuseOp& o = *seq[p.ops[0]];
    return prepare_op(n, m, o.k, o.targets, o.r, o.mats, o.adj, out, err, errlen, allow_native);
  }
  std::vector<double> M(2 * p.mat.size());
  for (size_t e = 0; e < p.mat.size(); ++e) {
    M[2 * e] = p.mat[e].real();
    M[2 * e + 1] = p.mat[e].imag();
  }
  if (p.unitary) return prepare_op(n, m, p.k, p.sorted, 1, M.data(), 0, out, err, errlen, allow_native);
  return prepare_transfer(n, m, p.k, p.sorted, M.data(), allow_native, out, err, errlen);
}

int fuse_ops(const std::vector<const FuseOp*>& seq, int max_q, int n, int m, int allow_native,
             std::vector<PreparedOp>* out, char* err, size_t errlen) {
  std::vector<FusePass> passes = fuse_plan(seq, max_q);
  out->resize(passes.size());
  for (size_t i = 0; i < passes.size(); ++i) {
    if (passes[i].ops.size() > 1) fuse_compose(passes[i], seq, false);
    if (fuse_prepare(passes[i], seq, n, m, allow_native, &(*out)[i], err, errlen) != 0) return 1;
  }
  return 0;
}

}  // namespace ht
