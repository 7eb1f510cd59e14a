// Fusion of neighbouring k-local ops into passes on at most two qubits
// (host only): planning, composition, preparation.  Used by circuits,
// batches and the server.
#pragma once

#include <complex>
#include <vector>

#include "ht_prep.h"

namespace ht {

// An op as given by the caller (matrices not owned); adj: the map applied is
// the adjoint one, sum_a L_a^dagger H L_a.
struct FuseOp {
  int k;
  int targets[3];
  int r;               // 1: unitary (mats holds U)
  int adj;
  const double* mats;  // r x 2^k x 2^k interleaved complex, caller's order
};

// A group of ops applied as one pass.
struct FusePass {
  std::vector<int> ops;                 // indices into the effective sequence, in order
  int k;                                // qubits of the pass
  int sorted[3];                        // ascending qubits
  bool unitary;                         // every op a unitary
  std::vector<std::complex<double>> mat;  // composed U (D x D) or S (D^2 x D^2); empty for one op
};

// Group a sequence of ops (applied in this order) into passes on at most
// max_q qubits (0: one pass per op).
std::vector<FusePass> fuse_plan(const std::vector<const FuseOp*>& seq, int max_q);

// Compose a pass: U = U_last ... U_first, or S = S_last ... S_first with
// S_op = sum_a A_a (x) conj(A_a), A_a = L_a or, for an adjoint op, L_a^dagger;
// as_transfer forces S.
void fuse_compose(FusePass& p, const std::vector<const FuseOp*>& seq, bool as_transfer);

// Prepare one planned pass for an n-qubit operator with effective tile
// exponent m: a one-op pass exactly as prepare_op would, a composed one from
// its U or S.  Returns 0 or nonzero with a message.
int fuse_prepare(const FusePass& p, const std::vector<const FuseOp*>& seq, int n, int m,
                 int allow_native, PreparedOp* out, char* err, size_t errlen);

// The whole pipeline for ops applied in the given order.
int fuse_ops(const std::vector<const FuseOp*>& seq, int max_q, int n, int m, int allow_native,
             std::vector<PreparedOp>* out, char* err, size_t errlen);

}  // namespace ht
