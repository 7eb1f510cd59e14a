// Host-side preparation of one k-local operation (no GPU involved).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ht {

// Doubles of coefficients an op can carry: 64 k = 3 Kraus operators.
constexpr int kPrepCoefDoubles = 2 * 64 * 64;

// Form of a k = 3 op that is not permutation-and-phase.
constexpr int kFormKraus3 = 3;

struct PreparedOp {
  int k;           // 1, 2 or 3
  int sorted[3];   // targets, ascending
  int ncross;      // targets >= the effective tile exponent
  // 0: direct (coef = A, 2^k x 2^k); 1: transfer (coef = S, 4^k x 4^k);
  // 2: native permutation-and-phase form (coef = c, 2^k x 2^k, with perm):
  //    w[u][v] = c[u][v] * h[perm[u]][perm[v]];
  // 3: k = 3 Kraus form (coef = the nkraus 8 x 8 operators A_a, one after
  //    the other): w = sum_a A_a h A_a^dagger
  int form;
  int nkraus;          // form 3: number of operators in coef (1..64)
  int perm[8];         // form 2: source row/column of local index u
  uint64_t active;     // form 2: bit u * 2^k + v set when entry (u, v) changes
  // form 2, k = 3: the changing entries in chunks of `chunk` (16 or 32)
  // entries, each chunk a union of whole orbits of (u, v) under
  // (u, v) -> (perm[u], perm[v]) and (u, v) -> (v, u), so that a chunk can be
  // updated in place once all its sources are loaded (the transpose joins
  // the two entries that share storage in blocks on the diagonal).  Entry:
  // bit 15 valid, bits 0-2 u, 3-5 v, 6-8 perm[u], 9-11 perm[v]; padding 0.
  int nchunks, chunk;
  uint16_t sched[256];
  double coef[kPrepCoefDoubles];
};


// allow_native value that restricts the native form to k = 3.
constexpr int kNativeK3Only = 2;
// allow_native value for operators whose passes stream from HBM: the native
// form for k = 3, and for k <= 2 only where it moved fewer bytes in
// measurement (see native_pays in ht_prep.cpp).
constexpr int kNativeWherePays = 3;

// Validate and prepare.  Returns 0 on success; otherwise writes a message to
// err (errlen bytes) and returns 1 (invalid argument).  m_eff is the effective tile
// exponent of the operator (min(tile_log2, n)).  allow_native: 1 = use form
// 2 when every Kraus operator has one nonzero entry per row, in the same
// column for all of them; kNativeWherePays = the same for k = 3, and for
// k <= 2 only where the native pass pays; kNativeK3Only = only for k = 3;
// 0 = never.  Other k = 3 ops take the Kraus form (kFormKraus3).
int prepare_op(int n, int m_eff, int k, const int* targets, int r, const double* kraus,
               int heisenberg, PreparedOp* out, char* err, size_t errlen, int allow_native = 1);

// Prepare a 1- or 2-qubit map given by its transfer matrix S (4^k x 4^k,
// row-major, interleaved complex; w = S vec(h) with vec row-major over local
// indices whose bit l belongs to sorted[l], ascending).  Uses the native
// form when S has one nonzero per row at (p(u), p(v)) for one permutation p
// and allow_native is 1 (or kNativeWherePays and the native pass pays); else
// form 1.
int prepare_transfer(int n, int m_eff, int k, const int* sorted, const double* S, int allow_native,
                     PreparedOp* out, char* err, size_t errlen);

}  // namespace ht
