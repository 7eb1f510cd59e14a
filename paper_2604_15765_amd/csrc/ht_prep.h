// Host-side preparation of one k-local operation (no GPU involved).
#pragma once

#include <stddef.h>

namespace ht {

struct PreparedOp {
  int k;           // 1 or 2
  int sorted[2];   // targets, ascending
  int ncross;      // targets >= the effective tile exponent
  int form;        // 0: direct (coef = A, 2^k x 2^k); 1: transfer (coef = S, 4^k x 4^k)
  double coef[2 * 256];
};

// Validate and prepare.  Returns 0 on success; otherwise writes a message to
// err (errlen bytes) and returns nonzero.  m_eff is the effective tile
// exponent of the operator (min(tile_log2, n)).
int prepare_op(int n, int m_eff, int k, const int* targets, int r, const double* kraus,
               int heisenberg, PreparedOp* out, char* err, size_t errlen);

}  // namespace ht
