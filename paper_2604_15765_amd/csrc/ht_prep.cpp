// Host-side preparation of one k-local operation.
//
// Section II-A: a k-local operation acts on each 2^k x 2^k block through its
// local Kraus operators L_a (Eq. (2)), or through the transfer matrix of
// Eq. (3).  The kernels index a block with its local bits in ascending target
// order and gather it row-major, so the host
//  1. adjoins every L_a for the Heisenberg picture (Phi*(O) = sum_a L_a^+ O L_a),
//  2. renumbers local bits from the caller's target order to ascending order,
//  3. keeps the single matrix for r = 1 (direct two-sided update), or builds
//     S = sum_a A_a (x) conj(A_a), the transfer matrix for a row-major block
//     vector.  (Eq. (3) stacks columns and uses conj(L) (x) L; gathering rows,
//     as the tile algorithms do, swaps the factors.)
#include "ht_prep.h"

#include <complex>
#include <cstdio>
#include <cstring>

namespace ht {

using cplx = std::complex<double>;

int prepare_op(int n, int m_eff, int k, const int* targets, int r, const double* kraus,
               int heisenberg, PreparedOp* out, char* err, size_t errlen) {
  auto fail = [&](const char* msg) {
    if (err && errlen) std::snprintf(err, errlen, "%s", msg);
    return 1;
  };
  if (!out) return fail("output pointer is NULL");
  if (k != 1 && k != 2) return fail("k must be 1 or 2");
  if (!targets) return fail("targets is NULL");
  if (!kraus) return fail("operator matrices pointer is NULL");
  const int D = 1 << k;
  if (r < 1 || r > D * D) return fail("Kraus rank r must satisfy 1 <= r <= 4^k");
  for (int l = 0; l < k; ++l) {
    if (targets[l] < 0 || targets[l] >= n) return fail("target qubit out of range [0, n)");
    for (int l2 = 0; l2 < l; ++l2)
      if (targets[l] == targets[l2]) return fail("targets must be distinct");
  }

  // perm[ls] = user local bit that becomes sorted local bit ls
  int perm[2] = {0, 1};
  if (k == 2 && targets[1] < targets[0]) {
    perm[0] = 1;
    perm[1] = 0;
  }
  for (int ls = 0; ls < k; ++ls) out->sorted[ls] = targets[perm[ls]];
  out->k = k;
  out->ncross = 0;
  for (int ls = 0; ls < k; ++ls)
    if (out->sorted[ls] >= m_eff) ++out->ncross;

  auto user_index = [&](int us) {
    int u = 0;
    for (int ls = 0; ls < k; ++ls) u |= ((us >> ls) & 1) << perm[ls];
    return u;
  };

  cplx A[16][16];  // up to r = 16 operators of 4x4
  for (int a = 0; a < r; ++a) {
    const double* L = kraus + (size_t)2 * D * D * a;
    for (int us = 0; us < D; ++us)
      for (int vs = 0; vs < D; ++vs) {
        const int u = user_index(us), v = user_index(vs);
        // entry (us, vs) of the renumbered operator; adjoint swaps and conjugates
        cplx e = heisenberg ? std::conj(cplx(L[2 * (v * D + u)], L[2 * (v * D + u) + 1]))
                            : cplx(L[2 * (u * D + v)], L[2 * (u * D + v) + 1]);
        A[a][us * D + vs] = e;
      }
  }

  if (r == 1) {
    out->form = 0;
    for (int e = 0; e < D * D; ++e) {
      out->coef[2 * e] = A[0][e].real();
      out->coef[2 * e + 1] = A[0][e].imag();
    }
    return 0;
  }
  out->form = 1;
  const int DD = D * D;
  for (int u = 0; u < D; ++u)
    for (int v = 0; v < D; ++v)
      for (int u2 = 0; u2 < D; ++u2)
        for (int v2 = 0; v2 < D; ++v2) {
          cplx s = 0.0;
          for (int a = 0; a < r; ++a) s += A[a][u * D + u2] * std::conj(A[a][v * D + v2]);
          const int e = (u * D + v) * DD + (u2 * D + v2);
          out->coef[2 * e] = s.real();
          out->coef[2 * e + 1] = s.imag();
        }
  return 0;
}

}  // namespace ht
