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
//  4. recognises permutation-and-phase operations (Section II-B: gates whose
//     matrix has one nonzero per row, such as X, Z, S, T, CNOT, SWAP or
//     Toffoli, and Kraus sets of such matrices sharing one permutation, such
//     as dephasing): there every output entry is one input entry times a
//     coefficient, w[u][v] = c[u][v] h[p(u)][p(v)] with
//     c[u][v] = sum_a A_a[u][p(u)] conj(A_a[v][p(v)]), and entries with
//     p(u) = u, p(v) = v and c[u][v] = 1 do not change at all, so the pass
//     need not touch them.
#include "ht_prep.h"

#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

namespace ht {

using cplx = std::complex<double>;

// Coefficients within this distance of one, on entries the permutation fixes,
// are taken as exactly one (|d|^2 of a unit phase such as exp(i pi / 4) is
// one only up to rounding): the entry is then left untouched, an error of at
// most 4 units in the last place instead of the product's own rounding.
constexpr double kUnitSnap = 1.0 / 1125899906842624.0;  // 2^-50

// Whether the native pass of a k <= 2 op moves fewer bytes than the generic
// pass in practice.  It skips the fixed entries, but HBM moves whole 128-byte
// lines (eight 16-byte entries, columns differing in bits 0..2): where a
// target below bit 3 decides whether a column's entry changes, every line
// still holds changing entries.  Measured on n = 16 operators (tile edge
// 32), the native pass was then 1-9 % slower for permutations (CNOT with a
// low control, SWAP) and for diagonal ops changing half the entries at bits
// 0, 1 (Z, T, dephasing), and faster for diagonal ops at bit 2 (+8 %) or
// changing at most 3/8 of the entries (CZ: +5-11 %), and for every op whose
// deciding targets lie at bit 3 or above (+22 % to 2.6x).
static bool native_pays(int k, int m_eff, const int* sorted, const int* pm, uint64_t active) {
  const int D = 1 << k;
  int lowest = 64;  // lowest intra target whose column bit decides whether an entry changes
  for (int l = 0; l < k; ++l) {
    if (sorted[l] >= m_eff) continue;  // selects tiles: no effect inside a line
    bool decides = false;
    for (int u = 0; u < D && !decides; ++u)
      for (int v = 0; v < D && !decides; ++v)
        decides = ((active >> (u * D + v)) & 1) != ((active >> (u * D + (v ^ (1 << l)))) & 1);
    if (decides && sorted[l] < lowest) lowest = sorted[l];
  }
  if (lowest >= 3) return true;
  bool diagonal = true;
  for (int u = 0; u < D; ++u) diagonal = diagonal && pm[u] == u;
  const int changing = __builtin_popcountll(active);
  return diagonal && (lowest == 2 || 8 * changing <= 3 * D * D);
}

// Fill the native form from the permutation pm and coefficients c (2^k x 2^k,
// w[u][v] = c[u][v] h[pm[u]][pm[v]]).  Returns 1 when the native form is
// used, 0 when the op should take a generic form instead (k <= 2 and every
// entry changes: the native pass would move the same bytes; or, under
// kNativeWherePays, the native pass does not pay), -1 on error.
static int native_form(int k, const int* pm, const cplx* c_in, int allow_native, int m_eff,
                       const int* sorted, PreparedOp* out, char* err, size_t errlen) {
  const int D = 1 << k;
  out->form = 2;
  out->active = 0;
  for (int u = 0; u < D; ++u) out->perm[u] = pm[u];
  for (int u = D; u < 8; ++u) out->perm[u] = u;
  for (int u = 0; u < D; ++u)
    for (int v = 0; v < D; ++v) {
      cplx c = c_in[u * D + v];
      const bool fixed = pm[u] == u && pm[v] == v;
      if (fixed && std::abs(c.real() - 1.0) <= kUnitSnap && std::abs(c.imag()) <= kUnitSnap) c = 1.0;
      if (!fixed || c != cplx(1.0, 0.0)) out->active |= (uint64_t)1 << (u * D + v);
      out->coef[2 * (u * D + v)] = c.real();
      out->coef[2 * (u * D + v) + 1] = c.imag();
    }
  // For k <= 2 the native pass pays off only when some entry stays in place
  // (it then moves fewer bytes); an op that changes every entry (X, Y, ...)
  // keeps the generic pass, which is exact for permutations too.
  if (k <= 2 && out->active == (((uint64_t)1 << (D * D)) - 1)) return 0;
  if (k <= 2 && allow_native == kNativeWherePays && !native_pays(k, m_eff, sorted, pm, out->active))
    return 0;
  // k = 3: chunks of whole orbits (first fit, largest orbits first); a cycle
  // of (u, v) -> (p(u), p(v)) is at most the lcm of two cycle lengths of p
  // (<= 15), an orbit at most two cycles
  out->nchunks = 0;
  out->chunk = 16;
  std::memset(out->sched, 0, sizeof out->sched);
  if (k == 3) {
    std::vector<std::vector<int>> orbits;
    uint64_t seen = 0;
    for (int e = 0; e < D * D; ++e) {
      if (!((out->active >> e) & 1) || ((seen >> e) & 1)) continue;
      std::vector<int> orb;
      for (int start : {e, (e % D) * D + e / D})
        for (int x = start; !((seen >> x) & 1); x = pm[x / D] * D + pm[x % D]) {
          seen |= (uint64_t)1 << x;
          orb.push_back(x);
        }
      if ((int)orb.size() > 16) out->chunk = 32;
      orbits.push_back(orb);
    }
    std::stable_sort(orbits.begin(), orbits.end(),
                     [](const std::vector<int>& a, const std::vector<int>& b) { return a.size() > b.size(); });
    const int cap = 256 / out->chunk;
    int fill[16] = {0};
    for (const auto& orb : orbits) {
      int ch = 0;
      while (ch < out->nchunks && fill[ch] + (int)orb.size() > out->chunk) ++ch;
      if (ch == cap) {
        if (err && errlen) std::snprintf(err, errlen, "internal: native schedule does not fit");
        return -1;
      }
      if (ch == out->nchunks) ++out->nchunks;
      for (int x : orb) {
        const int u = x / D, v = x % D;
        out->sched[ch * out->chunk + fill[ch]++] =
            (uint16_t)(0x8000 | u | (v << 3) | (pm[u] << 6) | (pm[v] << 9));
      }
    }
  }
  return 1;
}

int prepare_op(int n, int m_eff, int k, const int* targets, int r, const double* kraus,
               int heisenberg, PreparedOp* out, char* err, size_t errlen, int allow_native) {
  auto fail = [&](const char* msg) {
    if (err && errlen) std::snprintf(err, errlen, "%s", msg);
    return 1;
  };
  if (!out) return fail("output pointer is NULL");
  if (k < 1 || k > 3) return fail("k must be 1, 2 or 3");
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
  int perm[3] = {0, 1, 2};
  for (int a = 1; a < k; ++a)
    for (int b = a; b > 0 && targets[perm[b]] < targets[perm[b - 1]]; --b) {
      const int t = perm[b];
      perm[b] = perm[b - 1];
      perm[b - 1] = t;
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

  static thread_local cplx A[64][64];  // up to r = 64 operators of 8 x 8
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

  // permutation-and-phase form: one nonzero per row, same column in every A_a
  bool mono = allow_native == 1 || allow_native == kNativeWherePays ||
              (allow_native == kNativeK3Only && k == 3);
  int pm[8];
  for (int u = 0; u < D && mono; ++u) {
    pm[u] = -1;
    for (int a = 0; a < r && mono; ++a)
      for (int v = 0; v < D; ++v) {
        if (A[a][u * D + v] == cplx(0.0, 0.0)) continue;
        if (pm[u] < 0 && a == 0)
          pm[u] = v;
        else if (pm[u] != v)
          mono = false;
      }
    if (pm[u] < 0) mono = false;  // a zero row in the first operator
  }
  if (mono) {  // pm must be a permutation
    int seen = 0;
    for (int u = 0; u < D; ++u) seen |= 1 << pm[u];
    mono = seen == (1 << D) - 1;
  }
  if (mono) {
    cplx c[64];
    for (int u = 0; u < D; ++u)
      for (int v = 0; v < D; ++v) {
        c[u * D + v] = 0.0;
        for (int a = 0; a < r; ++a) c[u * D + v] += A[a][u * D + pm[u]] * std::conj(A[a][v * D + pm[v]]);
      }
    const int st = native_form(k, pm, c, allow_native, m_eff, out->sorted, out, err, errlen);
    if (st < 0) return 1;
    if (st == 1) return 0;
  }
  if (k == 3) {  // the Kraus operators themselves (a 64 x 64 transfer matrix would not pay)
    out->form = kFormKraus3;
    out->nkraus = r;
    for (int a = 0; a < r; ++a)
      for (int e = 0; e < D * D; ++e) {
        out->coef[2 * (a * D * D + e)] = A[a][e].real();
        out->coef[2 * (a * D * D + e) + 1] = A[a][e].imag();
      }
    return 0;
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

int prepare_transfer(int n, int m_eff, int k, const int* sorted, const double* S, int allow_native,
                     PreparedOp* out, char* err, size_t errlen) {
  auto fail = [&](const char* msg) {
    if (err && errlen) std::snprintf(err, errlen, "%s", msg);
    return 1;
  };
  if (!out || !sorted || !S) return fail("NULL argument");
  if (k != 1 && k != 2) return fail("a transfer matrix acts on 1 or 2 qubits");
  for (int l = 0; l < k; ++l) {
    if (sorted[l] < 0 || sorted[l] >= n) return fail("target qubit out of range [0, n)");
    if (l > 0 && sorted[l] <= sorted[l - 1]) return fail("targets must be ascending");
  }
  const int D = 1 << k, DD = D * D;
  out->k = k;
  out->ncross = 0;
  for (int l = 0; l < k; ++l) {
    out->sorted[l] = sorted[l];
    if (sorted[l] >= m_eff) ++out->ncross;
  }
  // native form if every row of S has one nonzero, at (p(u), p(v)) for one p
  if (allow_native == 1 || allow_native == kNativeWherePays) {
    int pm[4] = {-1, -1, -1, -1};
    bool mono = true;
    cplx c[16];
    for (int e = 0; e < DD && mono; ++e) {
      int f = -1;
      for (int g = 0; g < DD; ++g) {
        if (S[2 * (e * DD + g)] == 0.0 && S[2 * (e * DD + g) + 1] == 0.0) continue;
        if (f >= 0) mono = false;
        f = g;
      }
      if (f < 0) {
        mono = false;
        break;
      }
      const int u = e / D, v = e % D, fu = f / D, fv = f % D;
      if ((pm[u] >= 0 && pm[u] != fu) || (pm[v] >= 0 && pm[v] != fv)) mono = false;
      pm[u] = fu;
      pm[v] = fv;
      c[e] = cplx(S[2 * (e * DD + f)], S[2 * (e * DD + f) + 1]);
    }
    if (mono) {
      int seen = 0;
      for (int u = 0; u < D; ++u) seen |= 1 << pm[u];
      mono = seen == (1 << D) - 1;
    }
    if (mono) {
      const int st = native_form(k, pm, c, allow_native, m_eff, sorted, out, err, errlen);
      if (st < 0) return 1;
      if (st == 1) return 0;
    }
  }
  out->form = 1;
  for (int i = 0; i < 2 * DD * DD; ++i) out->coef[i] = S[i];
  return 0;
}

}  // namespace ht
