// Test driver for the host-side preparation and fusion code under the
// address and undefined-behaviour sanitizers (built by
// tests/test_host_sanitizers.py with g++, no GPU): random op sequences --
// unitaries, Kraus sets, permutation-and-phase matrices, k = 1, 2, 3, both
// pictures, every allow_native mode -- through prepare_op, prepare_transfer,
// fuse_plan and fuse_ops.  Exits non-zero on an unexpected result; the
// sanitizers abort on a memory or undefined-behaviour error.
#include <algorithm>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "ht_fuse.h"
#include "ht_prep.h"

using cplx = std::complex<double>;

static std::mt19937_64 rng(12345);

static double unif() { return std::uniform_real_distribution<double>(-1.0, 1.0)(rng); }

// r matrices of D x D interleaved complex: random, or permutation-and-phase.
static std::vector<double> mats(int D, int r, bool monomial) {
  std::vector<double> m((size_t)2 * r * D * D, 0.0);
  std::vector<int> p(D);
  for (int u = 0; u < D; ++u) p[u] = u;
  std::shuffle(p.begin(), p.end(), rng);
  for (int a = 0; a < r; ++a)
    for (int u = 0; u < D; ++u)
      for (int v = 0; v < D; ++v) {
        if (monomial && v != p[u]) continue;
        m[2 * ((size_t)a * D * D + u * D + v)] = unif();
        m[2 * ((size_t)a * D * D + u * D + v) + 1] = unif();
      }
  return m;
}

int main() {
  int failures = 0;
  char err[256];
  static ht::PreparedOp op;  // large: keep it off the stack
  for (int it = 0; it < 3000; ++it) {
    const int n = 3 + (int)(rng() % 9);
    const int m = 1 + (int)(rng() % 6) < n ? 1 + (int)(rng() % 6) : n;
    const int k = 1 + (int)(rng() % 3);
    const int D = 1 << k;
    int t[3];
    for (int l = 0; l < k; ++l) {
      bool again;
      do {
        t[l] = (int)(rng() % n);
        again = false;
        for (int l2 = 0; l2 < l; ++l2) again = again || t[l2] == t[l];
      } while (again);
    }
    const bool mono = rng() % 3 == 0;
    const int r = 1 + (int)(rng() % (mono ? 3 : (k == 3 ? 8 : D * D)));
    const std::vector<double> M = mats(D, r, mono);
    const int allow = (int)(rng() % 4);
    const int st = ht::prepare_op(n, m, k, t, r, M.data(), (int)(rng() % 2), &op, err, sizeof err, allow);
    if (st != 0) {
      std::printf("prepare_op failed unexpectedly: %s\n", err);
      ++failures;
    }
    // invalid arguments are rejected, not crashed on
    int bad[3] = {t[0], t[0], n};
    if (k > 1 && ht::prepare_op(n, m, k, bad, r, M.data(), 0, &op, err, sizeof err, allow) == 0) ++failures;
    if (ht::prepare_op(n, m, k, t, D * D + 1, M.data(), 0, &op, err, sizeof err, allow) == 0) ++failures;
  }
  // transfer matrices (k <= 2), random and monomial
  for (int it = 0; it < 500; ++it) {
    const int k = 1 + (int)(rng() % 2), D = 1 << k, DD = D * D;
    int s[2] = {0, 2};
    std::vector<double> S((size_t)2 * DD * DD, 0.0);
    for (auto& x : S) x = rng() % 4 == 0 ? unif() : 0.0;
    if (ht::prepare_transfer(6, 3, k, s, S.data(), (int)(rng() % 4), &op, err, sizeof err) != 0) ++failures;
  }
  // fusion of random sequences
  for (int it = 0; it < 300; ++it) {
    const int n = 3 + (int)(rng() % 6);
    const int len = 1 + (int)(rng() % 40);
    std::vector<std::vector<double>> store;
    std::vector<ht::FuseOp> fops(len);
    for (int i = 0; i < len; ++i) {
      ht::FuseOp& f = fops[i];
      f.k = 1 + (int)(rng() % (n >= 3 && rng() % 8 == 0 ? 3 : 2));
      const int D = 1 << f.k;
      for (int l = 0; l < 3; ++l) f.targets[l] = -1;
      for (int l = 0; l < f.k; ++l) {
        bool again;
        do {
          f.targets[l] = (int)(rng() % n);
          again = false;
          for (int l2 = 0; l2 < l; ++l2) again = again || f.targets[l2] == f.targets[l];
        } while (again);
      }
      f.r = 1 + (int)(rng() % 3);
      f.adj = (int)(rng() % 2);
      store.push_back(mats(D, f.r, rng() % 4 == 0));
      f.mats = store.back().data();
    }
    std::vector<const ht::FuseOp*> seq(len);
    for (int i = 0; i < len; ++i) seq[i] = &fops[i];
    std::vector<ht::PreparedOp> out;
    const int maxq = (int)(rng() % 3);
    const int mm = 1 + (int)(rng() % n);
    if (ht::fuse_ops(seq, maxq, n, mm, (int)(rng() % 4), &out, err, sizeof err) != 0) {
      std::printf("fuse_ops failed: %s\n", err);
      ++failures;
    }
    // every op in exactly one pass
    const std::vector<ht::FusePass> plan = ht::fuse_plan(seq, maxq);
    std::vector<int> seen(len, 0);
    for (const auto& p : plan)
      for (int i : p.ops) seen[i]++;
    for (int i = 0; i < len; ++i) failures += seen[i] != 1;
  }
  std::printf("failures %d\n", failures);
  return failures == 0 ? 0 : 1;
}
