// Host-side check of the conjugation pass's indexing (test support only; the
// library never loads this).  It runs the same per-lane body the GPU kernel
// runs (conj_group_lane from ht_geom.h) for every group and lane of a pass,
// sequentially on a host copy of the tiled storage, with a memory policy that
// rejects out-of-range accesses and counts reads and writes per entry.  Blocks
// of one pass touch disjoint entries, so the sequential order gives the same
// result as the parallel kernel.  Tests compare the result with the CPU
// oracle and require every stored entry to be written exactly once.
#include <cstdio>
#include <cstring>

#include "ht_geom.h"
#include "ht_internal.h"
#include "ht_k3.h"
#include "ht_native.h"
#include "ht_pair.h"
#include "ht_prep.h"

namespace {

struct CheckedMem {
  double2* h;
  uint64_t nelems;
  int32_t* wc;
  int32_t* rc;
  bool* oob;
  ht::cd load(uint64_t tb, uint32_t off) const {
    const uint64_t e = tb + off;
    if (e >= nelems) {
      *oob = true;
      return {0.0, 0.0};
    }
    if (rc) rc[e]++;
    return ht::load_c<double>(h + tb, off);
  }
  // held entries as the GPU holds 16-byte ones: FP64, conjugated at load
  using R = ht::cd;
  R load_x(uint64_t tb, uint32_t off, bool cj) const {
    ht::cd v = load(tb, off);
    if (cj) v.im = -v.im;
    return v;
  }
  static ht::cd widen(const R& r, bool) { return r; }
  void store(uint64_t tb, uint32_t off, ht::cd v) const {
    const uint64_t e = tb + off;
    if (e >= nelems) {
      *oob = true;
      return;
    }
    if (wc) wc[e]++;
    ht::store_c<double>(h + tb, off, v);
  }
  // the pair layout's accesses (ht_pair.h): a pair held as loaded (mirrored
  // entries conjugated when widened, as the GPU's narrow pairs are); the
  // GPU's 16-byte accesses are aligned, so off must be even
  struct H {
    ht::cd a, b;
  };
  H load_pair(uint64_t tb, uint32_t off) const {
    if (off & 1u) *oob = true;
    return {load(tb, off), load(tb, off + 1u)};
  }
  H load_two(uint64_t tb, uint32_t o0, uint32_t o1) const { return {load(tb, o0), load(tb, o1)}; }
  static void widen(const H& x, bool cj, ht::cd& a, ht::cd& b) {
    a = cj ? ht::conjg(x.a) : x.a;
    b = cj ? ht::conjg(x.b) : x.b;
  }
  static void set(H& x, int i, ht::cd w) { (i == 0 ? x.a : x.b) = w; }
  void store_pair(uint64_t tb, uint32_t off, const H& x) const {
    if (off & 1u) *oob = true;
    store(tb, off, x.a);
    store(tb, off + 1u, x.b);
  }
  void store_two_cj(uint64_t tb, uint32_t o0, uint32_t o1, const H& x) const {
    store(tb, o0, ht::conjg(x.a));
    store(tb, o1, ht::conjg(x.b));
  }
};

template <int JU, int K, int C, int FORM>
void run(const CheckedMem& mem, int n, int m, const ht::PreparedOp& op, int order, bool ilv,
         bool pairs, uint64_t* lanes_run) {
  ht::ConjGeom<K, C> g = ht::make_geom<K, C>(n, m, op.sorted, ilv);
  ht::Coef<K, FORM> cf;
  if constexpr (K == 2 && FORM == 1) {
    cf.p = op.coef;
  } else {
    for (int i = 0; i < 2 * ht::Coef<K, FORM>::NE; ++i) cf.c[i] = op.coef[i];
  }
  // the pair layout of complex64 passes (k = 1, and k = 2 in the direct
  // form), indexing checked on this complex128 copy (the same entries, in
  // pairs); JP pairs per step as on the GPU
  constexpr int JP = K == 1 ? 2 : 1;
  bool use_pairs = false;
  if constexpr (K == 1 || (K == 2 && FORM == 0)) use_pairs = pairs && g.F >= 4 && (K == C || g.ipos[0] != 0);
  if constexpr (K == 1 || (K == 2 && FORM == 0)) {
    if (use_pairs && order >= 2) {
      // the pair step kernel's split of the work (order 2..5: item order
      // 0..3): every (unit, wave) item of sync_item that is not past the end
      // and not a diagonal group, its pairs loaded and updated by every
      // lane; then, with a tile-selecting target, the diagonal groups in the
      // block layout (pair_diag_kernel)
      constexpr int LW = K == 1 ? 4 : 3;
      constexpr uint32_t WPB = 1u << LW;
      int sl, r, ps;
      ht::pair_sync_order(g.F, JP, LW, order - 2, sl, r, ps);
      const uint64_t nu = ht::sync_units(g.ngroups, sl, WPB, r, ps);
      for (uint64_t u = 0; u < nu; ++u)
        for (uint32_t w = 0; w < WPB; ++w) {
          uint64_t grp;
          uint32_t step;
          ht::sync_item(u, w, WPB, sl, r, ps, grp, step);
          if (grp >= g.ngroups) continue;
          ht::GroupCtx<C> gc;
          ht::group_ctx<K, C>(grp, g, gc);
          if (gc.diag) continue;
          for (uint32_t lane = 0; lane < 64; ++lane) {
            ht::PairStep<JP, K, CheckedMem> st;
            ht::pair_load<JP, K, C>(mem, g, gc, lane, step * JP, st);
            ht::pair_update_store<JP, K, C, FORM>(mem, g, gc, cf, st);
            ++*lanes_run;
          }
        }
      if (C > 0) {
        const uint64_t nts = ht::grid_rows(g.ngroups);
        for (uint64_t ti = 0; ti < nts; ++ti) {
          ht::GroupCtx<C> gc;
          ht::group_ctx<K, C>(ht::diag_group(ti), g, gc);
          if (!gc.diag) continue;
          for (uint32_t lane = 0; lane < 64; ++lane) {
            ht::conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane);
            ++*lanes_run;
          }
        }
      }
      return;
    }
  }
  for (uint64_t grp = 0; grp < g.ngroups; ++grp) {
    ht::GroupCtx<C> gc;
    ht::group_ctx<K, C>(grp, g, gc);
    if constexpr (K <= 2) {
      if (use_pairs && !gc.diag) {
        for (uint32_t lane = 0; lane < 64; ++lane) {
          if (order == 0) {
            ht::pair_group_lane<JP, K, C, FORM>(mem, g, gc, cf, lane, 0, 0xffffffffu);
          } else {
            for (uint32_t j0 = 0; j0 < ht::pair_jobs(g.F); j0 += JP)
              ht::pair_group_lane<JP, K, C, FORM>(mem, g, gc, cf, lane, j0, j0 + JP);
          }
          ++*lanes_run;
        }
        continue;
      }
    }
    for (uint32_t lane = 0; lane < 64; ++lane) {
      if (order == 0) {
        ht::conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane);
      } else {  // the per-step job ranges of the flattened work order
        for (uint32_t j0 = 0; j0 < g.jobs; j0 += JU)
          ht::conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane, j0, j0 + JU);
      }
      ++*lanes_run;
    }
  }
}

// The k = 3 Kraus form (ht_k3.h): 8 lanes share a block and exchange their
// left products through LDS, so the 64 lanes of a wave run here phase by
// phase -- every lane's left products written to the 8 blocks' tables, then
// every lane's row read back and its right products.
template <int C>
void run_k3(const CheckedMem& mem, int n, int m, const ht::PreparedOp& op, uint64_t* lanes_run) {
  const ht::ConjGeom<3, C> g = ht::make_geom<3, C>(n, m, op.sorted, false);
  const uint32_t nblk = 1u << (2 * g.F);
  for (uint64_t grp = 0; grp < g.ngroups; ++grp) {
    const ht::K3Group gr = ht::k3_group<C>(grp);
    ht::K3Tiles<C> tiles[8];
    for (int j = 0; j < 8; ++j) ht::k3_tiles<C>(g, gr, j, tiles[j]);
    for (uint32_t b0 = 0; b0 < nblk; b0 += 8) {
      ht::K3Block bk[64];
      ht::cd x[64][8], w[64][8], table[8][8][8];
      for (uint32_t lane = 0; lane < 64; ++lane) {
        bk[lane] = ht::k3_block<C>(g, gr, b0 + (lane >> 3));
        for (int u = 0; u < 8; ++u) x[lane][u] = w[lane][u] = ht::cd{0.0, 0.0};
        if (bk[lane].active) ht::k3_load_col<C>(mem, g, tiles[lane & 7], bk[lane], (int)(lane & 7), x[lane]);
      }
      for (int a = 0; a < op.nkraus; ++a) {
        const double* Aa = op.coef + 128 * a;
        for (uint32_t lane = 0; lane < 64; ++lane)
          ht::k3_left(Aa, x[lane], [&](int u, ht::cd t) { table[lane >> 3][u][lane & 7] = t; });
        for (uint32_t lane = 0; lane < 64; ++lane)
          ht::k3_right_acc(Aa, [&](int l) { return table[lane >> 3][lane & 7][l]; }, w[lane]);
      }
      for (uint32_t lane = 0; lane < 64; ++lane)
        if (bk[lane].active) ht::k3_store_row<C>(mem, g, gr, tiles[lane & 7], bk[lane], (int)(lane & 7), w[lane]);
      *lanes_run += 64;
    }
  }
}

template <int K, int C>
void run_native(const CheckedMem& mem, int n, int m, const ht::PreparedOp& pop, int order, bool ilv,
                uint64_t* lanes_run) {
  const ht::ConjGeom<K, C> g = ht::make_geom<K, C>(n, m, pop.sorted, ilv);
  ht::NativeOp<K> op;
  for (int u = 0; u < (1 << K); ++u) op.perm[u] = pop.perm[u];
  op.active = pop.active;
  op.nchunks = pop.nchunks;
  double data[512];
  ht::native_op_data(pop, data);
  op.c = data;
  for (uint64_t grp = 0; grp < g.ngroups; ++grp) {
    const ht::NativeGroup ng = ht::native_group<C>(grp);
    constexpr int JU = ht::native_unroll(K);
    for (uint32_t lane = 0; lane < 64; ++lane) {
      // order 1: the per-step job ranges of the flattened work order
      const uint32_t step = order == 0 ? 0xffffffffu : (uint32_t)JU;
      for (uint32_t j0 = 0; j0 < g.jobs; j0 += step) {
        const uint32_t j1 = order == 0 ? 0xffffffffu : j0 + JU;
        if constexpr (K == 3) {
          if (pop.chunk == 32)
            ht::native3_group_lane<C, 32>(mem, g, ng, op, lane, j0, j1);
          else
            ht::native3_group_lane<C, 16>(mem, g, ng, op, lane, j0, j1);
        } else {
          ht::native_group_lane<JU, K, C>(mem, g, ng, op, lane, j0, j1);
        }
        if (order == 0) break;
      }
      ++*lanes_run;
    }
  }
}

}  // namespace

extern "C" {

// raw: host c128 tiled storage of nelems entries (2*nelems doubles), updated
// in place.  write_counts / read_counts: nelems int32 each, zeroed by the
// caller, or NULL.  order: 0 = whole groups per lane, 1 = the per-step job
// ranges of the flattened work order; with pairs, 2..5 = the pair step
// kernel's split of the work in item order 0..3.  ilv: the alternating
// patch order (lane_block).  pairs: the pair layout of complex64
// passes (ht_pair.h) wherever it applies, checked on this complex128 copy.  native: allow the
// native pass for permutation-and-phase operations; *form (if not NULL)
// receives the form used.  Returns 0 on success, 1 on invalid op, 2 on an
// out-of-range access.  *lanes_run receives the number of lane bodies run.
int htc_emulate_conj(double* raw, uint64_t nelems, int n, int tile_log2, int k, const int* targets,
                     int r, const double* kraus, int heisenberg, int32_t* write_counts,
                     int32_t* read_counts, uint64_t* lanes_run, int order, int native,
                     int ilv, int pairs, int* form, char* err, size_t errlen) {
  const int m = tile_log2 < n ? tile_log2 : n;
  ht::PreparedOp op;
  if (ht::prepare_op(n, m, k, targets, r, kraus, heisenberg, &op, err, errlen, native) != 0)
    return 1;
  if (form) *form = op.form;
  bool oob = false;
  CheckedMem mem{reinterpret_cast<double2*>(raw), nelems, write_counts, read_counts, &oob};
  uint64_t lanes = 0;
#define HT_CASE(K_, C_, F_)                                 \
  if (op.k == K_ && op.ncross == C_ && op.form == F_)       \
    run<ht::conj_unroll(K_), K_, C_, F_>(mem, n, m, op, order, ilv != 0, pairs != 0, &lanes);
  HT_CASE(1, 0, 0)
  HT_CASE(1, 0, 1)
  HT_CASE(1, 1, 0)
  HT_CASE(1, 1, 1)
  HT_CASE(2, 0, 0)
  HT_CASE(2, 0, 1)
  HT_CASE(2, 1, 0)
  HT_CASE(2, 1, 1)
  HT_CASE(2, 2, 0)
  HT_CASE(2, 2, 1)
#undef HT_CASE
  if (op.form == ht::kFormKraus3) {
    if (op.ncross == 0) run_k3<0>(mem, n, m, op, &lanes);
    if (op.ncross == 1) run_k3<1>(mem, n, m, op, &lanes);
    if (op.ncross == 2) run_k3<2>(mem, n, m, op, &lanes);
    if (op.ncross == 3) run_k3<3>(mem, n, m, op, &lanes);
  }
#define HT_NATIVE(K_, C_) \
  if (op.form == 2 && op.k == K_ && op.ncross == C_) run_native<K_, C_>(mem, n, m, op, order, ilv != 0, &lanes);
  HT_NATIVE(1, 0)
  HT_NATIVE(1, 1)
  HT_NATIVE(2, 0)
  HT_NATIVE(2, 1)
  HT_NATIVE(2, 2)
  HT_NATIVE(3, 0)
  HT_NATIVE(3, 1)
  HT_NATIVE(3, 2)
  HT_NATIVE(3, 3)
#undef HT_NATIVE
  if (lanes_run) *lanes_run = lanes;
  if (oob) {
    if (err && errlen) std::snprintf(err, errlen, "out-of-range access");
    return 2;
  }
  return 0;
}

// lane_block for block index b: the block's base row and column indices
// (pidx, qidx) in [0, 2^F).
void htc_lane_block(uint32_t b, int F, int s, int ilv, uint32_t* pidx, uint32_t* qidx) {
  ht::lane_block(b, F, s, ilv != 0, *pidx, *qidx);
}

// The item order of the workgroup-wide step kernel: for every unit
// u < sync_units(...) and wave w < wpb, grp[u * wpb + w] and step[...] as
// sync_item gives them.  Returns the number of units, or 0 when they exceed
// max_units.
uint64_t htc_sync_items(uint64_t ngroups, int sl, uint32_t wpb, int r, int ps, uint64_t max_units,
                        uint64_t* grp, uint32_t* step) {
  const uint64_t nu = ht::sync_units(ngroups, sl, wpb, r, ps);
  if (nu > max_units) return 0;
  for (uint64_t u = 0; u < nu; ++u)
    for (uint32_t w = 0; w < wpb; ++w) ht::sync_item(u, w, wpb, sl, r, ps, grp[u * wpb + w], step[u * wpb + w]);
  return nu;
}

}  // extern "C"
