// k = 3 operations in Kraus form, shared by the GPU kernel (ht_k3.hip) and
// the host-side checker.
//
// Eq. (2) with 8 x 8 operators: every block of 64 entries becomes
// w = sum_a A_a h A_a^dagger.  One lane cannot hold a block (64 complex
// FP64 values), so 8 lanes share it: lane j first holds column j of the
// block and forms t[:, j] = A_a h[:, j] (left products), the 8 lanes
// exchange t through LDS, and lane j then holds row j of t and accumulates
// w[j][:] += t[j][:] A_a^dagger (right products); after the last operator
// it stores row j.  A 64-lane wave works on 8 blocks at a time whose base
// columns are consecutive, so a load (or store) instruction covers, for each
// of the 8 block columns (rows), eight consecutive entries.  Groups, blocks
// and the ownership rules of diagonal groups are those of the conjugation
// pass (ht_geom.h) with K = 3.
#pragma once

#include "ht_geom.h"

namespace ht {

constexpr int kK3Pad = 9;  // LDS row stride of a block (entries): 8 + 1 against bank conflicts

// A group of the pass: reduced tile indices Ti >= Tj (as in ht_geom.h).
struct K3Group {
  uint32_t Ti, Tj;
  bool diag;
};

template <int C>
HT_HD K3Group k3_group(uint64_t grp) {
  uint32_t Ti, Tj;
  tri_decode(grp, Ti, Tj);
  return {wave_uniform(Ti), wave_uniform(Tj), C > 0 && Ti == Tj};
}

// The stored tiles a lane reaches: its column j of a block lies in group
// tiles (X, j >> KI) for every X, its row j in tiles (j >> KI, Y) for every
// Y.  Tabulated per lane with the run-time index folded in, so that the
// loops below index these arrays by compile-time values only.
template <int C>
struct K3Tiles {
  uint64_t colb[1 << C], rowb[1 << C];  // element offsets of the stored tiles
  bool cold[1 << C], rowd[1 << C];      // stored in the group's orientation
};

template <int C>
HT_HD void k3_tiles(const ConjGeom<3, C>& g, const K3Group& gr, int j, K3Tiles<C>& t) {
  constexpr int KI = 3 - C;
  const uint32_t Xj = (uint32_t)(j >> KI);
  const uint32_t TRj = ins_cross<C>(gr.Ti, Xj, g.cpos), TCj = ins_cross<C>(gr.Tj, Xj, g.cpos);
#pragma unroll
  for (int X = 0; X < (1 << C); ++X) {
    const uint32_t TR = ins_cross<C>(gr.Ti, (uint32_t)X, g.cpos);
    const uint32_t TC = ins_cross<C>(gr.Tj, (uint32_t)X, g.cpos);
    // column j: tile (X, Xj); row j: tile (Xj, X)
    t.cold[X] = TR >= TCj;
    t.colb[X] = (tri64(t.cold[X] ? TR : TCj) + (t.cold[X] ? TCj : TR)) << (2 * g.m);
    t.rowd[X] = TRj >= TC;
    t.rowb[X] = (tri64(t.rowd[X] ? TRj : TC) + (t.rowd[X] ? TC : TRj)) << (2 * g.m);
  }
}

struct K3Block {
  uint32_t p, q;  // base row and column (target bits clear)
  bool active;
};

// Block b of a group (b < 4^F active).  The 8 blocks of a step (b >> 3)
// share a base row and have 8 consecutive free columns, so a stored tile is
// read in rows of 8 entries.  Consecutive steps advance the row first
// (F >= 3): in a mirrored tile, where those 8 blocks run down a column, the
// lines one step reads in 16-byte pieces are read again by the next steps
// while they are still cached.
template <int C>
HT_HD K3Block k3_block(const ConjGeom<3, C>& g, const K3Group& gr, uint32_t b) {
  constexpr int KI = 3 - C;
  const uint32_t nblk = 1u << (2 * g.F);
  const uint32_t fm = (1u << g.F) - 1u;
  K3Block r;
  r.active = b < nblk;
  if (!r.active) b = 0;
  uint32_t pi, qi;
  if (g.F >= 3) {
    pi = (b >> 3) & fm;
    qi = ((b >> (3 + g.F)) << 3) | (b & 7u);
  } else {
    pi = b >> g.F;
    qi = b & fm;
  }
  r.p = deposit_free<KI>(pi, g.ipos);
  r.q = deposit_free<KI>(qi, g.ipos);
  r.active = r.active && !(gr.diag && r.p < r.q);
  return r;
}

// Column j of the block in FP64 (mirrored tiles conjugated).
template <int C, typename Mem>
HT_HD void k3_load_col(const Mem& mem, const ConjGeom<3, C>& g, const K3Tiles<C>& t,
                       const K3Block& bk, int j, cd (&x)[8]) {
  constexpr int KI = 3 - C;
  constexpr int IM = (1 << KI) - 1;
  const uint32_t cv = bk.q + dep_intra<KI>(j & IM, g.ipos);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const uint32_t ru = bk.p + dep_intra<KI>(u & IM, g.ipos);
    const int X = u >> KI;
    const bool d = t.cold[X];
    const uint32_t off = d ? (ru << g.m) + cv : (cv << g.m) + ru;
    x[u] = Mem::widen(mem.load_x(t.colb[X], off, !d), !d);
  }
}

// The two products of one Kraus operator (A row-major 8 x 8, interleaved
// complex).  Both loop over rows or columns of A without unrolling the
// outer loop: fully unrolled, the compiler hoists all 128 uniform
// coefficient loads and spills most of them (about three register-spill
// instructions per FP64 FMA); one row or column at a time fits.  The
// results are exchanged through put / get rather than register arrays
// indexed by the loop counter.

// t = A x for one column: put(u, t[u]) for u = 0..7.
template <typename Put>
HT_HD void k3_left(const double* __restrict__ A, const cd (&x)[8], Put&& put) {
#pragma unroll 1
  for (int u = 0; u < 8; ++u) {
    cd acc = {0.0, 0.0};
#pragma unroll
    for (int l = 0; l < 8; ++l) acc = cfma(acc, cd{A[2 * (u * 8 + l)], A[2 * (u * 8 + l) + 1]}, x[l]);
    put(u, acc);
  }
}

// w[v] += sum_l t[l] conj(A[v][l]) for one row t of A x, t[l] = get(l); each
// w[v] takes its terms in the order l = 0..7.
template <typename Get>
HT_HD void k3_right_acc(const double* __restrict__ A, Get&& get, cd (&w)[8]) {
#pragma unroll 1
  for (int l = 0; l < 8; ++l) {
    const cd tl = get(l);
#pragma unroll
    for (int v = 0; v < 8; ++v) w[v] = cfma_cj(w[v], tl, cd{A[2 * (v * 8 + l)], A[2 * (v * 8 + l) + 1]});
  }
}

// Store row j of the block's result with the ownership rules of the
// conjugation pass (block_update_store): on a diagonal group, group tile
// (X, Y) is stored directly for X >= Y, and block (p, q), p > q, also writes
// the conjugate results of the skipped block (q, p).
template <int C, typename Mem>
HT_HD void k3_store_row(const Mem& mem, const ConjGeom<3, C>& g, const K3Group& gr,
                        const K3Tiles<C>& t, const K3Block& bk, int j, const cd (&w)[8]) {
  constexpr int KI = 3 - C;
  constexpr int IM = (1 << KI) - 1;
  const uint32_t ru = bk.p + dep_intra<KI>(j & IM, g.ipos);
  const int X = j >> KI;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const uint32_t cv = bk.q + dep_intra<KI>(v & IM, g.ipos);
    const int Y = v >> KI;
    const uint64_t tb = t.rowb[Y];
    const uint32_t offd = (ru << g.m) + cv;
    const uint32_t offm = (cv << g.m) + ru;
    if (!gr.diag) {
      if (t.rowd[Y])
        mem.store(tb, offd, w[v]);
      else
        mem.store(tb, offm, conjg(w[v]));
    } else if (X > Y) {
      mem.store(tb, offd, w[v]);
    } else if (X < Y) {
      if (bk.p != bk.q) mem.store(tb, offm, conjg(w[v]));
    } else {
      mem.store(tb, offd, w[v]);
      if (bk.p != bk.q) mem.store(tb, offm, conjg(w[v]));
    }
  }
}

}  // namespace ht
