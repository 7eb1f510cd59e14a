// Pair layout of the conjugation pass for 8-byte entries, shared by the GPU
// kernel (ht_conj.hip) and the host-side checker.
//
// In the block layout (ht_geom.h) a lane holds whole blocks and every load
// or store instruction moves one entry per lane: 8 bytes for complex64, so
// the 64 lanes of a patch row cover half of a 128-byte line.  In the pair
// layout a lane holds two blocks in adjacent columns q and q + 1: in a tile
// stored in the group's orientation the two blocks' entries at the same
// (u, v) are adjacent and travel as one 16-byte access, so an instruction
// covers whole lines (8 lanes x 16 bytes) like the complex128 pass; in a
// mirrored tile they lie in adjacent rows and take two 8-byte accesses.
// Requires k <= 2 without an intra target at bit 0 (so that q and q + 1 are
// both free columns) and at least 4 free bits per tile dimension; groups on
// the diagonal of the reduced grid keep the block layout (their ownership
// rules pair blocks (p, q) and (q, p)).
#pragma once

#include "ht_geom.h"

namespace ht {

// Pair patches per group: 4^F blocks, two per lane, 64 lanes.
HT_HD uint32_t pair_jobs(int F) { return 1u << (2 * F - 7); }

// Pair b of a group -> (pidx, qpidx): the lane's bits give the low three bits
// of the pair column index (8 lanes: 16 columns) and of the row index; the
// job bits go alternately to the next row bit and the next pair-column bit.
// Row bit first: in a mirrored tile a lane row of 8 rows x 8 B covers half a
// line, and the job that differs in row bit 3 covers the other half, so two
// consecutive jobs (one step, JP = 2) write whole lines there too.
HT_HD void pair_block(uint32_t b, int F, uint32_t& pidx, uint32_t& qpidx) {
  qpidx = b & 7u;
  pidx = (b >> 3) & 7u;
  uint32_t hi = b >> 6;
  int qs = 3, ps = 3;
  while (qs < F - 1 || ps < F) {
    if (ps < F) {
      pidx |= (hi & 1u) << ps;
      hi >>= 1;
      ++ps;
    }
    if (qs < F - 1) {
      qpidx |= (hi & 1u) << qs;
      hi >>= 1;
      ++qs;
    }
  }
}

// One step of a group off the reduced-grid diagonal: JP pair patches of a
// lane, loaded before any of them is updated.
// Mem holds a loaded pair as Mem::H:
//   load_pair(tb, off)        the entries at off and off + 1 of a stored tile;
//   load_two(tb, o0, o1)      two single entries (a mirrored tile);
//   widen(h, cj, a, b)        the pair in FP64, conjugated when cj;
//   set(h, i, w)              replace entry i (0 or 1) of the pair by w;
//   store_pair(tb, off, h)    and store_two_cj(tb, o0, o1, h) (conjugated).
template <int JP, int K, typename Mem>
struct PairStep {
  uint32_t P[JP], Q[JP];
  typename Mem::H x[JP][(1 << K) * (1 << K)];
};

// Load pair patches job .. job + JP - 1 of the lane.
template <int JP, int K, int C, typename Mem>
HT_HD void pair_load(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc, uint32_t lane, uint32_t job,
                     PairStep<JP, K, Mem>& ps) {
  constexpr int D = 1 << K;
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const int m = g.m;
#pragma unroll
  for (int jp = 0; jp < JP; ++jp) {
    uint32_t pidx, qpidx;
    pair_block((job + jp) * 64u + lane, g.F, pidx, qpidx);
    ps.P[jp] = deposit_free<KI>(pidx, g.ipos);
    ps.Q[jp] = deposit_free<KI>(2u * qpidx, g.ipos);  // even; the second block is at Q + 1
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
      const int u = e / D, v = e % D;
      const uint32_t ru = ps.P[jp] + dep_intra<KI>(u & IM, g.ipos);
      const uint32_t cv = ps.Q[jp] + dep_intra<KI>(v & IM, g.ipos);
      const int X = u >> KI, Y = v >> KI;
      const uint64_t tb = gc.tbase[X][Y];
      if (gc.dir[X][Y])
        ps.x[jp][e] = mem.load_pair(tb, (ru << m) + cv);
      else
        ps.x[jp][e] = mem.load_two(tb, (cv << m) + ru, ((cv + 1u) << m) + ru);
    }
  }
}

// Update the loaded pairs and write them back.  Each block of a pair is
// widened, transformed and written back into the held pair before the next
// one, so a lane holds one FP64 block at a time.
template <int JP, int K, int C, int FORM, typename Mem>
HT_HD void pair_update_store(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc,
                             const Coef<K, FORM>& cf, PairStep<JP, K, Mem>& ps) {
  constexpr int D = 1 << K;
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const int m = g.m;
#pragma unroll
  for (int jp = 0; jp < JP; ++jp) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      cd a[D * D];
#pragma unroll
      for (int e = 0; e < D * D; ++e) {
        const int u = e / D, v = e % D;
        cd lo, hi;
        Mem::widen(ps.x[jp][e], !gc.dir[u >> KI][v >> KI], lo, hi);
        a[e] = i == 0 ? lo : hi;
      }
      block_apply<K, FORM>(a, cf, [&](int u, int v, cd w) { Mem::set(ps.x[jp][u * D + v], i, w); });
    }
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
      const int u = e / D, v = e % D;
      const uint32_t ru = ps.P[jp] + dep_intra<KI>(u & IM, g.ipos);
      const uint32_t cv = ps.Q[jp] + dep_intra<KI>(v & IM, g.ipos);
      const int X = u >> KI, Y = v >> KI;
      const uint64_t tb = gc.tbase[X][Y];
      if (gc.dir[X][Y])
        mem.store_pair(tb, (ru << m) + cv, ps.x[jp][e]);
      else
        mem.store_two_cj(tb, (cv << m) + ru, ((cv + 1u) << m) + ru, ps.x[jp][e]);
    }
  }
}

// Jobs [job_begin, job_end) of a group off the reduced-grid diagonal, JP
// pairs per lane per step (all loads of a step issued before any store).
template <int JP, int K, int C, int FORM, typename Mem>
HT_HD void pair_group_lane(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc,
                           const Coef<K, FORM>& cf, uint32_t lane, uint32_t job_begin,
                           uint32_t job_end) {
  if (job_end > pair_jobs(g.F)) job_end = pair_jobs(g.F);
  for (uint32_t job = job_begin; job < job_end; job += JP) {
    PairStep<JP, K, Mem> ps;
    pair_load<JP, K, C>(mem, g, gc, lane, job, ps);
    pair_update_store<JP, K, C, FORM>(mem, g, gc, cf, ps);
  }
}

// The pair layout in workgroup-wide steps (pair_sync_kernel).  Steps per
// group: pair_jobs / JP.  Item order ord (0 whole groups, 1 the steps that
// share the tile's top row bit -- the pair patches' last job bit -- of
// consecutive groups, 2 of every other group, 3 of every fourth): r and ps
// of sync_item for wpb = 2^lw waves per workgroup.
HT_HD void pair_sync_order(int F, int JP, int lw, int ord, int& sl, int& r, int& ps) {
  const uint32_t steps = pair_jobs(F) / (uint32_t)JP;
  sl = 0;
  while ((1u << sl) < steps) ++sl;
  const int rmax = sl < lw ? sl : lw;
  r = (2 * F - 8) - (JP == 2 ? 1 : 0);
  if (ord == 0 || r > rmax) r = rmax;
  if (r < 0) r = 0;
  ps = ord == 2 ? 1 : ord == 3 ? 2 : 0;
}

// Group of reduced-grid row ti on the diagonal (Ti = Tj): ti (ti + 3) / 2.
HT_HD uint64_t diag_group(uint64_t ti) { return ti * (ti + 3) / 2; }

// The reduced grid's rows: ngroups = nts (nts + 1) / 2.
HT_HD uint64_t grid_rows(uint64_t ngroups) {
  uint64_t nts = 0;
  while ((nts + 1) * (nts + 2) / 2 <= ngroups) ++nts;
  return nts;
}

}  // namespace ht
