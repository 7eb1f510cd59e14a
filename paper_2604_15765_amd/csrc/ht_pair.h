// Pair layout of the one-qubit pass for 8-byte entries, shared by the GPU
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
// Requires k = 1 without an intra target at bit 0 (so that q and q + 1 are
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
// job bits go alternately to the next pair-column bit and the next row bit,
// so consecutive jobs first widen the patch to whole tile rows.
HT_HD void pair_block(uint32_t b, int F, uint32_t& pidx, uint32_t& qpidx) {
  qpidx = b & 7u;
  pidx = (b >> 3) & 7u;
  uint32_t hi = b >> 6;
  int qs = 3, ps = 3;
  while (qs < F - 1 || ps < F) {
    if (qs < F - 1) {
      qpidx |= (hi & 1u) << qs;
      hi >>= 1;
      ++qs;
    }
    if (ps < F) {
      pidx |= (hi & 1u) << ps;
      hi >>= 1;
      ++ps;
    }
  }
}

// Jobs [job_begin, job_end) of a group off the reduced-grid diagonal, JP
// pairs per lane per step (all loads of a step issued before any store).
// Mem: load / store of one entry, load_pair / store_pair of the entries at
// off and off + 1 (FP64 values).
template <int JP, int C, int FORM, typename Mem>
HT_HD void pair_group_lane(const Mem& mem, const ConjGeom<1, C>& g, const GroupCtx<C>& gc,
                           const Coef<1, FORM>& cf, uint32_t lane, uint32_t job_begin,
                           uint32_t job_end) {
  constexpr int KI = 1 - C;
  constexpr int IM = (1 << KI) - 1;
  const int m = g.m;
  if (job_end > pair_jobs(g.F)) job_end = pair_jobs(g.F);
  for (uint32_t job = job_begin; job < job_end; job += JP) {
    uint32_t P[JP], Q[JP];
    cd x[JP][2][4];
#pragma unroll
    for (int jp = 0; jp < JP; ++jp) {
      uint32_t pidx, qpidx;
      pair_block((job + jp) * 64u + lane, g.F, pidx, qpidx);
      P[jp] = deposit_free<KI>(pidx, g.ipos);
      Q[jp] = deposit_free<KI>(2u * qpidx, g.ipos);  // even; the second block is at Q + 1
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int u = e >> 1, v = e & 1;
        const uint32_t ru = P[jp] + dep_intra<KI>(u & IM, g.ipos);
        const uint32_t cv = Q[jp] + dep_intra<KI>(v & IM, g.ipos);
        const int X = u >> KI, Y = v >> KI;
        const uint64_t tb = gc.tbase[X][Y];
        if (gc.dir[X][Y]) {
          mem.load_pair(tb, (ru << m) + cv, x[jp][0][e], x[jp][1][e]);
        } else {
          x[jp][0][e] = conjg(mem.load(tb, (cv << m) + ru));
          x[jp][1][e] = conjg(mem.load(tb, ((cv + 1u) << m) + ru));
        }
      }
    }
#pragma unroll
    for (int jp = 0; jp < JP; ++jp) {
      cd w[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        block_apply<1, FORM>(x[jp][i], cf, [&](int u, int v, cd r) { w[i][u * 2 + v] = r; });
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int u = e >> 1, v = e & 1;
        const uint32_t ru = P[jp] + dep_intra<KI>(u & IM, g.ipos);
        const uint32_t cv = Q[jp] + dep_intra<KI>(v & IM, g.ipos);
        const int X = u >> KI, Y = v >> KI;
        const uint64_t tb = gc.tbase[X][Y];
        if (gc.dir[X][Y]) {
          mem.store_pair(tb, (ru << m) + cv, w[0][e], w[1][e]);
        } else {
          mem.store(tb, (cv << m) + ru, conjg(w[0][e]));
          mem.store(tb, ((cv + 1u) << m) + ru, conjg(w[1][e]));
        }
      }
    }
  }
}

}  // namespace ht
