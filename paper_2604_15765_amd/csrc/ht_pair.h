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

// Jobs [job_begin, job_end) of a group off the reduced-grid diagonal, JP
// pairs per lane per step (all loads of a step issued before any store).
// Mem holds a loaded pair as Mem::H:
//   load_pair(tb, off)        the entries at off and off + 1 of a stored tile;
//   load_two(tb, o0, o1)      two single entries (a mirrored tile);
//   widen(h, cj, a, b)        the pair in FP64, conjugated when cj;
//   set(h, i, w)              replace entry i (0 or 1) of the pair by w;
//   store_pair(tb, off, h)    and store_two_cj(tb, o0, o1, h) (conjugated).
// Each block of the pair is widened, transformed and written back into h
// before the next one, so a lane holds one FP64 block at a time.
template <int JP, int K, int C, int FORM, typename Mem>
HT_HD void pair_group_lane(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc,
                           const Coef<K, FORM>& cf, uint32_t lane, uint32_t job_begin,
                           uint32_t job_end) {
  constexpr int D = 1 << K;
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const int m = g.m;
  if (job_end > pair_jobs(g.F)) job_end = pair_jobs(g.F);
  for (uint32_t job = job_begin; job < job_end; job += JP) {
    uint32_t P[JP], Q[JP];
    typename Mem::H x[JP][D * D];
#pragma unroll
    for (int jp = 0; jp < JP; ++jp) {
      uint32_t pidx, qpidx;
      pair_block((job + jp) * 64u + lane, g.F, pidx, qpidx);
      P[jp] = deposit_free<KI>(pidx, g.ipos);
      Q[jp] = deposit_free<KI>(2u * qpidx, g.ipos);  // even; the second block is at Q + 1
#pragma unroll
      for (int e = 0; e < D * D; ++e) {
        const int u = e / D, v = e % D;
        const uint32_t ru = P[jp] + dep_intra<KI>(u & IM, g.ipos);
        const uint32_t cv = Q[jp] + dep_intra<KI>(v & IM, g.ipos);
        const int X = u >> KI, Y = v >> KI;
        const uint64_t tb = gc.tbase[X][Y];
        if (gc.dir[X][Y])
          x[jp][e] = mem.load_pair(tb, (ru << m) + cv);
        else
          x[jp][e] = mem.load_two(tb, (cv << m) + ru, ((cv + 1u) << m) + ru);
      }
    }
#pragma unroll
    for (int jp = 0; jp < JP; ++jp) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        cd a[D * D];
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
          const int u = e / D, v = e % D;
          cd lo, hi;
          Mem::widen(x[jp][e], !gc.dir[u >> KI][v >> KI], lo, hi);
          a[e] = i == 0 ? lo : hi;
        }
        block_apply<K, FORM>(a, cf, [&](int u, int v, cd w) { Mem::set(x[jp][u * D + v], i, w); });
      }
#pragma unroll
      for (int e = 0; e < D * D; ++e) {
        const int u = e / D, v = e % D;
        const uint32_t ru = P[jp] + dep_intra<KI>(u & IM, g.ipos);
        const uint32_t cv = Q[jp] + dep_intra<KI>(v & IM, g.ipos);
        const int X = u >> KI, Y = v >> KI;
        const uint64_t tb = gc.tbase[X][Y];
        if (gc.dir[X][Y])
          mem.store_pair(tb, (ru << m) + cv, x[jp][e]);
        else
          mem.store_two_cj(tb, (cv << m) + ru, ((cv + 1u) << m) + ru, x[jp][e]);
      }
    }
  }
}

}  // namespace ht
