// Per-lane body of the native pass for permutation-and-phase operations,
// shared by the GPU kernel (ht_native.hip) and the host-side checker.
//
// Section II-B: for a gate whose matrix has one nonzero per row (X, Z, S, T,
// CNOT, SWAP, Toffoli, ...) the update of a block is a permutation of its
// entries with phases, w[u][v] = c[u][v] h[p(u)][p(v)], and the entries that p
// fixes with c = 1 keep their value.  The pass therefore reads and writes only
// the entries that change: a diagonal gate on a tile-selecting qubit leaves
// the two tiles on the group's diagonal alone (half the bytes), a CNOT leaves
// the quarter with both control bits clear (three quarters of the bytes).
//
// Groups, blocks and the 8 x 8 lane patches are those of the conjugation pass
// (ht_geom.h).  Tile bases are computed from the group's reduced tile indices
// for each entry instead of being tabulated per group: a k = 3 group has up
// to 64 tiles, and the source tile of an entry depends on p at run time.
#pragma once

#include "ht_geom.h"
#include "ht_prep.h"

namespace ht {

// The operation: perm and the active mask travel by value; the 2^k x 2^k
// complex coefficients are read from device memory (uniform loads), and for
// k = 3 after them the chunk schedule of the prepared op, one entry per
// double (an exact integer).
template <int K>
struct NativeOp {
  static constexpr int D = 1 << K;
  int perm[D];
  uint64_t active;                 // bit u * D + v: entry (u, v) changes
  int nchunks;                     // k = 3: chunks of the schedule
  const double* __restrict__ c;    // 2 * D * D doubles, row-major complex [+ schedule]
  HT_HD bool act(int u, int v) const { return ((active >> (u * D + v)) & 1u) != 0; }
  HT_HD cd coef(int u, int v) const { return {c[2 * (u * D + v)], c[2 * (u * D + v) + 1]}; }
  HT_HD int sched(int i) const { return (int)c[2 * D * D + i]; }
};


// Blocks in flight per lane: 4 (k = 1, 16 entries) or 1 (k = 2, 16 entries);
// k = 3 walks its block in chunks of 16 or 32 entries (one block per step).
constexpr int native_unroll(int K) { return K == 1 ? 4 : 1; }

// The group: reduced tile indices Ti >= Tj.
struct NativeGroup {
  uint32_t Ti, Tj;
  bool diag;
};

template <int C>
HT_HD NativeGroup native_group(uint64_t grp) {
  uint32_t Ti, Tj;
  tri_decode(grp, Ti, Tj);
  NativeGroup r;
  r.Ti = wave_uniform(Ti);
  r.Tj = wave_uniform(Tj);
  r.diag = (C > 0) && (r.Ti == r.Tj);
  return r;
}

// Stored tile holding group tile (X, Y): element offset and orientation.
template <int K, int C>
HT_HD void native_tile(const ConjGeom<K, C>& g, const NativeGroup& ng, uint32_t X, uint32_t Y,
                       uint64_t& tb, bool& dir) {
  const uint32_t TR = ins_cross<C>(ng.Ti, X, g.cpos);
  const uint32_t TC = ins_cross<C>(ng.Tj, Y, g.cpos);
  dir = TR >= TC;
  const uint64_t hi = dir ? TR : TC, lo = dir ? TC : TR;
  tb = (tri64(hi) + lo) << (2 * g.m);
}

// Entry (a, b) of block (p, q): local row a, local column b (runtime values).
template <int K, int C, typename Mem>
HT_HD cd native_load(const Mem& mem, const ConjGeom<K, C>& g, const NativeGroup& ng, uint32_t p,
                     uint32_t q, int a, int b) {
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const uint32_t ru = p + dep_intra<KI>(a & IM, g.ipos);
  const uint32_t cv = q + dep_intra<KI>(b & IM, g.ipos);
  uint64_t tb;
  bool d;
  native_tile<K, C>(g, ng, (uint32_t)(a >> KI), (uint32_t)(b >> KI), tb, d);
  cd v = mem.load(tb, d ? (ru << g.m) + cv : (cv << g.m) + ru);
  if (!d) v.im = -v.im;
  return v;
}

// Write output entry (u, v) of block (p, q) with the ownership rules of the
// conjugation pass (mirrors conjugated; on diagonal groups block (p, q),
// p > q, also writes the mirror half, and block (p, p) only the stored side).
template <int K, int C, typename Mem>
HT_HD void native_store(const Mem& mem, const ConjGeom<K, C>& g, const NativeGroup& ng, uint32_t p,
                        uint32_t q, int u, int v, cd w) {
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const uint32_t ru = p + dep_intra<KI>(u & IM, g.ipos);
  const uint32_t cv = q + dep_intra<KI>(v & IM, g.ipos);
  const int X = u >> KI, Y = v >> KI;
  uint64_t tb;
  bool d;
  native_tile<K, C>(g, ng, (uint32_t)X, (uint32_t)Y, tb, d);
  const uint32_t offd = (ru << g.m) + cv;
  const uint32_t offm = (cv << g.m) + ru;
  if (!ng.diag) {
    if (d)
      mem.store(tb, offd, w);
    else
      mem.store(tb, offm, conjg(w));
  } else if (X > Y) {
    mem.store(tb, offd, w);
  } else if (X < Y) {
    if (p != q) mem.store(tb, offm, conjg(w));
  } else {
    mem.store(tb, offd, w);
    if (p != q) mem.store(tb, offm, conjg(w));
  }
}

// k = 3: a block has 64 entries, too many to hold at once at a useful
// occupancy; the lane walks its block chunk by chunk, CH entries each (each
// chunk closed under the permutation and under transposition, so loading
// all of a chunk's sources before writing it is safe in place, also where an
// entry and its transpose share storage).
// Jobs [job_begin, job_end) of the group (all by default), as in
// conj_group_lane.
template <int C, int CH, typename Mem>
HT_HD void native3_group_lane(const Mem& mem, const ConjGeom<3, C>& g, const NativeGroup& ng,
                              const NativeOp<3>& op, uint32_t lane, uint32_t job_begin = 0,
                              uint32_t job_end = 0xffffffffu) {
  constexpr int KI = 3 - C;
  const uint32_t nblk = 1u << (2 * g.F);
  if (job_end > g.jobs) job_end = g.jobs;
  for (uint32_t job = job_begin; job < job_end; ++job) {
    const uint32_t b = job * 64u + lane;
    uint32_t pidx, qidx;
    lane_block(b, g.F, g.s, g.ilv, pidx, qidx);
    const uint32_t p = deposit_free<KI>(pidx, g.ipos);
    const uint32_t q = deposit_free<KI>(qidx, g.ipos);
    if (b >= nblk || (ng.diag && p < q)) continue;
    for (int ch = 0; ch < op.nchunks; ++ch) {
      cd x[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int e = op.sched(ch * CH + i);
        if (e & 0x8000) x[i] = native_load<3, C>(mem, g, ng, p, q, (e >> 6) & 7, (e >> 9) & 7);
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int e = op.sched(ch * CH + i);
        if (e & 0x8000) {
          const int u = e & 7, v = (e >> 3) & 7;
          const cd c = op.coef(u, v);
          const bool one = c.re == 1.0 && c.im == 0.0;
          native_store<3, C>(mem, g, ng, p, q, u, v, one ? x[i] : cmul(c, x[i]));
        }
      }
    }
  }
}

// JU blocks of a lane: base rows and columns, whether each is the lane's,
// and the loaded sources of its changing entries.
template <int JU, int K>
struct NativeStep {
  uint32_t bp[JU], bq[JU];
  bool on[JU];
  cd x[JU][(1 << K) * (1 << K)];
};

// Load every changing entry of the lane's blocks job .. job + JU - 1 (those
// below job_end) from their permuted sources.  The sources of a block's
// entries lie in the same block, and blocks are disjoint.
template <int JU, int K, int C, typename Mem>
HT_HD void native_load_step(const Mem& mem, const ConjGeom<K, C>& g, const NativeGroup& ng, const NativeOp<K>& op,
                            uint32_t lane, uint32_t job, uint32_t job_end, NativeStep<JU, K>& st) {
  constexpr int D = 1 << K;
  constexpr int KI = K - C;
  const uint32_t nblk = 1u << (2 * g.F);
#pragma unroll
  for (int j = 0; j < JU; ++j) {
    const uint32_t b = (job + j) * 64u + lane;
    uint32_t pidx, qidx;
    lane_block(b, g.F, g.s, g.ilv, pidx, qidx);
    st.bp[j] = deposit_free<KI>(pidx, g.ipos);
    st.bq[j] = deposit_free<KI>(qidx, g.ipos);
    st.on[j] = job + j < job_end && b < nblk && !(ng.diag && st.bp[j] < st.bq[j]);
    if (st.on[j]) {
#pragma unroll
      for (int u = 0; u < D; ++u)
#pragma unroll
        for (int v = 0; v < D; ++v)
          if (op.act(u, v))
            st.x[j][u * D + v] = native_load<K, C>(mem, g, ng, st.bp[j], st.bq[j], op.perm[u], op.perm[v]);
    }
  }
}

// The products with the coefficients, written to the entries themselves.
template <int JU, int K, int C, typename Mem>
HT_HD void native_store_step(const Mem& mem, const ConjGeom<K, C>& g, const NativeGroup& ng, const NativeOp<K>& op,
                             const NativeStep<JU, K>& st) {
  constexpr int D = 1 << K;
#pragma unroll
  for (int j = 0; j < JU; ++j) {
    if (!st.on[j]) continue;
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int v = 0; v < D; ++v)
        if (op.act(u, v)) {
          const cd c = op.coef(u, v);
          // a coefficient of exactly one moves the entry unchanged (bitwise)
          const bool one = c.re == 1.0 && c.im == 0.0;
          native_store<K, C>(mem, g, ng, st.bp[j], st.bq[j], u, v,
                             one ? st.x[j][u * D + v] : cmul(c, st.x[j][u * D + v]));
        }
  }
}

// All blocks one lane owns in the current group, JU at a time: every
// changing entry of JU blocks loaded first, then written.
template <int JU, int K, int C, typename Mem>
HT_HD void native_group_lane(const Mem& mem, const ConjGeom<K, C>& g, const NativeGroup& ng,
                             const NativeOp<K>& op, uint32_t lane, uint32_t job_begin = 0,
                             uint32_t job_end = 0xffffffffu) {
  if (job_end > g.jobs) job_end = g.jobs;
  for (uint32_t job = job_begin; job < job_end; job += JU) {
    NativeStep<JU, K> st;
    native_load_step<JU, K, C>(mem, g, ng, op, lane, job, job_end, st);
    native_store_step<JU, K, C>(mem, g, ng, op, st);
  }
}

}  // namespace ht
