// Index arithmetic and the per-lane body of the tiled conjugation pass.
//
// Storage (Section III-B): tile (ti, tj), ti >= tj, is tile number
// ti(ti+1)/2 + tj; its M x M entries (M = 2^m) are row-major.
//
// Work decomposition (Section III-C generalised to k <= 2 targets):
//  * targets below m ("intra") address entries inside a tile, targets at or
//    above m ("cross", C of them) address tiles;
//  * removing the C cross bits from the tile indices leaves a reduced tile
//    grid of NtS = (N/M)/2^C rows; each pair (Ti >= Tj) of it is a "group":
//    the 2^C x 2^C tiles (ins(Ti, X), ins(Tj, Y)) that the operation mixes;
//  * a tile above the diagonal is reached through its stored mirror, read and
//    written conjugated and transposed (Algorithm 3 case B, Subroutine 3);
//  * inside a group, a block is fixed by its base row p and base column q
//    (positions inside a tile with the intra target bits cleared); block
//    (p, q) holds the 2^k x 2^k entries of Eq. (2): local row u = (X, ui),
//    local column v = (Y, vi), entry (X-tile, p + dep(ui), Y-tile, q + dep(vi)).
//  * one lane updates one block in registers; the 64 lanes of a wave take an
//    8 x 8 patch of (p, q) so that both a stored tile (rows p, 8 consecutive
//    columns q) and a mirrored one (rows q, 8 consecutive columns p) are read
//    as eight whole 128-byte lines per load instruction.
//  * groups on the diagonal of the reduced grid (Ti == Tj, C > 0) contain
//    each off-diagonal stored tile twice (directly and as a mirror); there
//    block (p, q) with p > q also writes the conjugate results of block
//    (q, p), which is skipped, and block (p, p) writes only entries whose
//    tile lies on or below the diagonal (the role of Subroutine 4).
// Every stored entry is written by exactly one lane per pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ht {

#define HT_HD __host__ __device__ inline

struct cd {
  double re, im;
};
HT_HD cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
HT_HD cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// acc + a * b
HT_HD cd cfma(cd acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + a * conj(b)
HT_HD cd cfma_cj(cd acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.im, b.re, acc.im);
  acc.im = fma(-a.re, b.im, acc.im);
  return acc;
}
HT_HD cd conjg(cd a) { return {a.re, -a.im}; }

// Storage element of the two dtypes: an interleaved (re, im) pair.
template <typename T>
struct store2;
template <>
struct store2<double> {
  using type = double2;
};
template <>
struct store2<float> {
  using type = float2;
};

template <typename T>
HT_HD cd load_c(const typename store2<T>::type* p, uint32_t off) {
  typename store2<T>::type v = p[off];
  return {(double)v.x, (double)v.y};
}
template <typename T>
HT_HD void store_c(typename store2<T>::type* p, uint32_t off, cd v) {
  typename store2<T>::type s;
  s.x = (T)v.re;
  s.y = (T)v.im;
  p[off] = s;
}

// Insert a zero bit at position pos: bits >= pos move up by one.
HT_HD uint32_t ins0(uint32_t x, int pos) {
  const uint32_t lo = x & ((1u << pos) - 1u);
  return ((x ^ lo) << 1) | lo;
}

HT_HD uint64_t tri64(uint64_t t) { return t * (t + 1) / 2; }

// g -> (ti, tj) with g = ti(ti+1)/2 + tj, 0 <= tj <= ti.
HT_HD void tri_decode(uint64_t g, uint32_t& ti, uint32_t& tj) {
  uint64_t t = (uint64_t)((sqrt(8.0 * (double)g + 1.0) - 1.0) * 0.5);
  while (tri64(t) > g) --t;
  while (tri64(t + 1) <= g) ++t;
  ti = (uint32_t)t;
  tj = (uint32_t)(g - tri64(t));
}

// Blocks in flight per lane: 16 entry loads for k = 1 (4 blocks) and for
// k = 2 (one block) of 16-byte entries -- 256 bytes per lane, the depth at
// which an in-place stream on MI355X reaches its best bandwidth.  8-byte
// entries stay in their storage type until their block is computed, which
// leaves room for two k = 2 blocks (measured +2..8 %; for k = 1 eight blocks
// measured slower than four).
constexpr int conj_unroll(int K, int entry_bytes = 16) {
  return K == 1 ? 4 : (entry_bytes == 8 ? 2 : 1);
}

// Geometry of one conjugation pass with K targets of which C are cross.
template <int K, int C>
struct ConjGeom {
  static constexpr int KI = K - C;
  int m;                       // effective tile exponent
  int F;                       // free bits per tile dimension: m - KI
  int s;                       // patch exponent: min(3, F)
  bool ilv;                    // alternate the high bits of p and q (lane_block)
  int ipos[KI > 0 ? KI : 1];   // intra target bits, ascending, < m
  int cpos[C > 0 ? C : 1];     // cross targets minus m, ascending
  uint32_t jobs;               // 64-block patches per group: ceil(4^F / 64)
  uint64_t ngroups;            // NtS (NtS + 1) / 2
};

// Deposit the bits of x into the positions that are not intra targets.
template <int KI>
HT_HD uint32_t deposit_free(uint32_t x, const int* ipos) {
#pragma unroll
  for (int l = 0; l < KI; ++l) x = ins0(x, ipos[l]);
  return x;
}

// Intra offset of local intra index ui: bit l of ui placed at ipos[l].
template <int KI>
HT_HD uint32_t dep_intra(int ui, const int* ipos) {
  uint32_t r = 0;
#pragma unroll
  for (int l = 0; l < KI; ++l) r |= (uint32_t)((ui >> l) & 1) << ipos[l];
  return r;
}

// Tile index with the cross bits of X inserted at cpos (ascending).
template <int C>
HT_HD uint32_t ins_cross(uint32_t t, uint32_t X, const int* cpos) {
#pragma unroll
  for (int l = 0; l < C; ++l) t = ins0(t, cpos[l]) | (((X >> l) & 1u) << cpos[l]);
  return t;
}

// Block index b (0 <= b < 4^F) -> base indices (pidx, qidx) in [0, 2^F):
// bits [0,s) -> q low, [s,2s) -> p low; the high bits either in two runs
// ([2s,F+s) -> q high, [F+s,2F) -> p high) or, with ilv, alternating
// (q high bit 0, p high bit 0, q high bit 1, ...), so that four consecutive
// patches cover 16 columns of 16 rows: whole 128-byte lines of 8-byte
// entries both in a stored tile (rows p) and in a mirrored one (rows q).
HT_HD void lane_block(uint32_t b, int F, int s, bool ilv, uint32_t& pidx, uint32_t& qidx) {
  const uint32_t ms = (1u << s) - 1u;
  if (!ilv) {
    const uint32_t mh = (1u << (F - s)) - 1u;
    qidx = (b & ms) | (((b >> (2 * s)) & mh) << s);
    pidx = ((b >> s) & ms) | ((b >> (F + s)) << s);
    return;
  }
  qidx = b & ms;
  pidx = (b >> s) & ms;
  const uint32_t hi = b >> (2 * s);
  for (int i = 0; i < F - s; ++i) {
    qidx |= ((hi >> (2 * i)) & 1u) << (s + i);
    pidx |= ((hi >> (2 * i + 1)) & 1u) << (s + i);
  }
}

// Items of one step of a workgroup of wpb waves (the step kernels), for
// groups of 2^sl steps: 2^r consecutive steps of each of wpb / 2^r groups
// (r <= sl, 2^r <= wpb), the groups consecutive (ps = 0) or every 2^ps-th
// of 2^ps times as many (the others in the next 2^ps - 1 units).
// r = min(sl, log2 wpb), ps = 0 takes whole groups; r = 0 gives every wave
// the same patches of its own group's tiles.  Every choice is a bijection
// of (unit, wave) onto (group, step), so results do not depend on it.
HT_HD uint64_t sync_units(uint64_t ngroups, int sl, uint32_t wpb, int r, int ps) {
  const uint64_t span = (uint64_t)(wpb >> r) << ps;  // groups one unit spans
  return ((ngroups + span - 1) / span) << (sl - r + ps);
}

HT_HD void sync_item(uint64_t u, uint32_t wib, uint32_t wpb, int sl, int r, int ps, uint64_t& grp,
                     uint32_t& step) {
  const int sr = sl - r;
  const uint64_t blk = u >> (sr + ps);
  const uint64_t h = (u >> sr) & ((1ull << ps) - 1u);
  const uint32_t sb = (uint32_t)u & ((1u << sr) - 1u);
  grp = blk * ((uint64_t)(wpb >> r) << ps) + ((uint64_t)(wib >> r) << ps) + h;
  step = (sb << r) | (wib & ((1u << r) - 1u));
}

// Per-group context: where each of the 2^C x 2^C tiles lives and whether it
// is stored in the orientation the group needs (dir) or as a mirror.
template <int C>
struct GroupCtx {
  uint64_t tbase[1 << C][1 << C];  // element offset of the stored tile
  bool dir[1 << C][1 << C];
  bool diag;
};

// A value every lane of a wave holds identically: on the GPU, tell the
// compiler so (it then keeps it in scalar registers).
HT_HD uint32_t wave_uniform(uint32_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_readfirstlane(x);
#else
  return x;
#endif
}

template <int K, int C>
HT_HD void group_ctx(uint64_t grp, const ConjGeom<K, C>& g, GroupCtx<C>& gc) {
  constexpr int NX = 1 << C;
  uint32_t Ti, Tj;
  tri_decode(grp, Ti, Tj);
  Ti = wave_uniform(Ti);  // grp is the same on every lane of the wave
  Tj = wave_uniform(Tj);
  gc.diag = (C > 0) && (Ti == Tj);
  uint32_t TR[NX], TC[NX];
#pragma unroll
  for (int X = 0; X < NX; ++X) {
    TR[X] = ins_cross<C>(Ti, (uint32_t)X, g.cpos);
    TC[X] = ins_cross<C>(Tj, (uint32_t)X, g.cpos);
  }
#pragma unroll
  for (int X = 0; X < NX; ++X) {
#pragma unroll
    for (int Y = 0; Y < NX; ++Y) {
      const bool d = TR[X] >= TC[Y];
      const uint64_t hi = d ? TR[X] : TC[Y];
      const uint64_t lo = d ? TC[Y] : TR[X];
      gc.dir[X][Y] = d;
      gc.tbase[X][Y] = (tri64(hi) + lo) << (2 * g.m);
    }
  }
}

// Coefficients of the operation.  Form 0 (direct): the 2^k x 2^k matrix A,
// applied as A h A^dagger.  Form 1 (transfer): the 4^k x 4^k matrix S acting
// on the row-major vector of h.  Small sets travel by value in the kernel
// arguments; the 16 x 16 transfer matrix of a two-qubit channel is read
// from device memory.
template <int K, int FORM>
struct Coef {
  static constexpr int D = 1 << K;
  static constexpr int NE = FORM == 0 ? D * D : D * D * D * D;
  double c[2 * NE];
  HT_HD cd at(int i) const { return {c[2 * i], c[2 * i + 1]}; }
};
template <>
struct Coef<2, 1> {
  static constexpr int NE = 256;
  const double* __restrict__ p;
  HT_HD cd at(int i) const { return {p[2 * i], p[2 * i + 1]}; }
};

// Apply the operation to the block x (row-major, 2^k x 2^k) and hand every
// output entry (u, v, w) to emit as soon as it is known.  The inputs stay in
// x until the end, so emit may overwrite the entries x was loaded from.
template <int K, int FORM, typename Emit>
HT_HD void block_apply(const cd (&x)[(1 << K) * (1 << K)], const Coef<K, FORM>& cf, Emit&& emit) {
  constexpr int D = 1 << K;
  if constexpr (FORM == 0) {
    // w = A x A^dagger, one output row at a time: t = (A x)[u, :], w[u, v] = t . conj(A[v, :])
#pragma unroll
    for (int u = 0; u < D; ++u) {
      cd t[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        cd acc = {0.0, 0.0};
#pragma unroll
        for (int l = 0; l < D; ++l) acc = cfma(acc, cf.at(u * D + l), x[l * D + j]);
        t[j] = acc;
      }
#pragma unroll
      for (int v = 0; v < D; ++v) {
        cd acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < D; ++j) acc = cfma_cj(acc, t[j], cf.at(v * D + j));
        emit(u, v, acc);
      }
    }
  } else {
    // w = S vec(x), vec row-major
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
      cd acc = {0.0, 0.0};
#pragma unroll
      for (int f = 0; f < D * D; ++f) acc = cfma(acc, cf.at(e * D * D + f), x[f]);
      emit(e / D, e % D, acc);
    }
  }
}

// Memory access of the pass: entry off of the stored tile at element offset tb.
// The kernels use plain loads and stores; a host-side checker substitutes a
// policy that verifies bounds and counts accesses.
// MODE bit 0: loads carry the nontemporal hint; bit 1: stores do.
template <typename T>
struct native2;
template <>
struct native2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct native2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};

// WIDE: hold loaded 8-byte entries as FP64 too (for kernels whose register
// budget is tight, and where it measured faster).
template <typename T, int MODE = 0, bool WIDE = false>
struct DirectMem {
  typename store2<T>::type* __restrict__ h;
  using V = typename native2<T>::type;
  // tile base (uniform) plus a 32-bit byte offset inside the tile
  HT_HD const V* at(uint64_t tb, uint32_t off) const {
    return reinterpret_cast<const V*>(reinterpret_cast<const char*>(h + tb) +
                                      (uint32_t)(off * (uint32_t)sizeof(V)));
  }
  HT_HD V load_v(uint64_t tb, uint32_t off) const {
    if constexpr ((MODE & 1) != 0)
      return __builtin_nontemporal_load(at(tb, off));
    else
      return *at(tb, off);
  }
  HT_HD cd load(uint64_t tb, uint32_t off) const {
    const V v = load_v(tb, off);
    return {(double)v.x, (double)v.y};
  }
  // A loaded entry as a lane holds it until its block is computed: as stored
  // (16-byte entries are FP64 values already; 8-byte ones take half the
  // registers, so twice the blocks in flight), conjugated only when the block
  // is widened.  Nothing is done to a loaded value before the block is
  // computed, so all loads of a step stay in flight together (a conjugation
  // at load time makes the compiler wait for every load at once).  WIDE
  // converts 8-byte entries to FP64 (and conjugates) at load instead.
  static constexpr bool kNarrow = sizeof(T) == 8 || !WIDE;
  struct Narrow {
    V v;
  };
  using R = typename std::conditional<kNarrow, Narrow, cd>::type;
  HT_HD R load_x(uint64_t tb, uint32_t off, bool cj) const {
    const V v = load_v(tb, off);
    if constexpr (kNarrow)
      return Narrow{v};
    else
      return cd{(double)v.x, cj ? -(double)v.y : (double)v.y};
  }
  // FP64 value of a held entry (cj: read through a mirror)
  HT_HD static cd widen(const R& r, bool cj) {
    if constexpr (kNarrow)
      return cd{(double)r.v.x, cj ? -(double)r.v.y : (double)r.v.y};
    else
      return r;
  }
  HT_HD void store(uint64_t tb, uint32_t off, cd w) const {
    V v;
    v.x = (T)w.re;
    v.y = (T)w.im;
    V* p = const_cast<V*>(at(tb, off));
    if constexpr ((MODE & 2) != 0)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  }
};

// Where block b of the current group sits: base row p and base column q
// inside a tile; inactive for the skipped half of diagonal groups and for
// padding lanes.
struct BlockPos {
  uint32_t p, q;
  bool active;
};

template <int K, int C>
HT_HD BlockPos block_pos(const ConjGeom<K, C>& g, const GroupCtx<C>& gc, uint32_t b, bool valid) {
  constexpr int KI = K - C;
  uint32_t pidx, qidx;
  lane_block(b, g.F, g.s, g.ilv, pidx, qidx);
  BlockPos r;
  r.p = deposit_free<KI>(pidx, g.ipos);
  r.q = deposit_free<KI>(qidx, g.ipos);
  r.active = valid && !(gc.diag && r.p < r.q);
  return r;
}

// Read the block's 2^k x 2^k entries (row-major, local bits in ascending
// target order); mirrored tiles are read transposed and their entries
// conjugated (when the block is widened, block_widen).  Called for inactive
// blocks too, which read the first entry of their tile instead: loads then
// never sit behind a branch, so the compiler keeps a whole step of them in
// flight (after a skipped load it could not count what is outstanding).
template <int K, int C, typename Mem>
HT_HD void block_load(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc,
                      const BlockPos& bp, typename Mem::R (&x)[(1 << K) * (1 << K)]) {
  constexpr int D = 1 << K;
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const int m = g.m;
#pragma unroll
  for (int u = 0; u < D; ++u) {
    const uint32_t ru = bp.p + dep_intra<KI>(u & IM, g.ipos);
#pragma unroll
    for (int v = 0; v < D; ++v) {
      const uint32_t cv = bp.q + dep_intra<KI>(v & IM, g.ipos);
      const int X = u >> KI, Y = v >> KI;
      const bool d = gc.dir[X][Y];
      const uint32_t off = d ? (ru << m) + cv : (cv << m) + ru;
      x[u * D + v] = mem.load_x(gc.tbase[X][Y], bp.active ? off : 0u, !d);
    }
  }
}

// The loaded block in FP64, mirrored entries conjugated.
template <int K, int C, typename Mem>
HT_HD void block_widen(const GroupCtx<C>& gc, const typename Mem::R (&x)[(1 << K) * (1 << K)],
                       cd (&w)[(1 << K) * (1 << K)]) {
  constexpr int D = 1 << K;
  constexpr int KI = K - C;
#pragma unroll
  for (int u = 0; u < D; ++u)
#pragma unroll
    for (int v = 0; v < D; ++v) w[u * D + v] = Mem::widen(x[u * D + v], !gc.dir[u >> KI][v >> KI]);
}

// Apply the operation to the loaded block and write the results back.
template <int K, int C, int FORM, typename Mem>
HT_HD void block_update_store(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc,
                              const Coef<K, FORM>& cf, const BlockPos& bp,
                              const typename Mem::R (&xr)[(1 << K) * (1 << K)]) {
  constexpr int KI = K - C;
  constexpr int IM = (1 << KI) - 1;
  const int m = g.m;
  const uint32_t p = bp.p, q = bp.q;
  cd x[(1 << K) * (1 << K)];
  block_widen<K, C, Mem>(gc, xr, x);
  block_apply<K, FORM>(x, cf, [&](int u, int v, cd w) {
    const uint32_t ru = p + dep_intra<KI>(u & IM, g.ipos);
    const uint32_t cv = q + dep_intra<KI>(v & IM, g.ipos);
    const int X = u >> KI, Y = v >> KI;
    const uint64_t tb = gc.tbase[X][Y];
    const uint32_t offd = (ru << m) + cv;
    const uint32_t offm = (cv << m) + ru;
    if (!gc.diag) {
      if (gc.dir[X][Y])
        mem.store(tb, offd, w);
      else
        mem.store(tb, offm, conjg(w));
    } else {
      // group on the diagonal of the reduced grid: dir[X][Y] == (X >= Y)
      if (X > Y) {
        mem.store(tb, offd, w);
      } else if (X < Y) {
        if (p != q) mem.store(tb, offm, conjg(w));
      } else {
        mem.store(tb, offd, w);
        if (p != q) mem.store(tb, offm, conjg(w));
      }
    }
  });
}

// All blocks one lane owns in the current group: patches of 64 blocks, JU
// patches per step, every load of a step issued before any update (JU
// blocks in flight per lane).
template <int JU, int K, int C, int FORM, typename Mem>
HT_HD void conj_group_lane(const Mem& mem, const ConjGeom<K, C>& g, const GroupCtx<C>& gc,
                           const Coef<K, FORM>& cf, uint32_t lane, uint32_t job_begin = 0,
                           uint32_t job_end = 0xffffffffu) {
  constexpr int D = 1 << K;
  const uint32_t nblk = 1u << (2 * g.F);
  if (job_end > g.jobs) job_end = g.jobs;
  for (uint32_t job = job_begin; job < job_end; job += JU) {
    BlockPos bp[JU];
    typename Mem::R x[JU][D * D];
#pragma unroll
    for (int j = 0; j < JU; ++j) {
      const uint32_t b = (job + j) * 64u + lane;
      bp[j] = block_pos<K, C>(g, gc, b, job + j < job_end && b < nblk);
      block_load<K, C>(mem, g, gc, bp[j], x[j]);
    }
#pragma unroll
    for (int j = 0; j < JU; ++j)
      if (bp[j].active) block_update_store<K, C, FORM>(mem, g, gc, cf, bp[j], x[j]);
  }
}

// Geometry of a pass for an n-qubit operator with effective tile exponent m
// and ascending targets sorted[0..K) of which the last C are cross targets.
template <int K, int C>
// ilv: the alternating patch order of lane_block.
HT_HD ConjGeom<K, C> make_geom(int n, int m, const int* sorted, bool ilv = false) {
  ConjGeom<K, C> g{};
  constexpr int KI = K - C;
  g.m = m;
  g.F = m - KI;
  g.s = g.F < 3 ? g.F : 3;
  g.ilv = ilv;
  for (int l = 0; l < KI; ++l) g.ipos[l] = sorted[l];
  for (int l = 0; l < C; ++l) g.cpos[l] = sorted[KI + l] - m;
  const uint32_t nblk = 1u << (2 * g.F);
  g.jobs = (nblk + 63u) / 64u;
  const uint64_t nts = (uint64_t)1 << (n - m - C);
  g.ngroups = nts * (nts + 1) / 2;
  return g;
}

}  // namespace ht
