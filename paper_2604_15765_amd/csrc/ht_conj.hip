// The conjugation pass: H -> sum_a K_a H K_a^dagger on tiled storage.
//
// One kernel template covers intra-tile operations (Algorithm 2, c = 0),
// operations whose targets select tiles (Algorithm 3 with Subroutines 2-4,
// c = 1) and two-qubit operations on two tile-selecting qubits (c = 2), for
// k = 1, 2 and for the direct (A h A^dagger) and transfer-matrix forms.  The
// per-lane arithmetic lives in ht_geom.h; this file holds the grid-stride
// driver and the runtime dispatch.
//
// The pass is a streaming read-modify-write of every stored entry (1-4 FP64
// flops per byte), so it is bound by HBM bandwidth; there is no matrix-core
// work in it.  Each wave owns whole groups, one at a time, and the blocks of a
// group are disjoint, so no synchronisation is needed.
#include "ht_geom.h"
#include "ht_internal.h"
#include "ht_pair.h"

namespace ht {

LaunchTuning& tuning() {
  static LaunchTuning t;
  return t;
}

template <typename T, int K, int C, int FORM, int MODE>
__global__ void __launch_bounds__(256)
    conj_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, C> g, Coef<K, FORM> cf,
                const double* __restrict__ coef, int order) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  // 8-byte entries: held as stored for intra-tile k = 1 and for k = 2 (two
  // blocks in flight), as FP64 for k = 1 with a tile-selecting target (the
  // faster choice per class, measured on one device: +7.5 % and +1.7 %)
  const DirectMem<T, MODE, (K == 1 && C > 0)> mem{h};
  if constexpr (K == 2 && FORM == 1) cf.p = coef;  // 16 x 16 transfer matrix, read-only
  constexpr int JU = conj_unroll(K, (int)sizeof(T) * 2);
  if (order == 0) {
    // one wave walks all patches of a group
    for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves) {
      GroupCtx<C> gc;
      group_ctx<K, C>(grp, g, gc);
      conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane);
    }
  } else {
    // (group, step of JU patches) items: neighbouring waves sweep one group
    const uint32_t steps = (g.jobs + JU - 1) / JU;  // a power of two
    const int sl = 31 - __builtin_clz(steps);
    const uint64_t items = g.ngroups << sl;
    for (uint64_t it = wave; it < items; it += nwaves) {
      GroupCtx<C> gc;
      group_ctx<K, C>(it >> sl, g, gc);
      const uint32_t j0 = (uint32_t)(it & (steps - 1)) * JU;
      conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane, j0, j0 + JU);
    }
  }
}

// ------------------------------------------------------- workgroup-wide steps

// The pass with its steps taken by a whole workgroup at once: the waves of a
// workgroup take (group, step) items (sync_item: whole groups of
// neighbouring tiles, or one quarter of the tiles of many groups), load all
// their blocks, meet at a barrier, then compute and store.  Every tile run
// that the workgroup covers in one step is then read completely before any
// of it is written back (measured on MI355X: in-place streams run faster in
// long read and write bursts than when each wave alternates on its own).
// The quarter orders keep the address bits just above a 4 KiB run equal
// across a workgroup step; an operator-sized probe measured in-place streams
// at 6.0-6.3 TB/s when every workgroup step's 4 KiB runs shared address
// bits 12-14, against 5.3-5.6 for contiguous 64 KiB runs.  Same lanes, same
// block arithmetic as conj_kernel: bitwise the same results.
template <typename T, int K, int C, int FORM, int MODE>
__global__ void __launch_bounds__(1024)
    conj_sync_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, C> g, Coef<K, FORM> cf,
                     const double* __restrict__ coef, int r, int ps) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wpb = blockDim.x >> 6;
  const DirectMem<T, MODE, (K == 1 && C > 0)> mem{h};
  using Mem = decltype(mem);
  if constexpr (K == 2 && FORM == 1) cf.p = coef;
  constexpr int JU = conj_unroll(K, (int)sizeof(T) * 2);
  constexpr int D = 1 << K;
  const uint32_t steps = (g.jobs + JU - 1) / JU;  // a power of two
  const int sl = 31 - __builtin_clz(steps);
  const uint64_t nu = sync_units(g.ngroups, sl, wpb, r, ps);
  const uint32_t nblk = 1u << (2 * g.F);
  // the loop bound is the same for every wave of the workgroup (barrier)
  for (uint64_t u = blockIdx.x; u < nu; u += gridDim.x) {
    uint64_t grp;
    uint32_t step;
    sync_item(u, wib, wpb, sl, r, ps, grp, step);
    const bool valid = grp < g.ngroups;
    GroupCtx<C> gc;
    group_ctx<K, C>(valid ? grp : 0, g, gc);
    const uint32_t j0 = step * JU;
    BlockPos bp[JU];
    typename Mem::R x[JU][D * D];
#pragma unroll
    for (int j = 0; j < JU; ++j) {
      const uint32_t b = (j0 + j) * 64u + lane;
      bp[j] = block_pos<K, C>(g, gc, b, valid && j0 + j < g.jobs && b < nblk);
      block_load<K, C>(mem, g, gc, bp[j], x[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < JU; ++j)
      if (bp[j].active) block_update_store<K, C, FORM>(mem, g, gc, cf, bp[j], x[j]);
  }
}

// The workgroup-wide steps with the next step's loads issued before the
// current step is computed: every wave holds two steps of blocks in
// registers, so the FP64 work of one step overlaps the loads of the next.
// All waves of the workgroup have their current step loaded before any of
// them stores it (a barrier after each wave's own wait).
template <int JU, int K, int C, typename Mem>
struct PipeSlot {
  GroupCtx<C> gc;
  BlockPos bp[JU];
  typename Mem::R x[JU][(1 << K) * (1 << K)];
};

template <int JU, int K, int C, typename Mem>
__device__ inline void pipe_load(const Mem& mem, const ConjGeom<K, C>& g, uint64_t it, uint64_t items, int sl,
                                 uint32_t lane, PipeSlot<JU, K, C, Mem>& sl_) {
  const bool valid = it < items;
  group_ctx<K, C>(valid ? (it >> sl) : 0, g, sl_.gc);
  const uint32_t steps_mask = (1u << sl) - 1u;
  const uint32_t j0 = (uint32_t)(it & steps_mask) * JU;
  const uint32_t nblk = 1u << (2 * g.F);
#pragma unroll
  for (int j = 0; j < JU; ++j) {
    const uint32_t b = (j0 + j) * 64u + lane;
    sl_.bp[j] = block_pos<K, C>(g, sl_.gc, b, valid && j0 + j < g.jobs && b < nblk);
    block_load<K, C>(mem, g, sl_.gc, sl_.bp[j], sl_.x[j]);
  }
}

// Wait for this lane's loads of a slot (an empty asm that reads every loaded
// register makes the compiler wait for them), then meet the other waves.
template <int JU, int K, int C, typename Mem, bool BAR>
__device__ inline void pipe_arrive(PipeSlot<JU, K, C, Mem>& sl_) {
#pragma unroll
  for (int j = 0; j < JU; ++j)
#pragma unroll
    for (int e = 0; e < (1 << K) * (1 << K); ++e) {
      if constexpr (Mem::kNarrow)
        asm volatile("" ::"v"(sl_.x[j][e].v));
      else
        asm volatile("" ::"v"(sl_.x[j][e].re), "v"(sl_.x[j][e].im));
    }
  if constexpr (BAR) __builtin_amdgcn_s_barrier();
}

template <int JU, int K, int C, int FORM, typename Mem>
__device__ inline void pipe_store(const Mem& mem, const ConjGeom<K, C>& g, const Coef<K, FORM>& cf,
                                  PipeSlot<JU, K, C, Mem>& sl_) {
#pragma unroll
  for (int j = 0; j < JU; ++j)
    if (sl_.bp[j].active) block_update_store<K, C, FORM>(mem, g, sl_.gc, cf, sl_.bp[j], sl_.x[j]);
}

template <typename T, int K, int C, int FORM, int MODE, int NTH, bool BAR>
__global__ void __launch_bounds__(NTH)
    conj_pipe_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, C> g, Coef<K, FORM> cf,
                     const double* __restrict__ coef) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr uint32_t wpb = NTH / 64;
  using Mem = DirectMem<T, MODE, (K == 1 && C > 0)>;
  const Mem mem{h};
  if constexpr (K == 2 && FORM == 1) cf.p = coef;
  constexpr int JU = conj_unroll(K, (int)sizeof(T) * 2);
  const uint32_t steps = (g.jobs + JU - 1) / JU;  // a power of two
  const int sl = 31 - __builtin_clz(steps);
  const uint64_t items = g.ngroups << sl;
  const uint64_t stride = (uint64_t)gridDim.x * wpb;
  uint64_t base = (uint64_t)blockIdx.x * wpb;
  if (base >= items) return;  // the whole workgroup
  PipeSlot<JU, K, C, Mem> a, b;
  pipe_load<JU, K, C>(mem, g, base + wib, items, sl, lane, a);
  // two steps per turn, so that the slots alternate without copies; every
  // bound below is the same for all waves of the workgroup
  // The prefetch is issued unconditionally (past the end it reads the first
  // entry of group 0's tiles): a load behind a branch would make the
  // compiler wait for every outstanding load, the prefetch included, before
  // the current step is used.
  for (;;) {
    uint64_t nb = base + stride;
    pipe_load<JU, K, C>(mem, g, nb + wib, items, sl, lane, b);
    pipe_arrive<JU, K, C, Mem, BAR>(a);
    pipe_store<JU, K, C, FORM>(mem, g, cf, a);
    if (nb >= items) break;
    base = nb;
    nb = base + stride;
    pipe_load<JU, K, C>(mem, g, nb + wib, items, sl, lane, a);
    pipe_arrive<JU, K, C, Mem, BAR>(b);
    pipe_store<JU, K, C, FORM>(mem, g, cf, b);
    if (nb >= items) break;
    base = nb;
  }
}

// ------------------------------------------------------- LDS-staged intra pass

// Intra-tile passes (Algorithm 2: every target inside the tile, every stored
// tile handled alike, diagonal tiles in both halves) staged through LDS.
// Tiles are contiguous in storage, so a workgroup step takes 16 KiB per
// wave of the threads (64 or 128 KiB: whole tiles of at most that size) --
// the next contiguous run of the buffer, or (PAR) every other 16 KiB
// granule of twice that span -- with 1 KiB nontemporal loads per wave
// instruction, puts it in LDS, applies the operation to every block of
// those tiles out of LDS, and writes it back the same way.  Global
// accesses are whole lines whatever the target bits; the block arithmetic
// is that of conj_kernel (block_apply), so results are bitwise the same.
constexpr int kStageVecs = 16;                 // 16-byte vectors per thread and step

// Workgroup barrier for LDS traffic only: waits for this wave's LDS accesses,
// not for its global loads (a prefetch may stay in flight across it).
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// PAR: a step takes every other 16 KiB granule of twice its span (the
// other step of the pair the granules in between), so that the granules a
// workgroup step touches share address bit 14; tiles of at most 16 KiB only
// (a granule then holds whole tiles).
constexpr uint32_t kGranVecs = 1024;  // 16-byte vectors per 16 KiB granule

template <typename T, int K, int FORM, int kStageThreads, bool PIPE, bool PAR = false>
__global__ void __launch_bounds__(kStageThreads)
    stage_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, 0> g, Coef<K, FORM> cf,
                 const double* __restrict__ coef, uint64_t total) {
  using S2 = typename store2<T>::type;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  constexpr uint32_t EPV = 16 / sizeof(S2);                 // entries per vector
  constexpr uint32_t CAPV = kStageVecs * kStageThreads;     // vectors per step
  constexpr uint32_t CAP = CAPV * EPV;                      // entries per step
  constexpr uint32_t GPS = CAPV / kGranVecs;                // granules per step
  constexpr int D = 1 << K;
  __shared__ u4 lds[CAPV];
  if constexpr (K == 2 && FORM == 1) cf.p = coef;
  const uint32_t t = threadIdx.x;
  const int m = g.m;
  const int F = g.F;
  const uint32_t bpt_log = 2u * (uint32_t)F;                // blocks per tile = 4^F
  const uint64_t tv = total / EPV;                          // vectors in the buffer
  const uint64_t nsteps =
      PAR ? 2 * ((tv + 2ull * CAPV - 1) / (2ull * CAPV)) : (total + CAP - 1) / CAP;
  u4* __restrict__ hv = reinterpret_cast<u4*>(h);
  S2* le = reinterpret_cast<S2*>(lds);
  // first granule of step st (PAR)
  auto gran0 = [&](uint64_t st) -> uint64_t { return (st >> 1) * (2ull * GPS) + (st & 1u); };
  // buffer vector of the step's i-th vector
  auto vaddr = [&](uint64_t st, uint32_t i) -> uint64_t {
    if constexpr (PAR) return (gran0(st) + 2ull * (i / kGranVecs)) * kGranVecs + (i % kGranVecs);
    return st * CAPV + i;
  };
  // vectors of step st that lie in the buffer (whole tiles; they form a
  // prefix of the step's vectors, since only the buffer's last granule can
  // be partial)
  auto count_v = [&](uint64_t st) -> uint32_t {
    if constexpr (PAR) {
      uint32_t c = 0;
      for (uint32_t i = 0; i < GPS; ++i) {
        const uint64_t g0 = (gran0(st) + 2ull * i) * kGranVecs;
        if (g0 < tv) c += (tv - g0 < kGranVecs) ? (uint32_t)(tv - g0) : kGranVecs;
      }
      return c;
    }
    const uint64_t left = total - st * CAP;
    return (left < CAP ? (uint32_t)left : CAP) / EPV;
  };
  auto load_step = [&](uint64_t st, u4 (&v)[kStageVecs]) {
    const uint32_t cntv = count_v(st);
    if (cntv == CAPV) {
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) v[j] = __builtin_nontemporal_load(hv + vaddr(st, j * kStageThreads + t));
    } else {
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) {
        const uint32_t i = j * kStageThreads + t;
        if (i < cntv) v[j] = __builtin_nontemporal_load(hv + vaddr(st, i));
      }
    }
  };
  u4 v[kStageVecs];
  uint64_t st = blockIdx.x;
  if (PIPE && st < nsteps) load_step(st, v);
  for (; st < nsteps; st += gridDim.x) {
    const uint32_t cntv = count_v(st);
    const uint32_t cnt = cntv * EPV;
    if constexpr (!PIPE) load_step(st, v);
    if (cntv == CAPV) {
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) lds[j * kStageThreads + t] = v[j];
    } else {
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) {
        const uint32_t i = j * kStageThreads + t;
        if (i < cntv) lds[i] = v[j];
      }
    }
    lds_barrier();
    if constexpr (PIPE) {
      // the next step's loads stay in flight while this one is computed and stored
      if (st + gridDim.x < nsteps) load_step(st + gridDim.x, v);
    }
    const uint32_t nb = cnt >> (2 * K);
    for (uint32_t b = t; b < nb; b += kStageThreads) {
      S2* tb = le + ((b >> bpt_log) << (2 * m));
      const uint32_t w = b & ((1u << bpt_log) - 1u);
      const uint32_t p = deposit_free<K>(w >> F, g.ipos);
      const uint32_t q = deposit_free<K>(w & ((1u << F) - 1u), g.ipos);
      cd x[D * D];
#pragma unroll
      for (int u = 0; u < D; ++u)
#pragma unroll
        for (int vv = 0; vv < D; ++vv) {
          const S2 e = tb[((p + dep_intra<K>(u, g.ipos)) << m) + q + dep_intra<K>(vv, g.ipos)];
          x[u * D + vv] = cd{(double)e.x, (double)e.y};
        }
      block_apply<K, FORM>(x, cf, [&](int u, int vv, cd r) {
        S2 e;
        e.x = (T)r.re;
        e.y = (T)r.im;
        tb[((p + dep_intra<K>(u, g.ipos)) << m) + q + dep_intra<K>(vv, g.ipos)] = e;
      });
    }
    lds_barrier();
    if (cntv == CAPV) {
      u4 o[kStageVecs];
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) o[j] = lds[j * kStageThreads + t];
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) __builtin_nontemporal_store(o[j], hv + vaddr(st, j * kStageThreads + t));
    } else {
#pragma unroll
      for (int j = 0; j < kStageVecs; ++j) {
        const uint32_t i = j * kStageThreads + t;
        if (i < cntv) __builtin_nontemporal_store(lds[i], hv + vaddr(st, i));
      }
    }
  }
}

// ------------------------------------------------------------- pair layout

// Complex64 entries for the pair layout (ht_pair.h): single entries and
// 16-byte pairs.  NARROW: a lane holds a loaded pair as it is stored (four
// floats), else as two FP64 values.  MODE as for DirectMem.
template <int MODE, bool NARROW>
struct PairMem {
  float2* __restrict__ h;
  typedef float V2 __attribute__((ext_vector_type(2)));
  typedef float V4 __attribute__((ext_vector_type(4)));
  struct Wide {
    cd a, b;
  };
  using H = typename std::conditional<NARROW, V4, Wide>::type;
  template <typename V>
  __device__ V* at(uint64_t tb, uint32_t off) const {
    return reinterpret_cast<V*>(reinterpret_cast<char*>(h + tb) + (uint32_t)(off * 8u));
  }
  template <typename V>
  __device__ V ld(uint64_t tb, uint32_t off) const {
    if constexpr ((MODE & 1) != 0)
      return __builtin_nontemporal_load(at<V>(tb, off));
    else
      return *at<V>(tb, off);
  }
  template <typename V>
  __device__ void st(uint64_t tb, uint32_t off, V v) const {
    if constexpr ((MODE & 2) != 0)
      __builtin_nontemporal_store(v, at<V>(tb, off));
    else
      *at<V>(tb, off) = v;
  }
  __device__ static H make(V4 v) {
    if constexpr (NARROW)
      return v;
    else
      return Wide{cd{(double)v.x, (double)v.y}, cd{(double)v.z, (double)v.w}};
  }
  __device__ static V4 narrow(const H& x) {
    if constexpr (NARROW)
      return x;
    else
      return V4{(float)x.a.re, (float)x.a.im, (float)x.b.re, (float)x.b.im};
  }
  __device__ H load_pair(uint64_t tb, uint32_t off) const { return make(ld<V4>(tb, off)); }
  __device__ H load_two(uint64_t tb, uint32_t o0, uint32_t o1) const {
    const V2 a = ld<V2>(tb, o0), b = ld<V2>(tb, o1);
    return make(V4{a.x, a.y, b.x, b.y});
  }
  __device__ static void widen(const H& x, bool cj, cd& a, cd& b) {
    if constexpr (NARROW) {
      a = cd{(double)x.x, cj ? -(double)x.y : (double)x.y};
      b = cd{(double)x.z, cj ? -(double)x.w : (double)x.w};
    } else {
      a = cj ? conjg(x.a) : x.a;
      b = cj ? conjg(x.b) : x.b;
    }
  }
  __device__ static void set(H& x, int i, cd w) {
    if constexpr (NARROW) {
      if (i == 0) {
        x.x = (float)w.re;
        x.y = (float)w.im;
      } else {
        x.z = (float)w.re;
        x.w = (float)w.im;
      }
    } else {
      (i == 0 ? x.a : x.b) = w;
    }
  }
  __device__ void store_pair(uint64_t tb, uint32_t off, const H& x) const { st<V4>(tb, off, narrow(x)); }
  __device__ void store_two_cj(uint64_t tb, uint32_t o0, uint32_t o1, const H& x) const {
    const V4 v = narrow(x);
    st<V2>(tb, o0, V2{v.x, -v.y});
    st<V2>(tb, o1, V2{v.z, -v.w});
  }
};

// The conjugation pass on complex64 storage in the pair layout, JP pairs
// per lane and step; groups on the diagonal of the reduced grid take the
// block layout with 2 JP blocks per step (the same step count).  k = 1
// holds pairs as FP64 values (as the block layout does for tile-selecting
// targets), k = 2 as stored (16 entries per block, one block in FP64 at a
// time).
template <int K, int C, int FORM, int MODE, int JP>
__global__ void __launch_bounds__(256)
    pair_kernel(float2* __restrict__ h, ConjGeom<K, C> g, Coef<K, FORM> cf, int order) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const DirectMem<float, MODE, K == 1> mem{h};
  const PairMem<MODE, K == 2> pm{h};
  static_assert(K == 1 || FORM == 0, "two-qubit pair passes take the direct form");
  constexpr int JU = 2 * JP;
  if (order == 0) {
    for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves) {
      GroupCtx<C> gc;
      group_ctx<K, C>(grp, g, gc);
      if (gc.diag)
        conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane);
      else
        pair_group_lane<JP, K, C, FORM>(pm, g, gc, cf, lane, 0, 0xffffffffu);
    }
  } else {
    const uint32_t steps = g.jobs / JU;  // = pair_jobs / JP, a power of two
    const int sl = 31 - __builtin_clz(steps);
    const uint64_t items = g.ngroups << sl;
    for (uint64_t it = wave; it < items; it += nwaves) {
      GroupCtx<C> gc;
      group_ctx<K, C>(it >> sl, g, gc);
      const uint32_t st = (uint32_t)(it & (steps - 1));
      if (gc.diag)
        conj_group_lane<JU, K, C, FORM>(mem, g, gc, cf, lane, st * JU, st * JU + JU);
      else
        pair_group_lane<JP, K, C, FORM>(pm, g, gc, cf, lane, st * JP, st * JP + JP);
    }
  }
}

// The pair layout in workgroup-wide steps (complex64): the waves of a
// workgroup take (group, step) items in the order of sync_item, load their
// pairs, meet at a barrier, then update and store, as conj_sync_kernel does
// for the block layout.  Groups on the reduced-grid diagonal keep the block
// layout (their ownership rules pair blocks (p, q) and (q, p)); they are
// skipped here and done by pair_diag_kernel, so that this kernel holds only
// the pair path's registers.  Same arithmetic as pair_kernel: bitwise the
// same results.
template <int K, int C, int FORM, int MODE, int JP, int NTH>
__global__ void __launch_bounds__(NTH)
    pair_sync_kernel(float2* __restrict__ h, ConjGeom<K, C> g, Coef<K, FORM> cf, int r, int ps) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr uint32_t wpb = NTH / 64;
  const PairMem<MODE, K == 2> pm{h};
  using PM = PairMem<MODE, K == 2>;
  static_assert(K == 1 || FORM == 0, "two-qubit pair passes take the direct form");
  const uint32_t steps = pair_jobs(g.F) / JP;  // a power of two
  const int sl = 31 - __builtin_clz(steps);
  const uint64_t nu = sync_units(g.ngroups, sl, wpb, r, ps);
  // the loop bound is the same for every wave of the workgroup (barrier)
  for (uint64_t u = blockIdx.x; u < nu; u += gridDim.x) {
    uint64_t grp;
    uint32_t step;
    sync_item(u, wib, wpb, sl, r, ps, grp, step);
    GroupCtx<C> gc;
    group_ctx<K, C>(grp < g.ngroups ? grp : 0, g, gc);
    const bool pair = grp < g.ngroups && !gc.diag;
    PairStep<JP, K, PM> st;
    if (pair) pair_load<JP, K, C>(pm, g, gc, lane, step * JP, st);
    __syncthreads();
    if (pair) pair_update_store<JP, K, C, FORM>(pm, g, gc, cf, st);
  }
}

// The reduced-grid diagonal groups (Ti = Tj: group Ti (Ti + 3) / 2) of a
// pair pass in the block layout, one group per wave.
template <int K, int C, int FORM, int MODE>
__global__ void __launch_bounds__(256)
    pair_diag_kernel(float2* __restrict__ h, ConjGeom<K, C> g, Coef<K, FORM> cf, uint64_t nts) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const DirectMem<float, MODE, K == 1> mem{h};
  for (uint64_t ti = wave; ti < nts; ti += nwaves) {
    GroupCtx<C> gc;
    group_ctx<K, C>(diag_group(ti), g, gc);
    // only groups that the pair path skips (C > 0: every Ti = Tj group)
    if (gc.diag) conj_group_lane<conj_unroll(K, 8), K, C, FORM>(mem, g, gc, cf, lane);
  }
}

// Memory mode of a complex64 pair pass in workgroup steps: nontemporal,
// except where many groups hold a mirrored tile: every target
// tile-selecting and the highest at bit n - 3 or above for k = 2, at the
// top bit n - 1 for k = 1 (in steps, both halves of a mirrored line are read
// in one step; measured at n = 16, k = 1 nontemporal: target 13 5.64 TB/s
// against 5.15 plain, 14 5.26 against 5.05, 15 4.67 against 4.96).
template <int K, int C>
static int smode_pair(const ConjGeom<K, C>& g, int n) {
  int pmode = tuning().mem_mode;
  if (pmode < 0) {
    pmode = 3;
    if constexpr (K - C == 0)
      if (g.cpos[C - 1] + g.m >= (K == 1 ? n - 1 : n - 3)) pmode = 0;
  }
  return pmode;
}

// Launch pair_sync_kernel and pair_diag_kernel: item order from the shape,
// the tuning or (-1) whole groups; the quarter orders give a workgroup step
// the steps that share the tile's top row bit (the pair patches' last job
// bit) and take every group, every other one or every fourth.  16 waves per
// workgroup for k = 1; k = 2 (above 128 registers) takes 8.
template <int K, int C, int FORM>
static hipError_t launch_pair_sync(float2* hp, const ConjGeom<K, C>& g, const Coef<K, FORM>& cf, int shape,
                                   int pmode, int num_cu, hipStream_t s) {
  constexpr int NTH = K == 1 ? 1024 : 512;
  constexpr uint32_t wpb = NTH / 64;
  // two pairs per lane and step for k = 1; one for k = 2 (two would spill)
  constexpr int jp = K == 1 ? 2 : 1;
  // automatic: every fourth group for k = 1 (measured at n = 16, tile bits
  // 0-5: 5.8-5.9 TB/s against 5.0-5.3 for pair_kernel), whole groups else
  int ord = tuning().sync_order;
  if (shape >= 0) ord = shape_sync_order(shape);
  if (ord < 0) ord = K == 1 ? 3 : 0;
  int sl, r, ps;
  pair_sync_order(g.F, jp, 31 - __builtin_clz(wpb), ord, sl, r, ps);
  uint64_t wg = sync_units(g.ngroups, sl, wpb, r, ps);
  // one workgroup per CU (measured 1-3 % faster than 3/4 in every order)
  uint64_t wcap = tuning().sync_grid > 0 ? (uint64_t)tuning().sync_grid
                                         : (uint64_t)num_cu * (uint64_t)tuning().sync_wg_per_cu;
  if (shape >= 0) wcap = shape_grid(shape, num_cu);
  if (wg > wcap) wg = wcap;
  const dim3 grid((unsigned)wg), block(NTH);
#define HT_PS(M_, J_) \
  hipLaunchKernelGGL((pair_sync_kernel<K, C, FORM, M_, J_, NTH>), grid, block, 0, s, hp, g, cf, r, ps)
  switch (pmode) {
    case 1: HT_PS(1, jp); break;
    case 2: HT_PS(2, jp); break;
    case 3: HT_PS(3, jp); break;
    default: HT_PS(0, jp);
  }
#undef HT_PS
  hipError_t e = hipGetLastError();
  // intra-tile passes (C = 0) have no diagonal groups: the pair path takes
  // diagonal tiles like any other
  if (e != hipSuccess || C == 0) return e;
  const uint64_t nts = grid_rows(g.ngroups);
  const unsigned dg = (unsigned)((nts + 3) / 4 < (uint64_t)num_cu ? (nts + 3) / 4 : (uint64_t)num_cu);
#define HT_PD(M_) hipLaunchKernelGGL((pair_diag_kernel<K, C, FORM, M_>), dim3(dg), dim3(256), 0, s, hp, g, cf, nts)
  switch (pmode) {
    case 1: HT_PD(1); break;
    case 2: HT_PD(2); break;
    case 3: HT_PD(3); break;
    default: HT_PD(0);
  }
#undef HT_PD
  return hipGetLastError();
}

template <typename T, int K, int C, int FORM>
static hipError_t launch_t(void* buf, int n, int m, const PreparedOp& op, const double* coef_dev,
                           int num_cu, hipStream_t s) {
  ConjGeom<K, C> g = make_geom<K, C>(n, m, op.sorted, use_interleave((int)sizeof(T) * 2));
  Coef<K, FORM> cf;
  if constexpr (K == 2 && FORM == 1) {
    cf.p = nullptr;  // the kernel reads coef_dev
  } else {
    for (int i = 0; i < 2 * Coef<K, FORM>::NE; ++i) cf.c[i] = op.coef[i];
  }
  const int threads = tuning().block_threads;
  const uint64_t waves_per_wg = (uint64_t)threads / 64;
  const uint64_t steps = (g.jobs + conj_unroll(K, (int)sizeof(T) * 2) - 1) / conj_unroll(K, (int)sizeof(T) * 2);
  // Automatic workgroups per CU for complex128 operators of 1 GiB and more:
  // 1 in the direct form, 2 in the transfer form (measured at n = 16 and 14:
  // fewer waves in flight keep the groups being worked on close together in
  // memory; the n = 16 layers ran 74.9 passes/s against 72.8 at 8; one wave
  // per SIMD cannot hide the transfer form's FP64 work).  Else 8: a
  // cache-resident n = 12 operator ran 13 % slower at 2, and complex64
  // slower in the block layout.
  const uint64_t nent = ((1ull << n) * ((1ull << n) + (1ull << g.m))) >> 1;
  const bool big = sizeof(T) == 8 && nent * 2 * sizeof(T) >= (1ull << 30);
  const uint64_t cap = (uint64_t)num_cu * (uint64_t)wg_per_cu_or(big ? (FORM == 0 ? 1 : 2) : 8);
  // automatic order: split groups over waves when whole groups would leave
  // the grid's waves idle (small operators, few large cross-tile groups)
  int order = tuning().order;
  if (order < 0) order = g.ngroups < cap * waves_per_wg ? 1 : 0;
  const uint64_t items = order == 0 ? g.ngroups : g.ngroups * steps;
  uint64_t wgs = (items + waves_per_wg - 1) / waves_per_wg;
  if (wgs > cap) wgs = cap;
  if (wgs < 1) wgs = 1;
  auto* hp = reinterpret_cast<typename store2<T>::type*>(buf);
  // Lowest intra target (none: 99).  Automatic choices for operators of
  // 1 GiB and more, measured at n = 16 (TB/s of algorithmic traffic):
  // intra-tile passes staged through LDS in 128 KiB steps of alternate
  // 16 KiB granules with the next step prefetched (c128 5.9-6.15, the
  // lane-patch kernel 4.7-5.7); complex128 passes with a tile-selecting
  // target in workgroup-wide steps of 16 waves whose item order follows the
  // target's tile bit (5.45-5.87, whole groups 5.2-5.5); an intra target
  // below bit 3 beside a tile-selecting one stays on the lane-patch kernel;
  // complex64 with a tile-selecting target takes the pair step kernel.
  constexpr int KI = K - C;
  const int low = KI > 0 ? g.ipos[0] : 99;
  // highest tile-selecting target at tile bit 4 or above
  const int far = (C > 0 && g.cpos[C > 0 ? C - 1 : 0] >= 4) ? 1 : 0;
  // a shape the pass tuner picked for this class and operator shape, used
  // while the launch tuning is automatic
  int shape = -1;
  if (tuning().stage < 0 && tuning().sync_waves < 0 && tuning().pipe_waves == 0)
    shape = tuned_shape(sizeof(T) == 8 ? 0 : 1, n, g.m, K, C, FORM, low < 3 ? 1 : 0, far);
  if constexpr (C == 0) {
    const uint64_t tile_bytes = (uint64_t)(2 * sizeof(T)) << (2 * g.m);
    int stage = tuning().stage;
    if (stage < 0) {
      // operators of 1 GiB and more; complex64 too (its lane-patch and pair
      // kernels ran 4.3-5.2 TB/s there, staged 5.0-5.75), except its k = 2
      // transfer form, whose 16 x 16 matrix the staged pass reads far slower
      const bool large = nent * 2 * sizeof(T) >= (1ull << 30);
      stage = large && !(sizeof(T) == 4 && K == 2 && FORM == 1) ? 1 : 0;
    }
    if (shape >= 0) stage = shape_is_stage(shape) ? 1 : 0;
    // The two-qubit transfer form (a 16 x 16 matrix per block) in 64 KiB
    // steps of two 256-thread workgroups per CU, so that one computes while
    // the other loads: measured 12.3 ms per n = 16 c128 pass against
    // 12.9-13.1 for one 512-thread workgroup per CU.
    const bool auto_shape = shape < 0 && tuning().stage < 0;
    const bool two_wg = (shape >= 0 && shape == kShapeStage2) || (auto_shape && K == 2 && FORM == 1);
    const int sth = two_wg ? 256 : shape >= 0 ? shape_stage_threads(shape) : tuning().stage_threads;
    const uint64_t step_bytes = 16ull * kStageVecs * (uint64_t)sth;
    if (stage == 1 && tile_bytes <= step_bytes) {
      const uint64_t steps_total = (nent * 2 * sizeof(T) + step_bytes - 1) / step_bytes;
      uint64_t sw = tuning().stage_grid > 0 ? (uint64_t)tuning().stage_grid
                                            : (uint64_t)num_cu * (uint64_t)tuning().stage_wg_per_cu;
      if (two_wg && auto_shape) sw = 2u * (uint64_t)num_cu;
      if (shape >= 0) sw = shape_grid(shape, num_cu);
      if (sw > steps_total) sw = steps_total;
      const bool pipe = tuning().stage_pipe != 0;
      // Every other 16 KiB granule per step (tiles of at most 16 KiB).
      // Measured at n = 16, c128 on one device: contiguous steps 5.17-5.33
      // TB/s for every intra class (4.4-4.8 at 3/4 and 5/8 of a workgroup
      // per CU), alternate granules 5.9-6.0 (6.12-6.14 at 3/4 for k = 1);
      // contiguous steps reached 6.05 on other devices.
      int sord = tuning().stage_order;
      if (shape >= 0) sord = shape_stage_order(shape);
      if (sord < 0) sord = 1;
      const bool par = sord == 1 && tile_bytes <= 16384;
#define HT_STAGE(TH, P, Q)                                                                                \
  hipLaunchKernelGGL((stage_kernel<T, K, FORM, TH, P, Q>), dim3((unsigned)sw), dim3(TH), 0, s, hp, g, cf, \
                     coef_dev, nent)
      if (par) {
        if (sth == 512) {
          if (pipe) HT_STAGE(512, true, true); else HT_STAGE(512, false, true);
        } else {
          if (pipe) HT_STAGE(256, true, true); else HT_STAGE(256, false, true);
        }
      } else if (sth == 512) {
        if (pipe) HT_STAGE(512, true, false); else HT_STAGE(512, false, false);
      } else {
        if (pipe) HT_STAGE(256, true, false); else HT_STAGE(256, false, false);
      }
#undef HT_STAGE
      return hipGetLastError();
    }
  }
  // memory mode of the step kernels below (as for conj_kernel's automatic one)
  int smode = tuning().mem_mode;
  if (smode < 0) smode = (sizeof(T) == 8 && low >= 3) ? 3 : 0;
  {
    // workgroup steps with the next step prefetched (tuning only)
    const int pw = tuning().pipe_waves;
    if (pw > 0) {
      const uint64_t items = g.ngroups * steps;
      uint64_t wg = (items + pw - 1) / pw;
      const uint64_t wcap = (uint64_t)num_cu * (uint64_t)tuning().sync_wg_per_cu;
      if (wg > wcap) wg = wcap;
#define HT_PIPE(M_, N_, B_) \
  hipLaunchKernelGGL((conj_pipe_kernel<T, K, C, FORM, M_, N_, B_>), dim3((unsigned)wg), dim3(N_), 0, s, hp, g, cf, coef_dev)
      const bool bar = tuning().pipe_barrier != 0;
      if (pw == 8) {
        if (smode == 3) HT_PIPE(3, 512, true); else HT_PIPE(0, 512, true);
      } else if (bar) {
        if (smode == 3) HT_PIPE(3, 256, true); else HT_PIPE(0, 256, true);
      } else {
        if (smode == 3) HT_PIPE(3, 256, false); else HT_PIPE(0, 256, false);
      }
#undef HT_PIPE
      return hipGetLastError();
    }
  }
  {
    // workgroup-wide steps
    int sw = tuning().sync_waves;
    // complex64 of 1 GiB and more: passes with a tile-selecting target and
    // no intra target below bit 3 in the pair layout's steps
    // (pair_sync_kernel; k = 2 direct form only, as the pair layout).
    // Measured at n = 16 against pair_kernel: k = 1 5.0-5.3 -> 5.8-5.9
    // TB/s at tile bits 0-5; k = 2 whole groups 5.09-5.12 -> 5.15-5.35 at
    // low tile bits, equal at the top ones, and the mirrored tiles'
    // half-line excess (+2.7 % traffic) gone; an intra target below bit 3
    // ran 3.2 TB/s in steps and stays on pair_kernel.
    const bool big64 = sizeof(T) == 4 && nent * 2 * sizeof(T) >= (1ull << 30);
    const bool pairs64 = big64 && C > 0 && (K == 1 || FORM == 0) && low >= 3 && g.F >= 4 && tuning().pairs != 0;
    // complex128: every pass with a tile-selecting target and no intra
    // target below bit 3 (k = 2 with one intra target: the quarter order
    // measured 12.3 ms at targets (4, 5) against 13.2-13.6 for the
    // lane-patch kernel, though its 16-wave form spills two registers)
    if (sw < 0) sw = ((big && C > 0 && low >= 3) || pairs64) ? 16 : 0;
    if (shape >= 0) sw = (C > 0 && shape_is_sync(shape)) ? 16 : 0;
    if (sw > 0) {
      // complex64 where the pair layout applies: the pair step kernel
      if constexpr (sizeof(T) == 4 && (K == 1 || FORM == 0)) {
        const bool pl = g.F >= 4 && (KI == 0 || g.ipos[0] != 0) && tuning().pairs != 0;
        if (pl) return launch_pair_sync<K, C, FORM>(hp, g, cf, shape, smode_pair(g, n), num_cu, s);
      }
      ConjGeom<K, C> gs = g;
      // Item order.  Measured at n = 16, c128 (TB/s of algorithmic traffic,
      // whole groups -> quarters -> quarters of every other group): k = 1
      // at tile bit 0 5.46 -> 5.67 -> 5.58, bit 3 5.32 -> 5.45 -> 5.38,
      // bit 5 5.33 -> 5.43 -> 5.65, bit 8 5.28 -> 5.50 -> 5.87, bit 10
      // 5.23 -> 5.20 -> 5.40; two tile-selecting targets at bits (0, 1)
      // 5.30 -> 5.44 (quarters), (4, 5) 5.26 -> 5.20, (9, 10) 5.08 -> 4.90.
      int ord = tuning().sync_order;
      if (shape >= 0) ord = shape_sync_order(shape);
      if (ord < 0) ord = C == 1 ? (far ? 2 : 1) : (K == 2 && C == 2 && !far) ? 1 : 0;
      if (ord > 2) ord = 2;  // a stride of 4 groups is for the pair layout's 8 KiB tiles
      int ilv = tuning().sync_interleave;
      // quarters need the row-run patch order (a step's patches then cover
      // whole rows of the tile)
      if (ilv < 0) ilv = (ord != 0 || C == 2) ? 0 : (use_interleave((int)sizeof(T) * 2) ? 1 : 0);
      gs.ilv = ilv != 0;
      const int sl = 31 - __builtin_clz((uint32_t)steps);
      const int lw = 31 - __builtin_clz((uint32_t)sw);
      const int rmax = sl < lw ? sl : lw;
      // steps that share the patches' row bits: 2^(F - s) patches of 64
      // blocks, conj_unroll of them per step
      constexpr int JU = conj_unroll(K, (int)sizeof(T) * 2);
      int r = g.F - g.s - (JU == 4 ? 2 : JU == 2 ? 1 : 0);
      if (ord == 0 || r > rmax) r = rmax;
      if (r < 0) r = 0;
      const int ps = ord == 2 ? 1 : 0;
      uint64_t wg = sync_units(g.ngroups, sl, (uint32_t)sw, r, ps);
      // grid: the quarter orders at 3/4 of a workgroup per CU (measured
      // 1-4 % faster than one per CU at most tile bits)
      uint64_t wcap = tuning().sync_grid > 0 ? (uint64_t)tuning().sync_grid
                      : ord != 0             ? (uint64_t)num_cu * 3u / 4u
                                             : (uint64_t)num_cu * (uint64_t)tuning().sync_wg_per_cu;
      if (shape >= 0) wcap = shape_grid(shape, num_cu);
      if (wg > wcap) wg = wcap;
      const dim3 grid((unsigned)wg), block((unsigned)(64 * sw));
      switch (smode) {
        case 1: hipLaunchKernelGGL((conj_sync_kernel<T, K, C, FORM, 1>), grid, block, 0, s, hp, gs, cf, coef_dev, r, ps); break;
        case 2: hipLaunchKernelGGL((conj_sync_kernel<T, K, C, FORM, 2>), grid, block, 0, s, hp, gs, cf, coef_dev, r, ps); break;
        case 3: hipLaunchKernelGGL((conj_sync_kernel<T, K, C, FORM, 3>), grid, block, 0, s, hp, gs, cf, coef_dev, r, ps); break;
        default: hipLaunchKernelGGL((conj_sync_kernel<T, K, C, FORM, 0>), grid, block, 0, s, hp, gs, cf, coef_dev, r, ps);
      }
      return hipGetLastError();
    }
  }
  if constexpr (sizeof(T) == 4 && (K == 1 || FORM == 0)) {
    // The pair layout (k = 1, and k = 2 in the direct form) needs a free
    // column bit 0 and F >= 4.  Automatic use (pairs == 1) is limited to
    // where it measured faster: every tile-selecting target set, and an
    // intra target at bit 4 or above (intra targets 1..3 split the 16-byte
    // accesses of a lane row across lines).  The k = 2 transfer form stays
    // in the block layout: at 128 FP64 flops per 16 bytes of complex64
    // traffic it is near the FP64 ridge, and pairs re-read its 16 x 16
    // matrix once per block.
    constexpr int KI = K - C;
    const bool applies = g.F >= 4 && (KI == 0 || g.ipos[0] != 0);
    const bool pays = KI == 0 || g.ipos[0] >= 4;
    if (applies && (tuning().pairs == 2 || (tuning().pairs == 1 && pays))) {
      // 16-byte accesses in stored tiles cover whole lines: nontemporal,
      // except where a quarter or more of the groups hold a mirrored tile
      // (every target tile-selecting, the highest at bit n - 3 or above):
      // a mirrored tile's lines are read in halves by neighbouring jobs,
      // and a nontemporal load lets the line go before its second half
      // (measured: plain 2-12 % faster there, nontemporal 1-3 % faster
      // below and 7-10 % with an intra target)
      int pmode = tuning().mem_mode;
      if (pmode < 0) {
        pmode = 3;
        if constexpr (KI == 0)
          if (g.cpos[C - 1] + g.m >= n - 3) pmode = 0;
      }
      constexpr int JP = K == 1 ? 2 : 1;  // 16 entries per lane and step either way
      const dim3 grid((unsigned)wgs), block(threads);
      if constexpr (K == 2 && KI == 0) {
        // two pairs per step, the second the first's row-bit-3 neighbour,
        // so that both halves of a mirrored tile's lines are read in one
        // step (measured 3-4 % faster at (13, 14), (14, 15), (5, 15); the
        // half-line stores still go out as separate instructions, so the
        // counted write traffic stays about the same)
        if (tuning().pair_jp2 == 1 && pmode == 0) {
          hipLaunchKernelGGL((pair_kernel<K, C, FORM, 0, 2>), grid, block, 0, s, hp, g, cf, order);
          return hipGetLastError();
        }
      }
      switch (pmode) {
        case 1: hipLaunchKernelGGL((pair_kernel<K, C, FORM, 1, JP>), grid, block, 0, s, hp, g, cf, order); break;
        case 2: hipLaunchKernelGGL((pair_kernel<K, C, FORM, 2, JP>), grid, block, 0, s, hp, g, cf, order); break;
        case 3: hipLaunchKernelGGL((pair_kernel<K, C, FORM, 3, JP>), grid, block, 0, s, hp, g, cf, order); break;
        default: hipLaunchKernelGGL((pair_kernel<K, C, FORM, 0, JP>), grid, block, 0, s, hp, g, cf, order);
      }
      return hipGetLastError();
    }
  }
  int mode = tuning().mem_mode;
  if (mode < 0) {
    // Nontemporal hints pay off only when every store instruction writes
    // whole 128-byte lines: 16-byte entries and no intra target below bit 3
    // (a lower column target splits the 8 lanes of a row across two lines).
    constexpr int KI = K - C;
    mode = (sizeof(T) == 8 && (KI == 0 || g.ipos[0] >= 3)) ? 3 : 0;
  }
  switch (mode) {
    case 1:
      hipLaunchKernelGGL((conj_kernel<T, K, C, FORM, 1>), dim3((unsigned)wgs), dim3(threads), 0, s,
                         hp, g, cf, coef_dev, order);
      break;
    case 2:
      hipLaunchKernelGGL((conj_kernel<T, K, C, FORM, 2>), dim3((unsigned)wgs), dim3(threads), 0, s,
                         hp, g, cf, coef_dev, order);
      break;
    case 3:
      hipLaunchKernelGGL((conj_kernel<T, K, C, FORM, 3>), dim3((unsigned)wgs), dim3(threads), 0, s,
                         hp, g, cf, coef_dev, order);
      break;
    default:
      hipLaunchKernelGGL((conj_kernel<T, K, C, FORM, 0>), dim3((unsigned)wgs), dim3(threads), 0, s,
                         hp, g, cf, coef_dev, order);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_dtype(void* buf, int n, int m, const PreparedOp& op,
                                 const double* coef_dev, int num_cu, hipStream_t s) {
  const int k = op.k, c = op.ncross, f = op.form;
#define HT_CASE(K_, C_, F_)                                                   \
  if (k == K_ && c == C_ && f == F_)                                          \
    return launch_t<T, K_, C_, F_>(buf, n, m, op, coef_dev, num_cu, s);
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
  return hipErrorInvalidValue;
}

hipError_t launch_conj(int dtype, void* buf, int n, int m, const PreparedOp& op,
                       const double* coef_dev, int num_cu, hipStream_t s) {
  if (dtype == 0) return dispatch_dtype<double>(buf, n, m, op, coef_dev, num_cu, s);
  if (dtype == 1) return dispatch_dtype<float>(buf, n, m, op, coef_dev, num_cu, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ coefficient upload

struct UploadChunk {
  double v[128];
};

__global__ void upload_kernel(double* __restrict__ dst, UploadChunk c, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = c.v[i];
}

hipError_t launch_upload(double* dst, const double* src, int count, hipStream_t s) {
  for (int off = 0; off < count; off += 128) {
    UploadChunk c;
    const int len = count - off < 128 ? count - off : 128;
    for (int i = 0; i < len; ++i) c.v[i] = src[off + i];
    hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(128), 0, s, dst + off, c, len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ht
