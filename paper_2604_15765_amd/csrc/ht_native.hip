// The native pass for permutation-and-phase operations (Section II-B):
// every changing entry is read once from its permuted source and written once
// with its phase; entries the operation fixes are not touched.  k = 1, 2, 3
// with any number of tile-selecting targets.  Per-lane body in ht_native.h;
// this file holds the grid-stride driver and the runtime dispatch.
//
// Like the conjugation pass it is a streaming read-modify-write of (part of)
// the storage, bound by HBM bandwidth.
#include "ht_internal.h"
#include "ht_native.h"

namespace ht {

// ORDER is a template parameter (not a run-time switch as in the
// conjugation pass): with both walks in one body the k = 2 intra-tile kernel
// needs one register more and loses a wave per SIMD.
template <typename T, int K, int C, int MODE, int CH, int ORDER>
__global__ void __launch_bounds__(256)
    native_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, C> g, NativeOp<K> op) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const DirectMem<T, MODE> mem{h};
  constexpr int JU = native_unroll(K);
  if constexpr (ORDER == 0) {
    // one wave walks all patches of a group
    for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves) {
      const NativeGroup ng = native_group<C>(grp);
      if constexpr (K == 3)
        native3_group_lane<C, CH>(mem, g, ng, op, lane);
      else
        native_group_lane<JU, K, C>(mem, g, ng, op, lane);
    }
  } else {
    // (group, step of JU patches) items: neighbouring waves sweep one group
    const uint32_t steps = (g.jobs + JU - 1) / JU;  // a power of two
    const int sl = 31 - __builtin_clz(steps);
    const uint64_t items = g.ngroups << sl;
    for (uint64_t it = wave; it < items; it += nwaves) {
      const NativeGroup ng = native_group<C>(it >> sl);
      const uint32_t j0 = (uint32_t)(it & (steps - 1)) * JU;
      if constexpr (K == 3)
        native3_group_lane<C, CH>(mem, g, ng, op, lane, j0, j0 + JU);
      else
        native_group_lane<JU, K, C>(mem, g, ng, op, lane, j0, j0 + JU);
    }
  }
}

// The native pass in workgroup-wide steps (k <= 2): the 16 waves of a
// workgroup take (group, step) items in the order of sync_item, load every
// changing entry of their blocks, meet at a barrier, then write them, as
// conj_sync_kernel does for the conjugation pass.  Same per-lane body:
// bitwise the same results.
template <typename T, int K, int C, int MODE>
__global__ void __launch_bounds__(1024)
    native_sync_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, C> g, NativeOp<K> op, int r, int ps) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr uint32_t wpb = 16;
  const DirectMem<T, MODE> mem{h};
  constexpr int JU = native_unroll(K);
  const uint32_t steps = (g.jobs + JU - 1) / JU;  // a power of two
  const int sl = 31 - __builtin_clz(steps);
  const uint64_t nu = sync_units(g.ngroups, sl, wpb, r, ps);
  // the loop bound is the same for every wave of the workgroup (barrier)
  for (uint64_t u = blockIdx.x; u < nu; u += gridDim.x) {
    uint64_t grp;
    uint32_t step;
    sync_item(u, wib, wpb, sl, r, ps, grp, step);
    const bool valid = grp < g.ngroups;
    const NativeGroup ng = native_group<C>(valid ? grp : 0);
    NativeStep<JU, K> st;
    const uint32_t j0 = step * JU;
    native_load_step<JU, K, C>(mem, g, ng, op, lane, j0, valid ? j0 + JU : j0, st);
    __syncthreads();
    native_store_step<JU, K, C>(mem, g, ng, op, st);
  }
}

template <typename T, int K, int C>
static hipError_t launch_t(void* buf, int n, int m, const PreparedOp& pop, const double* coef_dev,
                           int num_cu, hipStream_t s) {
  const ConjGeom<K, C> g = make_geom<K, C>(n, m, pop.sorted, use_interleave((int)sizeof(T) * 2));
  NativeOp<K> op;
  for (int u = 0; u < (1 << K); ++u) op.perm[u] = pop.perm[u];
  op.active = pop.active;
  op.nchunks = pop.nchunks;
  op.c = coef_dev;
  const int threads = tuning().block_threads;
  const uint64_t waves_per_wg = (uint64_t)threads / 64;
  // automatic: 8 workgroups per CU (2, as for the conjugation pass in
  // complex128, measured 5-50 % slower here)
  const uint64_t cap = (uint64_t)num_cu * (uint64_t)wg_per_cu_or(8);
  // work order as for the conjugation pass
  int order = tuning().order;
  if (order < 0) order = g.ngroups < cap * waves_per_wg ? 1 : 0;
  constexpr int JU = native_unroll(K);
  const uint64_t steps = (g.jobs + JU - 1) / JU;
  const uint64_t items = order == 0 ? g.ngroups : g.ngroups * steps;
  uint64_t wgs = (items + waves_per_wg - 1) / waves_per_wg;
  if (wgs > cap) wgs = cap;
  if (wgs < 1) wgs = 1;
  auto* hp = reinterpret_cast<typename store2<T>::type*>(buf);
  int mode = tuning().mem_mode;
  if (mode < 0) {
    // as for the conjugation pass: nontemporal only where stores cover
    // whole 128-byte lines
    constexpr int KI = K - C;
    mode = (sizeof(T) == 8 && (KI == 0 || g.ipos[0] >= 3)) ? 3 : 0;
  }
  // Workgroup-wide steps for complex128 operators of 1 GiB and more whose
  // highest tile-selecting target is at tile bit 4 or above and with no
  // intra target below bit 3, in the item order of the conjugation pass
  // (ht_conj.hip): quarters of every other group for one tile-selecting
  // target, whole groups for two.  Measured with CNOT at n = 16: targets
  // (8, 9) .. (14, 15) 11.4 -> 10.6-10.9 ms; nearer the tile bits, (4, 5) ..
  // (7, 8), the grid-stride kernel stayed faster (10.3-11.5 ms against
  // 11.5-12.6).
  if constexpr (K <= 2 && C > 0) {
    constexpr int KI = K - C;
    const int low = KI > 0 ? g.ipos[0] : 99;
    const uint64_t nent = ((1ull << n) * ((1ull << n) + (1ull << g.m))) >> 1;
    const bool big = sizeof(T) == 8 && nent * 2 * sizeof(T) >= (1ull << 30);
    const int far = g.cpos[C - 1] >= 4 ? 1 : 0;
    int sw = tuning().sync_waves;
    if (sw < 0) sw = (big && low >= 3 && far) ? 16 : 0;
    if (sw > 0 && (mode == 0 || mode == 3)) {
      int ord = tuning().sync_order;
      if (ord < 0) ord = C == 1 ? (far ? 2 : 1) : (far ? 0 : 1);
      if (ord > 2) ord = 2;
      ConjGeom<K, C> gs = g;
      int ilv = tuning().sync_interleave;
      if (ilv < 0) ilv = (ord != 0 || C == 2) ? 0 : (use_interleave((int)sizeof(T) * 2) ? 1 : 0);
      gs.ilv = ilv != 0;
      const uint32_t nsteps = (uint32_t)((g.jobs + JU - 1) / JU);
      const int sl = 31 - __builtin_clz(nsteps);
      const int rmax = sl < 4 ? sl : 4;
      int r = g.F - g.s - (JU == 4 ? 2 : JU == 2 ? 1 : 0);
      if (ord == 0 || r > rmax) r = rmax;
      if (r < 0) r = 0;
      const int ps = ord == 2 ? 1 : 0;
      uint64_t wg = sync_units(g.ngroups, sl, 16u, r, ps);
      const uint64_t wcap = tuning().sync_grid > 0 ? (uint64_t)tuning().sync_grid
                            : ord != 0             ? (uint64_t)num_cu * 3u / 4u
                                                   : (uint64_t)num_cu;
      if (wg > wcap) wg = wcap;
      if (mode == 3)
        hipLaunchKernelGGL((native_sync_kernel<T, K, C, 3>), dim3((unsigned)wg), dim3(1024), 0, s, hp, gs, op, r, ps);
      else
        hipLaunchKernelGGL((native_sync_kernel<T, K, C, 0>), dim3((unsigned)wg), dim3(1024), 0, s, hp, gs, op, r, ps);
      return hipGetLastError();
    }
  }
  const dim3 grid((unsigned)wgs), block(threads);
  if constexpr (K == 3) {
    if (pop.chunk == 32) {  // orbits longer than 16 entries (rare permutations)
      if (order == 1)
        hipLaunchKernelGGL((native_kernel<T, K, C, 0, 32, 1>), grid, block, 0, s, hp, g, op);
      else if (mode == 3)
        hipLaunchKernelGGL((native_kernel<T, K, C, 3, 32, 0>), grid, block, 0, s, hp, g, op);
      else
        hipLaunchKernelGGL((native_kernel<T, K, C, 0, 32, 0>), grid, block, 0, s, hp, g, op);
      return hipGetLastError();
    }
  }
  if (order == 1) {
    // few groups: an operator of at most a few hundred MB, plain hints
    hipLaunchKernelGGL((native_kernel<T, K, C, 0, 16, 1>), grid, block, 0, s, hp, g, op);
  } else if (mode == 3) {
    hipLaunchKernelGGL((native_kernel<T, K, C, 3, 16, 0>), grid, block, 0, s, hp, g, op);
  } else if (mode == 1) {
    hipLaunchKernelGGL((native_kernel<T, K, C, 1, 16, 0>), grid, block, 0, s, hp, g, op);
  } else if (mode == 2) {
    hipLaunchKernelGGL((native_kernel<T, K, C, 2, 16, 0>), grid, block, 0, s, hp, g, op);
  } else {
    hipLaunchKernelGGL((native_kernel<T, K, C, 0, 16, 0>), grid, block, 0, s, hp, g, op);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_dtype(void* buf, int n, int m, const PreparedOp& op,
                                 const double* coef_dev, int num_cu, hipStream_t s) {
  const int k = op.k, c = op.ncross;
#define HT_CASE(K_, C_) \
  if (k == K_ && c == C_) return launch_t<T, K_, C_>(buf, n, m, op, coef_dev, num_cu, s);
  HT_CASE(1, 0)
  HT_CASE(1, 1)
  HT_CASE(2, 0)
  HT_CASE(2, 1)
  HT_CASE(2, 2)
  HT_CASE(3, 0)
  HT_CASE(3, 1)
  HT_CASE(3, 2)
  HT_CASE(3, 3)
#undef HT_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_native(int dtype, void* buf, int n, int m, const PreparedOp& op,
                         const double* coef_dev, int num_cu, hipStream_t s) {
  if (op.form != 2) return hipErrorInvalidValue;
  if (dtype == 0) return dispatch_dtype<double>(buf, n, m, op, coef_dev, num_cu, s);
  if (dtype == 1) return dispatch_dtype<float>(buf, n, m, op, coef_dev, num_cu, s);
  return hipErrorInvalidValue;
}

}  // namespace ht
