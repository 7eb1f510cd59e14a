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
