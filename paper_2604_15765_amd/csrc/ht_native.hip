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

template <typename T, int K, int C, int MODE, int CH>
__global__ void __launch_bounds__(256)
    native_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<K, C> g, NativeOp<K> op) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const DirectMem<T, MODE> mem{h};
  for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves) {
    const NativeGroup ng = native_group<C>(grp);
    if constexpr (K == 3)
      native3_group_lane<C, CH>(mem, g, ng, op, lane);
    else
      native_group_lane<native_unroll(K), K, C>(mem, g, ng, op, lane);
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
  uint64_t wgs = (g.ngroups + waves_per_wg - 1) / waves_per_wg;
  const uint64_t cap = (uint64_t)num_cu * (uint64_t)tuning().wg_per_cu;
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
  if (K == 3 && pop.chunk == 32) {  // orbits longer than 16 entries (rare permutations)
    if (mode == 3)
      hipLaunchKernelGGL((native_kernel<T, K, C, 3, 32>), dim3((unsigned)wgs), dim3(threads), 0, s, hp, g, op);
    else
      hipLaunchKernelGGL((native_kernel<T, K, C, 0, 32>), dim3((unsigned)wgs), dim3(threads), 0, s, hp, g, op);
  } else if (mode == 3) {
    hipLaunchKernelGGL((native_kernel<T, K, C, 3, 16>), dim3((unsigned)wgs), dim3(threads), 0, s, hp, g, op);
  } else if (mode == 1) {
    hipLaunchKernelGGL((native_kernel<T, K, C, 1, 16>), dim3((unsigned)wgs), dim3(threads), 0, s, hp, g, op);
  } else if (mode == 2) {
    hipLaunchKernelGGL((native_kernel<T, K, C, 2, 16>), dim3((unsigned)wgs), dim3(threads), 0, s, hp, g, op);
  } else {
    hipLaunchKernelGGL((native_kernel<T, K, C, 0, 16>), dim3((unsigned)wgs), dim3(threads), 0, s, hp, g, op);
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
