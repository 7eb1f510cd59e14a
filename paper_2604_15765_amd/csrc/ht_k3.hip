// The k = 3 Kraus-form pass (ht_k3.h): 8 lanes per block, left products by
// columns, an LDS transpose inside the wave, right products by rows.
//
// Bytes: every stored entry is read and written once, as in the conjugation
// pass.  Flops: 2 x 64 complex multiply-adds per entry and operator (128 FP64
// flops per entry per Kraus operator), so one operator stays below the FP64
// ridge (32 bytes per entry of traffic) and a channel with more than about
// four Kraus operators becomes bound by FP64 arithmetic instead of HBM.
#include "ht_internal.h"
#include "ht_k3.h"

namespace ht {

// Order the LDS writes and reads of the lanes of one wave (a wave's LDS
// operations execute in order; the fences keep the compiler from moving
// them across).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kK3Threads = 256;  // 4 waves; the LDS array below has one region per wave

template <typename T, int C, int MODE>
__global__ void __launch_bounds__(kK3Threads)
    k3_kernel(typename store2<T>::type* __restrict__ h, ConjGeom<3, C> g,
              const double* __restrict__ A, int nkraus) {
  __shared__ double2 lds[kK3Threads / 64][8][8 * kK3Pad];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const DirectMem<T, MODE, true> mem{h};
  const int j = (int)(lane & 7u);
  double2* slot = lds[wib][lane >> 3];
  const uint32_t nblk = 1u << (2 * g.F);
  for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves) {
    const K3Group gr = k3_group<C>(grp);
    K3Tiles<C> tiles;
    k3_tiles<C>(g, gr, j, tiles);
    for (uint32_t b0 = 0; b0 < nblk; b0 += 8) {
      const K3Block bk = k3_block<C>(g, gr, b0 + (lane >> 3));
      cd x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = cd{0.0, 0.0};
      if (bk.active) k3_load_col<C>(mem, g, tiles, bk, j, x);
      cd w[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) w[v] = cd{0.0, 0.0};
      for (int a = 0; a < nkraus; ++a) {
        const double* Aa = A + 128 * a;
        wave_lds_sync();  // the previous operator's reads of this slot are done
        k3_left(Aa, x, [&](int u, cd t) { slot[u * kK3Pad + j] = make_double2(t.re, t.im); });
        wave_lds_sync();
        k3_right_acc(Aa, [&](int l) {
          const double2 v = slot[j * kK3Pad + l];
          return cd{v.x, v.y};
        }, w);
      }
      if (bk.active) k3_store_row<C>(mem, g, gr, tiles, bk, j, w);
      wave_lds_sync();
    }
  }
}

template <typename T, int C>
static hipError_t launch_t(void* buf, int n, int m, const PreparedOp& op, const double* coef_dev,
                           int num_cu, hipStream_t s) {
  const ConjGeom<3, C> g = make_geom<3, C>(n, m, op.sorted, false);
  const uint64_t waves_per_wg = kK3Threads / 64;
  // Workgroups per compute unit: for a single complex128 operator (memory
  // bound) fewer than the conjugation pass uses, as measured at n = 16: 1
  // when a group is one tile split into two steps (F <= 2), else 2.  Fewer
  // waves in flight leave more L2 per wave for the partial lines this pass
  // reads and writes (targets [0, 1, 2]: 21.0 -> 16.0 ms).  Channels (FP64
  // bound) and complex64 keep the tuning value: there fewer waves measured
  // slower.
  uint64_t per_cu = (uint64_t)wg_per_cu_or(8);
  if (sizeof(T) == 8 && op.nkraus == 1) {
    const uint64_t k3_cap = g.F <= 2 ? 1 : 2;
    if (per_cu > k3_cap) per_cu = k3_cap;
  }
  const uint64_t cap = (uint64_t)num_cu * per_cu;
  uint64_t wgs = (g.ngroups + waves_per_wg - 1) / waves_per_wg;
  if (wgs > cap) wgs = cap;
  if (wgs < 1) wgs = 1;
  // Automatic mode: plain loads and stores.  The 8 lanes of a block run down
  // the columns of a mirrored tile, so its lines are read in 16-byte pieces
  // by different steps; a nontemporal load lets a line go after its first
  // piece and the rest are fetched again (measured at n = 16, complex128:
  // 2.8x the algorithmic read bytes with all three targets tile-selecting,
  // +20 % with one or two).  With no mirrored tile the hint measured no
  // better either.
  int mode = tuning().mem_mode;
  if (mode < 0) mode = 0;
  auto* hp = reinterpret_cast<typename store2<T>::type*>(buf);
  const dim3 grid((unsigned)wgs), block(kK3Threads);
  if (mode == 3)
    hipLaunchKernelGGL((k3_kernel<T, C, 3>), grid, block, 0, s, hp, g, coef_dev, op.nkraus);
  else if (mode == 1)
    hipLaunchKernelGGL((k3_kernel<T, C, 1>), grid, block, 0, s, hp, g, coef_dev, op.nkraus);
  else if (mode == 2)
    hipLaunchKernelGGL((k3_kernel<T, C, 2>), grid, block, 0, s, hp, g, coef_dev, op.nkraus);
  else
    hipLaunchKernelGGL((k3_kernel<T, C, 0>), grid, block, 0, s, hp, g, coef_dev, op.nkraus);
  return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_dtype(void* buf, int n, int m, const PreparedOp& op,
                                 const double* coef_dev, int num_cu, hipStream_t s) {
  switch (op.ncross) {
    case 0: return launch_t<T, 0>(buf, n, m, op, coef_dev, num_cu, s);
    case 1: return launch_t<T, 1>(buf, n, m, op, coef_dev, num_cu, s);
    case 2: return launch_t<T, 2>(buf, n, m, op, coef_dev, num_cu, s);
    case 3: return launch_t<T, 3>(buf, n, m, op, coef_dev, num_cu, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_k3(int dtype, void* buf, int n, int m, const PreparedOp& op,
                     const double* coef_dev, int num_cu, hipStream_t s) {
  if (op.k != 3 || op.form != kFormKraus3 || op.nkraus < 1 || op.nkraus > 64)
    return hipErrorInvalidValue;
  if (dtype == 0) return dispatch_dtype<double>(buf, n, m, op, coef_dev, num_cu, s);
  if (dtype == 1) return dispatch_dtype<float>(buf, n, m, op, coef_dev, num_cu, s);
  return hipErrorInvalidValue;
}

}  // namespace ht
