// Batched execution: many independent operators, each with its own sequence
// of k-local operations, in one persistent launch.
//
// Every workgroup takes operators from a queue (a device counter, operators
// ordered largest first on the host) and runs the whole op sequence of one
// operator before taking the next: the passes of one op are spread over the
// workgroup's waves exactly as the grid-wide pass spreads them over all
// waves (same per-lane code, conj_group_lane), and a workgroup barrier
// separates consecutive ops.  An operator whose storage fits the LDS budget
// is copied into LDS once, evolved there through its whole sequence, and
// written back once, so its HBM traffic is 2 x its size per circuit instead
// of per op; larger operators are updated in place and stay warm in the
// XCD's L2 or the Infinity Cache between consecutive ops.
#include "ht_geom.h"
#include "ht_internal.h"
#include "ht_native.h"

namespace ht {

namespace {

template <typename T>
using S2 = typename store2<T>::type;

template <typename T, int K, int C, int FORM>
__device__ void batch_pass(S2<T>* base, int n, int m, const BatchOp& op,
                           const double* __restrict__ coefs, uint32_t wave, uint32_t nwaves,
                           uint32_t lane) {
  const ConjGeom<K, C> g = make_geom<K, C>(n, m, op.sorted);
  Coef<K, FORM> cf;
  if constexpr (K == 2 && FORM == 1) {
    cf.p = coefs + op.coef_off;
  } else {
#pragma unroll
    for (int i = 0; i < 2 * Coef<K, FORM>::NE; ++i) cf.c[i] = coefs[op.coef_off + i];
  }
  // base may point to LDS or to global memory (generic addressing); entries
  // held as FP64 (the kernel's budget at 1024 threads is 128 VGPRs)
  const DirectMem<T, 0, true> mem{base};
  for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves) {
    GroupCtx<C> gc;
    group_ctx<K, C>(grp, g, gc);
    conj_group_lane<conj_unroll(K), K, C, FORM>(mem, g, gc, cf, lane);
  }
}

// Native permutation-and-phase pass of one op over one operator, one block
// per lane at a time (the kernel's budget at 1024 threads is 128 VGPRs).
template <typename T, int K, int C>
__device__ void batch_native(S2<T>* base, int n, int m, const BatchOp& op,
                             const double* __restrict__ coefs, uint32_t wave, uint32_t nwaves,
                             uint32_t lane) {
  const ConjGeom<K, C> g = make_geom<K, C>(n, m, op.sorted);
  NativeOp<K> nop;
#pragma unroll
  for (int u = 0; u < (1 << K); ++u) nop.perm[u] = op.perm[u];
  nop.active = op.active;
  nop.nchunks = 0;  // k <= 2: whole blocks
  nop.c = coefs + op.coef_off;
  const DirectMem<T, 0> mem{base};
  for (uint64_t grp = wave; grp < g.ngroups; grp += nwaves)
    native_group_lane<1, K, C>(mem, g, native_group<C>(grp), nop, lane);
}

template <typename T>
__device__ void batch_dispatch(S2<T>* base, int n, int m, const BatchOp& op,
                               const double* __restrict__ coefs, uint32_t wave, uint32_t nwaves,
                               uint32_t lane) {
  const int k = op.k, c = op.ncross, f = op.form;
  if (f == 2) {
    if (k == 1 && c == 0) return batch_native<T, 1, 0>(base, n, m, op, coefs, wave, nwaves, lane);
    if (k == 1 && c == 1) return batch_native<T, 1, 1>(base, n, m, op, coefs, wave, nwaves, lane);
    if (k == 2 && c == 0) return batch_native<T, 2, 0>(base, n, m, op, coefs, wave, nwaves, lane);
    if (k == 2 && c == 1) return batch_native<T, 2, 1>(base, n, m, op, coefs, wave, nwaves, lane);
    if (k == 2 && c == 2) return batch_native<T, 2, 2>(base, n, m, op, coefs, wave, nwaves, lane);
    return;
  }
#define HT_CASE(K_, C_, F_) \
  if (k == K_ && c == C_ && f == F_) return batch_pass<T, K_, C_, F_>(base, n, m, op, coefs, wave, nwaves, lane);
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
}

__global__ void zero_counter_kernel(unsigned* counter) { *counter = 0u; }

template <typename T>
__global__ void __launch_bounds__(1024)
    batch_kernel(const BatchOperator* __restrict__ opers, unsigned nopers,
                 const BatchOp* __restrict__ ops, const double* __restrict__ coefs,
                 unsigned* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ unsigned s_next;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nwaves = blockDim.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned j = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();
    if (j >= nopers) break;  // the queue is drained: every wave of every workgroup exits here
    const BatchOperator o = opers[j];
    S2<T>* gbuf = reinterpret_cast<S2<T>*>(o.buf);
    S2<T>* base = gbuf;
    if (o.in_lds) {
      uint4* dst = reinterpret_cast<uint4*>(lds);
      const uint4* src = reinterpret_cast<const uint4*>(o.buf);
      for (uint32_t i = threadIdx.x; i < o.bytes / 16; i += blockDim.x) dst[i] = src[i];
      base = reinterpret_cast<S2<T>*>(lds);
      __syncthreads();
    }
    for (uint32_t oi = o.op_begin; oi < o.op_end; ++oi) {
      const BatchOp op = ops[oi];
      batch_dispatch<T>(base, o.n, o.m, op, coefs, wave, nwaves, lane);
      __syncthreads();  // the next op reads what this one wrote
    }
    if (o.in_lds) {
      uint4* dst = reinterpret_cast<uint4*>(o.buf);
      const uint4* src = reinterpret_cast<const uint4*>(lds);
      for (uint32_t i = threadIdx.x; i < o.bytes / 16; i += blockDim.x) dst[i] = src[i];
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_batch(int dtype, const BatchOperator* opers, unsigned nopers, const BatchOp* ops,
                        const double* coefs, unsigned* counter, int threads, int grid,
                        size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == 0)
    hipLaunchKernelGGL(batch_kernel<double>, dim3(grid), dim3(threads), lds_bytes, s, opers, nopers,
                       ops, coefs, counter);
  else
    hipLaunchKernelGGL(batch_kernel<float>, dim3(grid), dim3(threads), lds_bytes, s, opers, nopers,
                       ops, coefs, counter);
  return hipGetLastError();
}

hipError_t set_batch_lds_limit(int dtype, size_t bytes) {
  if (dtype == 0)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(batch_kernel<double>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipFuncSetAttribute(reinterpret_cast<const void*>(batch_kernel<float>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace ht
