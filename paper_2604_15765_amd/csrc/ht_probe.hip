// Streaming-bandwidth probe (measurement tool, not part of the library).
//
// Kernels that move a buffer the size of an operator with the access shapes
// the conjugation pass has, minus its arithmetic, to measure what HBM
// delivers for each shape on this device:
//   rmw_streams<NS>  in-place read-modify-write of NS far-apart regions
//                    advanced in lockstep (NS = 1: one contiguous stream; a
//                    cross-tile pass touches 4 or more tiles per group that
//                    lie in different parts of the buffer), 16 loads of 16 B
//                    in flight per lane, all loads of a step before its stores;
//   tile_rmw<PAT>    in-place read-modify-write of 16 KiB tiles (32 x 32
//                    16-byte entries), one tile per wave and step, 16 loads
//                    per lane: PAT 0 contiguous 1 KiB per instruction, PAT 1
//                    the conjugation pass's 8 x 8 lane patch (8 rows of
//                    128 B at a 512-byte stride per instruction);
//   read_stream      read-only; write_stream  write-only; copy_stream  copy.
// Every kernel is a grid-stride loop over whole work items that lie inside
// the buffer (items that would cross its end are not formed).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ inline u4 ld(const u4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT>
__device__ inline void st(u4* p, u4 v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <int NS, bool NT>
__global__ void __launch_bounds__(256) rmw_streams(u4* __restrict__ p, uint64_t n16, unsigned salt) {
  constexpr int PER = 16 / NS;  // 1-KiB wave instructions per stream and step
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t slen = n16 / NS;
  const uint64_t items = slen / (PER * 64);
  for (uint64_t it = wave; it < items; it += nwaves) {
    u4 v[16];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int i = 0; i < PER; ++i) v[s * PER + i] = ld<NT>(p + s * slen + (it * PER + i) * 64 + lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      v[i].x ^= salt;
      v[i].w += salt;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int i = 0; i < PER; ++i) st<NT>(p + s * slen + (it * PER + i) * 64 + lane, v[s * PER + i]);
  }
}

template <int PAT>
__global__ void __launch_bounds__(256) tile_rmw(u4* __restrict__ p, uint64_t ntiles, unsigned salt) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t t = wave; t < ntiles; t += nwaves) {
    u4* tile = p + t * 1024;
    uint32_t off[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if constexpr (PAT == 0)
        off[i] = i * 64 + lane;
      else
        off[i] = ((i >> 2) * 8 + (lane >> 3)) * 32 + (i & 3) * 8 + (lane & 7);
    }
    u4 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = __builtin_nontemporal_load(tile + off[i]);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      v[i].x ^= salt;
      v[i].w += salt;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(v[i], tile + off[i]);
  }
}

__global__ void __launch_bounds__(256) read_stream(const u4* __restrict__ p, uint64_t n16,
                                                   unsigned* __restrict__ out) {
  unsigned acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    const u4 v = __builtin_nontemporal_load(p + i);
    acc ^= v.x ^ v.w;
  }
  out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(256) write_stream(u4* __restrict__ p, uint64_t n16, unsigned salt) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    const u4 v = {salt, 0u, 0u, (unsigned)i};
    p[i] = v;
  }
}

__global__ void __launch_bounds__(256) copy_stream(u4* __restrict__ d, const u4* __restrict__ s,
                                                   uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) d[i] = s[i];
}

}  // namespace

extern "C" {

// Each returns the HIP error of the launch.  buf: n16 16-byte words.
int htp_rmw(int nstreams, int nontemporal, void* buf, uint64_t n16, int grid, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  u4* p = reinterpret_cast<u4*>(buf);
#define HTP_CASE(NS)                                                                           \
  if (nstreams == NS) {                                                                        \
    if (nontemporal)                                                                           \
      hipLaunchKernelGGL((rmw_streams<NS, true>), dim3(grid), dim3(256), 0, s, p, n16, 7u);    \
    else                                                                                       \
      hipLaunchKernelGGL((rmw_streams<NS, false>), dim3(grid), dim3(256), 0, s, p, n16, 7u);   \
    return (int)hipGetLastError();                                                             \
  }
  HTP_CASE(1)
  HTP_CASE(2)
  HTP_CASE(4)
  HTP_CASE(16)
#undef HTP_CASE
  return (int)hipErrorInvalidValue;
}

// buf: ntiles tiles of 16 KiB.
int htp_tile(int pattern, void* buf, uint64_t ntiles, int grid, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  u4* p = reinterpret_cast<u4*>(buf);
  if (pattern == 0)
    hipLaunchKernelGGL(tile_rmw<0>, dim3(grid), dim3(256), 0, s, p, ntiles, 7u);
  else if (pattern == 1)
    hipLaunchKernelGGL(tile_rmw<1>, dim3(grid), dim3(256), 0, s, p, ntiles, 7u);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

// out: grid * 256 unsigned
int htp_read(void* buf, uint64_t n16, int grid, void* out, void* stream) {
  hipLaunchKernelGGL(read_stream, dim3(grid), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const u4*>(buf), n16, reinterpret_cast<unsigned*>(out));
  return (int)hipGetLastError();
}

int htp_write(void* buf, uint64_t n16, int grid, void* stream) {
  hipLaunchKernelGGL(write_stream, dim3(grid), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<u4*>(buf), n16, 3u);
  return (int)hipGetLastError();
}

int htp_copy(void* dst, const void* src, uint64_t n16, int grid, void* stream) {
  hipLaunchKernelGGL(copy_stream, dim3(grid), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<u4*>(dst), reinterpret_cast<const u4*>(src), n16);
  return (int)hipGetLastError();
}

}  // extern "C"
