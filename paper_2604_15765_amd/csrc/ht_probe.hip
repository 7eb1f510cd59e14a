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
//   read_stream      read-only; write_stream  write-only; copy_stream  copy;
//   rmw_wg<NS,W,X>   workgroup bursts: W waves each move a 16 KiB chunk per
//                    step, the chunks spread over NS far-apart regions; all
//                    loads of a step complete (barrier) before any store; X:
//                    through LDS (write, update the next wave's chunk, read
//                    back) instead of in registers;
//   xstage<NS>       512 threads move 128 KiB per step through LDS, as NS
//                    runs in NS regions, with the next step's loads issued
//                    before the current step is updated and stored;
//   colour<MODE>     in-place (MODE 0), read-only (1) or write-only (2)
//                    streams of 1 KiB units, where a workgroup step takes
//                    64 units that share a "colour": bits [g, g + cbits) of
//                    the unit index equal bits [sel, sel + cbits) of the
//                    workgroup index (g = 2, cbits = 3: the 4 KiB runs of a
//                    step share address bits 12-14; cbits = 0: contiguous
//                    64 KiB per step).
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

template <int NS, int W, bool X>
__global__ void __launch_bounds__(W * 64) rmw_wg(u4* __restrict__ p, uint64_t n16, unsigned salt) {
  constexpr int WPR = W / NS;  // waves per region
  __shared__ u4 lds[X ? W * 1024 : 1];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t r = w / WPR, sub = w % WPR;
  const uint64_t slen = n16 / NS;
  const uint64_t steps = slen / (1024 * WPR);
  for (uint64_t it = blockIdx.x; it < steps; it += gridDim.x) {
    u4* base = p + r * slen + (it * WPR + sub) * 1024;
    u4 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = __builtin_nontemporal_load(base + i * 64 + lane);
    if constexpr (X) {
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[w * 1024 + i * 64 + lane] = v[i];
      __syncthreads();
      const uint32_t o = ((w + 1) % W) * 1024;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        u4 x = lds[o + i * 64 + lane];
        x.x ^= salt;
        x.w += salt;
        lds[o + i * 64 + lane] = x;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[w * 1024 + i * 64 + lane];
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        v[i].x ^= salt;
        v[i].w += salt;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(v[i], base + i * 64 + lane);
  }
}

template <int NS>
__global__ void __launch_bounds__(512) xstage(u4* __restrict__ p, uint64_t n16, unsigned salt) {
  constexpr int RUN = 8192 / NS;  // 16-byte words per run
  __shared__ u4 lds[8192];
  const uint32_t t = threadIdx.x;
  const uint64_t slen = n16 / NS;
  const uint64_t steps = slen / RUN;
  auto addr = [&](uint64_t st, int j) -> uint64_t {
    const uint32_t i = j * 512 + t;
    return (uint64_t)(i / RUN) * slen + st * RUN + (i % RUN);
  };
  u4 v[16];
  uint64_t st = blockIdx.x;
  if (st < steps)
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = __builtin_nontemporal_load(p + addr(st, j));
  for (; st < steps; st += gridDim.x) {
#pragma unroll
    for (int j = 0; j < 16; ++j) lds[j * 512 + t] = v[j];
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (st + gridDim.x < steps)
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = __builtin_nontemporal_load(p + addr(st + gridDim.x, j));
    const uint32_t o = (t + 256) & 511;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      u4 x = lds[j * 512 + o];
      x.x ^= salt;
      x.w += salt;
      lds[j * 512 + o] = x;
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    u4 q[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) q[j] = lds[j * 512 + t];
#pragma unroll
    for (int j = 0; j < 16; ++j) __builtin_nontemporal_store(q[j], p + addr(st, j));
  }
}

template <int MODE>
__global__ void __launch_bounds__(256) colour(u4* __restrict__ p, uint64_t nunits, int g, int cbits, int sel,
                                              unsigned salt, u4* __restrict__ sink) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t b = blockIdx.x;
  const uint32_t col = (b >> sel) & ((1u << cbits) - 1u);
  // workgroups of one colour, numbered without the colour bits
  const uint64_t lw = ((uint64_t)(b >> (sel + cbits)) << sel) | (b & ((1u << sel) - 1u));
  const uint64_t lg = gridDim.x >> cbits;
  const uint64_t steps = (nunits >> cbits) / 64;
  u4 acc = {0, 0, 0, 0};
  for (uint64_t st = lw; st < steps; st += lg) {
    u4 v[16];
    uint64_t off[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint64_t k = st * 64 + wave * 16 + i;  // unit within the colour
      const uint64_t u = ((k >> g) << (g + cbits)) | ((uint64_t)col << g) | (k & ((1ull << g) - 1));
      off[i] = u * 64 + lane;
    }
    if constexpr (MODE != 2) {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = __builtin_nontemporal_load(p + off[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = u4{salt, (unsigned)i, 0u, salt};
    }
    if constexpr (MODE == 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) acc ^= v[i];
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        v[i].x ^= salt;
        v[i].w += salt;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(v[i], p + off[i]);
    }
  }
  if constexpr (MODE == 1) sink[(uint64_t)blockIdx.x * 256 + threadIdx.x] = acc;
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

// Workgroup bursts: ns regions (1, 4 or 16), waves per workgroup (4, 8, 16;
// ns <= waves), xch: through LDS (4 or 8 waves).
int htp_wg(int ns, int waves, int xch, void* buf, uint64_t n16, int grid, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  u4* p = reinterpret_cast<u4*>(buf);
#define HTP_WG(NS, W, X)                                                                      \
  if (ns == NS && waves == W && (xch != 0) == X) {                                            \
    hipLaunchKernelGGL((rmw_wg<NS, W, X>), dim3(grid), dim3(W * 64), 0, s, p, n16, 7u);       \
    return (int)hipGetLastError();                                                            \
  }
  HTP_WG(1, 4, false)
  HTP_WG(1, 8, false)
  HTP_WG(1, 16, false)
  HTP_WG(1, 4, true)
  HTP_WG(1, 8, true)
  HTP_WG(4, 4, false)
  HTP_WG(4, 16, false)
  HTP_WG(16, 16, false)
#undef HTP_WG
  return (int)hipErrorInvalidValue;
}

// 128 KiB steps through LDS, prefetched: ns regions (1, 2 or 4).
int htp_xstage(int ns, void* buf, uint64_t n16, int grid, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  u4* p = reinterpret_cast<u4*>(buf);
  if (ns == 1)
    hipLaunchKernelGGL(xstage<1>, dim3(grid), dim3(512), 0, s, p, n16, 7u);
  else if (ns == 2)
    hipLaunchKernelGGL(xstage<2>, dim3(grid), dim3(512), 0, s, p, n16, 7u);
  else if (ns == 4)
    hipLaunchKernelGGL(xstage<4>, dim3(grid), dim3(512), 0, s, p, n16, 7u);
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

// buf: nunits 1 KiB units; sink: grid x 256 16-byte words (read-only mode).
// HIP's invalid-value error for shapes the colouring cannot cover exactly.
int htp_colour(int mode, void* buf, uint64_t nunits, int g, int cbits, int sel, int grid, void* sink,
               void* stream) {
  if (mode < 0 || mode > 2 || cbits < 0 || cbits > 6 || g < 0 || g > 20 || sel < 0 || sel + cbits > 12 ||
      grid <= 0 || (grid >> (sel + cbits)) == 0 || grid % (1 << (sel + cbits)) != 0 ||
      nunits % (64ull << (g + cbits)) != 0)
    return (int)hipErrorInvalidValue;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  u4* p = reinterpret_cast<u4*>(buf);
  u4* sk = reinterpret_cast<u4*>(sink);
  if (mode == 0)
    hipLaunchKernelGGL(colour<0>, dim3(grid), dim3(256), 0, s, p, nunits, g, cbits, sel, 7u, sk);
  else if (mode == 1)
    hipLaunchKernelGGL(colour<1>, dim3(grid), dim3(256), 0, s, p, nunits, g, cbits, sel, 7u, sk);
  else
    hipLaunchKernelGGL(colour<2>, dim3(grid), dim3(256), 0, s, p, nunits, g, cbits, sel, 7u, sk);
  return (int)hipGetLastError();
}

}  // extern "C"
