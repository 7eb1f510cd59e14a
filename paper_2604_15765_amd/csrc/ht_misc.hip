// Initialisation, IO and reductions over the tiled storage.
//
// Reductions (trace, tr(A B), Pauli sums) accumulate in FP64 for both storage
// types and are deterministic: every workgroup owns a fixed set of tiles or
// rows (fixed grid, grid-stride order), reduces in a fixed tree, and a single
// workgroup adds the partial sums in a fixed order.
#include "ht_geom.h"
#include "ht_internal.h"

namespace ht {

namespace {

constexpr int kThreads = 256;
constexpr int kReduceBlocks = 1024;  // fixed partial-sum count of the tile reductions
constexpr int kPauliBlocks = 64;     // partial sums per Pauli term

template <typename T>
using S2 = typename store2<T>::type;

__device__ inline uint64_t stored_off(uint64_t i, uint64_t j, int m) {
  // entry (i, j) with (i >> m) >= (j >> m): its element offset
  const uint64_t ti = i >> m, tj = j >> m, mask = (1ull << m) - 1ull;
  return ((tri64(ti) + tj) << (2 * m)) + ((i & mask) << m) + (j & mask);
}

__device__ inline double block_sum(double v, double* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) lds[t] += lds[t + w];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- elementwise

__global__ void fill_zero_kernel(uint4* __restrict__ p, uint64_t n16, uint8_t* __restrict__ tail,
                                 uint32_t ntail) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void copy_kernel(uint4* __restrict__ d, const uint4* __restrict__ s, uint64_t n16,
                            uint8_t* __restrict__ dt, const uint8_t* __restrict__ st,
                            uint32_t ntail) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    d[i] = s[i];
  if (blockIdx.x == 0 && threadIdx.x < ntail) dt[threadIdx.x] = st[threadIdx.x];
}

template <typename T>
__global__ void scale_kernel(S2<T>* __restrict__ h, uint64_t nelems, double alpha) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nelems; i += stride) {
    S2<T> v = h[i];
    v.x = (T)((double)v.x * alpha);
    v.y = (T)((double)v.y * alpha);
    h[i] = v;
  }
}

// h /= *denom (denom read from device memory, e.g. a trace just computed)
template <typename T>
__global__ void scale_inv_kernel(S2<T>* __restrict__ h, uint64_t nelems,
                                 const double* __restrict__ denom) {
  const double alpha = 1.0 / *denom;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nelems; i += stride) {
    S2<T> v = h[i];
    v.x = (T)((double)v.x * alpha);
    v.y = (T)((double)v.y * alpha);
    h[i] = v;
  }
}

template <typename T>
__global__ void set_diag_kernel(S2<T>* __restrict__ h, uint64_t N, int m, double value) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    store_c<T>(h + stored_off(i, i, m), 0u, cd{value, 0.0});
}

// One wave per tile (grid-stride over tiles); lanes walk the M^2 entries.
#define HT_TILE_LOOP(ntiles)                                                                   \
  const uint32_t lane = threadIdx.x & 63u;                                                     \
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) +                             \
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);                      \
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);                             \
  const uint32_t MM = 1u << (2 * m);                                                           \
  for (uint64_t t = wave; t < (ntiles); t += nwaves)

template <typename T>
__global__ void pack_dense_kernel(S2<T>* __restrict__ h, uint64_t ntiles, int m,
                                  const double* __restrict__ A, int64_t ld) {
  HT_TILE_LOOP(ntiles) {
    uint32_t ti, tj;
    tri_decode(t, ti, tj);
    S2<T>* tile = h + (t << (2 * m));
    for (uint32_t e = lane; e < MM; e += 64u) {
      const uint64_t i = ((uint64_t)ti << m) + (e >> m);
      const uint64_t j = ((uint64_t)tj << m) + (e & ((1u << m) - 1u));
      cd v;
      if (i >= j) {
        v = {A[2 * (i * ld + j)], A[2 * (i * ld + j) + 1]};
      } else {
        v = {A[2 * (j * ld + i)], -A[2 * (j * ld + i) + 1]};
      }
      store_c<T>(tile, e, v);
    }
  }
}

template <typename T>
__global__ void unpack_dense_kernel(const S2<T>* __restrict__ h, uint64_t N, int m,
                                    double* __restrict__ out, int64_t ld) {
  const uint64_t total = N * N;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const uint64_t i = e / N, j = e % N;
    const cd v = i >= j ? load_c<T>(h + stored_off(i, j, m), 0u)
                        : conjg(load_c<T>(h + stored_off(j, i, m), 0u));
    out[2 * (i * ld + j)] = v.re;
    out[2 * (i * ld + j) + 1] = v.im;
  }
}

// H = G G^dagger, one workgroup per tile (grid-stride).  The M rows of G
// that the tile's rows and columns need are staged in LDS transposed
// ([r][row]), so the lanes of a wave (consecutive columns) read consecutive
// LDS words.  Used when 2 M rank complex values fit the LDS budget.
template <typename T>
__global__ void __launch_bounds__(256) lowrank_lds_kernel(S2<T>* __restrict__ h, uint64_t ntiles,
                                                          int m, const double* __restrict__ G,
                                                          int rank) {
  extern __shared__ __align__(16) double lds[];
  const uint32_t M = 1u << m;
  double2* gi = reinterpret_cast<double2*>(lds);  // [rank][M]
  double2* gj = gi + (size_t)rank * M;            // [rank][M]
  const uint32_t MM = M * M;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t ti, tj;
    tri_decode(t, ti, tj);
    ti = wave_uniform(ti);
    tj = wave_uniform(tj);
    __syncthreads();  // the previous tile's reads are done
    for (uint32_t e = threadIdx.x; e < M * (uint32_t)rank; e += blockDim.x) {
      const uint32_t row = e / rank, r = e % rank;
      const uint64_t gr = ((uint64_t)ti << m) + row, gc = ((uint64_t)tj << m) + row;
      gi[(size_t)r * M + row] = make_double2(G[2 * (gr * rank + r)], G[2 * (gr * rank + r) + 1]);
      gj[(size_t)r * M + row] = make_double2(G[2 * (gc * rank + r)], G[2 * (gc * rank + r) + 1]);
    }
    __syncthreads();
    S2<T>* tile = h + (t << (2 * m));
    for (uint32_t e = threadIdx.x; e < MM; e += blockDim.x) {
      const uint32_t i = e >> m, j = e & (M - 1);
      cd acc = {0.0, 0.0};
      for (int r = 0; r < rank; ++r) {
        const double2 a = gi[(size_t)r * M + i], b = gj[(size_t)r * M + j];
        acc = cfma_cj(acc, cd{a.x, a.y}, cd{b.x, b.y});
      }
      store_c<T>(tile, e, acc);
    }
  }
}

template <typename T>
__global__ void lowrank_kernel(S2<T>* __restrict__ h, uint64_t ntiles, int m,
                               const double* __restrict__ G, int rank) {
  HT_TILE_LOOP(ntiles) {
    uint32_t ti, tj;
    tri_decode(t, ti, tj);
    S2<T>* tile = h + (t << (2 * m));
    for (uint32_t e = lane; e < MM; e += 64u) {
      const uint64_t i = ((uint64_t)ti << m) + (e >> m);
      const uint64_t j = ((uint64_t)tj << m) + (e & ((1u << m) - 1u));
      const double* gi = G + 2 * i * (uint64_t)rank;
      const double* gj = G + 2 * j * (uint64_t)rank;
      cd acc = {0.0, 0.0};
      for (int r = 0; r < rank; ++r)
        acc = cfma_cj(acc, cd{gi[2 * r], gi[2 * r + 1]}, cd{gj[2 * r], gj[2 * r + 1]});
      store_c<T>(tile, e, acc);
    }
  }
}

template <typename T>
__global__ void get_entries_kernel(const S2<T>* __restrict__ h, int m, uint64_t count,
                                   const int64_t* __restrict__ rows,
                                   const int64_t* __restrict__ cols, double* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
    const uint64_t i = (uint64_t)rows[e], j = (uint64_t)cols[e];
    const cd v = i >= j ? load_c<T>(h + stored_off(i, j, m), 0u)
                        : conjg(load_c<T>(h + stored_off(j, i, m), 0u));
    out[2 * e] = v.re;
    out[2 * e + 1] = v.im;
  }
}

// O[i, i^x] = sum over the strings with flip mask x of c (-i)^ny (-1)^popc(i & z).
// One thread per row i writes the entries of its row that are stored.
__device__ inline cd pauli_phase(int ny, uint32_t z, uint64_t i) {
  const double sgn = (__popcll(i & (uint64_t)z) & 1) ? -1.0 : 1.0;
  switch (ny & 3) {
    case 0: return {sgn, 0.0};
    case 1: return {0.0, -sgn};
    case 2: return {-sgn, 0.0};
    default: return {0.0, sgn};
  }
}

template <typename T>
__global__ void pauli_init_kernel(S2<T>* __restrict__ h, uint64_t N, int m,
                                  const PauliGroup* __restrict__ groups, int ngroups,
                                  const PauliTerm* __restrict__ terms) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    for (int gi = 0; gi < ngroups; ++gi) {
      const PauliGroup gr = groups[gi];
      const uint64_t j = i ^ (uint64_t)gr.x;
      if ((i >> m) < (j >> m)) continue;  // entry lives in the mirror tile
      cd acc = {0.0, 0.0};
      for (uint32_t t = gr.first; t < gr.first + gr.count; ++t) {
        const PauliTerm pt = terms[t];
        const cd ph = pauli_phase(pt.ny, pt.z, i);
        acc.re += pt.c * ph.re;
        acc.im += pt.c * ph.im;
      }
      store_c<T>(h + stored_off(i, j, m), 0u, acc);
    }
  }
}

// --------------------------------------------------------------- reductions

template <typename T>
__global__ void trace_partial_kernel(const S2<T>* __restrict__ h, uint64_t N, int m,
                                     double* __restrict__ partial) {
  __shared__ double lds[kThreads];
  double acc = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    acc += load_c<T>(h + stored_off(i, i, m), 0u).re;
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void expect_partial_kernel(const S2<T>* __restrict__ a, const S2<T>* __restrict__ b,
                                      uint64_t ntiles, int m, double* __restrict__ partial) {
  __shared__ double lds[kThreads];
  double acc = 0.0;
  HT_TILE_LOOP(ntiles) {
    uint32_t ti, tj;
    tri_decode(t, ti, tj);
    const double w = ti == tj ? 1.0 : 2.0;
    const S2<T>* ta = a + (t << (2 * m));
    const S2<T>* tb = b + (t << (2 * m));
    double s = 0.0;
    for (uint32_t e = lane; e < MM; e += 64u) {
      const cd x = load_c<T>(ta, e), y = load_c<T>(tb, e);
      s = fma(x.re, y.re, s);
      s = fma(x.im, y.im, s);
    }
    acc = fma(w, s, acc);
  }
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sum of `count` partials in a fixed order by one workgroup.
__global__ void finish_sum_kernel(const double* __restrict__ partial, int count,
                                  double* __restrict__ out) {
  __shared__ double lds[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) *out = s;
}

// Pauli expectation: S_t = sum_j (-1)^popc(j & z_t) H[j ^ x_t, j]; the
// result is sum_t c_t Re((-i)^ny_t S_t).  blockIdx.y = term.
template <typename T>
__global__ void pauli_partial_kernel(const S2<T>* __restrict__ h, uint64_t N, int m,
                                     const PauliTerm* __restrict__ terms,
                                     double* __restrict__ partial) {
  __shared__ double lds[kThreads];
  const PauliTerm pt = terms[blockIdx.y];
  double re = 0.0, im = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += stride) {
    const uint64_t i = j ^ (uint64_t)pt.x;
    const cd v = i >= j ? load_c<T>(h + stored_off(i, j, m), 0u)
                        : conjg(load_c<T>(h + stored_off(j, i, m), 0u));
    const double sgn = (__popcll(j & (uint64_t)pt.z) & 1) ? -1.0 : 1.0;
    re += sgn * v.re;
    im += sgn * v.im;
  }
  const double sr = block_sum(re, lds);
  const double si = block_sum(im, lds);
  if (threadIdx.x == 0) {
    double* p = partial + 2 * ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x);
    p[0] = sr;
    p[1] = si;
  }
}

__global__ void pauli_finish_kernel(const double* __restrict__ partial, int nblocks,
                                    const PauliTerm* __restrict__ terms, int nterms,
                                    double* __restrict__ out) {
  __shared__ double lds[kThreads];
  double acc = 0.0;
  for (int t = threadIdx.x; t < nterms; t += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      re += partial[2 * ((uint64_t)t * nblocks + b)];
      im += partial[2 * ((uint64_t)t * nblocks + b) + 1];
    }
    // Re((-i)^ny (re + i im))
    double v;
    switch (terms[t].ny & 3) {
      case 0: v = re; break;
      case 1: v = im; break;
      case 2: v = -re; break;
      default: v = -im; break;
    }
    acc = fma(terms[t].c, v, acc);
  }
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) *out = s;
}

inline unsigned grid_for(uint64_t work, uint64_t per_block, uint64_t cap) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

inline uint64_t ntiles_of(int n, int m) {
  const uint64_t nt = (uint64_t)1 << (n - m);
  return nt * (nt + 1) / 2;
}

}  // namespace

// ----------------------------------------------------------------- launchers

#define HT_DT_DISPATCH(dtype, call_double, call_float) \
  do {                                                 \
    if ((dtype) == 0) {                                \
      call_double;                                     \
    } else if ((dtype) == 1) {                         \
      call_float;                                      \
    } else {                                           \
      return hipErrorInvalidValue;                     \
    }                                                  \
  } while (0)

hipError_t launch_fill_zero(void* buf, size_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  const uint32_t tail = (uint32_t)(bytes % 16);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n16, kThreads, 8192)), dim3(kThreads), 0, s,
                     reinterpret_cast<uint4*>(buf), n16,
                     reinterpret_cast<uint8_t*>(buf) + n16 * 16, tail);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  const uint32_t tail = (uint32_t)(bytes % 16);
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n16, kThreads, 8192)), dim3(kThreads), 0, s,
                     reinterpret_cast<uint4*>(dst), reinterpret_cast<const uint4*>(src), n16,
                     reinterpret_cast<uint8_t*>(dst) + n16 * 16,
                     reinterpret_cast<const uint8_t*>(src) + n16 * 16, tail);
  return hipGetLastError();
}

hipError_t launch_scale(int dtype, void* buf, uint64_t nelems, double alpha, hipStream_t s) {
  const unsigned g = grid_for(nelems, kThreads, 8192);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(scale_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<double>*>(buf), nelems, alpha),
                 hipLaunchKernelGGL(scale_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<float>*>(buf), nelems, alpha));
  return hipGetLastError();
}

hipError_t launch_scale_inv(int dtype, void* buf, uint64_t nelems, const double* denom,
                            hipStream_t s) {
  const unsigned g = grid_for(nelems, kThreads, 8192);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(scale_inv_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<double>*>(buf), nelems, denom),
                 hipLaunchKernelGGL(scale_inv_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<float>*>(buf), nelems, denom));
  return hipGetLastError();
}

hipError_t launch_set_diag(int dtype, void* buf, int n, int m, double value, hipStream_t s) {
  const uint64_t N = (uint64_t)1 << n;
  const unsigned g = grid_for(N, kThreads, 4096);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(set_diag_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<double>*>(buf), N, m, value),
                 hipLaunchKernelGGL(set_diag_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<float>*>(buf), N, m, value));
  return hipGetLastError();
}

hipError_t launch_pack_dense(int dtype, void* buf, int n, int m, const double* A, int64_t ld,
                             hipStream_t s) {
  const uint64_t nt = ntiles_of(n, m);
  const unsigned g = grid_for(nt, kThreads / 64, 8192);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(pack_dense_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<double>*>(buf), nt, m, A, ld),
                 hipLaunchKernelGGL(pack_dense_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<float>*>(buf), nt, m, A, ld));
  return hipGetLastError();
}

hipError_t launch_unpack_dense(int dtype, const void* buf, int n, int m, double* out, int64_t ld,
                               hipStream_t s) {
  const uint64_t N = (uint64_t)1 << n;
  const unsigned g = grid_for(N * N, kThreads, 8192);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(unpack_dense_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<double>*>(buf), N, m, out, ld),
                 hipLaunchKernelGGL(unpack_dense_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<float>*>(buf), N, m, out, ld));
  return hipGetLastError();
}

hipError_t launch_lowrank(int dtype, void* buf, int n, int m, const double* G, int rank,
                          hipStream_t s) {
  const uint64_t nt = ntiles_of(n, m);
  const size_t lds = (size_t)2 * ((size_t)1 << m) * (size_t)rank * sizeof(double2);
  if (lds <= 64 * 1024) {
    const unsigned g = grid_for(nt, 1, 8192);
    HT_DT_DISPATCH(dtype,
                   hipLaunchKernelGGL(lowrank_lds_kernel<double>, dim3(g), dim3(kThreads), lds, s,
                                      reinterpret_cast<S2<double>*>(buf), nt, m, G, rank),
                   hipLaunchKernelGGL(lowrank_lds_kernel<float>, dim3(g), dim3(kThreads), lds, s,
                                      reinterpret_cast<S2<float>*>(buf), nt, m, G, rank));
    return hipGetLastError();
  }
  const unsigned g = grid_for(nt, kThreads / 64, 8192);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(lowrank_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<double>*>(buf), nt, m, G, rank),
                 hipLaunchKernelGGL(lowrank_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<float>*>(buf), nt, m, G, rank));
  return hipGetLastError();
}

hipError_t launch_get_entries(int dtype, const void* buf, int n, int m, int64_t count,
                              const int64_t* rows, const int64_t* cols, double* out,
                              hipStream_t s) {
  (void)n;
  const unsigned g = grid_for((uint64_t)count, kThreads, 4096);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(get_entries_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<double>*>(buf), m,
                                    (uint64_t)count, rows, cols, out),
                 hipLaunchKernelGGL(get_entries_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<float>*>(buf), m,
                                    (uint64_t)count, rows, cols, out));
  return hipGetLastError();
}

hipError_t launch_pauli_init(int dtype, void* buf, int n, int m, const PauliGroup* groups,
                             int ngroups, const PauliTerm* terms, hipStream_t s) {
  const uint64_t N = (uint64_t)1 << n;
  const unsigned g = grid_for(N, kThreads, 4096);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(pauli_init_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<double>*>(buf), N, m, groups, ngroups,
                                    terms),
                 hipLaunchKernelGGL(pauli_init_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<S2<float>*>(buf), N, m, groups, ngroups,
                                    terms));
  return hipGetLastError();
}

size_t reduce_scratch_doubles(int n, int m, int nterms) {
  (void)n;
  (void)m;
  const size_t a = kReduceBlocks;
  const size_t b = (size_t)2 * kPauliBlocks * (size_t)(nterms > 0 ? nterms : 0);
  return a > b ? a : b;
}

hipError_t launch_trace(int dtype, const void* buf, int n, int m, double* scratch,
                        double* out_dev, hipStream_t s) {
  const uint64_t N = (uint64_t)1 << n;
  const unsigned g = grid_for(N, kThreads, kReduceBlocks);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(trace_partial_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<double>*>(buf), N, m, scratch),
                 hipLaunchKernelGGL(trace_partial_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<float>*>(buf), N, m, scratch));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(kThreads), 0, s, scratch, (int)g, out_dev);
  return hipGetLastError();
}

hipError_t launch_expectation(int dtype, const void* a, const void* b, int n, int m,
                              double* scratch, double* out_dev, hipStream_t s) {
  const uint64_t nt = ntiles_of(n, m);
  const unsigned g = grid_for(nt, kThreads / 64, kReduceBlocks);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(expect_partial_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<double>*>(a),
                                    reinterpret_cast<const S2<double>*>(b), nt, m, scratch),
                 hipLaunchKernelGGL(expect_partial_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<float>*>(a),
                                    reinterpret_cast<const S2<float>*>(b), nt, m, scratch));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(kThreads), 0, s, scratch, (int)g, out_dev);
  return hipGetLastError();
}

hipError_t launch_pauli_expect(int dtype, const void* buf, int n, int m, const PauliTerm* terms,
                               int nterms, double* scratch, double* out_dev, hipStream_t s) {
  const uint64_t N = (uint64_t)1 << n;
  const unsigned gx = grid_for(N, kThreads, kPauliBlocks);
  const dim3 grid(gx, (unsigned)nterms);
  HT_DT_DISPATCH(dtype,
                 hipLaunchKernelGGL(pauli_partial_kernel<double>, grid, dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<double>*>(buf), N, m, terms,
                                    scratch),
                 hipLaunchKernelGGL(pauli_partial_kernel<float>, grid, dim3(kThreads), 0, s,
                                    reinterpret_cast<const S2<float>*>(buf), N, m, terms,
                                    scratch));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pauli_finish_kernel, dim3(1), dim3(kThreads), 0, s, scratch, (int)gx, terms,
                     nterms, out_dev);
  return hipGetLastError();
}

}  // namespace ht
