// Pauli-sum expectation without device allocation.
//
// ht_expectation_pauli_sum allocates its reduction partials and its term
// table on first use (and grows them with hipMalloc).  This variant runs the
// same kernels with both held in one fixed device array per GPU, so callers
// that must not allocate can read out tr(H O).  The array is a file-scope
// __device__ object: host code takes its device address once per device with
// hipGetSymbolAddress and passes that address on, never the symbol itself.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hermtile.h"
#include "ht_handle.h"
#include "ht_internal.h"

namespace {

constexpr int kMaxTerms = HT_NOALLOC_MAX_TERMS;
constexpr int kPauliBlocks = 64;  // partial sums per term (the reduction's fixed grid)
constexpr size_t kTermsBytes = ((size_t)kMaxTerms * sizeof(ht::PauliTerm) + 255) / 256 * 256;
constexpr size_t kPartialDoubles = (size_t)2 * kPauliBlocks * kMaxTerms;
constexpr size_t kOutOffset = kTermsBytes + kPartialDoubles * sizeof(double);
constexpr size_t kScratchBytes = kOutOffset + 256;
constexpr int kMaxDevices = 64;
static_assert(kScratchBytes == HT_NOALLOC_SCRATCH_BYTES, "the header states the array's size");

// Layout: [term table | partial sums | result].
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (device current).
ht_status scratch_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return ht_fail(HT_EDEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return ht_fail(HT_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_ptr[device]);
  return HT_OK;
}

struct TermChunk {
  static constexpr int kCap = 64;
  ht::PauliTerm t[kCap];
};

__global__ void store_terms_kernel(ht::PauliTerm* __restrict__ dst, TermChunk c, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = c.t[i];
}

}  // namespace

ht_status ht_expectation_pauli_sum_noalloc(const ht_herm* hc, int nterms, const uint8_t* codes,
                                           const double* coeffs, double* out) {
  ht_herm* h = const_cast<ht_herm*>(hc);
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!codes || !coeffs || !out) return ht_fail(HT_EINVAL, "codes, coeffs or out is NULL");
  if (nterms < 1 || nterms > kMaxTerms)
    return ht_fail(HT_EINVAL, "nterms = %d outside [1, %d], the limit of the fixed scratch array",
                   nterms, kMaxTerms);
  if (ht::reduce_scratch_doubles(h->n, h->m, nterms) > kPartialDoubles)
    return ht_fail(HT_EINVAL, "the reduction needs more partial sums than the fixed array holds");
  // Terms in the order ht_expectation_pauli_sum uses (stable by flip mask),
  // built on the stack: the summation order, and so every bit of the result,
  // is the same as there.
  ht::PauliTerm terms[kMaxTerms];
  for (int t = 0; t < nterms; ++t) {
    uint32_t x = 0, z = 0;
    int ny = 0;
    for (int q = 0; q < h->n; ++q) {
      const uint8_t c = codes[(size_t)t * h->n + q];
      if (c > 3) return ht_fail(HT_EINVAL, "Pauli code %d at term %d qubit %d is not in 0..3", c, t, q);
      if (c == 1 || c == 2) x |= 1u << q;
      if (c == 2 || c == 3) z |= 1u << q;
      if (c == 2) ++ny;
    }
    const ht::PauliTerm cur{x, z, ny & 3, 0, coeffs[t]};
    int j = t;
    while (j > 0 && terms[j - 1].x > cur.x) {  // insertion: stable
      terms[j] = terms[j - 1];
      --j;
    }
    terms[j] = cur;
  }
  ht_device_guard dg(h->device);
  unsigned char* base = nullptr;
  ht_status st = scratch_ptr(h->device, &base);
  if (st != HT_OK) return st;
  auto* dterms = reinterpret_cast<ht::PauliTerm*>(base);
  auto* partial = reinterpret_cast<double*>(base + kTermsBytes);
  auto* res = reinterpret_cast<double*>(base + kOutOffset);
  // Every partial slot the reduction reads is written by its first kernel,
  // and the result by its second, so nothing needs clearing between calls.
  for (int off = 0; off < nterms; off += TermChunk::kCap) {
    TermChunk c;
    const int len = nterms - off < TermChunk::kCap ? nterms - off : TermChunk::kCap;
    for (int i = 0; i < len; ++i) c.t[i] = terms[off + i];
    hipLaunchKernelGGL(store_terms_kernel, dim3(1), dim3(TermChunk::kCap), 0, h->stream, dterms + off,
                       c, len);
    HT_HIP(hipGetLastError());
  }
  HT_HIP(ht::launch_pauli_expect(h->dtype, h->buf, h->n, h->m, dterms, nterms, partial, res,
                                 h->stream));
  HT_HIP(hipMemcpyAsync(h->out_host, res, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HT_HIP(hipStreamSynchronize(h->stream));
  *out = h->out_host[0];
  return HT_OK;
}
