// C-ABI of the hermtile library: handle lifetime, validation, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hermtile.h"
#include "ht_handle.h"
#include "ht_internal.h"
#include "ht_prep.h"

namespace {

thread_local std::string g_err;

size_t elem_bytes(int dtype) { return dtype == HT_C128 ? 16 : 8; }

uint64_t stored_elems(int n, int m) {
  const uint64_t N = 1ull << n, M = 1ull << m;
  return N * (N + M) / 2;
}

}  // namespace

ht_status ht_fail(ht_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

namespace {

ht_status ensure_red(ht_herm* h, size_t doubles) {
  if (h->red_cap >= doubles) return HT_OK;
  if (h->red) {
    HT_HIP(hipStreamSynchronize(h->stream));
    HT_HIP(hipFree(h->red));
    h->red = nullptr;
    h->red_cap = 0;
  }
  if (hipMalloc(&h->red, doubles * sizeof(double)) != hipSuccess) {
    h->red = nullptr;
    return ht_fail(HT_ENOMEM, "could not allocate %zu bytes of reduction scratch", doubles * 8);
  }
  h->red_cap = doubles;
  return HT_OK;
}

ht_status ensure_tmp(ht_herm* h, size_t bytes) {
  if (h->tmp_cap >= bytes) return HT_OK;
  if (h->tmp) {
    HT_HIP(hipStreamSynchronize(h->stream));
    HT_HIP(hipFree(h->tmp));
    h->tmp = nullptr;
    h->tmp_cap = 0;
  }
  if (hipMalloc(&h->tmp, bytes) != hipSuccess) {
    h->tmp = nullptr;
    return ht_fail(HT_ENOMEM, "could not allocate %zu bytes of scratch", bytes);
  }
  h->tmp_cap = bytes;
  return HT_OK;
}

ht_status read_result(ht_herm* h, double* out) {
  HT_HIP(hipMemcpyAsync(h->out_host, h->out_dev, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HT_HIP(hipStreamSynchronize(h->stream));
  *out = h->out_host[0];
  return HT_OK;
}

hipEvent_t take_event(ht_herm* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Sort Pauli strings into device form: terms ordered by flip mask, runs of
// equal masks described by groups.
ht_status build_pauli(int n, int nterms, const uint8_t* codes, const double* coeffs,
                      std::vector<ht::PauliTerm>& terms, std::vector<ht::PauliGroup>& groups) {
  terms.resize(nterms);
  for (int t = 0; t < nterms; ++t) {
    uint32_t x = 0, z = 0;
    int ny = 0;
    for (int q = 0; q < n; ++q) {
      const uint8_t c = codes[(size_t)t * n + q];
      if (c > 3) return ht_fail(HT_EINVAL, "Pauli code %d at term %d qubit %d is not in 0..3", c, t, q);
      if (c == 1 || c == 2) x |= 1u << q;
      if (c == 2 || c == 3) z |= 1u << q;
      if (c == 2) ++ny;
    }
    terms[t] = ht::PauliTerm{x, z, ny & 3, 0, coeffs[t]};
  }
  std::stable_sort(terms.begin(), terms.end(),
                   [](const ht::PauliTerm& a, const ht::PauliTerm& b) { return a.x < b.x; });
  groups.clear();
  for (int t = 0; t < nterms; ++t) {
    if (groups.empty() || groups.back().x != terms[t].x)
      groups.push_back(ht::PauliGroup{terms[t].x, (uint32_t)t, 0, 0});
    groups.back().count++;
  }
  return HT_OK;
}

constexpr int kMaxPauliTerms = 4096;

}  // namespace

ht_status ht_launch_prepared(ht_herm* h, const ht::PreparedOp& op) {
  ht_device_guard dg(h->device);
  if (op.k == 2 && op.form == 1) HT_HIP(ht::launch_upload(h->coef_dev, op.coef, 512, h->stream));
  if (op.form == ht::kFormKraus3)
    HT_HIP(ht::launch_upload(h->coef_dev, op.coef, 128 * op.nkraus, h->stream));
  if (op.form == 2) {
    double data[512];
    const int nd = ht::native_op_data(op, data);
    HT_HIP(ht::launch_upload(h->coef_dev, data, nd, h->stream));
  }
  hipEvent_t a = nullptr, b = nullptr;
  // on a failure the events go back to the pool
  auto fail = [&](hipError_t e, const char* what) {
    if (a) h->pool.push_back(a);
    if (b) h->pool.push_back(b);
    return ht_fail(HT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  if (h->prof) {
    a = take_event(h);
    b = take_event(h);
    if (!a || !b) return fail(hipErrorOutOfMemory, "could not create profiling events");
    const hipError_t e = hipEventRecord(a, h->stream);
    if (e != hipSuccess) return fail(e, "hipEventRecord");
  }
  const hipError_t e =
      op.form == 2 ? ht::launch_native(h->dtype, h->buf, h->n, h->m, op, h->coef_dev, h->num_cu, h->stream)
      : op.form == ht::kFormKraus3
          ? ht::launch_k3(h->dtype, h->buf, h->n, h->m, op, h->coef_dev, h->num_cu, h->stream)
          : ht::launch_conj(h->dtype, h->buf, h->n, h->m, op, h->coef_dev, h->num_cu, h->stream);
  if (e != hipSuccess) return fail(e, "conjugation pass launch");
  if (h->prof) {
    const hipError_t eb = hipEventRecord(b, h->stream);
    if (eb != hipSuccess) return fail(eb, "hipEventRecord");
    const int cls = h->dtype * ht::kClassesPerDtype + ht::conj_class(op.k, op.ncross, op.form);
    // algorithmic bytes: every stored entry read and written once, or for the
    // native pass the changing fraction of them
    double frac = 1.0;
    if (op.form == 2) frac = (double)__builtin_popcountll(op.active) / (double)(1 << (2 * op.k));
    h->pending.push_back(ht_pending_event{cls, a, b, 2.0 * frac * (double)h->bytes});
  }
  return HT_OK;
}

extern "C" {

const char* ht_last_error(void) { return g_err.c_str(); }

int ht_effective_tile_log2(int n, int tile_log2) {
  if (n < 1 || n > HT_MAX_QUBITS || tile_log2 < HT_MIN_TILE_LOG2 || tile_log2 > HT_MAX_TILE_LOG2)
    return -1;
  return std::min(n, tile_log2);
}

size_t ht_storage_bytes(int n, int tile_log2, ht_dtype dtype) {
  const int m = ht_effective_tile_log2(n, tile_log2);
  if (m < 0 || (dtype != HT_C128 && dtype != HT_C64)) return 0;
  return (size_t)stored_elems(n, m) * elem_bytes(dtype);
}

ht_status ht_herm_create(int n, int tile_log2, ht_dtype dtype, void* dev_buf, size_t buf_bytes,
                         void* hip_stream, ht_herm** out) {
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > HT_MAX_QUBITS) return ht_fail(HT_EINVAL, "n = %d outside [1, %d]", n, HT_MAX_QUBITS);
  if (tile_log2 < HT_MIN_TILE_LOG2 || tile_log2 > HT_MAX_TILE_LOG2)
    return ht_fail(HT_EINVAL, "tile_log2 = %d outside [%d, %d]", tile_log2, HT_MIN_TILE_LOG2,
                HT_MAX_TILE_LOG2);
  if (dtype != HT_C128 && dtype != HT_C64) return ht_fail(HT_EINVAL, "unknown dtype %d", (int)dtype);
  const size_t need = ht_storage_bytes(n, tile_log2, dtype);
  if (dev_buf) {
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256 != 0)
      return ht_fail(HT_EINVAL, "borrowed buffer is not 256-byte aligned");
    if (buf_bytes < need)
      return ht_fail(HT_ENOMEM, "borrowed buffer holds %zu bytes, %zu needed", buf_bytes, need);
  }
  ht_herm* h = new ht_herm();
  h->n = n;
  h->m_req = tile_log2;
  h->m = std::min(n, tile_log2);
  h->dtype = dtype;
  h->nelems = stored_elems(n, h->m);
  h->bytes = need;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  auto cleanup = [&](ht_status st) {
    ht_herm_destroy(h);
    return st;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return cleanup(ht_fail(HT_EDEVICE, "no HIP device"));
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
      cus > 0)
    h->num_cu = cus;
  if (dev_buf) {
    h->buf = dev_buf;
    h->owned = false;
  } else {
    if (hipMalloc(&h->buf, need) != hipSuccess) {
      h->buf = nullptr;
      return cleanup(ht_fail(HT_ENOMEM, "could not allocate %zu bytes of tiled storage", need));
    }
    h->owned = true;
  }
  if (hipMalloc(&h->coef_dev, ht::kPrepCoefDoubles * sizeof(double)) != hipSuccess) {
    h->coef_dev = nullptr;
    return cleanup(ht_fail(HT_ENOMEM, "could not allocate coefficient buffer"));
  }
  if (hipMalloc(&h->out_dev, 8 * sizeof(double)) != hipSuccess) {
    h->out_dev = nullptr;
    return cleanup(ht_fail(HT_ENOMEM, "could not allocate result buffer"));
  }
  *out = h;
  return HT_OK;
}

ht_status ht_herm_destroy(ht_herm* h) {
  if (!h) return HT_OK;
  ht_device_guard dg(h->device);
  (void)hipStreamSynchronize(h->stream);
  for (auto& p : h->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->owned && h->buf) (void)hipFree(h->buf);
  if (h->coef_dev) (void)hipFree(h->coef_dev);
  if (h->out_dev) (void)hipFree(h->out_dev);
  if (h->red) (void)hipFree(h->red);
  if (h->tmp) (void)hipFree(h->tmp);
  delete h;
  return HT_OK;
}

ht_status ht_herm_set_stream(ht_herm* h, void* hip_stream) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(hipStreamSynchronize(h->stream));
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return HT_OK;
}

ht_status ht_herm_info(const ht_herm* h, int* n, int* tile_log2, int* dtype, void** dev_ptr,
                       size_t* bytes) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (n) *n = h->n;
  if (tile_log2) *tile_log2 = h->m;
  if (dtype) *dtype = h->dtype;
  if (dev_ptr) *dev_ptr = h->buf;
  if (bytes) *bytes = h->bytes;
  return HT_OK;
}

ht_status ht_herm_synchronize(ht_herm* h) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(hipStreamSynchronize(h->stream));
  return HT_OK;
}

ht_status ht_herm_init_zero(ht_herm* h) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(ht::launch_fill_zero(h->buf, h->bytes, h->stream));
  return HT_OK;
}

ht_status ht_herm_init_identity(ht_herm* h, double scale) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(ht::launch_fill_zero(h->buf, h->bytes, h->stream));
  HT_HIP(ht::launch_set_diag(h->dtype, h->buf, h->n, h->m, scale, h->stream));
  return HT_OK;
}

ht_status ht_herm_init_dense(ht_herm* h, const double* A, int64_t ld, int on_device) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!A) return ht_fail(HT_EINVAL, "A is NULL");
  const int64_t N = 1ll << h->n;
  if (ld < N) return ht_fail(HT_EINVAL, "ld = %lld < N = %lld", (long long)ld, (long long)N);
  ht_device_guard dg(h->device);
  if (on_device) {
    HT_HIP(ht::launch_pack_dense(h->dtype, h->buf, h->n, h->m, A, ld, h->stream));
    return HT_OK;
  }
  double* tmp = nullptr;
  const size_t bytes = (size_t)N * (size_t)ld * 16;
  if (hipMalloc(&tmp, bytes) != hipSuccess)
    return ht_fail(HT_ENOMEM, "could not allocate %zu bytes for the dense upload", bytes);
  hipError_t e = hipMemcpyAsync(tmp, A, bytes, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = ht::launch_pack_dense(h->dtype, h->buf, h->n, h->m, tmp, ld, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return ht_fail(HT_EDEVICE, "init_dense: %s", hipGetErrorString(e));
  return HT_OK;
}

ht_status ht_herm_init_lowrank(ht_herm* h, const double* G, int rank, int on_device) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!G) return ht_fail(HT_EINVAL, "G is NULL");
  if (rank < 1 || rank > 4096) return ht_fail(HT_EINVAL, "rank = %d outside [1, 4096]", rank);
  ht_device_guard dg(h->device);
  if (on_device) {
    HT_HIP(ht::launch_lowrank(h->dtype, h->buf, h->n, h->m, G, rank, h->stream));
    return HT_OK;
  }
  const size_t bytes = ((size_t)1 << h->n) * (size_t)rank * 16;
  double* tmp = nullptr;
  if (hipMalloc(&tmp, bytes) != hipSuccess)
    return ht_fail(HT_ENOMEM, "could not allocate %zu bytes for the factor upload", bytes);
  hipError_t e = hipMemcpyAsync(tmp, G, bytes, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = ht::launch_lowrank(h->dtype, h->buf, h->n, h->m, tmp, rank, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return ht_fail(HT_EDEVICE, "init_lowrank: %s", hipGetErrorString(e));
  return HT_OK;
}

ht_status ht_herm_init_pauli_sum(ht_herm* h, int nterms, const uint8_t* codes,
                                 const double* coeffs) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!codes || !coeffs) return ht_fail(HT_EINVAL, "codes or coeffs is NULL");
  if (nterms < 1 || nterms > kMaxPauliTerms)
    return ht_fail(HT_EINVAL, "nterms = %d outside [1, %d]", nterms, kMaxPauliTerms);
  std::vector<ht::PauliTerm> terms;
  std::vector<ht::PauliGroup> groups;
  ht_status st = build_pauli(h->n, nterms, codes, coeffs, terms, groups);
  if (st != HT_OK) return st;
  ht_device_guard dg(h->device);
  const size_t tb = terms.size() * sizeof(ht::PauliTerm), gb = groups.size() * sizeof(ht::PauliGroup);
  st = ensure_tmp(h, tb + gb);
  if (st != HT_OK) return st;
  HT_HIP(hipStreamSynchronize(h->stream));  // tmp may still be read by earlier work
  char* base = reinterpret_cast<char*>(h->tmp);
  HT_HIP(hipMemcpy(base, terms.data(), tb, hipMemcpyHostToDevice));
  HT_HIP(hipMemcpy(base + tb, groups.data(), gb, hipMemcpyHostToDevice));
  HT_HIP(ht::launch_fill_zero(h->buf, h->bytes, h->stream));
  HT_HIP(ht::launch_pauli_init(h->dtype, h->buf, h->n, h->m,
                               reinterpret_cast<const ht::PauliGroup*>(base + tb), (int)groups.size(),
                               reinterpret_cast<const ht::PauliTerm*>(base), h->stream));
  HT_HIP(hipStreamSynchronize(h->stream));
  return HT_OK;
}

ht_status ht_herm_to_dense(const ht_herm* hc, double* out, int64_t ld, int on_device) {
  ht_herm* h = const_cast<ht_herm*>(hc);
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  const int64_t N = 1ll << h->n;
  if (ld < N) return ht_fail(HT_EINVAL, "ld = %lld < N = %lld", (long long)ld, (long long)N);
  ht_device_guard dg(h->device);
  if (on_device) {
    HT_HIP(ht::launch_unpack_dense(h->dtype, h->buf, h->n, h->m, out, ld, h->stream));
    return HT_OK;
  }
  const size_t bytes = (size_t)N * (size_t)ld * 16;
  double* tmp = nullptr;
  if (hipMalloc(&tmp, bytes) != hipSuccess)
    return ht_fail(HT_ENOMEM, "could not allocate %zu bytes for the dense download", bytes);
  hipError_t e = ht::launch_fill_zero(tmp, bytes, h->stream);
  if (e == hipSuccess) e = ht::launch_unpack_dense(h->dtype, h->buf, h->n, h->m, tmp, ld, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return ht_fail(HT_EDEVICE, "to_dense: %s", hipGetErrorString(e));
  return HT_OK;
}

ht_status ht_herm_get_entries(const ht_herm* hc, int64_t count, const int64_t* rows,
                              const int64_t* cols, double* out) {
  ht_herm* h = const_cast<ht_herm*>(hc);
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!rows || !cols || !out) return ht_fail(HT_EINVAL, "rows, cols or out is NULL");
  if (count < 1 || count > (1ll << 24)) return ht_fail(HT_EINVAL, "count outside [1, 2^24]");
  const int64_t N = 1ll << h->n;
  for (int64_t e = 0; e < count; ++e)
    if (rows[e] < 0 || rows[e] >= N || cols[e] < 0 || cols[e] >= N)
      return ht_fail(HT_EINVAL, "entry %lld: (%lld, %lld) outside the matrix", (long long)e,
                  (long long)rows[e], (long long)cols[e]);
  ht_device_guard dg(h->device);
  const size_t ib = (size_t)count * 8, ob = (size_t)count * 16;
  ht_status st = ensure_tmp(h, 2 * ib + ob);
  if (st != HT_OK) return st;
  HT_HIP(hipStreamSynchronize(h->stream));
  char* base = reinterpret_cast<char*>(h->tmp);
  HT_HIP(hipMemcpy(base, rows, ib, hipMemcpyHostToDevice));
  HT_HIP(hipMemcpy(base + ib, cols, ib, hipMemcpyHostToDevice));
  HT_HIP(ht::launch_get_entries(h->dtype, h->buf, h->n, h->m, count,
                                reinterpret_cast<const int64_t*>(base),
                                reinterpret_cast<const int64_t*>(base + ib),
                                reinterpret_cast<double*>(base + 2 * ib), h->stream));
  HT_HIP(hipStreamSynchronize(h->stream));
  HT_HIP(hipMemcpy(out, base + 2 * ib, ob, hipMemcpyDeviceToHost));
  return HT_OK;
}

ht_status ht_herm_read_raw(const ht_herm* hc, size_t offset, size_t nbytes, void* out) {
  ht_herm* h = const_cast<ht_herm*>(hc);
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  if (offset > h->bytes || nbytes > h->bytes - offset)
    return ht_fail(HT_EINVAL, "range [%zu, %zu) outside the %zu-byte storage", offset, offset + nbytes,
                h->bytes);
  ht_device_guard dg(h->device);
  HT_HIP(hipStreamSynchronize(h->stream));
  HT_HIP(hipMemcpy(out, reinterpret_cast<char*>(h->buf) + offset, nbytes, hipMemcpyDeviceToHost));
  return HT_OK;
}

ht_status ht_herm_copy(ht_herm* dst, const ht_herm* src) {
  if (!dst || !src) return ht_fail(HT_EINVAL, "handle is NULL");
  if (dst->n != src->n || dst->m != src->m || dst->dtype != src->dtype)
    return ht_fail(HT_EINVAL, "copy needs equal n, tile edge and dtype");
  if (dst == src) return HT_OK;
  ht_device_guard dg(dst->device);
  if (src->stream != dst->stream) HT_HIP(hipStreamSynchronize(src->stream));
  HT_HIP(ht::launch_copy(dst->buf, src->buf, dst->bytes, dst->stream));
  return HT_OK;
}

static ht_status apply(ht_herm* h, int k, const int* targets, int r, const double* mats,
                       ht_picture picture) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (picture != HT_SCHRODINGER && picture != HT_HEISENBERG)
    return ht_fail(HT_EINVAL, "unknown picture %d", (int)picture);
  ht::PreparedOp op;
  char msg[256];
  const int pr = ht::prepare_op(h->n, h->m, k, targets, r, mats, picture == HT_HEISENBERG, &op, msg,
                                sizeof msg, ht::native_policy(h->bytes));
  if (pr != 0) return ht_fail(HT_EINVAL, "%s", msg);
  return ht_launch_prepared(h, op);
}

ht_status ht_apply_unitary(ht_herm* h, int k, const int* targets, const double* U,
                           ht_picture picture) {
  return apply(h, k, targets, 1, U, picture);
}

ht_status ht_apply_channel(ht_herm* h, int k, const int* targets, int r, const double* kraus,
                           ht_picture picture) {
  return apply(h, k, targets, r, kraus, picture);
}

ht_status ht_trace(const ht_herm* hc, double* out) {
  ht_herm* h = const_cast<ht_herm*>(hc);
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  ht_device_guard dg(h->device);
  ht_status st = ensure_red(h, ht::reduce_scratch_doubles(h->n, h->m, 0));
  if (st != HT_OK) return st;
  HT_HIP(ht::launch_trace(h->dtype, h->buf, h->n, h->m, h->red, h->out_dev, h->stream));
  return read_result(h, out);
}

ht_status ht_expectation(const ht_herm* a, const ht_herm* b, double* out) {
  ht_herm* h = const_cast<ht_herm*>(a);
  if (!a || !b) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!out) return ht_fail(HT_EINVAL, "out is NULL");
  if (a->n != b->n || a->m != b->m || a->dtype != b->dtype)
    return ht_fail(HT_EINVAL, "expectation needs equal n, tile edge and dtype");
  ht_device_guard dg(h->device);
  if (b->stream != a->stream) HT_HIP(hipStreamSynchronize(b->stream));
  ht_status st = ensure_red(h, ht::reduce_scratch_doubles(h->n, h->m, 0));
  if (st != HT_OK) return st;
  HT_HIP(ht::launch_expectation(h->dtype, a->buf, b->buf, h->n, h->m, h->red, h->out_dev,
                                h->stream));
  return read_result(h, out);
}

ht_status ht_expectation_pauli_sum(const ht_herm* hc, int nterms, const uint8_t* codes,
                                   const double* coeffs, double* out) {
  ht_herm* h = const_cast<ht_herm*>(hc);
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (!codes || !coeffs || !out) return ht_fail(HT_EINVAL, "codes, coeffs or out is NULL");
  if (nterms < 1 || nterms > kMaxPauliTerms)
    return ht_fail(HT_EINVAL, "nterms = %d outside [1, %d]", nterms, kMaxPauliTerms);
  std::vector<ht::PauliTerm> terms;
  std::vector<ht::PauliGroup> groups;
  ht_status st = build_pauli(h->n, nterms, codes, coeffs, terms, groups);
  if (st != HT_OK) return st;
  ht_device_guard dg(h->device);
  st = ensure_red(h, ht::reduce_scratch_doubles(h->n, h->m, nterms));
  if (st != HT_OK) return st;
  const size_t tb = terms.size() * sizeof(ht::PauliTerm);
  st = ensure_tmp(h, tb);
  if (st != HT_OK) return st;
  HT_HIP(hipStreamSynchronize(h->stream));
  HT_HIP(hipMemcpy(h->tmp, terms.data(), tb, hipMemcpyHostToDevice));
  HT_HIP(ht::launch_pauli_expect(h->dtype, h->buf, h->n, h->m,
                                 reinterpret_cast<const ht::PauliTerm*>(h->tmp), nterms, h->red,
                                 h->out_dev, h->stream));
  return read_result(h, out);
}

ht_status ht_scale(ht_herm* h, double alpha) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(ht::launch_scale(h->dtype, h->buf, h->nelems, alpha, h->stream));
  return HT_OK;
}

ht_status ht_profile_enable(ht_herm* h, int enable) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  h->prof = enable != 0;
  return HT_OK;
}

ht_status ht_profile_reset(ht_herm* h) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(hipStreamSynchronize(h->stream));
  for (auto& p : h->pending) {
    h->pool.push_back(p.a);
    h->pool.push_back(p.b);
  }
  h->pending.clear();
  std::fill(std::begin(h->prof_launches), std::end(h->prof_launches), 0);
  std::fill(std::begin(h->prof_ms), std::end(h->prof_ms), 0.0);
  std::fill(std::begin(h->prof_bytes), std::end(h->prof_bytes), 0.0);
  return HT_OK;
}

ht_status ht_profile_read(ht_herm* h, int max_classes, int* nclasses, int64_t* launches,
                          double* ms, double* bytes) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  ht_device_guard dg(h->device);
  HT_HIP(hipStreamSynchronize(h->stream));
  for (auto& p : h->pending) {
    float t = 0.f;
    HT_HIP(hipEventElapsedTime(&t, p.a, p.b));
    h->prof_launches[p.cls] += 1;
    h->prof_ms[p.cls] += t;
    h->prof_bytes[p.cls] += p.bytes;
    h->pool.push_back(p.a);
    h->pool.push_back(p.b);
  }
  h->pending.clear();
  const int total = 2 * ht::kClassesPerDtype;
  if (nclasses) *nclasses = total;
  for (int i = 0; i < total && i < max_classes; ++i) {
    if (launches) launches[i] = h->prof_launches[i];
    if (ms) ms[i] = h->prof_ms[i];
    if (bytes) bytes[i] = h->prof_bytes[i];
  }
  return HT_OK;
}

const char* ht_kernel_class_name(int idx) {
  static const char* names[ht::kClassesPerDtype] = {
      "k1_c0_direct", "k1_c0_transfer", "k1_c1_direct", "k1_c1_transfer", "k2_c0_direct",
      "k2_c0_transfer", "k2_c1_direct", "k2_c1_transfer", "k2_c2_direct", "k2_c2_transfer",
      "k1_c0_native", "k1_c1_native", "k2_c0_native", "k2_c1_native", "k2_c2_native",
      "k3_c0_native", "k3_c1_native", "k3_c2_native", "k3_c3_native",
      "k3_c0_kraus", "k3_c1_kraus", "k3_c2_kraus", "k3_c3_kraus"};
  static std::string full[2 * ht::kClassesPerDtype];
  static std::once_flag once;
  std::call_once(once, [] {
    for (int d = 0; d < 2; ++d)
      for (int i = 0; i < ht::kClassesPerDtype; ++i)
        full[d * ht::kClassesPerDtype + i] = std::string(d == 0 ? "c128_" : "c64_") + names[i];
  });
  if (idx < 0 || idx >= 2 * ht::kClassesPerDtype) return nullptr;
  return full[idx].c_str();
}

ht_status ht_set_tuning(const char* name, int64_t value) {
  if (!name) return ht_fail(HT_EINVAL, "name is NULL");
  const std::string k(name);
  if (k == "conj_wg_per_cu") {
    if (value != -1 && (value < 1 || value > 64))
      return ht_fail(HT_EINVAL, "conj_wg_per_cu must be -1 (automatic) or in [1, 64]");
    ht::tuning().wg_per_cu = (int)value;
    return HT_OK;
  }
  if (k == "conj_block_threads") {
    if (value != 64 && value != 128 && value != 256)
      return ht_fail(HT_EINVAL, "conj_block_threads must be 64, 128 or 256");
    ht::tuning().block_threads = (int)value;
    return HT_OK;
  }
  if (k == "conj_order") {
    if (value < -1 || value > 1) return ht_fail(HT_EINVAL, "conj_order must be -1, 0 or 1");
    ht::tuning().order = (int)value;
    return HT_OK;
  }
  if (k == "interleave") {
    if (value < 0 || value > 1) return ht_fail(HT_EINVAL, "interleave must be 0 or 1");
    ht::tuning().interleave = (int)value;
    return HT_OK;
  }
  if (k == "pairs") {
    if (value < 0 || value > 2) return ht_fail(HT_EINVAL, "pairs must be 0, 1 or 2");
    ht::tuning().pairs = (int)value;
    return HT_OK;
  }
  if (k == "native") {
    if (value < 0 || value > 2) return ht_fail(HT_EINVAL, "native must be 0, 1 or 2");
    ht::tuning().native = (int)value;
    return HT_OK;
  }
  if (k == "pair_jp2") {
    if (value < 0 || value > 1) return ht_fail(HT_EINVAL, "pair_jp2 must be 0 or 1");
    ht::tuning().pair_jp2 = (int)value;
    return HT_OK;
  }
  if (k == "stage") {
    if (value < -1 || value > 1) return ht_fail(HT_EINVAL, "stage must be -1, 0 or 1");
    ht::tuning().stage = (int)value;
    return HT_OK;
  }
  if (k == "stage_wg_per_cu") {
    if (value < 1 || value > 2) return ht_fail(HT_EINVAL, "stage_wg_per_cu must be 1 or 2");
    ht::tuning().stage_wg_per_cu = (int)value;
    return HT_OK;
  }
  if (k == "stage_grid" || k == "sync_grid") {
    if (value < 0 || value > 65536) return ht_fail(HT_EINVAL, "%s must be in [0, 65536]", name);
    (k == "stage_grid" ? ht::tuning().stage_grid : ht::tuning().sync_grid) = (int)value;
    return HT_OK;
  }
  if (k == "stage_order") {
    if (value < -1 || value > 1) return ht_fail(HT_EINVAL, "stage_order must be -1, 0 or 1");
    ht::tuning().stage_order = (int)value;
    return HT_OK;
  }
  if (k == "stage_pipe") {
    if (value < 0 || value > 1) return ht_fail(HT_EINVAL, "stage_pipe must be 0 or 1");
    ht::tuning().stage_pipe = (int)value;
    return HT_OK;
  }
  if (k == "stage_threads") {
    if (value != 256 && value != 512) return ht_fail(HT_EINVAL, "stage_threads must be 256 or 512");
    ht::tuning().stage_threads = (int)value;
    return HT_OK;
  }
  if (k == "sync_waves") {
    if (value != -1 && value != 0 && value != 4 && value != 8 && value != 16)
      return ht_fail(HT_EINVAL, "sync_waves must be -1, 0, 4, 8 or 16");
    ht::tuning().sync_waves = (int)value;
    return HT_OK;
  }
  if (k == "pipe_waves") {
    if (value != 0 && value != 4 && value != 8) return ht_fail(HT_EINVAL, "pipe_waves must be 0, 4 or 8");
    ht::tuning().pipe_waves = (int)value;
    return HT_OK;
  }
  if (k == "sync_interleave") {
    if (value < -1 || value > 1) return ht_fail(HT_EINVAL, "sync_interleave must be -1, 0 or 1");
    ht::tuning().sync_interleave = (int)value;
    return HT_OK;
  }
  if (k == "sync_order") {
    if (value < -1 || value > 3) return ht_fail(HT_EINVAL, "sync_order must be in [-1, 3]");
    ht::tuning().sync_order = (int)value;
    return HT_OK;
  }
  if (k == "pipe_barrier") {
    if (value < 0 || value > 1) return ht_fail(HT_EINVAL, "pipe_barrier must be 0 or 1");
    ht::tuning().pipe_barrier = (int)value;
    return HT_OK;
  }
  if (k == "sync_wg_per_cu") {
    if (value < 1 || value > 8) return ht_fail(HT_EINVAL, "sync_wg_per_cu must be in [1, 8]");
    ht::tuning().sync_wg_per_cu = (int)value;
    return HT_OK;
  }
  if (k == "conj_mem_mode") {
    if (value < -1 || value > 3) return ht_fail(HT_EINVAL, "conj_mem_mode must be in [-1, 3]");
    ht::tuning().mem_mode = (int)value;
    return HT_OK;
  }
  return ht_fail(HT_EINVAL, "unknown tuning parameter '%s'", name);
}

ht_status ht_prepare_op(int n, int tile_log2, int k, const int* targets, int r,
                        const double* kraus, ht_picture picture, int* sorted_targets, int* ncross,
                        int* form, double* coef) {
  const int m = ht_effective_tile_log2(n, tile_log2);
  if (m < 0) return ht_fail(HT_EINVAL, "n or tile_log2 out of range");
  if (picture != HT_SCHRODINGER && picture != HT_HEISENBERG)
    return ht_fail(HT_EINVAL, "unknown picture %d", (int)picture);
  ht::PreparedOp op;
  char msg[256];
  const int pr = ht::prepare_op(n, m, k, targets, r, kraus, picture == HT_HEISENBERG, &op, msg,
                                sizeof msg, ht::tuning().native != 0 ? 1 : 0);
  if (pr != 0) return ht_fail(HT_EINVAL, "%s", msg);
  if (sorted_targets)
    for (int l = 0; l < op.k; ++l) sorted_targets[l] = op.sorted[l];
  if (ncross) *ncross = op.ncross;
  if (form) *form = op.form;
  if (coef) {
    const int D = 1 << op.k;
    const int ne = op.form == 1 ? D * D * D * D : op.form == ht::kFormKraus3 ? op.nkraus * D * D : D * D;
    std::memcpy(coef, op.coef, sizeof(double) * 2 * ne);
    if (op.form == 2)
      for (int u = 0; u < D; ++u) coef[2 * ne + u] = (double)op.perm[u];
  }
  return HT_OK;
}

}  // extern "C"
