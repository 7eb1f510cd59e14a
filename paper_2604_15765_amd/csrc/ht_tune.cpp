// Launch-shape tuner of the conjugation pass.
//
// The pass is bound by HBM bandwidth, and which launch shape streams fastest
// differs by a few percent from one MI355X to another (measured across
// boxes: the LDS-staged intra-tile pass at one workgroup per CU ran 5.68 TB/s
// on some and 5.30 on others, where five workgroups per eight CUs ran 5.50).
// ht_tune_passes therefore times the candidate shapes of every pass class
// on the operator itself and keeps the fastest for operators of its storage
// type and shape.  The timed passes apply the identity (U = I in the direct
// form, S = I in the transfer form, native passes off), which leaves every
// represented entry unchanged; all shapes compute bitwise the same results,
// so the choice changes speed only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "hermtile.h"
#include "ht_handle.h"
#include "ht_internal.h"
#include "ht_prep.h"

namespace {

struct ShapeEntry {
  int dtype, n, m, k, c, form, low, far, shape;
};

std::mutex g_mu;
std::vector<ShapeEntry> g_shapes;

}  // namespace

namespace ht {

int tuned_shape(int dtype, int n, int m, int k, int c, int form, int low, int far) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& e : g_shapes)
    if (e.dtype == dtype && e.n == n && e.m == m && e.k == k && e.c == c && e.form == form && e.low == low &&
        e.far == far)
      return e.shape;
  return -1;
}

void set_tuned_shape(int dtype, int n, int m, int k, int c, int form, int low, int far, int shape) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& e : g_shapes)
    if (e.dtype == dtype && e.n == n && e.m == m && e.k == k && e.c == c && e.form == form && e.low == low &&
        e.far == far) {
      e.shape = shape;
      return;
    }
  g_shapes.push_back(ShapeEntry{dtype, n, m, k, c, form, low, far, shape});
}

}  // namespace ht

namespace {

// One pass class: k targets of which c select tiles, the form, whether an
// intra target lies below bit 3, whether the highest tile-selecting target
// is tile bit 4 or above (far), and the target sets timed for it.
struct TuneClass {
  int k, c, form, low, far;
  std::vector<std::vector<int>> targets;
};

std::vector<TuneClass> tune_classes(int n, int m) {
  std::vector<TuneClass> out;
  const int cross = n - m;  // tile-selecting qubits
  const bool has_far = cross >= 5;
  for (int form = 0; form < 2; ++form) {
    // intra-tile: low targets, and targets at bit 3 and above where the tile has them
    if (m >= 1) out.push_back({1, 0, form, 1, 0, {{0}}});
    if (m >= 4) out.push_back({1, 0, form, 0, 0, {{m - 1}}});
    if (m >= 2) out.push_back({2, 0, form, 1, 0, {{0, 1}}});
    if (m >= 5) out.push_back({2, 0, form, 0, 0, {{m - 2, m - 1}}});
    // one tile-selecting target: tile bits below 4 and from 4 up
    if (cross >= 1) {
      std::vector<std::vector<int>> t1 = {{m}};
      if (cross >= 3) t1.push_back({m + 2});
      out.push_back({1, 1, form, 0, 0, t1});
      if (has_far) {
        std::vector<std::vector<int>> tf = {{n - 1}};
        if (m + 5 < n - 1) tf.push_back({m + 5});
        out.push_back({1, 1, form, 0, 1, tf});
      }
      if (m >= 1) {
        out.push_back({2, 1, form, 1, 0, {{0, m}}});
        if (has_far) out.push_back({2, 1, form, 1, 1, {{0, n - 1}}});
      }
      if (m >= 4) {
        out.push_back({2, 1, form, 0, 0, {{m - 1, m}}});
        if (has_far) out.push_back({2, 1, form, 0, 1, {{m - 1, n - 1}}});
      }
    }
    if (cross >= 2) {
      out.push_back({2, 2, form, 0, 0, {{m, m + 1}}});
      if (has_far) out.push_back({2, 2, form, 0, 1, {{n - 2, n - 1}}});
    }
  }
  return out;
}

ht_status identity_op(const ht_herm* h, int k, int form, const std::vector<int>& targets, ht::PreparedOp* op) {
  const int D = 1 << k;
  char msg[256];
  int rc;
  if (form == 0) {
    std::vector<double> U(2 * D * D, 0.0);
    for (int i = 0; i < D; ++i) U[2 * (i * D + i)] = 1.0;
    rc = ht::prepare_op(h->n, h->m, k, targets.data(), 1, U.data(), 0, op, msg, sizeof msg, 0);
  } else {
    const int E = D * D;
    std::vector<double> S(2 * E * E, 0.0);
    for (int i = 0; i < E; ++i) S[2 * (i * E + i)] = 1.0;
    int sorted[2] = {targets[0], k > 1 ? targets[1] : 0};
    if (k > 1 && sorted[0] > sorted[1]) std::swap(sorted[0], sorted[1]);
    rc = ht::prepare_transfer(h->n, h->m, k, sorted, S.data(), 0, op, msg, sizeof msg);
  }
  if (rc != 0) return ht_fail(HT_EINVAL, "pass tuner: %s", msg);
  if (op->form != form) return ht_fail(HT_EINVAL, "pass tuner: identity op took form %d, not %d", op->form, form);
  return HT_OK;
}

}  // namespace

extern "C" ht_status ht_tune_passes(ht_herm* h, int reps, int max_rows, double* rows, int* nrows) {
  if (!h) return ht_fail(HT_EINVAL, "handle is NULL");
  if (reps < 1 || reps > 16) return ht_fail(HT_EINVAL, "reps = %d outside [1, 16]", reps);
  if (max_rows < 0 || (max_rows > 0 && !rows)) return ht_fail(HT_EINVAL, "rows is NULL");
  ht_device_guard dg(h->device);
  const ht::LaunchTuning saved = ht::tuning();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HT_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ht_fail(HT_EDEVICE, "hipEventCreate failed");
  }
  ht_status st = HT_OK;
  int nr = 0;
  const std::vector<TuneClass> classes = tune_classes(h->n, h->m);
  for (const TuneClass& tc : classes) {
    std::vector<ht::PreparedOp> ops(tc.targets.size());
    for (size_t i = 0; i < ops.size() && st == HT_OK; ++i) st = identity_op(h, tc.k, tc.form, tc.targets[i], &ops[i]);
    if (st != HT_OK) break;
    // the class's sorted targets all share ncross == tc.c by construction
    const bool skip_stage = h->dtype == HT_C64 && tc.k == 2 && tc.form == 1;  // measured 7x slower staged
    std::vector<int> cands = {ht::kShapeLane};
    for (int sh = 1; sh < ht::kShapeCount; ++sh)
      if ((tc.c == 0 && !skip_stage && ht::shape_is_stage(sh)) ||
          (tc.c > 0 && ht::shape_is_sync(sh) && (h->dtype == HT_C64 || ht::shape_sync_order(sh) < 3)))
        cands.push_back(sh);
    double best = 1e300, lane_ms = 0.0;
    int best_shape = ht::kShapeLane;
    for (int shape : cands) {
      ht::tuning() = saved;
      ht::tuning().pipe_waves = 0;
      ht::tuning().stage = ht::shape_is_stage(shape) ? 1 : 0;
      ht::tuning().stage_grid = ht::tuning().stage ? (int)ht::shape_grid(shape, h->num_cu) : 0;
      ht::tuning().stage_order = ht::tuning().stage ? ht::shape_stage_order(shape) : -1;
      ht::tuning().stage_threads = ht::tuning().stage ? ht::shape_stage_threads(shape) : saved.stage_threads;
      ht::tuning().sync_waves = ht::shape_is_sync(shape) ? 16 : 0;
      ht::tuning().sync_grid = ht::tuning().sync_waves ? (int)ht::shape_grid(shape, h->num_cu) : 0;
      ht::tuning().sync_order = ht::tuning().sync_waves ? ht::shape_sync_order(shape) : -1;
      ht::tuning().sync_interleave = -1;
      double tmin = 1e300;
      for (int r = 0; r <= reps && st == HT_OK; ++r) {  // the first round warms up
        double t = 0.0;
        for (const ht::PreparedOp& op : ops) {
          if (op.k == 2 && op.form == 1) {
            if (ht::launch_upload(h->coef_dev, op.coef, 512, h->stream) != hipSuccess) {
              st = ht_fail(HT_EDEVICE, "pass tuner: coefficient upload failed");
              break;
            }
          }
          hipError_t e = hipEventRecord(e0, h->stream);
          if (e == hipSuccess)
            e = ht::launch_conj(h->dtype, h->buf, h->n, h->m, op, h->coef_dev, h->num_cu, h->stream);
          if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) {
            st = ht_fail(HT_EDEVICE, "pass tuner: %s", hipGetErrorString(e));
            break;
          }
          t += ms;
        }
        if (r > 0) tmin = std::min(tmin, t);
      }
      if (st != HT_OK) break;
      if (shape == ht::kShapeLane) lane_ms = tmin;
      if (tmin < best) {
        best = tmin;
        best_shape = shape;
      }
    }
    if (st != HT_OK) break;
    ht::set_tuned_shape(h->dtype, h->n, h->m, tc.k, tc.c, tc.form, tc.low, tc.far, best_shape);
    if (nr < max_rows) {
      double* row = rows + 8 * nr;
      row[0] = tc.k;
      row[1] = tc.c;
      row[2] = tc.form;
      row[3] = tc.low;
      row[4] = tc.far;
      row[5] = best_shape;
      row[6] = best / (double)ops.size();
      row[7] = lane_ms / (double)ops.size();
    }
    ++nr;
  }
  ht::tuning() = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (nrows) *nrows = nr;
  return st;
}

extern "C" ht_status ht_set_pass_shape(int dtype, int n, int tile_log2, int k, int cross, int form, int low,
                                       int far, int shape) {
  if (dtype != HT_C128 && dtype != HT_C64) return ht_fail(HT_EINVAL, "unknown dtype %d", dtype);
  if (n < 1 || n > HT_MAX_QUBITS || tile_log2 < HT_MIN_TILE_LOG2 || tile_log2 > HT_MAX_TILE_LOG2)
    return ht_fail(HT_EINVAL, "invalid n = %d or tile_log2 = %d", n, tile_log2);
  const int m = std::min(n, tile_log2);
  // far: the highest tile-selecting target at tile bit 4 or above (n - m tile bits)
  if (k < 1 || k > 2 || cross < 0 || cross > k || cross > n - m || form < 0 || form > 1 || low < 0 || low > 1 ||
      (low == 1 && cross == k) || far < 0 || far > 1 || (far == 1 && (cross == 0 || n - m < 5)))
    return ht_fail(HT_EINVAL, "no pass class k = %d, cross = %d, form = %d, low = %d, far = %d at n = %d, m = %d",
                   k, cross, form, low, far, n, m);
  if (shape < -1 || shape >= ht::kShapeCount) return ht_fail(HT_EINVAL, "unknown shape %d", shape);
  if ((ht::shape_is_stage(shape) && cross != 0) || (ht::shape_is_sync(shape) && cross == 0))
    return ht_fail(HT_EINVAL, "shape %d does not apply to passes with %d tile-selecting targets", shape, cross);
  ht::set_tuned_shape(dtype, n, m, k, cross, form, low, far, shape);
  return HT_OK;
}
