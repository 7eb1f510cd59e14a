// Internal interfaces between the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ht_prep.h"

namespace ht {

// Number of kernel classes per dtype: (k, c, form) with c <= k.
constexpr int kClassesPerDtype = 23;
// Class index of (k, c, form) within a dtype: k=1 -> c*2+form (0..3),
// k=2 -> 4 + c*2 + form (4..9); native form (2): k=1 -> 10 + c,
// k=2 -> 12 + c, k=3 -> 15 + c (10..18); k = 3 Kraus form: 19 + c (19..22).
inline int conj_class(int k, int c, int form) {
  if (form == 2) return 10 + (k == 1 ? c : k == 2 ? 2 + c : 5 + c);
  if (form == kFormKraus3) return 19 + c;
  return (k == 1 ? 0 : 4) + c * 2 + form;
}

struct LaunchTuning {
  int block_threads = 256;  // 4 waves per workgroup
  int wg_per_cu = -1;       // cap on resident workgroups per CU of the grid-stride grid;
                            // -1: automatic (wg_per_cu_or below)
  int mem_mode = -1;        // -1: automatic; else bit 0: nontemporal loads, bit 1: stores
  int order = -1;           // 0: a wave walks a whole group; 1: waves share a group's
                            // patches; -1: 1 when there are fewer groups than the grid's waves
  int native = 1;           // native pass: 0 never, 1 on operators beyond the cache, 2 always
  int interleave = 1;       // patch order (lane_block): 0 runs, 1 alternating
  int pairs = 1;            // pair layout of complex64 passes (ht_pair.h): 0 off,
                            // 1 where it pays, 2 wherever it applies
  int pair_jp2 = 1;         // complex64 two-cross pair passes in plain mode: two pairs per step
  int stage = -1;           // intra-tile passes staged through LDS in 64 KiB steps:
                            // -1 automatic, 0 off, 1 wherever the tile fits
  int stage_wg_per_cu = 1;  // workgroups per CU of the staged pass
  int stage_grid = 0;       // staged pass: workgroups of the grid (0: stage_wg_per_cu per CU)
  int sync_grid = 0;        // synchronised pass: workgroups of the grid (0: sync_wg_per_cu per CU)
  int stage_pipe = 1;      // staged pass: prefetch the next step during compute
  int stage_order = -1;     // staged pass: -1 automatic, 0 contiguous steps, 1 every other 16 KiB
                            // granule per step
  int stage_threads = 512;  // threads per workgroup of the staged pass (256: 64 KiB steps, 512: 128 KiB)
  int sync_waves = -1;      // passes with a tile-selecting target in workgroup-wide
                            // steps: -1 automatic, 0 off, else waves per workgroup (4, 8, 16)
  int sync_wg_per_cu = 1;   // workgroups per CU of the synchronised pass
  int sync_order = -1;      // items of a synchronised workgroup step: -1 automatic, 0 whole
                            // groups, 1 one quarter of every tile of consecutive groups,
                            // 2 the same of every other group, 3 of every fourth (pair layout;
                            // the block layout takes 2 for it)
  int sync_interleave = -1; // patch order of the synchronised pass: -1 automatic (0 for two
                            // tile-selecting targets, else as "interleave"), 0 or 1
  int pipe_waves = 0;       // steps with the next one prefetched: 0 off, 4 or 8 waves per workgroup
  int pipe_barrier = 1;     // 4-wave prefetching workgroups meet at a barrier before each store phase
};
LaunchTuning& tuning();

// Launch shapes of the conjugation pass that the pass tuner (ht_tune_passes)
// chooses between for a class of passes.  Every shape computes the same
// blocks with the same arithmetic (bitwise equal results).  The grids are
// 1, 3/4 and 5/8 workgroups per CU; the 16-wave workgroup steps come in
// three item orders (conj_sync_kernel): whole groups, one quarter of every
// tile of 16 consecutive groups, and one quarter of every other group.
enum PassShape {
  kShapeLane = 0,      // lane-patch kernel (conj_kernel), automatic grid
  kShapeStage = 1,     // LDS-staged intra-tile pass, contiguous steps, 3 grids (1..3)
  kShapeSync = 4,      // 16-wave workgroup steps, whole groups (4..6)
  kShapeSyncQ = 7,     //   ... quarters of consecutive groups (7..9)
  kShapeSyncQA = 10,   //   ... quarters of every other group (10..12)
  kShapeStageA = 13,   // LDS-staged pass, every other 16 KiB granule per step (13..15)
  kShapeSyncQ4 = 16,   // 16-wave steps, quarters of every fourth group (16..18; complex64
                       // pair layout, the block layout takes every other group)
  kShapeStage2 = 19,   // LDS-staged pass, alternate granules, 64 KiB steps of 256-thread
                       // workgroups, two per CU
  kShapeCount = 20
};
inline bool shape_is_stage(int shape) {
  return (shape >= kShapeStage && shape < kShapeSync) || (shape >= kShapeStageA && shape < kShapeSyncQ4) ||
         shape == kShapeStage2;
}
inline bool shape_is_sync(int shape) {
  return (shape >= kShapeSync && shape < kShapeStageA) || (shape >= kShapeSyncQ4 && shape < kShapeStage2);
}
// Item order of a step shape: 0 whole groups, 1 quarters, 2 quarters of
// every other group, 3 of every fourth.
inline int shape_sync_order(int shape) { return shape >= kShapeSyncQ4 ? 3 : (shape - kShapeSync) / 3; }
// Step order of a staged shape: 0 contiguous, 1 every other 16 KiB granule.
inline int shape_stage_order(int shape) { return shape >= kShapeStageA ? 1 : 0; }
// Threads per workgroup of a staged shape.
inline int shape_stage_threads(int shape) { return shape == kShapeStage2 ? 256 : 512; }
// Grid of a shape: workgroups for num_cu compute units.
inline uint64_t shape_grid(int shape, int num_cu) {
  if (shape == kShapeStage2) return 2u * (uint64_t)num_cu;
  const int i = shape_is_stage(shape) ? (shape - (shape >= kShapeStageA ? kShapeStageA : kShapeStage))
                : shape_is_sync(shape) ? (shape - (shape >= kShapeSyncQ4 ? kShapeSyncQ4 : kShapeSync)) % 3
                                       : 0;
  const int f = i == 1 ? 6 : i == 2 ? 5 : 8;
  return (uint64_t)num_cu * (uint64_t)f / 8u;
}
// The tuned shape of a pass class on operators of this storage type and
// shape (n, effective tile exponent m); low: an intra target lies below
// bit 3; far: the highest tile-selecting target is tile bit 4 or above.
// -1 when none has been tuned.
int tuned_shape(int dtype, int n, int m, int k, int c, int form, int low, int far);
void set_tuned_shape(int dtype, int n, int m, int k, int c, int form, int low, int far, int shape);

// Workgroups per CU for a kernel family: the tuning value if set, else the
// family's measured default auto_value.
inline int wg_per_cu_or(int auto_value) {
  return tuning().wg_per_cu > 0 ? tuning().wg_per_cu : auto_value;
}

// allow_native for prepare_op on an operator of `bytes` bytes: the native
// pass only pays where the pass is bound by HBM (an operator larger than the
// 256 MiB Infinity Cache: on cache-resident operators it measured up to 1.8x
// slower than the generic pass), and there only where the op's fixed entries
// fill whole cache lines (kNativeWherePays); k = 3 always takes it (its only
// form).  (tuning "native": 0 never -- k = 3 then fails --, 1 where it pays,
// 2 always.)
inline int native_policy(size_t bytes) {
  if (tuning().native == 0) return 0;
  if (tuning().native == 2) return 1;
  return bytes > ((size_t)256 << 20) ? kNativeWherePays : kNativeK3Only;
}
// The patch order of a pass (alternating measured faster for both storage
// types: +1 % for 16-byte entries, up to +10 % for 8-byte ones).
inline bool use_interleave(int /*entry_bytes*/) { return tuning().interleave != 0; }

// Enqueue one conjugation pass.  dtype 0: c128, 1: c64.  coef_dev is a device
// buffer of >= 512 doubles that holds op.coef when the kernel reads its
// coefficients from memory (two-qubit transfer form); the caller uploads it.
hipError_t launch_conj(int dtype, void* buf, int n, int m, const PreparedOp& op,
                       const double* coef_dev, int num_cu, hipStream_t s);

// Enqueue one k = 3 Kraus-form pass (op.form == kFormKraus3); coef_dev holds
// op.coef's 128 * op.nkraus doubles (uploaded by the caller).
hipError_t launch_k3(int dtype, void* buf, int n, int m, const PreparedOp& op,
                     const double* coef_dev, int num_cu, hipStream_t s);

// Enqueue one native pass (op.form == 2); coef_dev holds what native_op_data
// wrote (uploaded by the caller).
hipError_t launch_native(int dtype, void* buf, int n, int m, const PreparedOp& op,
                         const double* coef_dev, int num_cu, hipStream_t s);
// Device data of a native op: the coefficients, then for k = 3 the chunk
// schedule, one entry per double.  Returns the number of doubles (<= 512).
inline int native_op_data(const PreparedOp& op, double* out) {
  const int nc = 2 << (2 * op.k);
  for (int i = 0; i < nc; ++i) out[i] = op.coef[i];
  if (op.k != 3) return nc;
  for (int i = 0; i < op.nchunks * op.chunk; ++i) out[nc + i] = (double)op.sched[i];
  return nc + op.nchunks * op.chunk;
}

// Elementwise and reduction kernels over the tiled storage.
hipError_t launch_fill_zero(void* buf, size_t bytes, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// h /= *denom with denom a device scalar.
hipError_t launch_scale_inv(int dtype, void* buf, uint64_t nelems, const double* denom,
                            hipStream_t s);
hipError_t launch_set_diag(int dtype, void* buf, int n, int m, double value, hipStream_t s);
hipError_t launch_scale(int dtype, void* buf, uint64_t nelems, double alpha, hipStream_t s);
hipError_t launch_pack_dense(int dtype, void* buf, int n, int m, const double* A, int64_t ld,
                             hipStream_t s);
hipError_t launch_unpack_dense(int dtype, const void* buf, int n, int m, double* out, int64_t ld,
                               hipStream_t s);
hipError_t launch_lowrank(int dtype, void* buf, int n, int m, const double* G, int rank,
                          hipStream_t s);
hipError_t launch_get_entries(int dtype, const void* buf, int n, int m, int64_t count,
                              const int64_t* rows, const int64_t* cols, double* out,
                              hipStream_t s);

// Pauli strings in device form: x = bits where the string flips (X or Y),
// z = bits with a sign (Y or Z), ny = number of Y factors mod 4.
struct PauliTerm {
  uint32_t x, z;
  int32_t ny, pad;
  double c;
};
// Terms sorted by x; groups[g] = {x, first term, count} for runs of equal x.
struct PauliGroup {
  uint32_t x, first, count, pad;
};
hipError_t launch_pauli_init(int dtype, void* buf, int n, int m, const PauliGroup* groups,
                             int ngroups, const PauliTerm* terms, hipStream_t s);

// Deterministic FP64 reductions; each writes one double to out_dev.
// scratch must hold at least reduce_scratch_doubles(...) doubles.
size_t reduce_scratch_doubles(int n, int m, int nterms);
hipError_t launch_trace(int dtype, const void* buf, int n, int m, double* scratch, double* out_dev,
                        hipStream_t s);
hipError_t launch_expectation(int dtype, const void* a, const void* b, int n, int m,
                              double* scratch, double* out_dev, hipStream_t s);
hipError_t launch_pauli_expect(int dtype, const void* buf, int n, int m, const PauliTerm* terms,
                               int nterms, double* scratch, double* out_dev, hipStream_t s);

// One op of a batch in device form (see ht_batch.hip).
struct BatchOp {
  int32_t k, ncross, form;
  int32_t sorted[2];
  uint32_t coef_off;  // offset (in doubles) of its coefficients in the batch's array
  int32_t perm[4];    // native form: source local index of local index u
  uint32_t active;    // native form: bit u * 2^k + v set when entry (u, v) changes
};
// Number of doubles of coefficients an op of this shape carries.
inline int op_coef_doubles(int k, int form) {
  const int D = 1 << k;
  return 2 * (form == 1 ? D * D * D * D : D * D);
}
// One operator of a batch: its storage, shape and op range.
struct BatchOperator {
  void* buf;
  uint64_t bytes;
  int32_t n, m;
  uint32_t op_begin, op_end;
  int32_t in_lds, pad;
};
// Enqueue a queue reset and one persistent batch launch (grid workgroups of
// threads threads; lds_bytes of dynamic LDS for operators staged in LDS).
hipError_t launch_batch(int dtype, const BatchOperator* opers, unsigned nopers, const BatchOp* ops,
                        const double* coefs, unsigned* counter, int threads, int grid,
                        size_t lds_bytes, hipStream_t s);
// Allow the batch kernel to use up to bytes of dynamic LDS.
hipError_t set_batch_lds_limit(int dtype, size_t bytes);

// Upload count doubles into a device buffer with stream-ordered kernels
// (the values travel as kernel arguments, so no host buffer must outlive the
// call and no pageable-memory copy is involved).
hipError_t launch_upload(double* dst, const double* src, int count, hipStream_t s);

}  // namespace ht
