/*
 * hermtile -- k-local quantum operations on n-qubit hermitian operators stored
 * as lower-triangle tiles, on AMD Instinct MI355X (gfx950).
 *
 * Method: "Orkan: cache-friendly simulation of quantum operations on
 * hermitian operators" (arXiv 2604.15765).
 * A hermitian N x N operator H (N = 2^n; a density matrix or an observable) is
 * stored as the tiles T(ti,tj), ti >= tj, of edge M = 2^m of its lower tile
 * triangle (Section III-B), and every k-local operation
 *     H -> sum_a K_a H K_a^dagger,  K_a = I (x) L_a          (Eq. (1), Eq. (2))
 * is applied in one read-modify-write pass over the stored tiles (Section
 * III-C, Algorithms 2 and 3 and their appendix subroutines).
 *
 * Conventions used throughout
 * ---------------------------
 *  - Qubit q is bit q of a basis index (little-endian).
 *  - Complex numbers are interleaved pairs of doubles (re, im).
 *  - A k-local matrix is 2^k x 2^k, row-major; its local index bit l belongs
 *    to targets[l] (the order the caller gives; the library sorts internally).
 *  - Storage: tile (ti, tj) is tile number ti(ti+1)/2 + tj; its M^2 entries are
 *    row-major; diagonal tiles hold all M^2 entries.  When N < M the library
 *    uses one N x N tile instead of padding (the effective tile edge is
 *    min(M, N)).  c128 entries are 16 bytes, c64 entries 8 bytes.
 *  - Device memory: "device" pointers are HIP device addresses on the device
 *    that was current when the handle was created.
 *  - Streams: every call is enqueued on the handle's stream in order.  Calls
 *    that return a value to a host pointer synchronise that stream first.
 *  - Errors: every function returns an ht_status.  Argument errors are
 *    detected before anything is enqueued and leave the operator untouched;
 *    ht_last_error() then describes the problem.  HIP failures return
 *    HT_EDEVICE with the HIP error string.
 *  - Thread safety: a handle must not be used from two threads at once;
 *    distinct handles are independent.
 */
#ifndef HERMTILE_H
#define HERMTILE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ht_herm ht_herm; /* opaque handle: one tiled hermitian operator */

typedef enum {
  HT_C128 = 0, /* complex double storage, FP64 arithmetic */
  HT_C64 = 1   /* complex float storage, FP64 arithmetic and reductions */
} ht_dtype;

typedef enum {
  HT_SCHRODINGER = 0, /* H -> sum_a L_a H L_a^dagger (states) */
  HT_HEISENBERG = 1   /* H -> sum_a L_a^dagger H L_a (observables) */
} ht_picture;

typedef enum {
  HT_OK = 0,
  HT_EINVAL = 1,       /* invalid argument; nothing was enqueued */
  HT_ENOMEM = 2,       /* device allocation failed or buffer too small */
  HT_EDEVICE = 3,      /* a HIP call failed */
  HT_EUNSUPPORTED = 4  /* valid request outside what this build implements */
} ht_status;

/* Smallest and largest tile edge exponent accepted by ht_herm_create. */
#define HT_MIN_TILE_LOG2 1
#define HT_MAX_TILE_LOG2 8
/* Largest qubit count accepted (c128 at n = 17 is 137 GB of storage). */
#define HT_MAX_QUBITS 18

/* ---------------------------------------------------------------- sizes -- */

/* Bytes of tiled storage for an n-qubit operator: N(N + M')/2 entries with
 * M' = min(2^tile_log2, N) (Section III-B; Table I gives the padded sizes).
 * Returns 0 if n or tile_log2 is out of range or the dtype is unknown.
 * Pure host function; needs no GPU. */
size_t ht_storage_bytes(int n, int tile_log2, ht_dtype dtype);

/* Effective tile edge exponent used for an n-qubit operator:
 * min(tile_log2, n).  Returns -1 on invalid input.  Pure host function. */
int ht_effective_tile_log2(int n, int tile_log2);

/* ------------------------------------------------------------- lifetime -- */

/* Create a handle for an n-qubit hermitian operator with tile edge
 * 2^tile_log2 and storage type dtype.
 *   dev_buf    NULL: the library allocates the storage and frees it in
 *              ht_herm_destroy.  Non-NULL: a device buffer of buf_bytes bytes
 *              owned by the caller (for example a torch tensor); it must hold
 *              ht_storage_bytes(...) bytes, be 256-byte aligned, and outlive
 *              the handle.  The library never frees it.
 *   hip_stream the hipStream_t every call of this handle is enqueued on
 *              (NULL: the null stream).  Owned by the caller.
 *   out        receives the handle.
 * The storage content is undefined until one of the init calls runs.
 * Errors: HT_EINVAL (n, tile_log2, dtype, alignment, out == NULL),
 * HT_ENOMEM (allocation failed or buf_bytes too small), HT_EDEVICE. */
ht_status ht_herm_create(int n, int tile_log2, ht_dtype dtype, void* dev_buf, size_t buf_bytes,
                         void* hip_stream, ht_herm** out);

/* Destroy a handle: waits for its stream, frees what the library allocated.
 * Accepts NULL. */
ht_status ht_herm_destroy(ht_herm* h);

/* Replace the stream future calls are enqueued on (NULL: null stream). */
ht_status ht_herm_set_stream(ht_herm* h, void* hip_stream);

/* Describe a handle.  Any output pointer may be NULL.  dev_ptr receives the
 * device address of the tiled storage (tile 0, entry 0). */
ht_status ht_herm_info(const ht_herm* h, int* n, int* tile_log2, int* dtype, void** dev_ptr,
                       size_t* bytes);

/* Wait until everything enqueued on the handle's stream has finished. */
ht_status ht_herm_synchronize(ht_herm* h);

/* ---------------------------------------------------------- init and IO -- */

/* The init calls below fill the tiled format of Section III-B (lower tile
 * triangle, full diagonal tiles) with an operand for the conjugation passes.
 * The paper assumes an operator already in that format; these calls are the
 * library's own way to build one on the device and name the operands the
 * paper works with.  Each is enqueued on the handle's stream; argument
 * errors return HT_EINVAL (NULL handle or pointer, out-of-range sizes) with
 * the storage untouched. */

/* H = 0. */
ht_status ht_herm_init_zero(ht_herm* h);

/* H = scale * I.  scale = 1/N gives the maximally mixed state, the fixed
 * point of the depolarising channel of Section IV-A; scale = 1 gives the
 * identity observable, which the Heisenberg map of a trace-preserving
 * channel keeps (Section II-A, duality). */
ht_status ht_herm_init_identity(ht_herm* h, double scale);

/* Section III-B: pack a dense operator into the tiled format.
 * H = the hermitian matrix whose lower triangle (i >= j) is that of the dense
 * complex N x N row-major matrix A with leading dimension ld >= N (complex
 * entries).  Entries above the diagonal of A are not read: the stored upper
 * halves of diagonal tiles are set to the conjugates of the lower ones.
 * on_device != 0: A is a device pointer; 0: a host pointer (copied in; this
 * needs a temporary N x N device buffer).  A is not retained. */
ht_status ht_herm_init_dense(ht_herm* h, const double* A, int64_t ld, int on_device);

/* A density matrix of rank <= rank without a dense host copy (Section IV-A
 * evolves randomly initialised operators; at n = 16 a dense one would be
 * 64 GiB on the host).
 * H = G G^dagger for a complex N x rank matrix G, row-major (rank entries per
 * row), 1 <= rank <= 4096.  on_device as above.  A normalised density matrix
 * follows with ht_trace and ht_scale. */
ht_status ht_herm_init_lowrank(ht_herm* h, const double* G, int rank, int on_device);

/* An observable for the Heisenberg picture (Section I: every prediction is
 * tr(rho O), and the map may act on O instead of rho).  Each Pauli string is
 * a permutation with signs (Section II-B: X swaps entries, Y swaps and
 * negates, Z negates), so H is built entry by entry without any product.
 * H = sum_t coeffs[t] P_t for Pauli strings P_t; codes is nterms x n (host,
 * row-major), codes[t*n + q] in {0=I, 1=X, 2=Y, 3=Z} acting on qubit q;
 * coeffs is host, real.  1 <= nterms <= 4096.  HT_EINVAL for a code > 3. */
ht_status ht_herm_init_pauli_sum(ht_herm* h, int nterms, const uint8_t* codes,
                                 const double* coeffs);

/* Write the dense N x N matrix represented by H (entries i >= j from storage,
 * entries i < j as conjugates of their mirrors) to out, row-major, leading
 * dimension ld >= N, complex128.  on_device: out is a device pointer (else
 * host; the call then synchronises). */
ht_status ht_herm_to_dense(const ht_herm* h, double* out, int64_t ld, int on_device);

/* Read count entries H[rows[e], cols[e]] of the represented matrix (any
 * 0 <= row, col < N; entries above the diagonal come back as conjugates of
 * their stored mirrors) into out (host, 2*count doubles).  rows and cols are
 * host arrays.  Synchronises.  1 <= count <= 2^24. */
ht_status ht_herm_get_entries(const ht_herm* h, int64_t count, const int64_t* rows,
                              const int64_t* cols, double* out);

/* Copy raw storage bytes [offset, offset + nbytes) to the host buffer out.
 * Synchronises. */
ht_status ht_herm_read_raw(const ht_herm* h, size_t offset, size_t nbytes, void* out);

/* dst = src (same n, tile edge and dtype).  Enqueued on dst's stream after
 * src's stream (if different) has been synchronised; src must not be
 * modified until dst's stream has passed the copy. */
ht_status ht_herm_copy(ht_herm* dst, const ht_herm* src);

/* ------------------------------------------------------------- hot path -- */

/* Apply a k-qubit unitary (or any 2^k x 2^k matrix) U by conjugation:
 * Schroedinger H -> U H U^dagger, Heisenberg H -> U^dagger H U
 * (Eq. (2) with one Kraus operator; Section II-A: unitaries keep the direct
 * two-sided block update).  k in {1, 2, 3}; targets: k distinct qubits in
 * [0, n); U: host, 2 * 4^k doubles, row-major, interleaved complex.  U is not
 * checked for unitarity.  Enqueued asynchronously; U is copied before return.
 *
 * Permutation-and-phase matrices (one nonzero per row: X, Y, Z, S, T, RZ,
 * CNOT, CZ, SWAP, Toffoli, ... -- the gates of Section II-B) take a native
 * pass that moves every changing entry once, with its phase, and does not
 * touch the entries the gate fixes (a diagonal gate on a tile-selecting
 * qubit touches half of the storage, a CNOT three quarters).  Fixed entries
 * keep their bits; a phase product within 2^-50 of one on an entry the
 * permutation fixes counts as one.  Other k = 3 operations take a Kraus-form
 * pass (8 lanes per block of 64 entries, an LDS exchange between the left
 * and right products): every entry read and written once, 128 FP64 flops
 * per entry per Kraus operator.  For k <= 2 the native pass is used on
 * operators larger than the 256 MiB Infinity Cache, where the pass is bound
 * by HBM (on cache-resident ones the generic pass is faster), when some
 * entry stays in place, and when the fixed entries fill whole 128-byte
 * lines, i.e. whether an entry changes is decided by targets at bit 3 or
 * above (for diagonal matrices also bit 2, or any bits when at most 3/8 of
 * the entries change); otherwise the generic pass, measured faster there.
 * ht_set_tuning("native", v): 0 off (k <= 2 generic, k = 3 Kraus form), 1
 * as described (default), 2 whenever the matrix allows it, at every size. */
ht_status ht_apply_unitary(ht_herm* h, int k, const int* targets, const double* U,
                           ht_picture picture);

/* Apply the quantum operation with Kraus operators L_0..L_{r-1}:
 * Schroedinger H -> sum_a L_a H L_a^dagger (Eq. (1)), Heisenberg
 * H -> sum_a L_a^dagger H L_a.  k in {1, 2, 3}; 1 <= r <= 4^k; kraus: host,
 * r consecutive 2^k x 2^k row-major complex matrices (2 * r * 4^k doubles).
 * For r > 1 and k <= 2 the map is applied through its transfer matrix
 * (Eq. (3), built on the host in FP64); for k = 3 as the sum of the r
 * two-sided products (the Kraus-form pass described at ht_apply_unitary).
 * Kraus sets whose operators all have one nonzero per row in the same
 * columns (dephasing, for example) take the native pass described at
 * ht_apply_unitary.
 * Trace-preservation is not required (the algorithms hold for trace
 * non-increasing maps, Section IV-A).  Enqueued asynchronously; kraus is
 * copied before return. */
ht_status ht_apply_channel(ht_herm* h, int k, const int* targets, int r, const double* kraus,
                           ht_picture picture);

/* ----------------------------------------------------------- reductions -- */

/* The trace, tr(H I): the prediction of Section I for the identity
 * observable, and what a trace-preserving map keeps (Section II-A: the maps
 * are trace non-increasing; Section IV-A: the benchmarked channels preserve
 * it).  The N diagonal entries live in the diagonal tiles (Section III-B).
 * tr H = sum_i Re h_ii, accumulated in FP64 in a fixed order (deterministic,
 * also for complex64 storage).  out: host.  Synchronises.  HT_EINVAL for a
 * NULL handle or out. */
ht_status ht_trace(const ht_herm* h, double* out);

/* tr(A B) = Re sum_ij a_ij conj(b_ij) over the represented matrices, from the
 * tiles (Section III-C closing formula, with the off-diagonal tile sum strict:
 * diagonal tiles once, strictly lower tiles twice).  A and B must have the
 * same n, tile edge and dtype.  FP64, deterministic.  Synchronises. */
ht_status ht_expectation(const ht_herm* a, const ht_herm* b, double* out);

/* Section I's prediction tr(H O) for a Pauli-sum observable
 * O = sum_t coeffs[t] P_t (codes/coeffs as in ht_herm_init_pauli_sum,
 * 1 <= nterms <= 4096).  A string with flip mask x and sign mask z touches
 * N entries, tr(H P) = (-i)^ny sum_j (-1)^popcount(j & z) H[j ^ x, j]
 * (the permutation-with-signs form of Section II-B), so no dense O is built.
 * FP64, deterministic.  out: host.  Synchronises.  HT_EINVAL for a NULL
 * argument, nterms out of range or a code > 3. */
ht_status ht_expectation_pauli_sum(const ht_herm* h, int nterms, const uint8_t* codes,
                                   const double* coeffs, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as ht_expectation_pauli_sum, bit for bit (the same kernels, the
 * same term order and summation order), with the term table, the partial
 * sums and the result held in one fixed device array of
 * HT_NOALLOC_SCRATCH_BYTES bytes per GPU instead of buffers the handle
 * allocates.  The array is taken on a GPU's first call and held by that GPU
 * until the process ends.  Makes no device allocation or free.
 * 1 <= nterms <= HT_NOALLOC_MAX_TERMS; more terms return HT_EINVAL (use
 * ht_expectation_pauli_sum).  Other arguments and errors as for
 * ht_expectation_pauli_sum; out: host; synchronises the handle's stream.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (every slot a call reads is written by that call first): calls
 * that overlap on one GPU (from several threads, or on several handles of
 * one GPU with their streams running concurrently) race and must be
 * serialised by the caller. */
#define HT_NOALLOC_MAX_TERMS 256
#define HT_NOALLOC_SCRATCH_BYTES 268544
ht_status ht_expectation_pauli_sum_noalloc(const ht_herm* h, int nterms, const uint8_t* codes,
                                           const double* coeffs, double* out);

/* H = alpha * H, in FP64 before the store.  Not an operation of the paper
 * (its benchmark operator is not normalised, Section IV-A): the library's
 * normalisation step, e.g. alpha = 1 / tr H for rho = G G^dagger / tr.
 * Enqueued asynchronously.  HT_EINVAL for a NULL handle. */
ht_status ht_scale(ht_herm* h, double alpha);

/* ------------------------------------------------------------- batches -- */

/* A batch queues k-local operations for many independent operators and runs
 * them all in ONE persistent launch (the conjugation pass of Section III-C,
 * applied per operator in the order queued).  Each workgroup of the launch
 * takes operators from a queue (largest work first) and runs an operator's
 * whole sequence, with a barrier between consecutive ops; an operator whose
 * storage fits the LDS budget is evolved in LDS and written back once.
 * Results are bitwise identical to applying the same ops one call at a time.
 * Operators must live on one device; a batch may mix c128 and c64 operators
 * (one launch per storage type).  Not thread-safe. */
typedef struct ht_batch ht_batch;

ht_status ht_batch_create(ht_batch** out);
/* Waits for the batch's last run and frees its tables.  Accepts NULL. */
ht_status ht_batch_destroy(ht_batch* b);

/* Schedule parameters: "threads" (64..1024, power of two, default 256) per
 * workgroup; "wg_per_cu" (1..32, default 2) workgroups per compute unit;
 * "lds_max_bytes" (0..163584 = 160 KiB less the kernel's own LDS, default
 * 65536): operators up to this size run in LDS (0 disables LDS staging);
 * "fuse_qubits" (0, 1 or 2, default 0): run each operator's queued ops
 * fused into passes on at most that many qubits, as ht_circuit does (0: one
 * pass per op).  HT_EINVAL for an unknown name or value. */
ht_status ht_batch_set_param(ht_batch* b, const char* name, int64_t value);

/* Queue one op for operator h; arguments as ht_apply_unitary /
 * ht_apply_channel, with k in {1, 2} and the generic forms only (the batch
 * kernel has no native pass).  The matrices are prepared and copied before
 * return.
 * h must stay alive until the run that executes the op has finished. */
ht_status ht_batch_add_unitary(ht_batch* b, ht_herm* h, int k, const int* targets, const double* U,
                               ht_picture picture);
ht_status ht_batch_add_channel(ht_batch* b, ht_herm* h, int k, const int* targets, int r,
                               const double* kraus, ht_picture picture);

/* Number of operators and of ops queued (either pointer may be NULL). */
ht_status ht_batch_size(const ht_batch* b, int64_t* noperators, int64_t* nops);

/* Enqueue every queued op on hip_stream (one launch per storage type) and
 * return.  Work already enqueued on the operators' own streams is waited for
 * first.  The queue is kept: ht_batch_clear empties it. */
ht_status ht_batch_run(ht_batch* b, void* hip_stream);
ht_status ht_batch_clear(ht_batch* b);

/* Autotuner of batched launches (the tile edge 2^b is a free parameter of
 * the tiled format, Section III-B; here it is picked per qubit count by
 * measurement, together with the launch shape).  Times candidates on a
 * sample of the queued batch: at most sample_operators operators (0 = 512),
 * stratified by qubit count and storage type, as zero-initialised scratch
 * copies evolved by their own queued ops (re-prepared for each candidate
 * edge; run time does not depend on the values).  Searches, in turn: per
 * qubit count n, tile exponents 2..min(n, 7) and the operators' own; launch
 * shapes threads x wg_per_cu (at most 2048 threads per compute unit) x
 * lds_max_bytes in {0, 65536, 163584}; then the tile exponents again at the
 * chosen shape.  The fastest shape is stored in the batch (as by
 * ht_batch_set_param).  The queued operators are not changed: an operator's
 * tile edge is fixed when it is created, so to use the chosen edges create
 * the operators with out->tile_log2[n] and queue the ops again.
 * Synchronous.  Scratch: the sample's storage at one set of edges, from
 * hipMalloc on the batch's device; HT_ENOMEM if that exceeds half the free
 * device memory.  HT_EINVAL for an empty batch or a NULL argument. */
typedef struct {
  int tile_log2[HT_MAX_QUBITS + 1]; /* chosen exponent per qubit count; 0 where none */
  int threads;                      /* chosen launch shape (stored in the batch) */
  int wg_per_cu;
  int64_t lds_max_bytes;
  int sample_operators;             /* operators in the timed sample */
  int configs_timed;                /* candidate configurations timed */
  double sample_seconds_before;     /* sample at the queued edges and the batch's former shape */
  double sample_seconds_after;      /* sample at the chosen edges and shape */
  double tuning_seconds;            /* wall time of the whole search */
} ht_batch_tuning;
ht_status ht_batch_autotune(ht_batch* b, int sample_operators, ht_batch_tuning* out);

/* ------------------------------------------------------------ circuits -- */

/* A circuit: an op sequence applied with fusion.  Every conjugation pass
 * streams the whole operator (Section III-C), so neighbouring ops that
 * together act on at most max_qubits qubits are composed on the host in FP64
 * into one map (unitaries multiply; channels compose through their transfer
 * matrices, Eq. (3)) and applied in one pass.  The planner takes the
 * earliest op not yet applied and absorbs later ops that keep the group
 * within max_qubits (growing towards the qubits of the next op that couples
 * the group to other qubits), skipping past ops it cannot absorb as long as
 * no skipped op shares a qubit with an absorbed one (ops on disjoint qubits
 * commute).  A group of one op runs exactly as ht_apply_* runs it.  The
 * result equals applying the ops one by one up to rounding.  Not
 * thread-safe. */
typedef struct ht_circuit ht_circuit;
ht_status ht_circuit_create(ht_circuit** out);
ht_status ht_circuit_destroy(ht_circuit* c); /* accepts NULL */
/* Append an op (arguments as ht_apply_unitary / ht_apply_channel; k <= 3;
 * targets in [0, HT_MAX_QUBITS), checked against n when applied).  The
 * matrices are copied. */
ht_status ht_circuit_add_unitary(ht_circuit* c, int k, const int* targets, const double* U);
ht_status ht_circuit_add_channel(ht_circuit* c, int k, const int* targets, int r,
                                 const double* kraus);
ht_status ht_circuit_size(const ht_circuit* c, int64_t* nops);
/* Group the ops into passes for picture (Heisenberg: the adjoint maps in
 * reverse order) with at most max_qubits (0: no fusion, 1 or 2) qubits per
 * pass; *npasses (may be NULL) receives the number of passes.  Pure host
 * computation. */
ht_status ht_circuit_plan(ht_circuit* c, ht_picture picture, int max_qubits, int64_t* npasses);
/* Pass i of the last plan: *k qubits targets[0..k) (ascending), *nops ops
 * with their indices in the circuit as added (op_indices, nops entries, in
 * the order they are composed), and its transfer matrix (transfer: 2 * 16^k
 * doubles, row-major on the row-major block vector with local bit l at
 * targets[l]; k <= 2).  Any output may be NULL. */
ht_status ht_circuit_pass_info(const ht_circuit* c, int64_t i, int* k, int* targets, int64_t* nops,
                               int64_t* op_indices, double* transfer);
/* Enqueue the passes of the last plan on h's stream.  Every pass is prepared
 * before any is enqueued: on an error (a target >= n, ...) h is untouched. */
ht_status ht_circuit_apply(ht_circuit* c, ht_herm* h);

/* --------------------------------------------------------------- graphs -- */

/* Capture hot-path calls into a HIP graph and replay them with one launch.
 * Between ht_capture_begin(s) and ht_capture_end(s, &g), calls of handles
 * whose stream is s are recorded instead of executed (set the stream with
 * ht_herm_set_stream before beginning; reductions, init and IO calls must
 * not be made while capturing).  ht_graph_launch replays the recorded ops on
 * the same operators.  s must not be the null stream. */
typedef struct ht_graph ht_graph;
ht_status ht_capture_begin(void* hip_stream);
ht_status ht_capture_end(void* hip_stream, ht_graph** out);
ht_status ht_graph_launch(ht_graph* g, void* hip_stream);
ht_status ht_graph_destroy(ht_graph* g);

/* --------------------------------------------------------------- server -- */

/* A request server with continuous batching.  A scheduler thread admits
 * requests first-come first-served (per lane: small and large) when a slot
 * and enough of the HBM budget are free, keeps each operator resident until
 * its readout, advances small
 * operators (n <= batch_max_qubits) in rounds of one batched launch each
 * (requests join and leave between rounds) and large ones on their own
 * streams in chunks of plain passes, so the work of different requests
 * overlaps on the device.  A request's result does not depend on what else
 * is being served.  fifo = 1 serves one request at a time with plain
 * launches (the baseline).  One device (current at creation). */
typedef struct ht_server ht_server;

typedef struct {
  size_t budget_bytes;   /* HBM for resident operators (and their inputs) */
  int max_active;        /* requests resident at once, 1..256 */
  int batch_max_qubits;  /* n <= this: batched rounds; larger: plain passes */
  int chunk_ops;         /* ops per small request per batched round */
  int large_chunk_ops;   /* ops per chunk of a large request */
  int tile_log2;         /* tile edge exponent of every operator */
  int fifo;              /* 1: one request at a time, plain launches */
  int batch_threads;     /* see ht_batch_set_param */
  int batch_wg_per_cu;
  size_t lds_max_bytes;
  int max_large_active;  /* large requests running passes at once */
  int medium_max_qubits; /* n <= this (and > batch_max_qubits): medium lane */
  int max_medium_active; /* medium requests running passes at once */
  int fuse_qubits;       /* 0: one pass per op; 1, 2: a request's ops fused into
                            passes on at most that many qubits (as ht_circuit) */
} ht_server_config;

/* Defaults: 200 GiB budget, 32 active, batched rounds up to n = 8 (an
 * operator a single workgroup evolves from cache), medium lane up to n = 12
 * with 4 at once (their passes do not fill the GPU alone), large requests one
 * at a time (a large pass saturates HBM on its own; two at once only make
 * their access streams compete); 64 ops per round, 4 ops per chunk, tile
 * edge 32.  Each plain-pass lane also admits one request ahead of its limit
 * so that its initial state is built while the others run. */
void ht_server_config_default(ht_server_config* cfg);

/* A request: initial state G G^dagger / tr(G G^dagger) for the host N x rank
 * complex matrix G (row-major, 1 <= rank <= 4096); nops ops, op i acting on
 * op_k[i] in {1, 2} qubits op_targets[2i..2i+op_k[i]) with op_r[i] matrices
 * (1 = unitary) read consecutively from op_mats (row-major complex, as
 * ht_apply_channel); picture applies to every op; readout: tr(rho O) for the
 * Pauli sum (codes/coeffs as ht_herm_init_pauli_sum, nterms <= 4096) or, with
 * nterms = 0, the trace.  Everything is copied during ht_server_submit. */
typedef struct {
  int n;
  int dtype;
  int rank;
  const double* G;
  int nops;
  const int* op_k;
  const int* op_targets;
  const int* op_r;
  const double* op_mats;
  int picture;
  int nterms;
  const uint8_t* codes;
  const double* coeffs;
} ht_request;

ht_status ht_server_create(const ht_server_config* cfg, ht_server** out);
/* Validate and queue a request (HT_EINVAL for a malformed request or one
 * larger than the budget; nothing is queued then).  *id receives its id. */
ht_status ht_server_submit(ht_server* s, const ht_request* req, int64_t* id);
/* Block until every submitted request has completed (HT_EDEVICE on timeout). */
ht_status ht_server_wait_idle(ht_server* s, double timeout_s);
/* Move up to max completed requests out of the server: id, status (HT_OK or
 * the failure: HT_ENOMEM when the device cannot allocate the request's
 * operator, HT_EDEVICE when a launch failed; either way only that request
 * fails and the server keeps serving), readout value and the times (seconds on the server's
 * monotonic clock) of submission, admission and completion.  Any output
 * array may be NULL.  *count receives the number written. */
ht_status ht_server_poll(ht_server* s, int64_t max, int64_t* ids, int* status, double* values,
                         double* t_submit, double* t_admit, double* t_done, int64_t* count);
/* Current time on the server's clock. */
ht_status ht_server_now(const ht_server* s, double* t);
/* First asynchronous failure seen by the scheduler ("" if none). */
ht_status ht_server_last_error(ht_server* s, char* buf, size_t len);
/* Finish every submitted request, stop the scheduler, free everything. */
ht_status ht_server_destroy(ht_server* s);

/* --------------------------------------------------------- diagnostics -- */

/* Message describing the last error on the calling thread ("" if none). */
const char* ht_last_error(void);

/* Per-kernel timing of hot-path launches, for measurement.  When enabled,
 * every conjugation launch of this handle is bracketed by HIP events on the
 * handle's stream.  ht_profile_read synchronises and returns, per kernel
 * class (one class per storage type, k, number of tile-selecting targets and
 * form; ht_kernel_class_name(i) names class i), the number of launches, the
 * summed event time in milliseconds and the summed algorithmic bytes (every
 * stored entry read once and written once).  Entries 0..max_classes-1 of the
 * three arrays are written (any may be NULL); *nclasses receives the total
 * number of classes.  ht_profile_reset clears the sums. */
ht_status ht_profile_enable(ht_herm* h, int enable);
ht_status ht_profile_read(ht_herm* h, int max_classes, int* nclasses, int64_t* launches,
                          double* ms, double* bytes);
ht_status ht_profile_reset(ht_herm* h);
/* Name of kernel class idx ("c128_k1_c0_direct", ...); NULL if out of range. */
const char* ht_kernel_class_name(int idx);

/* Launch tuning of the conjugation pass, process-wide; it changes speed, never
 * results.  "conj_wg_per_cu" (-1 or 1..64, default -1): workgroups per
 * compute unit of the grid-stride grid; -1 = automatic: for the complex128
 * conjugation pass on operators of 1 GiB and more 1 (unitaries) or 2
 * (channels), 8 for smaller ones, complex64, the native pass and the three-qubit
 * Kraus-form pass (which itself caps single-operator complex128 passes at 2,
 * or 1 when a group is one tile).  "conj_block_threads" (64, 128 or 256, default
 * 256): workgroup size.  "conj_mem_mode" (-1..3, default -1 = automatic:
 * nontemporal loads and stores when every store writes whole cache lines);
 * 0..3: bit 0 marks the pass's loads nontemporal, bit 1 its stores.  "conj_order" (-1, 0 or 1,
 * default -1): 0 = each wave processes whole tile groups, 1 = the patches of
 * a group are spread over neighbouring waves, -1 = 1 when there are fewer
 * groups than the grid has waves, else 0.  "native" (0, 1 or 2, default 1):
 * the native pass for permutation-and-phase operations (see
 * ht_apply_unitary).  "interleave" (0 or 1,
 * default 1): the order in which a lane walks its patches of a tile group,
 * 1 alternating column and row patches (whole cache lines of 8-byte entries
 * in mirrored tiles too).  "pairs" (0, 1 or 2, default 1): the pair layout of
 * complex64 passes (one-qubit ops, and two-qubit ops in the direct form), in
 * which a lane holds two blocks in adjacent columns and moves their entries
 * as 16-byte accesses; 0 off, 1 where it pays (every target tile-selecting,
 * or the intra target at bit 4 or above), 2 wherever it applies (no intra
 * target at bit 0, at least 4 free bits per tile dimension).  Further names
 * select the launch shapes of the pass (every shape computes bitwise the
 * same result; -1 = automatic where allowed): "stage" (-1, 0, 1) the
 * LDS-staged intra-tile pass, "stage_threads" (256 or 512: 64 or 128 KiB
 * steps), "stage_pipe" (0 or 1: prefetch the next step), "stage_grid" and
 * "sync_grid" (0 = one workgroup per CU, else the number of workgroups),
 * "stage_wg_per_cu" (1 or 2), "sync_waves" (-1, 0, 4, 8, 16: workgroup-wide
 * steps for passes with a tile-selecting target), "sync_wg_per_cu",
 * "stage_order" (-1 automatic, 0 contiguous steps, 1 every other 16 KiB
 * granule per step), "sync_interleave" (-1, 0, 1), "sync_order" (-1 automatic; 0 a workgroup
 * step takes whole groups, 1 one quarter of every tile of consecutive
 * groups, 2 the same of every other group, 3 of every fourth group in the
 * complex64 pair layout, else as 2), "pipe_waves" (0, 4, 8: steps with the next
 * one prefetched), "pipe_barrier" (0 or 1), "pair_jp2" (0 or 1, default 1:
 * complex64 pair passes with two tile-selecting targets in plain mode take
 * two pairs per step).  A shape tuned by ht_tune_passes is used only while
 * "stage" and "sync_waves" are -1 and "pipe_waves" is 0.  HT_EINVAL for an unknown name or value.  Set it
 * while no other thread enqueues work (a server's scheduler thread reads it). */
ht_status ht_set_tuning(const char* name, int64_t value);

/* Launch-shape tuning of the conjugation pass by measurement on h.  The pass
 * streams every stored entry from and to HBM (Algorithms 2 and 3); which
 * launch shape streams fastest differs by a few percent between devices.
 * For every pass class of h's shape (storage type, n, tile edge) -- k = 1
 * and 2 targets, 0 to 2 of them tile-selecting, direct and transfer form,
 * an intra target below bit 3 or not, the highest tile-selecting target
 * below tile bit 4 or not -- this times each candidate shape (the
 * lane-patch kernel; the LDS-staged intra-tile pass in two step orders or
 * workgroup steps in three item orders, four for complex64 (in the pair
 * layout where it applies), each at grids of 1, 3/4 and 5/8 workgroups per
 * CU) on identity passes of h, reps timed rounds after one warm-up round,
 * and keeps the
 * fastest for operators of that shape.  The choice is process-wide and is
 * used while the launch tuning (ht_set_tuning "stage", "sync_waves",
 * "pipe_waves") is automatic; every shape computes bitwise the same result.
 * The identity passes leave every represented entry of h unchanged (a
 * negative zero may become a positive one, and the stored upper halves of
 * diagonal tiles are rewritten as the conjugates of the lower ones, which
 * is the same matrix).  Synchronises h's stream; at n = 16 it takes about
 * 10 s.  rows (host, may be NULL when max_rows = 0): up to max_rows records
 * of 8 doubles per class: k, tile-selecting targets, form (0 direct, 1
 * transfer), low (1: an intra target below bit 3), far (1: the highest
 * tile-selecting target at tile bit 4 or above), chosen shape (0 lane
 * patch, 1-3 staged at 1, 3/4, 5/8 workgroups per CU, 4-6 workgroup steps
 * of whole groups at the same grids, 7-9 steps of one quarter of every tile
 * of 16 groups, 10-12 the same of every other group of 32, 13-15 staged
 * with every other 16 KiB granule per step, 16-18 steps of every fourth
 * group, complex64 only, 19 staged with alternate granules in 64 KiB steps
 * of two 256-thread workgroups per CU), its ms per pass, the lane-patch
 * kernel's ms per pass;
 * nrows (may be NULL): classes tuned.  HT_EINVAL for a NULL handle, reps
 * outside [1, 16] or rows NULL with max_rows > 0.  Call it while no other
 * thread enqueues passes (it switches the process-wide launch tuning). */
ht_status ht_tune_passes(ht_herm* h, int reps, int max_rows, double* rows, int* nrows);

/* Set the launch shape of one pass class on operators of the given storage
 * type, n and tile edge, as ht_tune_passes would (for example from the
 * records of an earlier ht_tune_passes run; k, cross, form, low, far and
 * shape as in those records); shape -1 returns the class to the automatic
 * choice.  No GPU work.  HT_EINVAL for a class the operator shape cannot
 * have, a staged shape with a tile-selecting target or a step shape without
 * one. */
ht_status ht_set_pass_shape(int dtype, int n, int tile_log2, int k, int cross, int form, int low, int far,
                            int shape);

/* Pure host function (no GPU): the per-op preparation the library performs
 * before a launch, exposed for testing.  Given the same arguments as
 * ht_apply_channel (r = 1 for a unitary) and an operator shape (n, tile_log2),
 * writes
 *   sorted_targets[k]  targets in ascending order,
 *   *ncross            how many targets lie at or above the effective tile
 *                      exponent (they select tiles rather than entries),
 *   *form              0: direct two-sided form (coef holds the 2^k x 2^k
 *                      matrix A, applied as A h A^dagger), 1: transfer form
 *                      (coef holds the 4^k x 4^k matrix S acting on the
 *                      row-major vector of a block, S = sum_a A_a (x) conj(A_a)),
 *                      2: native permutation-and-phase form (coef holds the
 *                      2^k x 2^k coefficients c, then 2^k doubles p(0..2^k-1);
 *                      block entry w[u][v] = c[u][v] h[p(u)][p(v)]),
 *                      3: k = 3 Kraus form (coef holds the r 8 x 8 operators
 *                      A_a one after the other; w = sum_a A_a h A_a^dagger),
 *   coef               interleaved complex, row-major: 2 * 4^k doubles for
 *                      form 0, 2 * 16^k for form 1, 2 * 4^k + 2^k for form 2,
 *                      2 * 64 * r for form 3 (8192 always suffice),
 * where the A_a are the caller's operators with their local bits reordered to
 * ascending target order and, in the Heisenberg picture, adjoined.  The
 * native form is reported whenever the op has it (as for an operator beyond
 * the cache), unless ht_set_tuning("native", 0). */
ht_status ht_prepare_op(int n, int tile_log2, int k, const int* targets, int r,
                        const double* kraus, ht_picture picture, int* sorted_targets,
                        int* ncross, int* form, double* coef);

#ifdef __cplusplus
}
#endif

#endif /* HERMTILE_H */
