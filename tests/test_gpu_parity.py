"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Small operators are compared entry by entry with the dense oracle (relative
Frobenius error <= 1e-12 in complex128).  Full-size operators (n = 14 and
n = 16, in the launch configuration the benchmark uses) are checked on sampled
blocks of Eq. (2) read before and after each op, plus invariants.
"""

import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import layout
from tests import sampling

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ht():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_15765_amd as ht
    return ht


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lower_hermitian(H):
    return np.tril(H) + np.tril(H, -1).conj().T


def make(ht, n, m, H=None, dtype="c128"):
    h = ht.Herm(n, m, dtype)
    if H is not None:
        h.init_dense(H)
    return h


# ----------------------------------------------------------------- storage


@pytest.mark.parametrize("n,m", [(1, 5), (3, 2), (5, 5), (6, 2), (7, 3), (9, 5), (10, 6)])
def test_init_dense_roundtrip_and_layout(ht, n, m):
    rng = synth.make_rng(10 * n + m)
    H = synth.random_hermitian_dense(n, rng)
    h = make(ht, n, m, H)
    assert np.array_equal(h.to_dense(), lower_hermitian(H))
    # raw storage is exactly the paper's tiled format (decoded independently)
    me = ht.effective_tile_log2(n, m)
    assert np.array_equal(h.raw_entries(), layout.encode(lower_hermitian(H), me))


def test_init_kernels(ht):
    rng = synth.make_rng(3)
    n, m = 7, 3
    h = make(ht, n, m)
    h.init_identity(0.25)
    assert np.array_equal(h.to_dense(), 0.25 * np.eye(1 << n))
    h.init_zero()
    assert not h.to_dense().any()
    G = synth.ginibre_factor(n, 5, rng)
    h.init_lowrank(G)
    assert rel(h.to_dense(), G @ G.conj().T) < 1e-14
    Gd = torch.from_numpy(G).cuda()
    h2 = make(ht, n, m)
    h2.init_lowrank(Gd)
    assert rel(h2.to_dense(), G @ G.conj().T) < 1e-14
    codes, coeffs = synth.random_pauli_sum(n, 40, rng)
    h.init_pauli_sum(codes, coeffs)
    assert rel(h.to_dense(), oracle.pauli_sum_matrix(codes, coeffs)) < 1e-14
    h.scale(-2.5)
    assert rel(h.to_dense(), -2.5 * oracle.pauli_sum_matrix(codes, coeffs)) < 1e-14


def test_get_entries_and_copy(ht):
    rng = synth.make_rng(4)
    n, m = 6, 2
    H = synth.random_hermitian_dense(n, rng)
    h = make(ht, n, m, H)
    r = rng.integers(0, 1 << n, size=500)
    c = rng.integers(0, 1 << n, size=500)
    assert np.array_equal(h.get_entries(r, c), lower_hermitian(H)[r, c])
    h2 = make(ht, n, m).copy_from(h)
    assert np.array_equal(h2.to_dense(), h.to_dense())


# ----------------------------------------------------------- single ops


def _check_op(ht, n, m, targets, kraus, picture, rng, dtype="c128"):
    H = synth.random_hermitian_dense(n, rng)
    h = make(ht, n, m, H)
    if kraus.shape[0] == 1 and rng.random() < 0.5:
        h.apply_unitary(targets, kraus[0], picture)
    else:
        h.apply_channel(targets, kraus, picture)
    ref = (oracle.kraus_map_adjoint if picture else oracle.kraus_map)(H, kraus, targets)
    e = rel(h.to_dense(), ref)
    assert e <= TOL, (n, m, targets, kraus.shape[0], picture, e)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_single_qubit_ops_every_position(ht, m):
    rng = synth.make_rng(100 + m)
    for n in (1, 2, 4, 6, 8):
        for a in range(n):
            for picture in (0, 1):
                _check_op(ht, n, m, [a], synth.haar_unitary(2, rng)[None], picture, rng)
                _check_op(ht, n, m, [a], synth.random_kraus_set(1, 4, rng), picture, rng)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_two_qubit_ops_every_ordered_pair(ht, m):
    rng = synth.make_rng(200 + m)
    for n in (2, 3, 5, 7):
        for a, b in itertools.permutations(range(n), 2):
            picture = int(rng.integers(2))
            _check_op(ht, n, m, [a, b], synth.haar_unitary(4, rng)[None], picture, rng)
            _check_op(ht, n, m, [a, b], synth.random_kraus_set(2, int(rng.integers(2, 17)), rng),
                      picture, rng)


def test_complex_nonsymmetric_channels(ht):
    """The transfer-matrix order only shows with complex non-symmetric Kraus
    operators."""
    rng = synth.make_rng(300)
    S, T = synth.named_gate("S"), synth.named_gate("T")
    ry = synth.named_gate("RY", 0.7) @ synth.named_gate("RZ", 0.3)
    kr = np.stack([np.sqrt(0.5) * S, np.sqrt(0.3) * T, np.sqrt(0.2) * ry])
    for m in (2, 5):
        for a in range(8):
            _check_op(ht, 8, m, [a], kr, 0, rng)


def test_work_orders_give_bitwise_equal_results(ht):
    """Whole groups per wave (order 0) and group steps spread over waves
    (order 1, the default below one group per wave) update the same blocks
    with the same arithmetic: bitwise equal storage, generic and native
    passes, every class.  So do grids of 1, 2 and 8 workgroups per CU and
    the automatic choice."""
    rng = synth.make_rng(470)
    n = 9
    H = synth.random_hermitian_dense(n, rng)
    ops = []
    for _ in range(30):
        k = int(rng.integers(1, 3))
        t = [int(x) for x in rng.choice(n, k, replace=False)]
        c = rng.random()
        mats = (synth.haar_unitary(1 << k, rng)[None] if c < 0.4 else
                synth.random_kraus_set(k, 2, rng) if c < 0.7 else
                (synth.cnot_matrix() if k == 2 else synth.named_gate("T"))[None])
        ops.append((t, mats))
    ops.append(([1, 7, 4], synth.permutation_gate("TOFFOLI")[None]))
    ht.set_tuning("native", 2)
    try:
        for m in (3, 5):
            out = []
            for order, wg in ((0, -1), (1, -1), (0, 1), (1, 2), (0, 8)):
                ht.set_tuning("conj_order", order)
                ht.set_tuning("conj_wg_per_cu", wg)
                h = make(ht, n, m, H)
                for t, mats in ops:
                    h.apply_channel(t, mats)
                out.append(h.raw_entries())
                h.close()
            for i in range(1, len(out)):
                assert np.array_equal(out[0], out[i]), (m, i)
    finally:
        ht.set_tuning("conj_order", -1)
        ht.set_tuning("conj_wg_per_cu", -1)
        ht.set_tuning("native", 1)


STEP_TUNINGS = [
    # LDS-staged intra-tile pass: 64 and 128 KiB steps, with and without the prefetch
    {"stage": 1, "stage_threads": 256, "stage_pipe": 1},
    {"stage": 1, "stage_threads": 512, "stage_pipe": 1},
    {"stage": 1, "stage_threads": 256, "stage_pipe": 0},
    # ... every other 16 KiB granule per step
    {"stage": 1, "stage_threads": 512, "stage_pipe": 1, "stage_order": 1},
    {"stage": 1, "stage_threads": 256, "stage_pipe": 0, "stage_order": 1},
    {"stage": 1, "stage_threads": 256, "stage_pipe": 1, "stage_order": 1, "stage_grid": 8},
    # workgroup-wide steps, both patch orders, the three item orders
    {"sync_waves": 16, "sync_order": 0},
    {"sync_waves": 8, "sync_interleave": 0, "sync_order": 0},
    {"sync_waves": 4, "sync_interleave": 1, "sync_order": 0},
    {"sync_waves": 16, "sync_order": 1},
    {"sync_waves": 16, "sync_order": 2},
    {"sync_waves": 8, "sync_order": 2},
    {"sync_waves": 4, "sync_order": 1, "sync_interleave": 1},
    # complex64: the pair layout in workgroup steps (every group, every
    # fourth), and the block layout in steps
    {"sync_waves": 16, "sync_order": 3},
    {"sync_waves": 8, "sync_order": 3, "pair_jp2": 0},
    {"sync_waves": 16, "sync_order": 1, "pairs": 0},
    # complex64 pair passes with two tile-selecting targets in plain mode: one pair per step
    {"pair_jp2": 0},
    # steps with the next one prefetched, with and without the barrier
    {"pipe_waves": 4},
    {"pipe_waves": 4, "pipe_barrier": 0},
    {"pipe_waves": 8},
]
STEP_DEFAULTS = {"stage": -1, "stage_threads": 512, "stage_pipe": 1, "sync_waves": -1, "sync_interleave": -1,
                 "sync_order": -1, "stage_order": -1, "pairs": 1, "stage_grid": 0,
                 "pipe_waves": 0, "pipe_barrier": 1, "native": 1, "pair_jp2": 1}


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_step_kernels_give_bitwise_equal_results(ht, dtype):
    """The LDS-staged intra-tile pass, the workgroup-wide step kernels and
    the prefetching ones apply the same block arithmetic (Eq. (2) direct,
    Eq. (3) transfer) to the same blocks as the lane-patch kernel: bitwise
    equal storage for every class, at tile edges 8 (the staged pass's last
    step is then partial) and 32, against the lane-patch kernel (all of
    them off), and the result matches the oracle."""
    rng = synth.make_rng(471)
    n = 9
    H = synth.random_hermitian_dense(n, rng)
    ops = []
    for _ in range(24):
        k = int(rng.integers(1, 3))
        t = [int(x) for x in rng.choice(n, k, replace=False)]
        c = rng.random()
        mats = (synth.haar_unitary(1 << k, rng)[None] if c < 0.5 else synth.random_kraus_set(k, 2, rng))
        ops.append((t, mats))
    # every class at least once: intra (low and high bits), one and two tile-selecting targets
    ops += [([0], synth.haar_unitary(2, rng)[None]), ([2, 1], synth.haar_unitary(4, rng)[None]),
            ([4, 3], synth.random_kraus_set(2, 3, rng)), ([8], synth.haar_unitary(2, rng)[None]),
            ([6, 1], synth.haar_unitary(4, rng)[None]), ([8, 6], synth.haar_unitary(4, rng)[None]),
            ([7, 5], synth.random_kraus_set(2, 2, rng))]
    want = oracle.apply_ops(H, [synth.random_ops.channel_op(t, mats) for t, mats in ops])

    def run(tune, m):
        for k, v in STEP_DEFAULTS.items():
            ht.set_tuning(k, v)
        ht.set_tuning("native", 0)
        ht.set_tuning("stage", 0)
        ht.set_tuning("sync_waves", 0)
        for k, v in tune.items():
            ht.set_tuning(k, v)
        h = make(ht, n, m, H, dtype)
        for t, mats in ops:
            h.apply_channel(t, mats)
        raw, dense = h.raw_entries(), h.to_dense()
        h.close()
        return raw, dense

    try:
        for m in (3, 5):
            base, dense = run({}, m)
            tol = 1e-12 if dtype == "c128" else 4e-5
            assert rel(dense, want) <= tol, (m, rel(dense, want))
            for tune in STEP_TUNINGS:
                raw, _ = run(tune, m)
                assert np.array_equal(base, raw), (m, tune)
    finally:
        for k, v in STEP_DEFAULTS.items():
            ht.set_tuning(k, v)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_every_pass_shape_gives_bitwise_equal_results(ht, dtype):
    """Every launch shape the pass tuner can choose (ht_set_pass_shape,
    shapes 0-19: lane patches, staged steps in both orders, grids and
    workgroup sizes, workgroup steps in every item order and grid), set for
    every pass class it applies to, gives bitwise the lane-patch kernel's
    result on a sequence of one- and two-qubit unitaries and channels, at
    tile edges 8 (tile bits up to 5, both buckets of the highest
    tile-selecting target) and 32 (the complex64 pair layout applies)."""
    rng = synth.make_rng(473)
    n = 9
    H = synth.random_hermitian_dense(n, rng)
    ops = []
    for _ in range(24):
        k = int(rng.integers(1, 3))
        t = [int(x) for x in rng.choice(n, k, replace=False)]
        ops.append((t, synth.haar_unitary(1 << k, rng)[None] if rng.random() < 0.5
                    else synth.random_kraus_set(k, 2, rng)))
    f = ht.lib.ht_set_pass_shape
    dt = {"c128": 0, "c64": 1}[dtype]
    classes = [(k, c, form, low, far) for k in (1, 2) for c in range(k + 1) for form in (0, 1)
               for low in (0, 1) for far in (0, 1)]

    def run(m):
        g = make(ht, n, m, H, dtype)
        for t, mats in ops:
            g.apply_channel(t, mats)
        raw = g.raw_entries()
        g.close()
        return raw

    for m in (3, 5):
        try:
            base = run(m)  # no tuned shapes: the automatic choice
            for shape in range(len(ht.PASS_SHAPES)):
                applied = [cl for cl in classes if f(dt, n, m, *cl, shape) == 0]
                assert applied or shape == 0, (m, shape)
                raw = run(m)
                assert np.array_equal(base, raw), (dtype, m, ht.PASS_SHAPES[shape])
                for cl in applied:
                    f(dt, n, m, *cl, -1)
        finally:
            for cl in classes:
                f(dt, n, m, *cl, -1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pass_tuner_keeps_the_operator_and_the_results(ht, dtype):
    """ht_tune_passes times identity passes on the operator: the represented
    matrix is unchanged, every class gets a shape, and passes launched with
    the tuned shapes give bitwise the results of the lane-patch kernel."""
    rng = synth.make_rng(472)
    n, m = 9, 3
    H = synth.random_hermitian_dense(n, rng)
    h = make(ht, n, m, H, dtype)
    before = h.to_dense()
    rows = h.tune_passes(1)
    assert np.array_equal(h.to_dense(), before)
    classes = {(r["k"], r["cross"], r["form"], r["low_intra"]) for r in rows}
    # k = 1 and 2, 0-2 tile-selecting targets, both forms; m = 3 has no intra target at bit 3
    assert (1, 0, "direct", True) in classes and (1, 1, "transfer", False) in classes
    assert (2, 2, "direct", False) in classes and (2, 1, "transfer", True) in classes
    assert all(r["ms"] > 0 and r["lane_ms"] > 0 for r in rows)
    # tile bits 0..5: both buckets of the highest tile-selecting target
    assert {(r["cross"], r["far"]) for r in rows if r["k"] == 1} >= {(1, False), (1, True)}
    assert all(r["shape"] in ht.PASS_SHAPES for r in rows)
    h.close()
    ops = []
    for _ in range(20):
        k = int(rng.integers(1, 3))
        t = [int(x) for x in rng.choice(n, k, replace=False)]
        ops.append((t, synth.haar_unitary(1 << k, rng)[None] if rng.random() < 0.5
                    else synth.random_kraus_set(k, 2, rng)))
    out = []
    for tune in ({}, {"stage": 0, "sync_waves": 0}):
        for key, v in tune.items():
            ht.set_tuning(key, v)
        try:
            g = make(ht, n, m, H, dtype)
            for t, mats in ops:
                g.apply_channel(t, mats)
            out.append(g.raw_entries())
            g.close()
        finally:
            for key in tune:
                ht.set_tuning(key, -1)
    assert np.array_equal(out[0], out[1])


def test_native_gate_exactness(ht):
    """X twice is the identity bitwise; CNOT leaves the control-0 quarter
    bitwise unchanged; S leaves entries with equal target bits unchanged."""
    rng = synth.make_rng(301)
    n, m = 8, 3
    H = synth.random_hermitian_dense(n, rng)
    h = make(ht, n, m, H)
    X = synth.named_gate("X")
    for a in range(n):
        h.apply_unitary([a], X)
        h.apply_unitary([a], X)
    assert np.array_equal(h.to_dense(), lower_hermitian(H))
    N = 1 << n
    idx = np.arange(N)
    for c, t in ((1, 6), (6, 1), (0, 2), (4, 7)):
        h.init_dense(H)
        h.apply_unitary([c, t], synth.cnot_matrix())
        zero = ((idx >> c) & 1) == 0
        assert np.array_equal(h.to_dense()[np.ix_(zero, zero)], lower_hermitian(H)[np.ix_(zero, zero)])
    for a in (0, 5):
        h.init_dense(H)
        h.apply_unitary([a], synth.named_gate("S"))
        same = (((idx[:, None] ^ idx[None, :]) >> a) & 1) == 0
        assert np.array_equal(h.to_dense()[same], lower_hermitian(H)[same])


# --------------------------------------------------------------- circuits


def test_plain_n8_circuit(ht):
    """200 random ops at n = 8 (Ginibre state), whole circuit vs the dense
    oracle, plus the reductions."""
    G, ops = synth.circuit_plain_n8(seed=1234)
    rho0 = oracle.density_from_factor(G)
    for m in (3, 5):
        h = ht.Herm(8, m)
        h.init_lowrank(G)
        h.scale(1.0 / h.trace())
        for op in ops:
            h.apply_op(op)
        ref = oracle.apply_ops(rho0, ops)
        assert rel(h.to_dense(), ref) <= TOL
        assert abs(h.trace() - oracle.trace(ref)) < 1e-13
        # the stored upper halves of diagonal tiles (Section III-B keeps all
        # M^2 entries; Subroutine 4 writes them) match the conjugated lower ones
        assert layout.diagonal_tile_asymmetry(h.raw_entries(), 8, h.tile_log2) <= 1e-14


def test_sweep_circuit_and_heisenberg_duality(ht):
    """Every op class on every position (n = 10), then the same circuit in the
    Heisenberg picture on a Pauli-sum observable: tr(O Phi(rho)) computed both
    ways on the GPU agrees with the oracle."""
    n, m = 10, 3
    G, ops, (codes, coeffs) = synth.circuit_sweep(n=n, seed=77)
    rho0 = oracle.density_from_factor(G)
    rho = ht.Herm(n, m)
    rho.init_lowrank(G)
    rho.scale(1.0 / rho.trace())
    for op in ops:
        rho.apply_op(op)
    ref = oracle.apply_ops_local(rho0, ops)
    assert rel(rho.to_dense(), ref) <= TOL
    assert layout.diagonal_tile_asymmetry(rho.raw_entries(), n, m) <= 1e-14
    O = ht.Herm(n, m).init_pauli_sum(codes, coeffs)
    for op in reversed(ops):
        O.apply_op(op, ht.HEISENBERG)
    O_ref = oracle.apply_ops_local(oracle.pauli_sum_matrix(codes, coeffs), list(reversed(ops)), adjoint=True)
    assert rel(O.to_dense(), O_ref) <= TOL
    assert layout.diagonal_tile_asymmetry(O.raw_entries(), n, m) <= 1e-14
    rho_init = ht.Herm(n, m)
    rho_init.init_lowrank(G)
    rho_init.scale(1.0 / rho_init.trace())
    want = oracle.pauli_sum_expectation(ref, codes, coeffs)
    got_s = rho.expectation_pauli_sum(codes, coeffs)
    got_h = O.expectation(rho_init)
    assert abs(got_s - want) < 1e-12 * max(1.0, abs(want))
    assert abs(got_h - want) < 1e-12 * max(1.0, abs(want))


# ------------------------------------------------------------- reductions


def test_reductions_against_oracle(ht):
    rng = synth.make_rng(400)
    for n, m in ((3, 5), (6, 2), (9, 4)):
        A = synth.random_hermitian_dense(n, rng)
        B = synth.random_hermitian_dense(n, rng)
        a, b = make(ht, n, m, A), make(ht, n, m, B)
        assert abs(a.trace() - oracle.trace(A)) < 1e-12 * (1 << n)
        assert abs(a.expectation(b) - oracle.expectation(A, B)) < 1e-12 * np.linalg.norm(A) * np.linalg.norm(B)
        codes, coeffs = synth.random_pauli_sum(n, 30, rng)
        want = oracle.pauli_sum_expectation(A, codes, coeffs)
        assert abs(a.expectation_pauli_sum(codes, coeffs) - want) < 1e-12 * np.linalg.norm(A) * np.abs(coeffs).sum()
        # deterministic: identical bits on repetition
        assert a.trace() == a.trace() and a.expectation(b) == a.expectation(b)


# ------------------------------------------------------------- errors


def test_invalid_arguments_leave_state_untouched(ht):
    rng = synth.make_rng(500)
    n, m = 5, 2
    H = synth.random_hermitian_dense(n, rng)
    h = make(ht, n, m, H)
    U = synth.haar_unitary(2, rng)
    for t in ([5], [-1]):
        with pytest.raises(ht.HermError):
            h.apply_unitary(t, U)
    with pytest.raises(ht.HermError):
        h.apply_unitary([1, 1], synth.haar_unitary(4, rng))
    with pytest.raises(ht.HermError):
        h.apply_channel([0], np.stack([U] * 5))
    with pytest.raises(ht.HermError):
        h.expectation(make(ht, 6, 2))
    assert np.array_equal(h.to_dense(), lower_hermitian(H))


def test_error_paths_through_the_c_abi(ht):
    """Every argument error of create, init, apply and the reductions returns
    its status code through the C ABI and leaves the storage bitwise as it
    was (HT_EINVAL = 1, HT_ENOMEM = 2)."""
    import ctypes

    lib = ht.lib
    EINVAL, ENOMEM = 1, 2
    out = ctypes.c_void_p()
    for n, m in ((5, 0), (5, 9), (0, 5), (19, 5), (-1, 3)):
        assert lib.ht_herm_create(n, m, 0, None, 0, None, ctypes.byref(out)) == EINVAL, (n, m)
        assert out.value is None
    assert lib.ht_herm_create(5, 2, 2, None, 0, None, ctypes.byref(out)) == EINVAL   # dtype
    assert lib.ht_herm_create(5, 2, 0, None, 0, None, None) == EINVAL                # out NULL
    need = ht.storage_bytes(5, 2)
    raw = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    base = (raw.data_ptr() + 255) // 256 * 256
    assert lib.ht_herm_create(5, 2, 0, ctypes.c_void_p(base + 16), need, None, ctypes.byref(out)) == EINVAL
    assert lib.ht_herm_create(5, 2, 0, ctypes.c_void_p(base), need - 1, None, ctypes.byref(out)) == ENOMEM
    assert out.value is None
    assert lib.ht_herm_create(5, 2, 0, ctypes.c_void_p(base), need, None, ctypes.byref(out)) == 0
    assert lib.ht_herm_destroy(out) == 0

    rng = synth.make_rng(501)
    n, m = 5, 2
    H = synth.random_hermitian_dense(n, rng)
    a = make(ht, n, m, H)
    b64 = make(ht, n, m, H, dtype="c64")
    b3 = make(ht, n, 3, H)
    before = [x.read_raw() for x in (a, b64, b3)]
    res = ctypes.c_double(12345.0)
    for other in (b64, b3, make(ht, 6, m)):
        assert lib.ht_expectation(a.handle, other.handle, ctypes.byref(res)) == EINVAL
    assert lib.ht_expectation(a.handle, a.handle, None) == EINVAL
    assert lib.ht_expectation(None, a.handle, ctypes.byref(res)) == EINVAL
    assert lib.ht_trace(a.handle, None) == EINVAL
    assert lib.ht_trace(None, ctypes.byref(res)) == EINVAL
    assert res.value == 12345.0
    codes = np.zeros((2, n), np.uint8)
    coeffs = np.ones(2)
    P = lambda x: ctypes.c_void_p(x.ctypes.data)
    for nt in (0, 4097):
        assert lib.ht_expectation_pauli_sum(a.handle, nt, P(codes), P(coeffs), ctypes.byref(res)) == EINVAL
    assert lib.ht_expectation_pauli_sum(a.handle, 2, None, P(coeffs), ctypes.byref(res)) == EINVAL
    assert lib.ht_expectation_pauli_sum(a.handle, 2, P(codes), None, ctypes.byref(res)) == EINVAL
    assert lib.ht_expectation_pauli_sum(a.handle, 2, P(codes), P(coeffs), None) == EINVAL
    bad_codes = codes.copy()
    bad_codes[1, 3] = 4
    assert lib.ht_expectation_pauli_sum(a.handle, 2, P(bad_codes), P(coeffs), ctypes.byref(res)) == EINVAL
    assert lib.ht_herm_init_pauli_sum(a.handle, 2, P(bad_codes), P(coeffs)) == EINVAL
    assert lib.ht_herm_init_pauli_sum(a.handle, 0, P(codes), P(coeffs)) == EINVAL
    G = synth.ginibre_factor(n, 2, rng)
    for rank in (0, 4097):
        assert lib.ht_herm_init_lowrank(a.handle, P(G), rank, 0) == EINVAL
    assert lib.ht_herm_init_lowrank(a.handle, None, 2, 0) == EINVAL
    D = np.ascontiguousarray(H)
    assert lib.ht_herm_init_dense(a.handle, P(D), (1 << n) - 1, 0) == EINVAL
    assert lib.ht_herm_init_dense(a.handle, None, 1 << n, 0) == EINVAL
    U = np.ascontiguousarray(synth.haar_unitary(4, rng))
    t = np.array([0, 3, 4], np.int32)
    for k in (0, 4):
        assert lib.ht_apply_unitary(a.handle, k, P(t), P(U), 0) == EINVAL
    assert lib.ht_apply_unitary(a.handle, 2, None, P(U), 0) == EINVAL
    assert lib.ht_apply_unitary(a.handle, 2, P(t), None, 0) == EINVAL
    assert lib.ht_apply_unitary(a.handle, 2, P(t), P(U), 2) == EINVAL                 # picture
    assert lib.ht_apply_channel(a.handle, 2, P(t), 0, P(U), 0) == EINVAL               # r = 0
    assert lib.ht_apply_channel(a.handle, 2, P(t), 17, P(U), 0) == EINVAL              # r > 4^k
    assert lib.ht_apply_unitary(None, 2, P(t), P(U), 0) == EINVAL
    assert lib.ht_scale(None, 2.0) == EINVAL
    assert lib.ht_herm_init_zero(None) == EINVAL
    assert lib.ht_herm_init_identity(None, 1.0) == EINVAL
    assert lib.ht_last_error()  # a message was recorded
    after = [x.read_raw() for x in (a, b64, b3)]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert np.array_equal(a.to_dense(), lower_hermitian(H))


def test_borrowed_buffer_survives_destroy(ht):
    h = ht.Herm(6, 3)
    buf = h.buffer
    h.init_identity(1.0)
    h.close()
    buf.fill_(7)
    torch.cuda.synchronize()
    assert int(buf[0].item()) == 7


# --------------------------------------------------------- full sizes


def _sampled_op_check(h, op, picture, n, rng, nblocks=1500):
    """Blocks drawn with at least 120 in diagonal tile groups and 120 in the
    last tile row (tests/sampling.py), the rest uniform."""
    R, C, d = sampling.block_entries(n, op.targets, h.tile_log2, nblocks, rng)
    ndiag, nlast = sampling.strata_counts(n, op.targets, h.tile_log2, R, C, d)
    assert ndiag >= 100 and nlast >= 100, (ndiag, nlast)
    before = h.get_entries(R, C).reshape(nblocks, d, d)
    h.apply_op(op, picture)
    after = h.get_entries(R, C).reshape(nblocks, d, d)
    want = oracle.block_update(before, op.mats, adjoint=bool(picture))
    return rel(after, want)


@pytest.mark.parametrize("n,dtype", [(14, "c128"), (16, "c128"), (16, "c64")])
def test_full_size_sampled_blocks(ht, n, dtype):
    """Full-size operators (n = 14: 2.15 GB, n = 16: 34.4 GB of c128 tiles or
    17.2 GB of c64, tile edge 32, the benchmark's launch configuration):
    every op class at intra and cross positions, checked on 1500 sampled
    blocks per op, plus trace preservation over the whole operator.  In
    complex64 the extra ops take the pair layout in both of its memory modes
    (nontemporal, and plain where the highest target is at n - 3 or above);
    each result lies within one float rounding of the FP64 map of its
    stored input."""
    rng = synth.make_rng(900 + n + (7 if dtype == "c64" else 0))
    G = synth.ginibre_factor(n, 16, rng)
    h = ht.Herm(n, 5, dtype)
    h.init_lowrank(G)
    h.scale(1.0 / h.trace())
    ops = [
        synth.random_ops.unitary_op([2], synth.haar_unitary(2, rng)),                 # k=1 c=0
        synth.random_ops.unitary_op([n - 1], synth.haar_unitary(2, rng)),             # k=1 c=1 (top)
        synth.random_ops.unitary_op([5], synth.haar_unitary(2, rng)),                 # k=1 c=1 (lowest cross)
        synth.random_ops.channel_op([9], synth.depolarising_kraus(0.07)),
        synth.random_ops.channel_op([3], synth.amplitude_damping_kraus(0.05)),
        synth.random_ops.unitary_op([1, 3], synth.haar_unitary(4, rng)),             # k=2 c=0
        synth.random_ops.unitary_op([4, 5], synth.haar_unitary(4, rng)),             # k=2 c=1
        synth.random_ops.unitary_op([n - 1, 6], synth.haar_unitary(4, rng)),         # k=2 c=2
        synth.random_ops.channel_op([7, 12], synth.random_kraus_set(2, 3, rng)),     # k=2 c=2 transfer
        synth.random_ops.channel_op([1, 3], synth.random_kraus_set(2, 3, rng)),      # k=2 c=0 transfer (staged)
        synth.random_ops.unitary_op([0, n - 2], synth.cnot_matrix()),                # k=2 c=1
    ]
    if dtype == "c64":
        ops += [
            synth.random_ops.unitary_op([4], synth.haar_unitary(2, rng)),             # pairs, intra bit 4
            synth.random_ops.channel_op([10], synth.amplitude_damping_kraus(0.05)),   # pairs, transfer
            synth.random_ops.unitary_op([n - 2], synth.haar_unitary(2, rng)),         # pairs, plain
            synth.random_ops.unitary_op([9, 10], synth.haar_unitary(4, rng)),         # k=2 pairs
            synth.random_ops.unitary_op([n - 1, n - 2], synth.haar_unitary(4, rng)),  # k=2 pairs, plain
            synth.random_ops.unitary_op([10, 4], synth.haar_unitary(4, rng)),         # k=2 pairs, intra 4
        ]
    tol = TOL if dtype == "c128" else 2 * C64_EPS
    for i, op in enumerate(ops):
        pic = i % 2 if op.kind == "unitary" else 0
        e = _sampled_op_check(h, op, pic, n, rng)
        assert e <= tol, (op.label, op.targets, e)
    assert abs(h.trace() - 1.0) < (1e-12 if dtype == "c128" else 1e-6)
    h.close()


def test_largest_operator(ht):
    """The largest c128 operator that fits one MI355X: n = 17 (131072 x 131072,
    137.5 GB of tiles, element offsets beyond 2^32), with ops whose targets
    select the farthest tiles, on sampled blocks, plus the trace."""
    n = 17
    free, _ = torch.cuda.mem_get_info()
    if free < ht.storage_bytes(n, 5) + (8 << 30):
        pytest.skip("needs about 146 GB of free device memory")
    rng = synth.make_rng(917)
    h = ht.Herm(n, 5)
    h.init_lowrank(synth.ginibre_factor(n, 8, rng))
    h.scale(1.0 / h.trace())
    assert h.nbytes == 137_472_507_904
    ops = [synth.random_ops.unitary_op([n - 1], synth.haar_unitary(2, rng)),
           synth.random_ops.channel_op([n - 2, 0], synth.random_kraus_set(2, 2, rng)),
           synth.random_ops.unitary_op([n - 1, n - 3], synth.cnot_matrix())]
    for i, op in enumerate(ops):
        e = _sampled_op_check(h, op, i % 2 if op.kind == "unitary" else 0, n, rng, nblocks=800)
        assert e <= TOL, (op.targets, e)
    assert abs(h.trace() - 1.0) < 1e-12
    h.close()
    torch.cuda.empty_cache()


def test_largest_c64_operator(ht):
    """The largest operator one MI355X holds: n = 18 in complex64 storage
    (262144 x 262144, 274.9 GB of tiles, element offsets beyond 2^34), with a
    tile-selecting unitary, a channel across the farthest tiles and a native
    CNOT, each within one float rounding on sampled blocks, plus the trace."""
    n = 18
    torch.cuda.empty_cache()
    need = ht.storage_bytes(n, 5, "c64")
    free, _ = torch.cuda.mem_get_info()
    if free < need + (6 << 30):
        pytest.skip(f"needs about {(need >> 30) + 6} GiB of free device memory")
    rng = synth.make_rng(918)
    h = ht.Herm(n, 5, "c64")
    assert h.nbytes == need == 274_911_461_376
    h.init_lowrank(synth.ginibre_factor(n, 8, rng))
    h.scale(1.0 / h.trace())
    ops = [synth.random_ops.unitary_op([n - 1], synth.haar_unitary(2, rng)),
           synth.random_ops.channel_op([n - 2, 0], synth.random_kraus_set(2, 2, rng)),
           synth.random_ops.unitary_op([n - 1, n - 3], synth.cnot_matrix())]
    for i, op in enumerate(ops):
        e = _sampled_op_check(h, op, i % 2 if op.kind == "unitary" else 0, n, rng, nblocks=800)
        assert e <= 2 * C64_EPS, (op.targets, e)
    assert abs(h.trace() - 1.0) < 1e-6
    h.close()
    torch.cuda.empty_cache()


# ------------------------------------------------------------- complex64

C64_EPS = 2.0 ** -24  # unit roundoff of float32 (round to nearest)


def quantise_c64(H):
    return H.astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("m", [2, 5])
def test_c64_single_ops_within_one_rounding(ht, m):
    """complex64 storage, FP64 arithmetic: one pass rounds each FP64 result
    to float32 once, so against the oracle applied to the same stored input
    the relative Frobenius error is at most 2^-24 (checked with margin 2)."""
    rng = synth.make_rng(700 + m)
    n = 7
    for targets in ([0], [4], [6], [1, 2], [5, 1], [3, 6], [6, 5]):
        k = len(targets)
        for kraus in (synth.haar_unitary(1 << k, rng)[None], synth.random_kraus_set(k, 3, rng)):
            H = synth.random_hermitian_dense(n, rng)
            h = make(ht, n, m, H, dtype="c64")
            Hq = lower_hermitian(quantise_c64(H))
            assert np.array_equal(h.to_dense(), Hq)
            h.apply_channel(targets, kraus)
            e = rel(h.to_dense(), oracle.kraus_map(Hq, kraus, targets))
            assert e <= 2 * C64_EPS, (targets, kraus.shape[0], e)


def test_c64_pair_layout_is_bitwise_equal_to_the_block_layout(ht):
    """The pair layout of complex64 passes (two blocks in adjacent columns
    per lane, 16-byte accesses) applies the same FP64 arithmetic to every
    block as the block layout: bitwise equal storage for every target set
    it applies to (one-qubit unitaries and channels, two-qubit unitaries),
    both work orders, both pictures, both memory modes of the automatic
    choice (targets at n - 3 and above, and below), and within one rounding
    of the oracle."""
    rng = synth.make_rng(720)
    n = 9
    H = synth.random_hermitian_dense(n, rng)
    Hq = lower_hermitian(quantise_c64(H))
    cases = []
    for a in range(1, n):
        cases += [([a], synth.haar_unitary(2, rng)[None]), ([a], synth.random_kraus_set(1, 3, rng))]
    for a, b in ([5, 6], [8, 7], [6, 8], [1, 7], [4, 8], [7, 2], [3, 6], [8, 5]):
        cases.append(([a, b], synth.haar_unitary(4, rng)[None]))
    try:
        for m in (5, 6, 7, 8):
            for i, (targets, kraus) in enumerate(cases):
                pic = (i + m) % 2
                out = []
                for pairs, order in ((0, 0), (2, 0), (2, 1)):
                    ht.set_tuning("pairs", pairs)
                    ht.set_tuning("conj_order", order)
                    h = make(ht, n, m, H, dtype="c64")
                    h.apply_channel(targets, kraus, pic)
                    out.append((h.raw_entries(), h.to_dense()))
                    h.close()
                assert np.array_equal(out[0][0], out[1][0]), (m, targets, pic)
                assert np.array_equal(out[0][0], out[2][0]), (m, targets, pic)
                ref = (oracle.kraus_map_adjoint if pic else oracle.kraus_map)(Hq, kraus, targets)
                e = rel(out[1][1], ref)
                assert e <= 2 * C64_EPS, (m, targets, pic, e)
    finally:
        ht.set_tuning("pairs", 1)
        ht.set_tuning("conj_order", -1)


def test_c64_circuit_error_bound_and_fp64_reductions(ht):
    """The n = 8 circuit in complex64 storage: error vs the FP64 oracle stays
    within (passes + 1) * 2^-24 relative (one rounding per pass plus the
    input), and trace / Pauli-sum reductions accumulate in FP64."""
    G, ops = synth.circuit_plain_n8(seed=1234)
    rho0 = oracle.density_from_factor(G)
    h = ht.Herm(8, 5, "c64")
    h.init_lowrank(G)
    h.scale(1.0 / h.trace())
    for op in ops:
        h.apply_op(op)
    ref = oracle.apply_ops(rho0, ops)
    e = rel(h.to_dense(), ref)
    assert e <= (len(ops) + 1) * C64_EPS, e
    # reductions of the stored (float) entries are exact to FP64 rounding
    D = h.to_dense()
    assert abs(h.trace() - float(np.real(np.trace(D)))) < 1e-13
    codes, coeffs = synth.random_pauli_sum(8, 32, synth.make_rng(5))
    assert abs(h.expectation_pauli_sum(codes, coeffs) - oracle.pauli_sum_expectation(D, codes, coeffs)) < 1e-12
