"""The conjugation pass's per-lane body, run on the CPU, against the oracle.

``_hostcheck.so`` compiles the same ``conj_group_lane`` the GPU kernel runs (from
csrc/ht_geom.h) for the host and drives it over every group, patch and lane
of a pass with a memory policy that rejects out-of-range accesses and counts
writes.  These tests establish, before anything runs on a GPU, that every
pass stays inside the storage, writes every stored entry exactly once, and
computes the oracle's result (decoded with the oracle's own model of the
tiled layout) -- for all tile edges, qubit positions, target orders, Kraus
ranks and both pictures at small n.
"""

import ctypes
import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from tests.native_masks import changing_entries, expected_writes
from oracle import layout

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(os.path.dirname(HERE), "paper_2604_15765_amd", "_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(SO):
        pytest.skip("_hostcheck.so not built")
    lib = ctypes.CDLL(SO)
    f = lib.htc_emulate_conj
    vp = ctypes.c_void_p
    f.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp,
                  ctypes.c_int, vp, vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_char_p, ctypes.c_size_t]
    f.restype = ctypes.c_int
    return f


def emulate(f, raw, n, m, targets, kraus, heis, order=0, native=0, want_form=False, ilv=0, pairs=0):
    """Run one pass on the CPU.  native=0 keeps the generic forms (direct,
    transfer); native=1 lets permutation-and-phase ops take the native pass;
    ilv=1 the alternating patch order; pairs=1 the pair layout of complex64
    one-qubit passes (indexing checked on complex128 storage)."""
    raw = np.ascontiguousarray(raw, dtype=np.complex128).copy()
    kraus = np.ascontiguousarray(kraus, dtype=np.complex128)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    wc = np.zeros(raw.size, dtype=np.int32)
    lanes = ctypes.c_uint64()
    form = ctypes.c_int(-1)
    err = ctypes.create_string_buffer(256)
    rc = f(raw.ctypes.data, raw.size, n, m, len(targets), t.ctypes.data, kraus.shape[0], kraus.ctypes.data,
           int(heis), wc.ctypes.data, None, ctypes.byref(lanes), order, native, ilv, pairs, ctypes.byref(form),
           err, 256)
    assert rc == 0, err.value.decode()
    if want_form:
        return raw, wc, form.value
    return raw, wc


def reference(H, kraus, targets, heis):
    return (oracle.kraus_map_adjoint if heis else oracle.kraus_map)(H, kraus, targets)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check(f, n, m, targets, kraus, heis, rng):
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    order = int(rng.integers(2))  # both work orders of the kernel
    ilv = int(rng.integers(2))    # both patch orders
    pairs = int(rng.integers(2))  # both layouts of complex64 one-qubit passes
    out, wc = emulate(f, raw, n, m, targets, kraus, heis, order, ilv=ilv, pairs=pairs)
    assert np.all(wc == 1), f"write counts {np.unique(wc)} for n={n} m={m} t={targets}"
    got = layout.decode(out, n, m)
    ref = reference(H, kraus, targets, heis)
    e = rel(got, ref)
    assert e < 1e-13, (n, m, targets, kraus.shape[0], heis, e)
    return out


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_single_qubit_every_position(hc, m):
    rng = synth.make_rng(100 + m)
    for n in range(1, 7):
        for a in range(n):
            for heis in (False, True):
                check(hc, n, m, [a], synth.haar_unitary(2, rng)[None], heis, rng)          # direct form
                check(hc, n, m, [a], synth.random_kraus_set(1, 3, rng), heis, rng)        # transfer form


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_two_qubit_every_ordered_pair(hc, m):
    rng = synth.make_rng(200 + m)
    for n in range(2, 7):
        for a, b in itertools.permutations(range(n), 2):
            heis = bool(rng.integers(2))
            check(hc, n, m, [a, b], synth.haar_unitary(4, rng)[None], heis, rng)
            check(hc, n, m, [a, b], synth.random_kraus_set(2, 3, rng), heis, rng)


def test_complex_nonsymmetric_channel_orders(hc):
    """Transfer-matrix ordering is only visible with complex, non-symmetric
    Kraus operators (for real or depolarising sets both orders agree)."""
    rng = synth.make_rng(300)
    S, T = synth.named_gate("S"), synth.named_gate("T")
    ry = synth.named_gate("RY", 0.7) @ synth.named_gate("RZ", 0.3)
    kr = np.stack([np.sqrt(0.5) * S, np.sqrt(0.3) * T, np.sqrt(0.2) * ry])
    for m in (1, 2, 3):
        for a in range(5):
            check(hc, 5, m, [a], kr, False, rng)


def test_large_tile_edges_and_single_tile(hc):
    rng = synth.make_rng(400)
    for n, m in ((7, 6), (7, 7), (8, 8), (3, 8), (6, 3)):
        for t in ([0], [n - 1], [0, n - 1], [n - 1, 1 % n] if n > 1 else [0]):
            if len(set(t)) != len(t):
                continue
            check(hc, n, m, t, synth.haar_unitary(1 << len(t), rng)[None], False, rng)


def test_diagonal_tile_halves_consistent_after_cross_op(hc):
    """After an op whose targets select tiles, the stored upper halves of the
    diagonal tiles are rewritten as conjugates of the lower ones."""
    rng = synth.make_rng(500)
    n, m = 6, 2
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    for t in ([4], [2, 5], [5, 3]):
        raw, _ = emulate(hc, raw, n, m, t, synth.haar_unitary(1 << len(t), rng)[None], False)
        assert layout.diagonal_tile_asymmetry(raw, n, m) < 1e-14


@pytest.mark.parametrize("native", [0, 1])
def test_pauli_x_twice_is_bitwise_identity(hc, native):
    rng = synth.make_rng(600)
    n, m = 6, 3
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    X = synth.named_gate("X")[None]
    for a in range(n):
        once, _ = emulate(hc, raw, n, m, [a], X, False, native=native)
        twice, _ = emulate(hc, once, n, m, [a], X, False, native=native)
        assert np.array_equal(twice, raw)


# ------------------------------------------------------ native pass (form 2)

def check_native(f, n, m, targets, kraus, heis, rng, order=None):
    """Native pass: form 2 unless k <= 2 and every entry changes (then the
    generic pass, which moves the same bytes); exactly the changing entries
    are written, once each, in either work order of the kernel."""
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    order = int(rng.integers(2)) if order is None else order
    out, wc, form = emulate(f, raw, n, m, targets, kraus, heis, order=order, native=1, want_form=True,
                            ilv=int(rng.integers(2)))
    changing = changing_entries(kraus, targets, heis)
    assert form == (2 if len(targets) == 3 or not changing.all() else (0 if kraus.shape[0] == 1 else 1)), \
        (targets, form)
    expect = expected_writes(n, m, targets, changing)
    assert np.array_equal(wc, expect), (n, m, targets, np.unique(wc - expect))
    ref = reference(H, kraus, targets, heis)
    e = rel(layout.decode(out, n, m), ref)
    assert e < 1e-13, (n, m, targets, heis, e)
    # untouched entries keep their bits; the rest agree with the generic pass
    assert np.array_equal(out[expect == 0], raw[expect == 0])
    if len(targets) < 3:
        gen, _ = emulate(f, raw, n, m, targets, kraus, heis, native=0)
        assert rel(layout.decode(gen, n, m), layout.decode(out, n, m)) < 1e-14


NAMED_1Q = ["X", "Y", "Z", "S", "T"]


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_native_single_qubit_gates_every_position(hc, m):
    rng = synth.make_rng(700 + m)
    gates = [synth.named_gate(g)[None] for g in NAMED_1Q]
    gates.append(synth.named_gate("RZ", 0.37)[None])
    gates.append(synth.dephasing_kraus(0.2))                 # diagonal Kraus set
    X, Y = synth.named_gate("X"), synth.named_gate("Y")
    gates.append(np.stack([np.sqrt(0.3) * X, np.sqrt(0.7) * (X @ synth.named_gate("S"))]))  # shared permutation
    for n in range(1, 7):
        for a in range(n):
            for g in gates:
                check_native(hc, n, m, [a], g, bool(rng.integers(2)), rng)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_native_two_qubit_gates_every_ordered_pair(hc, m):
    rng = synth.make_rng(800 + m)
    gates = [synth.cnot_matrix()[None]] + [synth.permutation_gate(g)[None] for g in ("CZ", "SWAP", "ISWAP")]
    for n in range(2, 7):
        for a, b in itertools.permutations(range(n), 2):
            for g in gates:
                check_native(hc, n, m, [a, b], g, bool(rng.integers(2)), rng)
            check_native(hc, n, m, [a, b], synth.random_monomial(2, rng)[None], bool(rng.integers(2)), rng)
            check_native(hc, n, m, [a, b], synth.random_monomial(2, rng, diagonal=True)[None], False, rng)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_native_three_qubit_gates(hc, m):
    """k = 3 (Toffoli, CCZ, Fredkin, random permutation-and-phase matrices,
    including permutations that are not involutions) on every ordered
    triple at n = 3..5 and a sample at n = 6, every count of tile-selecting
    targets."""
    rng = synth.make_rng(900 + m)
    gates = [synth.permutation_gate(g)[None] for g in ("TOFFOLI", "CCZ", "FREDKIN")]
    for n in range(3, 7):
        triples = list(itertools.permutations(range(n), 3))
        if n == 6:
            triples = [triples[i] for i in rng.choice(len(triples), 30, replace=False)]
        for t in triples:
            for g in gates:
                check_native(hc, n, m, list(t), g, bool(rng.integers(2)), rng)
            check_native(hc, n, m, list(t), synth.random_monomial(3, rng)[None], bool(rng.integers(2)), rng)


def test_native_split_work_order_at_the_benchmark_tile_edge(hc):
    """Tile edge 32, where a group has several steps of patches: the work
    order that spreads a group's steps over waves writes the same entries
    once each, for k = 1, 2, 3 and every count of tile-selecting targets."""
    rng = synth.make_rng(940)
    n, m = 7, 5
    cases = [([2], synth.named_gate("X")), ([6], synth.named_gate("T")), ([5], synth.named_gate("Y")),
             ([1, 3], synth.cnot_matrix()), ([6, 2], synth.cnot_matrix()), ([5, 6], synth.permutation_gate("CZ")),
             ([0, 4, 2], synth.permutation_gate("TOFFOLI")), ([6, 1, 3], synth.permutation_gate("FREDKIN")),
             ([5, 6, 0], synth.random_monomial(3, rng)), ([4, 5, 6], synth.permutation_gate("CCZ"))]
    for t, g in cases:
        check_native(hc, n, m, t, g[None], bool(rng.integers(2)), rng, order=1)


def test_native_policy_for_operators_beyond_the_cache(hc):
    """Under the size-based policy (native = 3 here) a k <= 2 op takes the
    native pass only where its fixed entries fill whole 128-byte lines:
    whether an entry changes is decided by targets at bit 3 or above (for
    diagonal ops also bit 2, or any bits when at most 3/8 of the entries
    change); k = 3 always.  Tile edge 32, so bits 5 and 6 select tiles."""
    rng = synth.make_rng(945)
    n, m = 7, 5
    Z, X = synth.named_gate("Z")[None], synth.named_gate("X")[None]
    cnot, cz, swap = (synth.cnot_matrix()[None], synth.permutation_gate("CZ")[None],
                      synth.permutation_gate("SWAP")[None])
    expect = [([0], Z, False), ([1], Z, False), ([2], Z, True), ([3], Z, True), ([6], Z, True),
              ([2], synth.dephasing_kraus(0.2), True), ([0], synth.dephasing_kraus(0.2), False),
              ([0, 1], cnot, False), ([1, 2], cnot, False), ([2, 3], cnot, False), ([3, 4], cnot, True),
              ([2, 6], cnot, False), ([6, 2], cnot, True), ([5, 6], cnot, True), ([0, 4], cnot, False),
              ([0, 1], cz, True), ([1, 2], cz, True), ([2, 6], cz, True),
              ([0, 1], swap, False), ([2, 3], swap, False), ([3, 4], swap, True), ([2, 6], swap, False),
              ([0], X, False), ([0, 1, 2], synth.permutation_gate("TOFFOLI")[None], True)]
    raw = layout.encode(synth.random_hermitian_dense(n, rng), m)
    for t, g, native in expect:
        out, wc, form = emulate(hc, raw, n, m, t, g, False, native=3, want_form=True)
        assert (form == 2) == native, (t, g.shape, form)
        ref = reference(layout.decode(raw, n, m), g, t, False)
        assert rel(layout.decode(out, n, m), ref) < 1e-13


def test_native_is_chosen_only_for_permutation_and_phase_ops(hc):
    rng = synth.make_rng(950)
    n, m = 4, 2
    raw = layout.encode(synth.random_hermitian_dense(n, rng), m)
    cases = [([1], synth.named_gate("H")[None]), ([0], synth.haar_unitary(2, rng)[None]),
             ([2], synth.amplitude_damping_kraus(0.1)), ([3], synth.depolarising_kraus(0.1)),
             ([0, 3], synth.haar_unitary(4, rng)[None])]
    for t, g in cases:
        _, _, form = emulate(hc, raw, n, m, t, g, False, native=1, want_form=True)
        assert form in (0, 1), (t, form)


# -------------------------------------- pair layout (complex64, k = 1, 2)

@pytest.mark.parametrize("m", [4, 5, 6, 7])
def test_pair_layout_covers_every_entry_once(hc, m):
    """The pair layout of complex64 one-qubit passes (two blocks in adjacent
    columns per lane, 16-byte accesses in stored tiles): every entry read and
    written once, 16-byte accesses aligned, results those of the block
    layout, for intra and tile-selecting targets, both forms, both pictures
    and both work orders (diagonal groups keep the block layout)."""
    rng = synth.make_rng(1300 + m)
    for n in (m + 1, m + 2):
        H = synth.random_hermitian_dense(n, rng)
        raw = layout.encode(H, m)
        for a in range(1, n):
            for kraus in (synth.haar_unitary(2, rng)[None], synth.random_kraus_set(1, 3, rng)):
                heis = bool(rng.integers(2))
                order = int(rng.integers(2))
                p, wp = emulate(hc, raw, n, m, [a], kraus, heis, order, pairs=1)
                b, _ = emulate(hc, raw, n, m, [a], kraus, heis, order, pairs=0)
                assert np.all(wp == 1), (n, m, a, np.unique(wp))
                assert np.array_equal(p, b), (n, m, a)


@pytest.mark.parametrize("m", [4, 5, 6])
def test_pair_layout_two_qubit_ops(hc, m):
    """The pair layout of complex64 two-qubit passes in the direct form (16
    entries per block, pairs held as loaded and transformed one block at a
    time): every entry read and written once, results those of the block
    layout, on every ordered pair of targets (the layout applies where both
    targets select tiles, or the intra one is above bit 0 and 4 free bits
    remain; channels take the block layout)."""
    rng = synth.make_rng(1400 + m)
    n = m + 2
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            kraus = synth.haar_unitary(4, rng)[None] if rng.random() < 0.8 else synth.random_kraus_set(2, 3, rng)
            heis = bool(rng.integers(2))
            order = int(rng.integers(2))
            p, wp = emulate(hc, raw, n, m, [a, b], kraus, heis, order, pairs=1)
            q, _ = emulate(hc, raw, n, m, [a, b], kraus, heis, order, pairs=0)
            assert np.all(wp == 1), (n, m, a, b, np.unique(wp))
            assert np.array_equal(p, q), (n, m, a, b)


@pytest.mark.parametrize("m", [4, 5])
def test_pair_step_kernel_split_covers_every_entry_once(hc, m):
    """The pair layout in workgroup-wide steps (pair_sync_kernel): the work
    split of its four item orders -- sync_item's (unit, wave) items minus
    the diagonal groups, then the diagonal groups in the block layout when a
    target selects tiles (pair_diag_kernel) -- writes every stored entry
    exactly once and gives bitwise the block layout's result, for one-qubit
    ops at every position (unitaries and channels, both pictures) and
    two-qubit unitaries on a sample of ordered pairs, intra and
    tile-selecting."""
    rng = synth.make_rng(1450 + m)
    for n in (m + 1, m + 3):
        H = synth.random_hermitian_dense(n, rng)
        raw = layout.encode(H, m)
        cases = [([a], synth.haar_unitary(2, rng)[None]) for a in range(1, n)]
        cases += [([a], synth.random_kraus_set(1, 3, rng)) for a in range(1, n, 2)]
        pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
        for i in rng.choice(len(pairs), 8, replace=False):
            cases.append((list(pairs[i]), synth.haar_unitary(4, rng)[None]))
        for targets, kraus in cases:
            heis = bool(rng.integers(2))
            want, _ = emulate(hc, raw, n, m, targets, kraus, heis, 0, pairs=0)
            for order in (2, 3, 4, 5):
                got, wc = emulate(hc, raw, n, m, targets, kraus, heis, order, pairs=1)
                assert np.all(wc == 1), (n, m, targets, order, np.unique(wc))
                assert np.array_equal(got, want), (n, m, targets, order)


# ----------------------------------------------- k = 3 Kraus form (form 3)

def check_k3(f, n, m, targets, kraus, heis, rng, native=0):
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    out, wc, form = emulate(f, raw, n, m, targets, kraus, heis, native=native, want_form=True)
    assert form == 3, (targets, form)
    assert np.all(wc == 1), (n, m, targets, np.unique(wc))
    e = rel(layout.decode(out, n, m), reference(H, kraus, targets, heis))
    assert e < 1e-13, (n, m, targets, kraus.shape[0], heis, e)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_k3_kraus_form_every_triple(hc, m):
    """General three-qubit unitaries and channels (8 lanes per block, the
    LDS exchange emulated phase by phase) on every ordered triple at
    n = 3..5 and a sample at n = 6, 7: every stored entry written once,
    results vs the oracle, both pictures, every count of tile-selecting
    targets."""
    rng = synth.make_rng(1100 + m)
    for n in range(3, 8):
        triples = list(itertools.permutations(range(n), 3))
        if n >= 6:
            triples = [triples[i] for i in rng.choice(len(triples), 12, replace=False)]
        for t in triples:
            heis = bool(rng.integers(2))
            check_k3(hc, n, m, list(t), synth.haar_unitary(8, rng)[None], heis, rng)
            check_k3(hc, n, m, list(t), synth.random_kraus_set(3, int(rng.integers(2, 6)), rng), heis, rng)


def test_k3_kraus_form_full_rank_and_permutations(hc):
    """A channel with 64 Kraus operators (the largest rank), and a Toffoli
    with the native pass off: the Kraus form gives the oracle's result."""
    rng = synth.make_rng(1200)
    n, m = 7, 5
    check_k3(hc, n, m, [6, 1, 5], synth.random_kraus_set(3, 64, rng), False, rng)
    check_k3(hc, n, m, [2, 6, 0], synth.permutation_gate("TOFFOLI")[None], True, rng, native=0)


def test_step_kernel_item_orders_cover_every_item_once():
    """The workgroup-wide step kernels' item orders (sync_item): for every
    group count, steps per group, waves per workgroup, steps per group in
    one workgroup step (r) and group stride (1, 2 or 4), the (unit, wave)
    pairs reach each (group, step) of the pass exactly once, every step
    index is in range, and whole groups (r = min(sl, log2 waves), stride 1)
    are the consecutive items u * waves + w."""
    if not os.path.exists(SO):
        pytest.skip("_hostcheck.so not built")
    f = ctypes.CDLL(SO).htc_sync_items
    f.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_uint64
    cap = 4096
    for ng in (1, 2, 3, 15, 16, 17, 31, 33, 100, 528):
        for sl in range(5):
            for lw in (2, 3, 4):
                wpb = 1 << lw
                for r in range(min(sl, lw) + 1):
                    for ps in (0, 1, 2):
                        grp = np.zeros(cap * wpb, dtype=np.uint64)
                        step = np.zeros(cap * wpb, dtype=np.uint32)
                        nu = f(ng, sl, wpb, r, ps, cap, grp.ctypes.data, step.ctypes.data)
                        assert 0 < nu <= cap
                        g, s = grp[:nu * wpb], step[:nu * wpb]
                        assert np.all(s < (1 << sl))
                        live = g < ng
                        key = g[live] * (1 << sl) + s[live]
                        assert np.array_equal(np.sort(key), np.arange(ng << sl, dtype=np.uint64)), \
                            (ng, sl, wpb, r, ps)
                        if r == min(sl, lw) and ps == 0:
                            it = np.arange(nu * wpb, dtype=np.uint64)
                            assert np.array_equal(g, it >> np.uint64(sl))
                            assert np.array_equal(s, (it & np.uint64((1 << sl) - 1)).astype(np.uint32))


def test_quarter_order_steps_cover_one_row_band():
    """The step kernel's quarter order gives a workgroup step the 2^r
    consecutive steps of a group with r = F - s - log2(blocks per lane and
    step) (complex128 JU = 4 for k = 1, 1 for k = 2; row-run patches,
    s = 3).  Those steps must cover exactly one 8-row band of base row
    indices (the same high bits for every block) and every base column.
    With no intra target (F = 5 at M = 32) that is one 4 KiB run of each
    stored tile, so all runs of a workgroup step share address bits
    12-13."""
    if not os.path.exists(SO):
        pytest.skip("_hostcheck.so not built")
    f = ctypes.CDLL(SO).htc_lane_block
    f.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                  ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
    p, q = ctypes.c_uint32(), ctypes.c_uint32()
    # (F, JU): k = 1 one tile-selecting target (F = m = 5), k = 2 two (F = 5),
    # k = 2 one intra + one tile-selecting (F = 4)
    for F, ju in ((5, 4), (5, 1), (4, 1)):
        s = min(3, F)
        jobs = (1 << (2 * F)) // 64
        steps = jobs // ju
        r = F - s - {4: 2, 2: 1, 1: 0}[ju]
        per = 1 << r  # steps per unit
        for u in range(steps // per):
            rows, cols = set(), set()
            for step in range(u * per, (u + 1) * per):
                for job in range(step * ju, step * ju + ju):
                    for lane in range(64):
                        f(job * 64 + lane, F, s, 0, ctypes.byref(p), ctypes.byref(q))
                        rows.add(p.value)
                        cols.add(q.value)
            assert cols == set(range(1 << F)), (F, ju, u)
            assert len(rows) == 8 and len({r_ >> 3 for r_ in rows}) == 1, (F, ju, u, sorted(rows))
