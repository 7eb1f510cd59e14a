"""The native pass for permutation-and-phase operations (gates of Section II-B
and k = 3) on the GPU, against the CPU oracle: results, untouched entries,
agreement with the generic pass, complex64, full-size sampled blocks, and
the batch and graph paths."""

import itertools

import numpy as np
import pytest
import torch

import oracle
from tests import sampling
import synth
from oracle import layout
from tests.native_masks import changing_entries, expected_writes

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ht():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_15765_amd as ht
    ht.set_tuning("native", 2)  # the native pass at every size (these operators are small)
    yield ht
    ht.set_tuning("native", 1)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gate_set(k, rng):
    if k == 1:
        out = [synth.named_gate(g)[None] for g in ("X", "Y", "Z", "S", "T")]
        out += [synth.named_gate("RZ", 1.1)[None], synth.dephasing_kraus(0.15), synth.random_monomial(1, rng)[None]]
        return out
    if k == 2:
        return [synth.cnot_matrix()[None]] + [synth.permutation_gate(g)[None] for g in ("CZ", "SWAP", "ISWAP")] + \
            [synth.random_monomial(2, rng)[None], synth.random_monomial(2, rng, diagonal=True)[None]]
    return [synth.permutation_gate(g)[None] for g in ("TOFFOLI", "CCZ", "FREDKIN")] + \
        [synth.random_monomial(3, rng)[None]]


def _run(ht, n, m, targets, kraus, picture, rng, dtype="c128"):
    H = synth.random_hermitian_dense(n, rng)
    h = ht.Herm(n, m, dtype).init_dense(H)
    before = h.raw_entries()
    if kraus.shape[0] == 1:
        h.apply_unitary(targets, kraus[0], picture)
    else:
        h.apply_channel(targets, kraus, picture)
    return H, h, before


@pytest.mark.parametrize("m", [2, 3, 5])
def test_native_ops_match_oracle_and_leave_fixed_entries(ht, m):
    """Every gate of the set on every target tuple (sampled for k = 3) at
    n = 3..7: the result matches the oracle and every stored entry the op
    fixes keeps its bits."""
    rng = synth.make_rng(1300 + m)
    for n in range(3, 8):
        for k in (1, 2, 3):
            tuples = list(itertools.permutations(range(n), k))
            if len(tuples) > 24:
                tuples = [tuples[i] for i in rng.choice(len(tuples), 24, replace=False)]
            for t in tuples:
                for g in gate_set(k, rng):
                    pic = int(rng.integers(2))
                    H, h, before = _run(ht, n, m, list(t), g, pic, rng)
                    ref = (oracle.kraus_map_adjoint if pic else oracle.kraus_map)(H, g, list(t))
                    e = rel(h.to_dense(), ref)
                    assert e <= TOL, (n, m, t, pic, e)
                    fixed = expected_writes(n, m, list(t), changing_entries(g, list(t), pic)) == 0
                    assert np.array_equal(h.raw_entries()[fixed], before[fixed]), (n, m, t)


def test_native_agrees_with_generic_pass(ht):
    rng = synth.make_rng(1400)
    n, m = 8, 3
    try:
        for k in (1, 2):
            for t in ([0], [4], [7]) if k == 1 else ([0, 1], [2, 6], [7, 3], [5, 6]):
                for g in gate_set(k, rng):
                    H = synth.random_hermitian_dense(n, rng)
                    outs = []
                    for native in (2, 0):
                        ht.set_tuning("native", native)
                        h = ht.Herm(n, m).init_dense(H)
                        h.apply_channel(t, g)
                        outs.append(h.to_dense())
                    assert rel(outs[0], outs[1]) < 1e-14, (t, rel(outs[0], outs[1]))
    finally:
        ht.set_tuning("native", 2)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_native_step_kernel_bitwise_equal(ht, dtype):
    """The native pass in workgroup-wide steps (native_sync_kernel, k <= 2,
    a tile-selecting target) gives bitwise the grid-stride native pass's
    storage for every gate of the set on intra, tile-selecting and mixed
    target pairs, in the three item orders and with 16 waves per workgroup,
    at tile edges 8 and 32 (n = 9: tile bits up to 5)."""
    rng = synth.make_rng(1410)
    n = 9
    H = synth.random_hermitian_dense(n, rng)
    cases = []
    for t in ([3], [5], [8], [2, 7], [6, 8], [8, 5], [4, 6]):
        for g in gate_set(len(t), rng):
            cases.append((t, g, int(rng.integers(2))))
    tunings = [{"sync_waves": 16, "sync_order": o} for o in (0, 1, 2)] + [{"sync_waves": 16, "sync_grid": 7}]
    try:
        for m in (3, 5):
            base = []
            ht.set_tuning("sync_waves", 0)
            for t, g, pic in cases:
                h = ht.Herm(n, m, dtype).init_dense(H)
                h.apply_channel(t, g, pic)
                base.append(h.raw_entries())
                h.close()
            for tune in tunings:
                for key, v in tune.items():
                    ht.set_tuning(key, v)
                for (t, g, pic), want in zip(cases, base):
                    h = ht.Herm(n, m, dtype).init_dense(H)
                    h.apply_channel(t, g, pic)
                    assert np.array_equal(h.raw_entries(), want), (dtype, m, t, tune)
                    h.close()
                for key in tune:
                    ht.set_tuning(key, -1 if key != "sync_grid" else 0)
            ht.set_tuning("sync_waves", -1)
    finally:
        for key, v in (("sync_waves", -1), ("sync_order", -1), ("sync_grid", 0)):
            ht.set_tuning(key, v)


def test_native_c64_one_rounding(ht):
    rng = synth.make_rng(1500)
    n, m = 7, 3
    for t in ([1], [5], [0, 6], [6, 2], [1, 4, 6], [6, 5, 4]):
        for g in gate_set(len(t), rng):
            H, h, _ = _run(ht, n, m, t, g, 0, rng, dtype="c64")
            Hq = H.astype(np.complex64).astype(np.complex128)
            e = rel(h.to_dense(), oracle.kraus_map(Hq, g, t))
            assert e <= 2 * 2.0 ** -24, (t, e)


def test_toffoli_circuit_and_involutions(ht):
    """A circuit of native and generic ops at n = 9 against the dense oracle;
    Toffoli, Fredkin and CNOT applied twice return the state bitwise."""
    rng = synth.make_rng(1600)
    n, m = 9, 3
    H = synth.random_hermitian_dense(n, rng)
    h = ht.Herm(n, m).init_dense(H)
    ops = []
    for _ in range(40):
        c = rng.random()
        if c < 0.3:
            t = [int(x) for x in rng.choice(n, 3, replace=False)]
            ops.append(synth.random_ops.unitary_op(t, synth.permutation_gate(str(rng.choice(["TOFFOLI", "FREDKIN", "CCZ"])))))
        elif c < 0.5:
            t = [int(x) for x in rng.choice(n, 2, replace=False)]
            ops.append(synth.random_ops.unitary_op(t, synth.cnot_matrix()))
        elif c < 0.7:
            ops.append(synth.random_ops.channel_op([int(rng.integers(n))], synth.dephasing_kraus(0.1)))
        else:
            ops.append(synth.random_ops.unitary_op([int(rng.integers(n))], synth.haar_unitary(2, rng)))
    for op in ops:
        h.apply_op(op)
    assert rel(h.to_dense(), oracle.apply_ops(H, ops)) <= TOL
    raw = h.raw_entries()
    for t, g in (([0, 4, 8], "TOFFOLI"), ([8, 2, 5], "FREDKIN"), ([3, 7], None)):
        U = synth.permutation_gate(g) if g else synth.cnot_matrix()
        h.apply_unitary(t, U)
        h.apply_unitary(t, U)
        assert np.array_equal(h.raw_entries(), raw)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_k3_kraus_form_matches_oracle(ht, m):
    """General three-qubit unitaries and channels (the Kraus-form pass: 8
    lanes per block, LDS exchange) against the oracle at n = 3..8 on sampled
    target triples, both pictures, complex128 and complex64."""
    rng = synth.make_rng(1750 + m)
    for n in range(3, 9):
        tuples = list(itertools.permutations(range(n), 3))
        tuples = [tuples[i] for i in rng.choice(len(tuples), min(len(tuples), 10), replace=False)]
        for t in tuples:
            for kraus in (synth.haar_unitary(8, rng)[None], synth.random_kraus_set(3, int(rng.integers(2, 7)), rng)):
                pic = int(rng.integers(2))
                H, h, _ = _run(ht, n, m, list(t), kraus, pic, rng)
                ref = (oracle.kraus_map_adjoint if pic else oracle.kraus_map)(H, kraus, list(t))
                assert rel(h.to_dense(), ref) <= TOL, (n, m, t, kraus.shape[0], pic)
        t = [int(x) for x in rng.choice(n, 3, replace=False)]
        kraus = synth.random_kraus_set(3, 3, rng)
        H, h, _ = _run(ht, n, m, t, kraus, 0, rng, dtype="c64")
        e = rel(h.to_dense(), oracle.kraus_map(H.astype(np.complex64).astype(np.complex128), kraus, t))
        assert e <= 2 * 2.0 ** -24, (n, m, t, e)


def test_k3_kraus_form_agrees_with_native_pass(ht):
    """A Toffoli and a random permutation-and-phase matrix through the Kraus
    form (native pass off) and the native pass; a channel of full rank 64."""
    rng = synth.make_rng(1760)
    n, m = 8, 3
    H = synth.random_hermitian_dense(n, rng)
    try:
        for t, U in (([0, 5, 7], synth.permutation_gate("TOFFOLI")), ([6, 2, 3], synth.random_monomial(3, rng))):
            outs = []
            for native in (0, 2):
                ht.set_tuning("native", native)
                h = ht.Herm(n, m).init_dense(H)
                h.apply_unitary(t, U)
                outs.append(h.to_dense())
            assert rel(outs[0], outs[1]) <= 1e-14, t
    finally:
        ht.set_tuning("native", 2)
    K = synth.random_kraus_set(3, 64, rng)
    h = ht.Herm(n, m).init_dense(H)
    h.apply_channel([7, 0, 4], K)
    assert rel(h.to_dense(), oracle.kraus_map(H, K, [7, 0, 4])) <= TOL


def test_k3_bad_kraus_count_leaves_state(ht):
    rng = synth.make_rng(1700)
    h = ht.Herm(6, 3).init_dense(synth.random_hermitian_dense(6, rng))
    raw = h.raw_entries()
    with pytest.raises(ht.HermError) as ei:
        h.apply_channel([0, 2, 5], np.stack([np.eye(8)] * 65))
    assert ei.value.status == 1
    assert np.array_equal(h.raw_entries(), raw)


@pytest.mark.parametrize("n", [14, 16])
def test_native_full_size_sampled_blocks(ht, n):
    """Full-size operators at the benchmark's tile edge: native ops at intra
    and tile-selecting positions on 1500 sampled blocks each (k <= 2 with a
    tile-selecting target at tile bit 4 or above in workgroup steps, nearer
    ones grid-stride), plus trace."""
    rng = synth.make_rng(1800 + n)
    h = ht.Herm(n, 5).init_lowrank(synth.ginibre_factor(n, 16, rng))
    h.scale(1.0 / h.trace())
    ops = [
        synth.random_ops.unitary_op([3], synth.named_gate("X")),
        synth.random_ops.unitary_op([n - 1], synth.named_gate("T")),
        synth.random_ops.channel_op([7], synth.dephasing_kraus(0.2)),
        synth.random_ops.unitary_op([4, n - 3], synth.cnot_matrix()),
        synth.random_ops.unitary_op([9, 6], synth.permutation_gate("SWAP")),
        synth.random_ops.unitary_op([n - 1, n - 2], synth.cnot_matrix()),      # workgroup steps, top tiles
        synth.random_ops.unitary_op([5, 6], synth.permutation_gate("CZ")),     # grid-stride (near)
        synth.random_ops.unitary_op([1, 2, 4], synth.permutation_gate("TOFFOLI")),
        synth.random_ops.unitary_op([0, 8, n - 1], synth.permutation_gate("FREDKIN")),
        synth.random_ops.unitary_op([n - 1, 10, 5], synth.permutation_gate("TOFFOLI")),
        synth.random_ops.unitary_op([6, 11, 12], synth.random_monomial(3, rng)),
        synth.random_ops.unitary_op([2, n - 2, 9], synth.haar_unitary(8, rng)),       # Kraus form
        synth.random_ops.channel_op([n - 1, 0, 6], synth.random_kraus_set(3, 2, rng)),  # Kraus form
    ]
    for i, op in enumerate(ops):
        nblocks = 1500
        R, C, d = sampling.block_entries(n, op.targets, h.tile_log2, nblocks, rng)
        before = h.get_entries(R, C).reshape(nblocks, d, d)
        pic = i % 2
        h.apply_op(op, pic)
        after = h.get_entries(R, C).reshape(nblocks, d, d)
        want = oracle.block_update(before, op.mats, adjoint=bool(pic))
        assert rel(after, want) <= TOL, (op.targets, rel(after, want))
    assert abs(h.trace() - 1.0) < 1e-12


def test_batch_with_native_ops_equals_plain_bitwise(ht):
    """Native ops inside the persistent batch launch (LDS-resident and not)
    give bitwise the results of one launch per op."""
    rng = synth.make_rng(1900)
    batch = ht.Batch()
    pairs = []
    for i in range(24):
        n = int(rng.integers(2, 10))
        m = int(rng.choice([2, 3, 5]))
        H = synth.random_hermitian_dense(n, rng)
        a = ht.Herm(n, m).init_dense(H)
        b = ht.Herm(n, m).init_dense(H)
        ops = []
        for _ in range(int(rng.integers(5, 20))):
            k = 1 if n < 2 or rng.random() < 0.5 else 2
            t = [int(x) for x in rng.choice(n, k, replace=False)]
            g = gate_set(k, rng)[int(rng.integers(len(gate_set(k, rng))))]
            if rng.random() < 0.3:
                g = synth.haar_unitary(1 << k, rng)[None]
            ops.append(synth.random_ops.channel_op(t, g))
        for op in ops:
            batch.add_op(a, op)
            b.apply_op(op)
        pairs.append((a, b, H, ops))
    batch.run()
    torch.cuda.synchronize()
    for a, b, H, ops in pairs:
        assert np.array_equal(a.raw_entries(), b.raw_entries()), (a.n, a.tile_log2)
        assert rel(a.to_dense(), oracle.apply_ops(H, ops)) <= TOL
    batch.close()
