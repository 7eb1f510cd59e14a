"""Batched persistent launches and captured graphs, against one-call-at-a-time
application and the CPU oracle."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ht():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_15765_amd as ht
    return ht


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _random_circuit(n, nops, rng):
    ops = []
    for _ in range(nops):
        c = rng.random()
        if c < 0.4 or n < 2:
            ops.append(synth.random_ops.unitary_op([int(rng.integers(n))], synth.haar_unitary(2, rng)))
        elif c < 0.7:
            t = [int(x) for x in rng.choice(n, 2, replace=False)]
            ops.append(synth.random_ops.unitary_op(t, synth.haar_unitary(4, rng)))
        elif c < 0.9:
            ops.append(synth.random_ops.channel_op([int(rng.integers(n))], synth.random_kraus_set(1, 3, rng)))
        else:
            t = [int(x) for x in rng.choice(n, 2, replace=False)]
            ops.append(synth.random_ops.channel_op(t, synth.random_kraus_set(2, 3, rng)))
    return ops


def _cases(rng, count):
    out = []
    for i in range(count):
        n = int(rng.integers(1, 10))
        m = int(rng.choice([2, 3, 5]))
        dtype = "c64" if i % 5 == 4 else "c128"
        out.append((n, m, dtype, synth.random_hermitian_dense(n, rng), _random_circuit(n, int(rng.integers(5, 30)), rng)))
    return out


@pytest.mark.parametrize("params", [dict(), dict(lds_max_bytes=0), dict(threads=1024, wg_per_cu=1),
                                    dict(threads=64, wg_per_cu=8)])
def test_batch_equals_plain_bitwise(ht, params):
    """One persistent launch over 40 operators of mixed n, tile edge and
    storage type gives bitwise the same storage as applying every op with its
    own launch, and matches the oracle."""
    rng = synth.make_rng(1000)
    cases = _cases(rng, 40)
    batch = ht.Batch(**params)
    pairs = []
    for n, m, dtype, H, ops in cases:
        a = ht.Herm(n, m, dtype).init_dense(H)
        b = ht.Herm(n, m, dtype).init_dense(H)
        for op in ops:
            batch.add_op(a, op)
            b.apply_op(op)
        pairs.append((a, b, H, ops, dtype))
    assert batch.size() == (len(cases), sum(len(c[4]) for c in cases))
    batch.run()
    torch.cuda.synchronize()
    for a, b, H, ops, dtype in pairs:
        assert np.array_equal(a.read_raw(), b.read_raw()), (a.n, a.tile_log2, dtype)
        ref = oracle.apply_ops(H if dtype == "c128" else H.astype(np.complex64).astype(np.complex128), ops)
        tol = 1e-12 if dtype == "c128" else (len(ops) + 1) * 2.0 ** -24 * 4
        assert rel(a.to_dense(), ref) <= tol, (a.n, dtype, rel(a.to_dense(), ref))
    batch.close()


def test_batch_heisenberg_and_reuse(ht):
    """Heisenberg-picture ops in a batch; a batch can be cleared and refilled."""
    rng = synth.make_rng(1001)
    batch = ht.Batch()
    for round_ in range(2):
        hs = []
        for n in (3, 6, 8):
            H = synth.random_hermitian_dense(n, rng)
            ops = _random_circuit(n, 12, rng)
            h = ht.Herm(n, 3).init_dense(H)
            for op in reversed(ops):
                batch.add_op(h, op, ht.HEISENBERG)
            hs.append((h, H, ops))
        batch.run()
        torch.cuda.synchronize()
        for h, H, ops in hs:
            ref = oracle.apply_ops(H, list(reversed(ops)), adjoint=True)
            assert rel(h.to_dense(), ref) <= 1e-12
        batch.clear()
        assert batch.size() == (0, 0)


def test_graph_replays_match_eager(ht):
    """A captured op sequence replayed three times, with eager work and
    synchronisation between replays: every replay equals eager application."""
    rng = synth.make_rng(1002)
    n, m = 7, 3
    H = synth.random_hermitian_dense(n, rng)
    ops = _random_circuit(n, 25, rng)
    s = torch.cuda.Stream()
    h = ht.Herm(n, m, stream=s).init_dense(H)
    ref = ht.Herm(n, m).init_dense(H)
    for op in ops:
        ref.apply_op(op)
    expect = ref.read_raw()
    torch.cuda.synchronize()
    ht.capture_begin(s)
    for op in ops:
        h.apply_op(op)
    g = ht.capture_end(s)
    for rep in range(3):
        h.init_dense(H)
        tr = h.trace()  # eager work between replays
        assert abs(tr - oracle.trace(H)) < 1e-12
        g.launch(s)
        s.synchronize()
        assert np.array_equal(h.read_raw(), expect), rep
    g.close()


def test_autotune_picks_valid_settings_and_results_stay_exact(ht):
    """The autotuner returns a tile exponent for every qubit count present
    (and none for the others) and a valid launch shape; operators created
    with the chosen edges and run as one batch at the chosen shape give
    bitwise the storage of one launch per op, and match the oracle.  The
    operators queued for tuning are left untouched."""
    rng = synth.make_rng(1200)
    cases = []
    for i in range(36):
        n = int(rng.integers(3, 9))
        dtype = "c64" if i % 6 == 5 else "c128"
        cases.append((n, dtype, synth.random_hermitian_dense(n, rng), _random_circuit(n, int(rng.integers(5, 25)), rng)))
    tune = ht.Batch()
    probes = []
    for n, dtype, H, ops in cases:
        h = ht.Herm(n, 5, dtype).init_dense(H)
        for op in ops:
            tune.add_op(h, op)
        probes.append((h, h.read_raw().copy()))
    res = tune.autotune()
    present = sorted({c[0] for c in cases})
    assert sorted(res["tile_log2"]) == present
    for n, m in res["tile_log2"].items():
        assert 1 <= m <= min(n, 7) or m == min(n, 5), (n, m)
    assert res["threads"] in (256, 512, 1024) and res["wg_per_cu"] in (1, 2, 4, 8)
    assert res["threads"] * res["wg_per_cu"] <= 2048
    assert res["lds_max_bytes"] in (0, 65536, 163584)
    assert res["sample_operators"] == len(cases) and res["configs_timed"] > 0
    assert res["sample_seconds_after"] > 0 and res["tuning_seconds"] > 0
    for h, raw in probes:  # tuning evolves scratch copies only
        assert np.array_equal(h.read_raw(), raw)
    tune.close()

    batch = ht.Batch(threads=res["threads"], wg_per_cu=res["wg_per_cu"],
                     lds_max_bytes=res["lds_max_bytes"])
    pairs = []
    for n, dtype, H, ops in cases:
        m = res["tile_log2"][n]
        a = ht.Herm(n, m, dtype).init_dense(H)
        b = ht.Herm(n, m, dtype).init_dense(H)
        for op in ops:
            batch.add_op(a, op)
            b.apply_op(op)
        pairs.append((a, b, H, ops, dtype))
    batch.run()
    torch.cuda.synchronize()
    for a, b, H, ops, dtype in pairs:
        assert np.array_equal(a.read_raw(), b.read_raw()), (a.n, a.tile_log2, dtype)
        ref = oracle.apply_ops(H if dtype == "c128" else H.astype(np.complex64).astype(np.complex128), ops)
        tol = 1e-12 if dtype == "c128" else (len(ops) + 1) * 2.0 ** -24 * 4
        assert rel(a.to_dense(), ref) <= tol, (a.n, dtype, rel(a.to_dense(), ref))
    batch.close()


def test_autotune_rejects_an_empty_batch(ht):
    b = ht.Batch()
    with pytest.raises(ht.HermError):
        b.autotune()
    b.close()


def test_fused_batch_equals_fused_circuits(ht):
    """fuse_qubits = 2: each operator's ops run as the fused passes a circuit
    plans (bitwise equal to ht_circuit_apply on a copy), fewer passes than
    ops, and the oracle's result."""
    rng = synth.make_rng(1300)
    batch = ht.Batch(fuse_qubits=2)
    rows = []
    for i in range(20):
        n = int(rng.integers(2, 9))
        m = int(rng.choice([2, 3, 5]))
        H = synth.random_hermitian_dense(n, rng)
        ops = _random_circuit(n, int(rng.integers(10, 40)), rng)
        a = ht.Herm(n, m).init_dense(H)
        b = ht.Herm(n, m).init_dense(H)
        for op in ops:
            batch.add_op(a, op)
        c = ht.Circuit(ops)
        npass = c.plan(0, 2)
        c.apply(b)
        rows.append((a, b, H, ops, npass, c))
    batch.run()
    torch.cuda.synchronize()
    assert sum(r[4] for r in rows) < sum(len(r[3]) for r in rows)
    for a, b, H, ops, npass, c in rows:
        assert np.array_equal(a.read_raw(), b.read_raw()), (a.n, npass, len(ops))
        assert rel(a.to_dense(), oracle.apply_ops(H, ops)) <= 1e-12
        c.close()
    batch.close()
