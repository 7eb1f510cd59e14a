"""The continuous-batching server: results against the oracle, independent of
what else is being served, and equal to the one-at-a-time baseline."""

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


def _requests(seed, count, n_choices):
    rng = synth.make_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(n_choices))
        G = synth.ginibre_factor(n, min(8, 1 << n), rng)
        ops = [synth.circuits._random_mixed_op(n, rng, "dephase") for _ in range(int(rng.integers(10, 60)))]
        pauli = synth.random_pauli_sum(n, 16, rng) if i % 2 == 0 else None
        dtype = "c64" if i % 4 == 3 else "c128"
        out.append(dict(n=n, G=G, ops=ops, pauli=pauli, dtype=dtype))
    return out


def _serve(ht, reqs, **cfg):
    srv = ht.Server(**cfg)
    ids = [srv.submit(r["n"], r["G"], r["ops"], r["pauli"], r["dtype"]) for r in reqs]
    srv.wait_idle(300)
    res = {d["id"]: d for d in srv.poll()}
    assert srv.last_error() == "", srv.last_error()
    srv.close()
    assert all(res[i]["status"] == 0 for i in ids)
    return [res[i]["value"] for i in ids], [res[i] for i in ids]


def _oracle_value(r):
    rho = oracle.apply_ops(oracle.density_from_factor(r["G"]), r["ops"])
    if r["pauli"] is None:
        return oracle.trace(rho)
    return oracle.pauli_sum_expectation(rho, *r["pauli"])


def test_server_results_alone_mix_and_fifo(ht):
    reqs = _requests(77, 26, [3, 4, 5, 6, 7, 8, 9]) + _requests(78, 2, [12, 13])
    cfg = dict(batch_max_qubits=7, medium_max_qubits=9, chunk_ops=16, large_chunk_ops=3)
    alone, _ = _serve(ht, [reqs[0]], **cfg)
    mixed, recs = _serve(ht, reqs, **cfg)
    fifo, _ = _serve(ht, reqs, fifo=1)
    # the same request gives bitwise the same value alone and in the mix
    assert alone[0] == mixed[0]
    # batched rounds and plain passes compute identical bits
    assert mixed == fifo
    for r, v in zip(reqs, mixed):
        if r["n"] > 9:
            continue
        want = _oracle_value(r)
        if r["dtype"] == "c128":
            tol = 1e-12 * max(1.0, abs(want))
        else:
            # |d tr(rho O)| <= ||d rho||_F ||O||_F with ||d rho||_F <= (passes + 1) 2^-24 and
            # ||O||_F <= sqrt(N) sum|c| (sqrt(N) for the trace); factor 2 margin
            wsum = float(np.abs(r["pauli"][1]).sum()) if r["pauli"] is not None else 1.0
            tol = 2 * (len(r["ops"]) + 3) * 2.0 ** -24 * np.sqrt(1 << r["n"]) * wsum
        assert abs(v - want) <= tol, (r["n"], r["dtype"], v, want)
    # timestamps are ordered per request
    for d in recs:
        assert d["t_submit"] <= d["t_admit"] <= d["t_done"]


def test_server_tight_budget_queues_and_completes(ht):
    reqs = _requests(79, 12, [6, 8, 9])
    want, _ = _serve(ht, reqs)
    biggest = max(ht.storage_bytes(r["n"], 5, r["dtype"]) for r in reqs)
    got, recs = _serve(ht, reqs, budget_bytes=2 * biggest + (1 << 20), max_active=3)
    assert got == want
    assert max(d["t_admit"] for d in recs) > min(d["t_done"] for d in recs)  # later ones waited


def test_server_rejects_bad_requests(ht):
    srv = ht.Server(budget_bytes=1 << 20)
    rng = synth.make_rng(80)
    G = synth.ginibre_factor(10, 4, rng)  # n = 10 needs ~8.6 MB > 1 MB budget
    with pytest.raises(ht.HermError):
        srv.submit(10, G, [])
    G = synth.ginibre_factor(4, 2, rng)
    bad = synth.random_ops.unitary_op([7], synth.haar_unitary(2, rng))  # qubit 7 of a 4-qubit operator
    with pytest.raises(ht.HermError):
        srv.submit(4, G, [bad])
    ok = srv.submit(4, G, [synth.random_ops.unitary_op([1], synth.haar_unitary(2, rng))])
    srv.wait_idle(60)
    (d,) = srv.poll()
    assert d["id"] == ok and d["status"] == 0 and abs(d["value"] - 1.0) < 1e-12
    srv.close()


def test_server_with_fusion(ht):
    """Requests fused into 2-qubit passes: the same value alone, in the mix
    and one at a time (bitwise), and the oracle's value within tolerance."""
    reqs = _requests(81, 20, [3, 5, 6, 7, 8, 9]) + _requests(82, 2, [12])
    cfg = dict(batch_max_qubits=7, medium_max_qubits=9, chunk_ops=8, large_chunk_ops=2, fuse_qubits=2)
    alone, _ = _serve(ht, [reqs[1]], **cfg)
    mixed, _ = _serve(ht, reqs, **cfg)
    fifo, _ = _serve(ht, reqs, fifo=1, fuse_qubits=2)
    plain, _ = _serve(ht, reqs, fifo=1)
    assert alone[0] == mixed[1]
    assert mixed == fifo
    for r, v, p in zip(reqs, mixed, plain):
        if r["dtype"] == "c128":
            assert abs(v - p) <= 1e-12 * max(1.0, abs(p))
            if r["n"] <= 9:
                want = _oracle_value(r)
                assert abs(v - want) <= 1e-12 * max(1.0, abs(want)), (r["n"], v, want)


def test_server_fails_only_the_request_the_device_cannot_hold(ht):
    """An n = 18 complex128 request (about 550 GB, more than the device holds)
    within a 1 TiB budget: it fails with HT_ENOMEM, alone, whether other
    requests are resident or not, and the requests around it complete."""
    reqs = _requests(83, 6, [4, 6, 9])
    cfg = dict(batch_max_qubits=5, medium_max_qubits=7)
    want, _ = _serve(ht, reqs, **cfg)
    rng = synth.make_rng(84)
    n_big = 18
    assert ht.storage_bytes(n_big, 5, "c128") > torch.cuda.get_device_properties(0).total_memory
    big = synth.ginibre_factor(n_big, 1, rng)
    srv = ht.Server(budget_bytes=1 << 40, **cfg)
    ids = [srv.submit(r["n"], r["G"], r["ops"], r["pauli"], r["dtype"]) for r in reqs[:3]]
    bad = [srv.submit(n_big, big, [])]  # while the first ones are resident
    ids += [srv.submit(r["n"], r["G"], r["ops"], r["pauli"], r["dtype"]) for r in reqs[3:]]
    srv.wait_idle(300)
    bad.append(srv.submit(n_big, big, []))  # with nothing else resident
    ok = srv.submit(reqs[0]["n"], reqs[0]["G"], reqs[0]["ops"], reqs[0]["pauli"], reqs[0]["dtype"])
    srv.wait_idle(300)
    res = {d["id"]: d for d in srv.poll()}
    assert "cannot hold" in srv.last_error()
    srv.close()
    assert [res[i]["status"] for i in bad] == [2, 2]  # HT_ENOMEM
    assert [res[i]["status"] for i in ids + [ok]] == [0] * (len(ids) + 1)
    assert [res[i]["value"] for i in ids] == want
    assert res[ok]["value"] == want[0]


def test_server_heisenberg_requests(ht):
    """Requests in the Heisenberg picture: every op applied as its adjoint
    map, in the order given, in the batched, medium and large lanes and with
    fusion; the readout matches the oracle."""
    rng = synth.make_rng(85)
    reqs = []
    for n in (4, 6, 8, 9):
        G = synth.ginibre_factor(n, 4, rng)
        ops = [synth.circuits._random_mixed_op(n, rng, "dephase") for _ in range(25)]
        reqs.append(dict(n=n, G=G, ops=ops, pauli=synth.random_pauli_sum(n, 8, rng)))
    for cfg in (dict(batch_max_qubits=5, medium_max_qubits=8), dict(fuse_qubits=2)):
        srv = ht.Server(**cfg)
        ids = [srv.submit(r["n"], r["G"], r["ops"], r["pauli"], "c128", ht.HEISENBERG) for r in reqs]
        srv.wait_idle(300)
        res = {d["id"]: d for d in srv.poll()}
        srv.close()
        for i, r in zip(ids, reqs):
            assert res[i]["status"] == 0
            rho = oracle.apply_ops(oracle.density_from_factor(r["G"]), r["ops"], adjoint=True)
            want = oracle.pauli_sum_expectation(rho, *r["pauli"])
            assert abs(res[i]["value"] - want) <= 1e-12 * max(1.0, abs(want)), (cfg, r["n"])
