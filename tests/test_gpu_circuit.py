"""Fused circuits on the GPU against the CPU oracle and against op-by-op
application."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.test_circuit_cpu import random_circuit

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


@pytest.mark.parametrize("picture", [0, 1])
def test_fused_circuit_matches_oracle(ht, picture):
    rng = synth.make_rng(2500 + picture)
    for n, m in ((3, 2), (6, 2), (7, 3), (8, 5), (9, 3)):
        ops = random_circuit(n, 60, rng)
        ops.append(synth.random_ops.unitary_op([0, n - 1, 1], synth.permutation_gate("TOFFOLI")))
        ops += random_circuit(n, 10, rng)
        H = synth.random_hermitian_dense(n, rng)
        ref = oracle.apply_ops(H, ops[::-1], adjoint=True) if picture else oracle.apply_ops(H, ops)
        c = ht.Circuit(ops)
        for max_q in (0, 1, 2):
            npass = c.plan(picture, max_q)
            h = ht.Herm(n, m).init_dense(H)
            c.apply(h)
            e = rel(h.to_dense(), ref)
            assert e <= TOL, (n, m, max_q, npass, e)
        c.close()


def test_unfused_plan_is_bitwise_op_by_op(ht):
    rng = synth.make_rng(2600)
    n, m = 8, 3
    ops = random_circuit(n, 50, rng)
    H = synth.random_hermitian_dense(n, rng)
    for picture in (0, 1):
        a = ht.Herm(n, m).init_dense(H)
        for op in (ops[::-1] if picture else ops):
            a.apply_op(op, picture)
        c = ht.Circuit(ops)
        assert c.plan(picture, 0) == len(ops)
        b = ht.Herm(n, m).init_dense(H)
        c.apply(b)
        assert np.array_equal(a.raw_entries(), b.raw_entries())
        c.close()


def test_fused_diagonal_groups_take_the_native_pass(ht):
    """A group of diagonal gates composes to a diagonal map, which runs as a
    native pass (fixed entries untouched)."""
    rng = synth.make_rng(2700)
    n, m = 7, 3
    ops = [synth.random_ops.unitary_op([2], synth.named_gate("T")),
           synth.random_ops.unitary_op([2, 5], synth.permutation_gate("CZ")),
           synth.random_ops.unitary_op([5], synth.named_gate("RZ", 0.4)),
           synth.random_ops.channel_op([5], synth.dephasing_kraus(0.1))]
    H = synth.random_hermitian_dense(n, rng)
    c = ht.Circuit(ops)
    assert c.plan(0, 2) == 1
    h = ht.Herm(n, m).init_dense(H)
    h.profile_enable(True)
    ht.set_tuning("native", 2)  # at every size (this operator is small)
    try:
        c.apply(h)
    finally:
        ht.set_tuning("native", 1)
    prof = h.profile_read()
    assert list(prof) == ["c128_k2_c1_native"], prof
    assert rel(h.to_dense(), oracle.apply_ops(H, ops)) <= TOL
    c.close()


def test_fused_c64_within_bound(ht):
    rng = synth.make_rng(2800)
    n, m = 8, 3
    ops = random_circuit(n, 80, rng)
    H = synth.random_hermitian_dense(n, rng)
    Hq = H.astype(np.complex64).astype(np.complex128)
    ref = oracle.apply_ops(Hq, ops)
    c = ht.Circuit(ops)
    npass = c.plan(0, 2)
    h = ht.Herm(n, m, "c64").init_dense(H)
    c.apply(h)
    e = rel(h.to_dense(), ref)
    assert e <= (npass + 1) * 2.0 ** -24, (npass, e)
    c.close()


def test_fused_layers_full_size(ht):
    """Two layers of the n = 16 workload: fused (at most 8 + 9 passes; the
    planner also merges across the layer boundary) against op by op (79
    passes) on the GPU, compared on 200,000 sampled entries, and the trace."""
    rng = synth.make_rng(2900)
    n = 16
    G = synth.ginibre_factor(n, 16, rng)
    ops = synth.layer_n16(0, rng, n=n) + synth.layer_n16(1, rng, n=n)
    a = ht.Herm(n, 5).init_lowrank(G)
    a.scale(1.0 / a.trace())
    for op in ops:
        a.apply_op(op)
    rows = rng.integers(0, 1 << n, size=200000)
    cols = rng.integers(0, 1 << n, size=200000)
    want = a.get_entries(rows, cols)
    tr = a.trace()
    a.close()
    torch.cuda.empty_cache()
    b = ht.Herm(n, 5).init_lowrank(G)
    b.scale(1.0 / b.trace())
    c = ht.Circuit(ops)
    assert c.plan(0, 2) <= 17
    c.apply(b)
    assert rel(b.get_entries(rows, cols), want) <= 1e-13
    assert abs(b.trace() - tr) < 1e-13
    c.close()


def test_apply_checks_qubits_and_leaves_state(ht):
    rng = synth.make_rng(3000)
    h = ht.Herm(4, 2).init_dense(synth.random_hermitian_dense(4, rng))
    raw = h.raw_entries()
    c = ht.Circuit([synth.random_ops.unitary_op([0], synth.haar_unitary(2, rng)),
                    synth.random_ops.unitary_op([5], synth.haar_unitary(2, rng))])
    c.plan(0, 2)
    with pytest.raises(ht.HermError):
        c.apply(h)
    assert np.array_equal(h.raw_entries(), raw)
    with pytest.raises(ht.HermError):
        ht.Circuit().apply(h)  # not planned
    c.close()


def test_empty_inputs_are_no_ops(ht):
    """An empty circuit, an empty batch and a circuit of one op on the
    smallest operator (n = 1) leave or update the state as they should."""
    rng = synth.make_rng(3100)
    h = ht.Herm(5, 2).init_dense(synth.random_hermitian_dense(5, rng))
    raw = h.raw_entries()
    c = ht.Circuit()
    assert c.plan(0, 2) == 0
    c.apply(h)
    b = ht.Batch()
    b.run()
    torch.cuda.synchronize()
    assert np.array_equal(h.raw_entries(), raw)
    c.close()
    b.close()
    H1 = synth.random_hermitian_dense(1, rng)
    ops = [synth.random_ops.unitary_op([0], synth.haar_unitary(2, rng)),
           synth.random_ops.channel_op([0], synth.dephasing_kraus(0.3))]
    c = ht.Circuit(ops)
    assert c.plan(0, 2) == 1
    h1 = ht.Herm(1, 5).init_dense(H1)
    c.apply(h1)
    assert rel(h1.to_dense(), oracle.apply_ops(H1, ops)) <= TOL
    c.close()
