"""Circuit fusion planned on the host (no GPU): every op lands in exactly
one pass, dependencies are kept, and the composed transfer matrices applied
pass by pass reproduce the oracle's op-by-op result in both pictures."""

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def ht():
    import paper_2604_15765_amd as ht
    return ht


def apply_transfer(H, S, sorted_t):
    """Dense application of a transfer matrix on the blocks of Eq. (2), local
    bits in ascending target order (Subroutine 1)."""
    n = H.shape[0].bit_length() - 1
    k = len(sorted_t)
    d = 1 << k
    out = H.copy()
    for s in range(1 << (n - k)):
        r = [oracle.insert_bits(s, a, sorted_t) for a in range(d)]
        for s2 in range(1 << (n - k)):
            c = [oracle.insert_bits(s2, a, sorted_t) for a in range(d)]
            out[np.ix_(r, c)] = (S @ H[np.ix_(r, c)].reshape(-1)).reshape(d, d)
    return out


def random_circuit(n, nops, rng):
    ops = []
    for _ in range(nops):
        c = rng.random()
        if c < 0.35:
            ops.append(synth.random_ops.unitary_op([int(rng.integers(n))], synth.haar_unitary(2, rng)))
        elif c < 0.6:
            t = [int(x) for x in rng.choice(n, 2, replace=False)]
            ops.append(synth.random_ops.unitary_op(t, synth.haar_unitary(4, rng)))
        elif c < 0.8:
            ops.append(synth.random_ops.channel_op([int(rng.integers(n))], synth.random_kraus_set(1, 2, rng)))
        elif c < 0.9:
            t = [int(x) for x in rng.choice(n, 2, replace=False)]
            ops.append(synth.random_ops.channel_op(t, synth.random_kraus_set(2, 3, rng)))
        else:
            ops.append(synth.random_ops.channel_op([int(rng.integers(n))], synth.dephasing_kraus(0.2)))
    return ops


def passes_of(c, npasses):
    return [c.pass_info(i) for i in range(npasses)]


@pytest.mark.parametrize("max_q", [0, 1, 2])
@pytest.mark.parametrize("picture", [0, 1])
def test_fused_passes_reproduce_the_oracle(ht, max_q, picture):
    rng = synth.make_rng(2100 + 10 * max_q + picture)
    for trial in range(6):
        n = int(rng.integers(2, 6))
        ops = random_circuit(n, int(rng.integers(5, 40)), rng)
        c = ht.Circuit(ops)
        npass = c.plan(picture, max_q)
        ps = passes_of(c, npass)
        # every op in exactly one pass, within the size bound
        seen = sorted(i for p in ps for i in p["ops"])
        assert seen == list(range(len(ops)))
        for p in ps:
            assert len(p["targets"]) <= max(max_q, max(len(ops[i].targets) for i in p["ops"]))
            assert set().union(*[set(ops[i].targets) for i in p["ops"]]) == set(p["targets"])
        if max_q == 0:
            assert npass == len(ops)
        H = synth.random_hermitian_dense(n, rng)
        got = H.copy()
        for p in ps:
            got = apply_transfer(got, p["transfer"], p["targets"])
        ref = oracle.apply_ops(H, ops[::-1], adjoint=True) if picture else oracle.apply_ops(H, ops)
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert e < 1e-13, (trial, n, len(ops), npass, e)
        c.close()


def test_dependencies_are_kept(ht):
    """Within a pass the ops keep their order; an op is never moved across an
    op it shares a qubit with."""
    rng = synth.make_rng(2200)
    for trial in range(20):
        n = int(rng.integers(3, 7))
        ops = random_circuit(n, 40, rng)
        c = ht.Circuit(ops)
        npass = c.plan(0, 2)
        order = [i for p in passes_of(c, npass) for i in p["ops"]]
        pos = {op: j for j, op in enumerate(order)}
        for a in range(len(ops)):
            for b in range(a + 1, len(ops)):
                if set(ops[a].targets) & set(ops[b].targets):
                    assert pos[a] < pos[b], (trial, a, b)
        c.close()


def test_layer_workload_fuses_to_qubit_pairs(ht):
    """One layer of the n = 16 workload (Haar U(2) on every qubit, brickwork
    Haar U(4), amplitude damping on every qubit) fuses into one pass per
    brickwork pair plus one per unpaired qubit."""
    rng = synth.make_rng(2300)
    for layer, want in ((0, 8), (1, 9)):
        ops = synth.layer_n16(layer, rng, n=16)
        c = ht.Circuit(ops)
        assert c.plan(0, 2) == want
        assert c.plan(1, 2) == want
        # a qubit's U(2) and damping are separated by its 2-qubit gate, so
        # single-qubit groups merge them only on the qubits without one (0
        # and 15 on odd layers)
        assert c.plan(0, 1) == len(ops) - (0 if layer == 0 else 2)
        c.close()


def test_three_qubit_ops_stay_single(ht):
    rng = synth.make_rng(2400)
    ops = [synth.random_ops.unitary_op([0], synth.named_gate("Z")),
           synth.random_ops.unitary_op([0, 1, 2], synth.permutation_gate("TOFFOLI")),
           synth.random_ops.unitary_op([1], synth.haar_unitary(2, rng)),
           synth.random_ops.unitary_op([3], synth.haar_unitary(2, rng))]
    c = ht.Circuit(ops)
    npass = c.plan(0, 2)
    ps = [c.pass_info(i, transfer=False) for i in range(npass)]
    assert [p["ops"] for p in ps] == [[0, 3], [1], [2]]  # Z(0) and U(3) commute past the rest
    p1 = c.pass_info(1)
    assert p1["targets"] == [0, 1, 2] and "transfer" not in p1  # none for a 3-qubit pass
    S = np.zeros(2 * 64 * 64)
    assert ht.lib.ht_circuit_pass_info(c._c, 1, None, None, None, None, S.ctypes.data) == 4
    c.close()


def test_circuit_argument_errors(ht):
    c = ht.Circuit()
    with pytest.raises(ht.HermError):
        c.add_unitary([0, 0], np.eye(4))
    with pytest.raises(ht.HermError):
        c.add_channel([0], np.stack([np.eye(2)] * 5))
    with pytest.raises(ht.HermError):
        c.plan(0, 3)
    with pytest.raises(ht.HermError):
        c.pass_info(0)  # not planned
    c.add_unitary([0], np.eye(2))
    assert c.size() == 1 and c.plan(0, 2) == 1
    c.close()
