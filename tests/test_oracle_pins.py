"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle is the reference every GPU result is compared with, so it is
checked here against things other than itself: library routines (np.kron),
closed forms of textbook channels, invariants of Kraus maps, the identity
behind Eq. (3), the values printed in Table I and hand-derived 2x2 results.
"""

import os
import re

import numpy as np
import pytest

import oracle
import synth
from oracle import layout
from tests import oracle_checks as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return synth.make_rng(seed)


def test_expand_single_target_is_kron():
    assert C.single_target_kron_error(oracle.expand_local, 5, rng(1)) < 1e-15


def test_expand_pair_is_kron():
    assert C.pair_kron_error(oracle.expand_local, 5, rng(2)) < 1e-15


def test_vec_identity_eq3():
    assert C.vec_identity_error(oracle.block_update, rng(3)) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_local_block_matches_kronecker(n):
    if n == 1:
        H = synth.random_hermitian_dense(1, rng(4))
        kraus = synth.random_kraus_set(1, 3, rng(5))
        assert C.rel(oracle.local_block_map(H, kraus, [0]), oracle.kraus_map(H, kraus, [0])) < 1e-14
        return
    assert C.local_vs_dense_error(oracle.local_block_map, oracle.kraus_map, n, rng(6 + n)) < 1e-14
    adj_local = lambda H, k, t: oracle.local_block_map(H, k, t, adjoint=True)
    assert C.local_vs_dense_error(adj_local, oracle.kraus_map_adjoint, n, rng(16 + n)) < 1e-14


def test_hermiticity_preserved():
    assert C.hermiticity_error(oracle.kraus_map, 5, rng(20)) < 1e-15


def test_trace_preservation():
    assert C.trace_preservation_error(oracle.kraus_map, 5, rng(21)) < 1e-13


def test_positivity():
    assert C.positivity_error(oracle.kraus_map, 5, rng(22)) < 1e-13


def test_pauli_conjugation_closed_form():
    for s in range(4):
        assert C.pauli_conjugation_error(oracle.kraus_map, 5, rng(30 + s)) < 1e-15


def test_pauli_x_twice_is_bitwise_identity():
    H = synth.random_hermitian_dense(4, rng(35))
    X = synth.named_gate("X")[None]
    for a in range(4):
        assert np.array_equal(oracle.kraus_map(oracle.kraus_map(H, X, [a]), X, [a]), H)


def test_depolarising_closed_form():
    assert C.depolarising_closed_form_error(oracle.kraus_map, 4, rng(40)) < 1e-14


def test_amplitude_damping_closed_form():
    assert C.amplitude_damping_error(oracle.kraus_map, 4, rng(41)) < 1e-14


def test_dephasing_closed_form():
    assert C.dephasing_error(oracle.kraus_map, 4, rng(42)) < 1e-15


def test_duality_and_unitality():
    assert C.duality_error(oracle.kraus_map, oracle.kraus_map_adjoint, 4, rng(43)) < 1e-13


def test_unitary_roundtrip():
    assert C.unitary_roundtrip_error(oracle.kraus_map, 4, rng(44)) < 1e-14


def test_cnot_basis_action_and_untouched_quarter():
    assert C.cnot_basis_error(oracle.kraus_map, 4, rng(45)) == 0.0


def test_diagonal_gate_leaves_equal_bit_entries():
    assert C.diagonal_gate_error(oracle.kraus_map, 4, rng(46)) == 0.0


def test_worked_2x2_examples():
    """Hand-derived single-qubit results."""
    ket0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    ket1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
    H = synth.named_gate("H")[None]
    assert np.allclose(oracle.kraus_map(ket0, H, [0]), 0.5 * np.ones((2, 2)), atol=1e-15)
    a, b, d = 0.3, 0.2 - 0.7j, 0.7
    rho = np.array([[a, b], [np.conj(b), d]])
    X = synth.named_gate("X")[None]
    assert np.array_equal(oracle.kraus_map(rho, X, [0]), np.array([[d, np.conj(b)], [b, a]]))
    g = 0.25
    assert np.allclose(oracle.kraus_map(ket1, synth.amplitude_damping_kraus(g), [0]),
                       np.diag([g, 1 - g]), atol=1e-16)
    p = 0.09
    assert np.allclose(oracle.kraus_map(ket0, synth.depolarising_kraus(p), [0]),
                       np.diag([1 - 2 * p / 3, 2 * p / 3]), atol=1e-16)
    # Y rho Y on a 2x2: swaps the diagonal, conjugates and negates b
    Y = synth.named_gate("Y")[None]
    assert np.allclose(oracle.kraus_map(rho, Y, [0]), np.array([[d, -np.conj(b)], [-b, a]]), atol=1e-16)


def test_heisenberg_is_reverse_adjoint_circuit():
    """tr(O Phi_L...Phi_1(rho)) = tr(Phi_1*...Phi_L*(O) rho)."""
    r = rng(50)
    n = 4
    g, ops = synth.circuit_plain_n8(seed=51, n=n, nops=12)
    rho = oracle.density_from_factor(g)
    codes, coeffs = synth.random_pauli_sum(n, 8, r)
    O = oracle.pauli_sum_matrix(codes, coeffs)
    fwd = oracle.apply_ops(rho, ops)
    back = oracle.apply_ops(O, list(reversed(ops)), adjoint=True)
    assert abs(oracle.expectation(fwd, O) - oracle.expectation(rho, back)) < 1e-13


def test_insert_bits_bijection_and_bit_placement():
    """Subroutine 1 against a construction on binary digit strings."""
    n = 6
    for positions in ([0], [3], [5], [0, 1], [1, 4], [2, 5], [0, 5]):
        k = len(positions)
        seen = set()
        for s in range(1 << (n - k)):
            for a in range(1 << k):
                g = oracle.insert_bits(s, a, positions)
                digits = []  # little-endian digits of the result
                s_bits = [(s >> b) & 1 for b in range(n - k)]
                for q in range(n):
                    if q in positions:
                        digits.append((a >> positions.index(q)) & 1)
                    else:
                        digits.append(s_bits.pop(0))
                assert g == sum(d << q for q, d in enumerate(digits))
                seen.add(g)
        assert seen == set(range(1 << n))


def _parse_size(tok: str):
    num, unit = tok.split()
    scale = {"B": 1, "KiB": 1024, "MiB": 1024 ** 2, "GiB": 1024 ** 3}[unit]
    decimals = len(num.split(".")[1]) if "." in num else 0
    return float(num) * scale, 0.5 * 10 ** (-decimals) * scale


def test_table1_memory_footprint():
    rows = []
    with open(os.path.join(GOLDEN, "table1_memory_footprint.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([c.strip() for c in line.split("|")])
    assert len(rows) == 5
    for n_s, full_s, packed_s, tiled_s, ratio_s in rows:
        n = int(n_s)
        full = 16 * layout.full_elems(n)
        packed = 16 * layout.packed_elems(n)
        tiled = 16 * layout.tiled_elems(n, 5, pad=True)
        for val, tok in ((full, full_s), (packed, packed_s), (tiled, tiled_s)):
            printed, half = _parse_size(tok)
            assert abs(val - printed) <= half, (n, tok, val)
        r = float(re.sub("x$", "", ratio_s))
        dec = len(ratio_s.rstrip("x").split(".")[1]) if "." in ratio_s else 0
        assert abs(tiled / packed - r) <= 0.5 * 10 ** (-dec) + 1e-12, (n, ratio_s, tiled / packed)


def test_layout_roundtrip_and_padding():
    r = rng(60)
    for n, m in ((1, 5), (3, 2), (5, 3), (6, 5), (7, 2)):
        H = synth.random_hermitian_dense(n, r)
        for pad in (False, True):
            raw = layout.encode(H, m, pad=pad)
            assert raw.size == layout.tiled_elems(n, m, pad=pad)
            assert np.array_equal(layout.decode(raw, n, m, pad=pad), np.tril(H) + np.tril(H, -1).conj().T)
            assert layout.diagonal_tile_asymmetry(raw, n, m, pad=pad) < 1e-15
    # tile numbering follows the row-major order of the lower tile triangle
    order = [(ti, tj) for ti in range(6) for tj in range(ti + 1)]
    assert [layout.tile_number(ti, tj) for ti, tj in order] == list(range(len(order)))


@pytest.mark.parametrize("n,m", [(5, 1), (6, 2), (7, 3)])
def test_algorithm3_case_counts_and_ownership(n, m):
    """Case C occurs once per base tile row, the three cases cover every base
    pair, and every stored tile is touched by exactly one base pair."""
    nt = (1 << n) >> m
    for a in range(m, n):
        res = layout.cross_tile_cases(n, m, a)
        nb = res["nb"]
        c = res["counts"]
        assert c["C"] == nb
        assert c["A"] + c["B"] + c["C"] == nb * (nb + 1) // 2
        if a == m:
            assert c["B"] == 0 or nb == 1
        seen = {}
        for tiles in res["touched"]:
            for t in tiles:
                assert t[0] >= t[1]
                seen[t] = seen.get(t, 0) + 1
        assert set(seen) == {(ti, tj) for ti in range(nt) for tj in range(ti + 1)}
        assert all(v == 1 for v in seen.values())
    if n - m >= 3:
        # case A dominates for the lowest cross bit, case B for the highest
        lo = layout.cross_tile_cases(n, m, m)["counts"]
        hi = layout.cross_tile_cases(n, m, n - 1)["counts"]
        assert lo["A"] > lo["B"] and hi["B"] > hi["A"]


def test_expectation_readouts():
    r = rng(70)
    n = 5
    rho = C.random_density(n, r)
    assert abs(oracle.expectation(rho, np.eye(1 << n)) - oracle.trace(rho)) < 1e-15
    # single Pauli strings against the closed form sum_j phase(j) rho_{j^x, j}
    for _ in range(6):
        codes = r.integers(0, 4, size=n)
        x = sum(1 << q for q, c in enumerate(codes) if c in (1, 2))
        z = sum(1 << q for q, c in enumerate(codes) if c in (2, 3))
        ny = sum(1 for c in codes if c == 2)
        tot = 0.0
        for j in range(1 << n):
            sign = -1.0 if bin(j & z).count("1") & 1 else 1.0
            tot += ((-1j) ** ny) * sign * rho[j ^ x, j]
        assert abs(oracle.expectation(rho, oracle.pauli_string_matrix(codes)) - tot.real) < 1e-14
        assert abs(tot.imag) < 1e-14


def test_tiled_expectation_strict_formula():
    """The tiled expectation with a strict off-diagonal sum equals tr(rho O);
    counting the diagonal tiles twice (the printed >=) does not."""
    r = rng(71)
    n, m = 6, 3
    rho = C.random_density(n, r)
    O = synth.random_hermitian_dense(n, r)
    a, b = layout.encode(rho, m), layout.encode(O, m)
    exact = oracle.expectation(rho, O)
    assert abs(layout.tiled_expectation(a, b, n, m) - exact) < 1e-13
    nt = (1 << n) >> m
    diag = sum(float(np.real(np.sum(layout.stored_tile(b, n, m, t, t).conj() * layout.stored_tile(a, n, m, t, t))))
               for t in range(nt))
    printed = layout.tiled_expectation(a, b, n, m) + 2 * diag
    assert abs(printed - exact) > 1e-3


def test_generators_are_deterministic():
    g1, ops1 = synth.circuit_plain_n8(seed=9, n=5, nops=20)
    g2, ops2 = synth.circuit_plain_n8(seed=9, n=5, nops=20)
    assert np.array_equal(g1, g2)
    for a, b in zip(ops1, ops2):
        assert a.targets == b.targets and np.array_equal(a.mats, b.mats)
    cats = [op.label for op in synth.circuit_plain_n8(seed=3, n=8, nops=200)[1]]
    assert 80 <= cats.count("haar1") <= 120 and 40 <= cats.count("haar2") <= 80
    U = synth.haar_unitary(4, rng(80))
    assert np.allclose(U @ U.conj().T, np.eye(4), atol=1e-14)
    for kr in (synth.depolarising_kraus(0.1), synth.amplitude_damping_kraus(0.3),
               synth.dephasing_kraus(0.2), synth.random_kraus_set(2, 5, rng(81))):
        assert np.allclose(sum(L.conj().T @ L for L in kr), np.eye(kr.shape[1]), atol=1e-14)


def test_block_indices_partition_and_digits():
    """Subroutine 1 as used by Eq. (2): block_indices against a digit-string
    construction, for sorted, unsorted, adjacent and distant target tuples;
    the subspaces partition the index range."""
    sets = [[0], [4], [1, 3], [3, 1], [4, 0], [0, 4], [2, 5], [5, 2, 0], [1, 4, 3]]
    assert C.block_indices_error(oracle.block_indices, 6, sets) == 0


def test_block_form_matches_whole_matrix_map():
    """Every block h_{s,s'} of the mapped matrix equals Eq. (2) applied to the
    gathered block (n = 5, every pair of subspaces, both pictures)."""
    err = C.block_form_consistency_error(oracle.block_indices, oracle.block_update,
                                         oracle.local_block_map, 5, rng(90))
    assert err < 1e-14


def test_pauli_sum_matrix_entrywise_closed_form():
    for n in (1, 3, 5):
        assert C.pauli_sum_matrix_error(oracle.pauli_sum_matrix, n, rng(91 + n)) < 1e-15


def test_pauli_sum_expectation_closed_form():
    for n in (1, 3, 5):
        assert C.pauli_sum_expectation_error(oracle.pauli_sum_expectation, n, rng(95 + n)) < 1e-14


def test_circuit_order_dense_and_local():
    """Both circuit runners apply ops in the order given (hand-derived
    results for X and amplitude damping, which do not commute)."""
    assert C.op_order_error(oracle.apply_ops) < 1e-15
    assert C.op_order_error(oracle.apply_ops_local) < 1e-15
    assert C.op_order_error(oracle.apply_ops, n=4, q=3, gamma=0.05) < 1e-15


def test_trace_and_density_from_factor():
    assert C.trace_error(oracle.trace, 4, rng(99)) < 1e-12
    assert C.density_from_factor_error(oracle.density_from_factor, 4, rng(100)) < 1e-13
