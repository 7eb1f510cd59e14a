"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pins catch each one.  This is evidence that the pins constrain the oracle:
a dropped term, a wrong sign, a wrong index or a transposed operand anywhere in
it would fail at least one of them."""

import numpy as np

import oracle
import synth
from tests import oracle_checks as C


def rng(s):
    return synth.make_rng(s)


def expand_big_endian(L, targets, n):
    """Mistake: qubit q read as bit n-1-q."""
    return oracle.expand_local(L, [n - 1 - t for t in targets], n)


def expand_swapped_local_bits(L, targets, n):
    """Mistake: local bit l attached to targets[k-1-l]."""
    return oracle.expand_local(L, list(reversed(targets)), n)


def kmap_with(expand):
    def f(H, kraus, targets):
        n = H.shape[0].bit_length() - 1
        out = np.zeros_like(H, dtype=np.complex128)
        for L in kraus:
            K = expand(L, targets, n)
            out += K @ H @ K.conj().T
        return out
    return f


def kmap_transpose(H, kraus, targets):
    """Mistake: K H K^T instead of K H K^dagger."""
    n = H.shape[0].bit_length() - 1
    out = np.zeros_like(H, dtype=np.complex128)
    for L in kraus:
        K = oracle.expand_local(L, targets, n)
        out += K @ H @ K.T
    return out


def kmap_drop_last(H, kraus, targets):
    """Mistake: the last Kraus operator is dropped."""
    kr = np.asarray(kraus)
    return oracle.kraus_map(H, kr[:-1] if len(kr) > 1 else kr, targets)


def kmap_adjoint_wrong(H, kraus, targets):
    """Mistake: the Heisenberg map applies K O K^dagger (the forward map)."""
    return oracle.kraus_map(H, kraus, targets)


def block_update_no_conj(blk, kraus, adjoint=False):
    """Mistake: h -> sum L h L^T."""
    return sum(L @ blk @ L.T for L in kraus)


def local_map_no_conj(H, kraus, targets, adjoint=False):
    """Mistake: the column side contracts L instead of conj(L)."""
    from oracle.local_block import _apply_on_axes

    N = H.shape[0]
    n = N.bit_length() - 1
    T = np.asarray(H, np.complex128).reshape((2,) * (2 * n))
    out = np.zeros_like(T)
    for L in kraus:
        R = _apply_on_axes(T, L, [n - 1 - t for t in targets])
        out += _apply_on_axes(R, L, [2 * n - 1 - t for t in targets])
    return out.reshape(N, N)


def test_big_endian_is_caught():
    assert C.single_target_kron_error(expand_big_endian, 4, rng(1)) > 0.1
    assert C.pauli_conjugation_error(kmap_with(expand_big_endian), 4, rng(2)) > 0.1


def test_swapped_local_bits_is_caught():
    assert C.pair_kron_error(expand_swapped_local_bits, 4, rng(3)) > 0.1
    assert C.cnot_basis_error(kmap_with(expand_swapped_local_bits), 4, rng(4)) > 0.1


def test_transpose_instead_of_adjoint_is_caught():
    # (the U, U^dagger roundtrip is blind to this one: U^T and conj(U) cancel)
    assert C.hermiticity_error(kmap_transpose, 4, rng(6)) > 0.1
    assert C.trace_preservation_error(kmap_transpose, 4, rng(5)) > 1e-3


def test_dropped_kraus_term_is_caught():
    assert C.trace_preservation_error(kmap_drop_last, 4, rng(7)) > 1e-3
    assert C.depolarising_closed_form_error(kmap_drop_last, 3, rng(8)) > 1e-3


def test_wrong_heisenberg_map_is_caught():
    assert C.duality_error(oracle.kraus_map, kmap_adjoint_wrong, 4, rng(9)) > 1e-3


def test_missing_conjugate_in_block_update_is_caught():
    assert C.vec_identity_error(block_update_no_conj, rng(10)) > 0.1


def test_missing_conjugate_in_local_map_is_caught():
    assert C.local_vs_dense_error(local_map_no_conj, oracle.kraus_map, 3, rng(11)) > 0.1


# -- blocks, Pauli sums, op order, readouts ----------------------------------

def block_indices_ignore_s(s, targets):
    """Mistake: the subspace label is ignored (every sample is block 0)."""
    return oracle.block_indices(0, targets)


def block_indices_sorted(s, targets):
    """Mistake: local bits attached to the targets in ascending order."""
    return oracle.block_indices(s, sorted(targets))


def block_indices_reversed(s, targets):
    """Mistake: local bit l attached to targets[k-1-l]."""
    return oracle.block_indices(s, list(reversed(targets)))


def block_indices_s_high_first(s, targets):
    """Mistake: the label's bits fill the free positions from the top down."""
    n_free = 6 - len(targets)
    rev = int(format(s, f"0{n_free}b")[::-1], 2)
    return oracle.block_indices(rev, targets)


def test_block_index_mistakes_are_caught():
    sets = [[0], [4], [1, 3], [3, 1], [4, 0], [5, 2, 0]]
    for bad in (block_indices_ignore_s, block_indices_sorted, block_indices_reversed,
                block_indices_s_high_first):
        assert C.block_indices_error(bad, 6, sets) > 0, bad.__name__
    for bad in (block_indices_sorted, block_indices_reversed):
        assert C.block_form_consistency_error(bad, oracle.block_update, oracle.local_block_map, 5,
                                              rng(12)) > 0.1, bad.__name__


def pauli_matrix_big_endian(codes, coeffs):
    """Mistake: qubit 0 taken as the most significant index bit."""
    return oracle.pauli_sum_matrix(np.asarray(codes)[:, ::-1], coeffs)


def pauli_matrix_y_transposed(codes, coeffs):
    """Mistake: Y written as [[0, i], [-i, 0]]."""
    out = None
    for row, c in zip(np.asarray(codes), coeffs):
        M = np.ones((1, 1), dtype=np.complex128)
        for code in reversed([int(x) for x in row]):
            P = oracle.pauli_string_matrix([code])
            M = np.kron(M, P.T if code == 2 else P)
        out = c * M if out is None else out + c * M
    return out


def pauli_matrix_coeffs_shifted(codes, coeffs):
    """Mistake: coefficients paired with the wrong strings."""
    return oracle.pauli_sum_matrix(codes, np.roll(np.asarray(coeffs), 1))


def pauli_expectation_no_transpose(rho, codes, coeffs):
    """Mistake: tr(rho O) taken as Re sum_ij rho_ij O_ij."""
    O = oracle.pauli_sum_matrix(codes, coeffs)
    return float(np.real(np.sum(np.asarray(rho) * O)))


def pauli_expectation_drop_last(rho, codes, coeffs):
    """Mistake: the last term is dropped."""
    return oracle.pauli_sum_expectation(rho, np.asarray(codes)[:-1], np.asarray(coeffs)[:-1])


def test_pauli_sum_mistakes_are_caught():
    for bad in (pauli_matrix_big_endian, pauli_matrix_y_transposed, pauli_matrix_coeffs_shifted):
        assert C.pauli_sum_matrix_error(bad, 3, rng(13)) > 0.1, bad.__name__
    for bad in (pauli_expectation_no_transpose, pauli_expectation_drop_last):
        assert C.pauli_sum_expectation_error(bad, 3, rng(14)) > 1e-3, bad.__name__


def apply_ops_reversed(H, ops, adjoint=False):
    """Mistake: the circuit runs back to front."""
    return oracle.apply_ops(H, list(ops)[::-1], adjoint=adjoint)


def apply_ops_local_reversed(H, ops, adjoint=False):
    return oracle.apply_ops_local(H, list(ops)[::-1], adjoint=adjoint)


def apply_ops_forward_map_in_heisenberg(H, ops, adjoint=False):
    """Mistake: the Heisenberg flag is ignored."""
    return oracle.apply_ops(H, ops)


def test_op_order_mistakes_are_caught():
    for bad in (apply_ops_reversed, apply_ops_local_reversed, apply_ops_forward_map_in_heisenberg):
        assert C.op_order_error(bad) > 0.1, bad.__name__


def trace_abs(A):
    """Mistake: sum of moduli of the diagonal."""
    return float(np.sum(np.abs(np.diag(A))))


def density_unnormalised(G):
    G = np.asarray(G, dtype=np.complex128)
    return G @ G.conj().T


def density_transpose(G):
    """Mistake: G G^T / tr."""
    G = np.asarray(G, dtype=np.complex128)
    R = G @ G.T
    return R / np.trace(R)


def test_readout_mistakes_are_caught():
    assert C.trace_error(trace_abs, 3, rng(15)) > 0.1
    for bad in (density_unnormalised, density_transpose):
        assert C.density_from_factor_error(bad, 3, rng(16)) > 0.1, bad.__name__
