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
