"""Scalar readouts of a hermitian operator -- test infrastructure.

Section I: predictions are expectation values tr(rho O); Section III-C closes
with the same quantity computed on tiled operands.  Here they are computed on
plain dense matrices.
"""

from __future__ import annotations

import numpy as np

_PAULI = [
    np.eye(2, dtype=np.complex128),
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def trace(H: np.ndarray) -> float:
    """tr H = sum_i Re h_ii (the imaginary part vanishes for hermitian H)."""
    return float(np.real(np.trace(np.asarray(H))))


def expectation(rho: np.ndarray, O: np.ndarray) -> float:
    """Re tr(rho O) = Re sum_ij rho_ij O_ji."""
    rho = np.asarray(rho)
    O = np.asarray(O)
    return float(np.real(np.sum(rho * O.T)))


def pauli_string_matrix(codes_row) -> np.ndarray:
    """Dense matrix of a Pauli string; codes 0=I 1=X 2=Y 3=Z, entry q acting on
    qubit q.  Qubit 0 is the least significant index bit, so it is the last
    factor of the Kronecker product."""
    M = np.ones((1, 1), dtype=np.complex128)
    for c in reversed([int(x) for x in codes_row]):
        M = np.kron(M, _PAULI[c])
    return M


def pauli_sum_matrix(codes, coeffs) -> np.ndarray:
    """sum_t coeffs[t] P_t as a dense hermitian matrix."""
    codes = np.asarray(codes)
    out = None
    for row, c in zip(codes, coeffs):
        P = float(c) * pauli_string_matrix(row)
        out = P if out is None else out + P
    return out


def pauli_sum_expectation(rho: np.ndarray, codes, coeffs) -> float:
    """tr(rho O) for O = sum_t coeffs[t] P_t, via the dense matrices."""
    return expectation(rho, pauli_sum_matrix(codes, coeffs))


def density_from_factor(G: np.ndarray) -> np.ndarray:
    """rho = G G^dagger / tr(G G^dagger)."""
    G = np.asarray(G, dtype=np.complex128)
    R = G @ G.conj().T
    return R / np.real(np.trace(R))
