"""Dense Kraus map with Kronecker-expanded operators -- test infrastructure.

Section II-A, Eq. (1): Phi(H) = sum_a K_a H K_a^dagger on an N x N complex
matrix, N = 2^n.  For a k-local operation K_a = I (x) L_a up to the ordering of
qubits (Section II-A, the factorisation below Eq. (1)).  Section IV-A uses this
form, with the extended Kraus matrices assembled beforehand and plain matrix
products, as its naive baseline; that is what this module is.
"""

from __future__ import annotations

from typing import Iterable, Sequence

import numpy as np


def expand_local(L: np.ndarray, targets: Sequence[int], n: int) -> np.ndarray:
    """The N x N matrix K = I (x) L with L acting on ``targets``.

    Index convention: qubit q is bit q of a basis index (little-endian, the
    reading that makes Section II-B's X swap h_{i,j} <-> h_{i xor 2^a, j xor 2^a}
    act on qubit a).  Local index bit l of L belongs to ``targets[l]``.
    K[i, j] = L[loc(i), loc(j)] when i and j agree on every non-target bit,
    and 0 otherwise, where loc(i) collects the target bits of i.
    """
    L = np.asarray(L, dtype=np.complex128)
    N = 1 << n
    idx = np.arange(N, dtype=np.int64)
    loc = np.zeros(N, dtype=np.int64)
    mask = 0
    for l, t in enumerate(targets):
        loc |= ((idx >> t) & 1) << l
        mask |= 1 << t
    rest = idx & ~mask
    same = rest[:, None] == rest[None, :]
    return np.where(same, L[loc[:, None], loc[None, :]], 0.0).astype(np.complex128)


def kraus_map(H: np.ndarray, kraus: np.ndarray, targets: Sequence[int]) -> np.ndarray:
    """Schroedinger picture, Eq. (1): sum_a K_a H K_a^dagger with K_a the
    extended form of each local Kraus operator (dense matrix products)."""
    H = np.asarray(H, dtype=np.complex128)
    n = H.shape[0].bit_length() - 1
    out = np.zeros_like(H)
    for L in np.asarray(kraus, dtype=np.complex128):
        K = expand_local(L, targets, n)
        out += K @ H @ K.conj().T
    return out


def kraus_map_adjoint(H: np.ndarray, kraus: np.ndarray, targets: Sequence[int]) -> np.ndarray:
    """Heisenberg picture: the adjoint map Phi*(O) = sum_a K_a^dagger O K_a,
    dual to Eq. (1) under the trace inner product <A,B> = tr(A^dagger B)
    (Section II-A, the sentence after Eq. (1))."""
    H = np.asarray(H, dtype=np.complex128)
    n = H.shape[0].bit_length() - 1
    out = np.zeros_like(H)
    for L in np.asarray(kraus, dtype=np.complex128):
        K = expand_local(L, targets, n)
        out += K.conj().T @ H @ K
    return out


def apply_ops(H: np.ndarray, ops: Iterable, adjoint: bool = False) -> np.ndarray:
    """Apply a sequence of ops (objects with ``targets`` and ``mats``) one after
    the other, each as :func:`kraus_map` (or :func:`kraus_map_adjoint` when
    ``adjoint``).  The order is the order given; a Heisenberg evolution of a
    circuit passes the ops reversed."""
    out = np.asarray(H, dtype=np.complex128).copy()
    f = kraus_map_adjoint if adjoint else kraus_map
    for op in ops:
        out = f(out, op.mats, op.targets)
    return out
