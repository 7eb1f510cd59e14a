"""Block form of a k-local Kraus map -- test infrastructure.

Section II-A, Eq. (2): a k-local operation splits the index space into
2^(n-k) invariant subspaces and maps every 2^k x 2^k block h_{s,s'} to
sum_a L_a h_{s,s'} L_a^dagger.  Subroutine 1 (insertBits) rebuilds the global
indices of a block from its subspace label.  This module implements that
mathematics twice: once over a whole dense matrix by tensor contraction (used
where the Kronecker form is too slow, n up to ~14) and once for single blocks
(used to check sampled blocks of operators too large to hold densely; the
tests gather a block's rows and columns with :func:`block_indices`).
"""

from __future__ import annotations

from typing import Iterable, Sequence

import numpy as np


def insert_bits(s: int, a: int, positions: Sequence[int]) -> int:
    """Subroutine 1: insert the bits of the local index ``a`` into the label
    ``s`` at the ascending global bit positions ``positions``; bit l of ``a``
    lands at ``positions[l]`` and the bits of ``s`` fill the other positions
    in order."""
    g = int(s)
    for l, pos in enumerate(positions):
        low = g & ((1 << pos) - 1)
        high = (g >> pos) << 1
        high |= (int(a) >> l) & 1
        g = (high << pos) | low
    return g


def block_indices(s: int, targets: Sequence[int]) -> np.ndarray:
    """Global indices of the 2^k members of invariant subspace ``s``: entry
    ``u`` is the index whose target bits spell ``u`` (local bit l <-> targets[l])
    and whose other bits spell ``s``."""
    k = len(targets)
    base = insert_bits(s, 0, sorted(targets))
    out = np.empty(1 << k, dtype=np.int64)
    for u in range(1 << k):
        g = base
        for l, t in enumerate(targets):
            g |= ((u >> l) & 1) << t
        out[u] = g
    return out


def block_update(blk: np.ndarray, kraus: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """Eq. (2) for one block (or a stack of blocks, leading axis): sum_a
    L_a h L_a^dagger; with ``adjoint`` the Heisenberg form sum_a L_a^dagger h L_a."""
    blk = np.asarray(blk, dtype=np.complex128)
    out = np.zeros_like(blk)
    for L in np.asarray(kraus, dtype=np.complex128):
        A = L.conj().T if adjoint else L
        out += A @ blk @ A.conj().T
    return out


def _apply_on_axes(T: np.ndarray, A: np.ndarray, axes_of_local_bit: Sequence[int]) -> np.ndarray:
    """Contract the k-local matrix A (output index, input index) with the
    tensor axes that carry its local bits; local bit l sits on
    ``axes_of_local_bit[l]``.  The output bits are put back on the same axes."""
    k = len(axes_of_local_bit)
    At = A.reshape((2,) * (2 * k))  # axis k-1-l: output bit l; axis 2k-1-l: input bit l
    in_axes = [2 * k - 1 - l for l in range(k)]
    R = np.tensordot(At, T, axes=(in_axes, list(axes_of_local_bit)))
    # R's first k axes are At's output axes, i.e. local bits k-1, ..., 0
    dest = [axes_of_local_bit[k - 1 - i] for i in range(k)]
    return np.moveaxis(R, list(range(k)), dest)


def local_block_map(H: np.ndarray, kraus: np.ndarray, targets: Sequence[int],
                    adjoint: bool = False) -> np.ndarray:
    """Eq. (2) applied to every block of a dense matrix at once.

    The N x N matrix is viewed as a tensor with one binary axis per row bit and
    per column bit (row bit q on axis n-1-q, column bit q on axis 2n-1-q); L_a
    is contracted with the target row axes and conj(L_a) with the target
    column axes, and the results are summed over a.
    """
    H = np.asarray(H, dtype=np.complex128)
    N = H.shape[0]
    n = N.bit_length() - 1
    T = H.reshape((2,) * (2 * n))
    row_axes = [n - 1 - t for t in targets]
    col_axes = [2 * n - 1 - t for t in targets]
    out = np.zeros_like(T)
    for L in np.asarray(kraus, dtype=np.complex128):
        A = L.conj().T if adjoint else L
        R = _apply_on_axes(T, A, row_axes)
        out += _apply_on_axes(R, A.conj(), col_axes)
    return out.reshape(N, N)


def apply_ops_local(H: np.ndarray, ops: Iterable, adjoint: bool = False) -> np.ndarray:
    """Apply a sequence of ops with :func:`local_block_map`, in the order given."""
    out = np.asarray(H, dtype=np.complex128)
    for op in ops:
        out = local_block_map(out, op.mats, op.targets, adjoint=adjoint)
    return out
