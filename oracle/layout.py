"""The tiled lower-triangle format -- test infrastructure.

Section III-B: the N x N hermitian matrix is covered by square tiles of edge
M = 2^m; only tiles T_{ti,tj} with ti >= tj are stored, tiles one after the
other in row-major order of the tile grid (tile (ti, tj) is number
ti(ti+1)/2 + tj, the tile pointer arithmetic of Algorithm 3) and the M^2
entries of each tile row-major.  Diagonal tiles hold all M^2 entries.  The
paper pads N < M up to one full tile; Table I lists the resulting sizes.

The library does not pad: when N < M it uses a single N x N tile.  Both sizes
are provided here (``pad``).  This module is an independent model of the
format, used to pin Table I and to decode raw storage taken from the device.
"""

from __future__ import annotations

import numpy as np


def full_elems(n: int) -> int:
    """Table I, 'Full': N^2 entries."""
    return (1 << n) ** 2


def packed_elems(n: int) -> int:
    """Table I, 'Packed': the N(N+1)/2 entries of the lower triangle."""
    N = 1 << n
    return N * (N + 1) // 2


def tile_edge(n: int, m: int, pad: bool) -> int:
    """Tile edge used for an n-qubit operator: M = 2^m, or N when N < M and the
    storage is not padded."""
    M = 1 << m
    N = 1 << n
    return M if (pad or N >= M) else N


def tiled_elems(n: int, m: int, pad: bool = True) -> int:
    """Section III-B: N(N+M)/2 stored entries, with N raised to M when the
    matrix is padded to one tile."""
    N = 1 << n
    M = tile_edge(n, m, pad)
    Np = max(N, M)
    return Np * (Np + M) // 2


def tile_number(ti: int, tj: int) -> int:
    """Position of stored tile (ti, tj), ti >= tj, in the tile sequence."""
    assert ti >= tj
    return ti * (ti + 1) // 2 + tj


def encode(H: np.ndarray, m: int, pad: bool = False) -> np.ndarray:
    """Raw tiled storage (1-D complex array) of a dense hermitian matrix."""
    H = np.asarray(H, dtype=np.complex128)
    N = H.shape[0]
    n = N.bit_length() - 1
    M = tile_edge(n, m, pad)
    Np = max(N, M)
    if Np != N:
        Hp = np.zeros((Np, Np), dtype=np.complex128)
        Hp[:N, :N] = H
        H = Hp
    nt = Np // M
    out = np.empty(tiled_elems(n, m, pad), dtype=np.complex128)
    for ti in range(nt):
        for tj in range(ti + 1):
            t = tile_number(ti, tj)
            out[t * M * M:(t + 1) * M * M] = H[ti * M:(ti + 1) * M, tj * M:(tj + 1) * M].reshape(-1)
    return out


def stored_tile(raw: np.ndarray, n: int, m: int, ti: int, tj: int, pad: bool = False) -> np.ndarray:
    """The stored M x M tile (ti, tj), ti >= tj, as a view-free copy."""
    M = tile_edge(n, m, pad)
    t = tile_number(ti, tj)
    return np.asarray(raw[t * M * M:(t + 1) * M * M]).reshape(M, M).copy()


def decode(raw: np.ndarray, n: int, m: int, pad: bool = False) -> np.ndarray:
    """Dense hermitian matrix represented by raw tiled storage: entries with
    i >= j are read from their stored tile, the others are the conjugates of
    their mirrors.  (The upper halves of diagonal tiles are a redundant copy
    and are not used here.)"""
    N = 1 << n
    M = tile_edge(n, m, pad)
    Np = max(N, M)
    nt = Np // M
    D = np.zeros((Np, Np), dtype=np.complex128)
    for ti in range(nt):
        for tj in range(ti + 1):
            D[ti * M:(ti + 1) * M, tj * M:(tj + 1) * M] = stored_tile(raw, n, m, ti, tj, pad)
    low = np.tril(D)
    D = low + np.tril(D, -1).conj().T
    return D[:N, :N]


def diagonal_tile_asymmetry(raw: np.ndarray, n: int, m: int, pad: bool = False) -> float:
    """max over diagonal tiles of |T - T^dagger| / max|T|: how far the stored
    upper halves of diagonal tiles are from the conjugates of the lower ones."""
    N = 1 << n
    M = tile_edge(n, m, pad)
    nt = max(N, M) // M
    worst = 0.0
    for t in range(nt):
        T = stored_tile(raw, n, m, t, t, pad)
        scale = max(np.abs(T).max(), 1e-300)
        worst = max(worst, float(np.abs(T - T.conj().T).max() / scale))
    return worst


def cross_tile_cases(n: int, m: int, a: int) -> dict:
    """Algorithm 3's case analysis for a single-qubit op on qubit a >= m.

    For every pair of base tile indices tj <= ti < N/2M the four tiles are
    (ti0, tj0), (ti0, tj1), (ti1, tj0), (ti1, tj1) with bit a-m of the tile
    index inserted as 0/1.  Tile (ti0, tj1) is stored when ti0 > tj1 (case
    A), lies above the diagonal with a stored mirror (tj1, ti0) when ti != tj
    (case B), and is the adjoint of tile (ti1, tj0) when ti == tj (case C).
    Returns the case counts and the list of tiles each pair touches.
    """
    from .local_block import insert_bits

    ap = a - m
    N = 1 << n
    M = 1 << m
    nb = N // (2 * M)
    counts = {"A": 0, "B": 0, "C": 0}
    touched = []
    for ti in range(nb):
        ti0 = insert_bits(ti, 0, [ap])
        ti1 = ti0 + (1 << ap)
        for tj in range(ti + 1):
            tj0 = insert_bits(tj, 0, [ap])
            tj1 = tj0 + (1 << ap)
            tiles = [(ti0, tj0), (ti1, tj0), (ti1, tj1)]
            if ti0 > tj1:
                counts["A"] += 1
                tiles.append((ti0, tj1))
            elif ti != tj:
                counts["B"] += 1
                tiles.append((tj1, ti0))
            else:
                counts["C"] += 1
            touched.append(tiles)
    return {"counts": counts, "touched": touched, "nb": nb}


def tiled_expectation(raw_rho: np.ndarray, raw_O: np.ndarray, n: int, m: int, pad: bool = False) -> float:
    """tr(rho O) from two tiled operands (Section III-C, closing formula): the
    Frobenius products of the diagonal tiles once, plus twice the real parts
    of the Frobenius products of the strictly lower tiles.  (The printed
    formula's second sum runs over ti >= tj, which would count the diagonal
    tiles a second time; the strict reading is the one that equals tr(rho O).)"""
    N = 1 << n
    M = tile_edge(n, m, pad)
    nt = max(N, M) // M
    total = 0.0
    for ti in range(nt):
        for tj in range(ti + 1):
            a = stored_tile(raw_O, n, m, ti, tj, pad)
            b = stored_tile(raw_rho, n, m, ti, tj, pad)
            f = float(np.real(np.sum(a.conj() * b)))
            total += f if ti == tj else 2.0 * f
    return total
