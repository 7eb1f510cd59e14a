"""Stratified choice of blocks h_{s,s'} (Eq. (2)) for full-size parity checks.

Uniform labels rarely land where the conjugation pass has its special cases
at full size: groups on the diagonal of the reduced tile grid (ti = tj after
the tile-selecting target bits are removed; there a group holds a tile and
its mirror, Algorithm 3 case C and its two-target generalisation) and the
last tile row (the largest tile numbers, where element offsets are widest).
This module draws a fixed number of labels from each of those strata and the
rest uniformly.  It uses only index arithmetic; the blocks' indices come from
the oracle's block_indices."""

from __future__ import annotations

import numpy as np

import oracle


def free_positions(n, targets):
    return [q for q in range(n) if q not in set(targets)]


def block_labels(n, targets, m, nblocks, rng, per_stratum=120):
    """(s, s') label pairs: ``per_stratum`` in diagonal tile groups, as many in
    the last tile row (some of them also diagonal), the rest uniform.  m is
    the effective tile exponent."""
    k = len(targets)
    nfree = n - k
    free = free_positions(n, targets)
    low_bits = sum(1 for q in free if q < m)         # label bits that lie inside a tile
    low_mask = (1 << low_bits) - 1
    all_mask = (1 << nfree) - 1
    high_mask = all_mask & ~low_mask                  # label bits that select the tile
    s = rng.integers(0, 1 << nfree, size=nblocks, dtype=np.int64)
    s2 = rng.integers(0, 1 << nfree, size=nblocks, dtype=np.int64)
    a = min(per_stratum, nblocks)
    b = min(2 * per_stratum, nblocks)
    # diagonal tile groups: s' shares the tile-selecting bits of s
    s2[:a] = (s[:a] & high_mask) | (s2[:a] & low_mask)
    # last tile row: every tile-selecting bit of the row label set
    s[a:b] |= high_mask
    # a few of them also on the diagonal
    c = a + (b - a) // 4
    s2[a:c] = (s[a:c] & high_mask) | (s2[a:c] & low_mask)
    return s, s2


def block_entries(n, targets, m, nblocks, rng, per_stratum=120):
    """Row and column indices of the sampled blocks' entries, flattened
    (block-major, row-major inside a block), and the block edge 2^k."""
    s, s2 = block_labels(n, targets, m, nblocks, rng, per_stratum)
    k = len(targets)
    rows = np.stack([oracle.block_indices(int(x), targets) for x in s])
    cols = np.stack([oracle.block_indices(int(x), targets) for x in s2])
    d = 1 << k
    R = np.repeat(rows[:, :, None], d, axis=2).reshape(nblocks, -1)
    C = np.repeat(cols[:, None, :], d, axis=1).reshape(nblocks, -1)
    return R.reshape(-1), C.reshape(-1), d


def strata_counts(n, targets, m, R, C, d):
    """How many blocks touch a diagonal group / the last tile row (for the
    tests' own check that the strata are populated)."""
    k = len(targets)
    cross = [t for t in targets if t >= m]
    keep = ~sum(1 << t for t in cross) if cross else ~0
    nb = R.shape[0] // (d * d)
    Rb = R.reshape(nb, d * d)
    Cb = C.reshape(nb, d * d)
    diag = np.all(((Rb[:, :1] & keep) >> m) == ((Cb[:, :1] & keep) >> m), axis=1)
    last_tile = ((1 << n) - 1) >> m
    last = np.any(((np.maximum(Rb, Cb)) >> m) == last_tile, axis=1)
    return int(diag.sum()), int(last.sum())
