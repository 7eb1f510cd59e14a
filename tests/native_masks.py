"""Which stored entries a permutation-and-phase op changes, derived from the
op's transfer matrix (test helper, independent of the library)."""

import numpy as np

from oracle import layout


def sorted_local(kraus, targets):
    """The Kraus matrices with local bits renumbered to ascending targets."""
    k = len(targets)
    order = np.argsort(targets)  # sorted bit ls is user bit order[ls]
    d = 1 << k
    user = np.array([sum(((us >> ls) & 1) << int(order[ls]) for ls in range(k)) for us in range(d)])
    return np.asarray(kraus)[:, user[:, None], user[None, :]]


def changing_entries(kraus, targets, heis):
    """Local entries (u, v), ascending target order, that the map does not
    leave exactly in place: row (u, v) of the row-major transfer matrix
    differs from the unit vector (entries equal to it within 2^-50 count as
    unchanged, the tolerance the library applies to unit phases)."""
    A = sorted_local(kraus, targets)
    if heis:
        A = np.conj(np.transpose(A, (0, 2, 1)))
    d = A.shape[1]
    S = sum(np.kron(a, np.conj(a)) for a in A)
    return np.abs(S - np.eye(d * d)).max(axis=1).reshape(d, d) > 2.0 ** -50


def expected_writes(n, m, targets, changing):
    """Per stored entry of the tiled layout: 1 if the op changes it, else 0."""
    N = 1 << n
    idx = np.arange(N)
    loc = np.zeros(N, dtype=np.int64)
    for ls, t in enumerate(sorted(targets)):
        loc |= ((idx >> t) & 1) << ls
    E = changing[loc[:, None], loc[None, :]].astype(np.complex128)
    return layout.encode(E, m).real.astype(np.int32)
