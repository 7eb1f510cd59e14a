"""Checks that pin the CPU oracle to facts fixed by the paper and by the
mathematics, written so that each takes the oracle function it checks as an
argument.  The pin tests call them with the real oracle; the mutation tests
call them with deliberately broken variants and expect them to fail.

Every check returns a non-negative error; the caller compares it with a
tolerance.  Closed forms are computed here with plain index arithmetic, never
by calling the oracle.
"""

from __future__ import annotations

import numpy as np

import synth

PAULI_1Q = {
    1: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    2: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    3: np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_density(n, rng, rank=None):
    g = synth.ginibre_factor(n, rank or (1 << n), rng)
    r = g @ g.conj().T
    return r / np.trace(r).real


def pauli_conjugation_error(kmap, n, rng) -> float:
    """P rho P for a Pauli string P (applied one single-qubit Pauli at a time
    through ``kmap``) against the sign/permutation closed form
    (P rho P)_{ij} = (-1)^{popcount((i^j) & z)} rho_{i^x, j^x}, where x marks
    X/Y positions and z marks Y/Z positions (Section II-B: X swaps entries,
    Y swaps and negates, Z negates)."""
    rho = synth.random_hermitian_dense(n, rng)
    codes = rng.integers(0, 4, size=n)
    out = rho.copy()
    x = z = 0
    for q, c in enumerate(codes):
        c = int(c)
        if c == 0:
            continue
        out = kmap(out, PAULI_1Q[c][None], [q])
        if c in (1, 2):
            x |= 1 << q
        if c in (2, 3):
            z |= 1 << q
    N = 1 << n
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    par = np.vectorize(lambda v: bin(int(v)).count("1") & 1)((i ^ j) & z)
    expect = np.where(par == 1, -1.0, 1.0) * rho[i ^ x, j ^ x]
    return float(np.abs(out - expect).max())


def single_target_kron_error(expand, n, rng) -> float:
    """K = I (x) L for one target q equals kron(I_{2^(n-1-q)}, L, I_{2^q})."""
    worst = 0.0
    for q in range(n):
        L = synth.haar_unitary(2, rng)
        ref = np.kron(np.kron(np.eye(1 << (n - 1 - q)), L), np.eye(1 << q))
        worst = max(worst, float(np.abs(expand(L, [q], n) - ref).max()))
    return worst


def pair_kron_error(expand, n, rng) -> float:
    """Adjacent ascending targets (q, q+1): K = kron(I, L, I) with L's local
    index b_q + 2 b_{q+1}; the reversed order (q+1, q) uses SWAP L SWAP."""
    swap = np.eye(4)[[0, 2, 1, 3]]
    worst = 0.0
    for q in range(n - 1):
        L = synth.haar_unitary(4, rng)
        ref = np.kron(np.kron(np.eye(1 << (n - 2 - q)), L), np.eye(1 << q))
        worst = max(worst, float(np.abs(expand(L, [q, q + 1], n) - ref).max()))
        worst = max(worst, float(np.abs(expand(swap @ L @ swap, [q + 1, q], n) - ref).max()))
    return worst


def vec_identity_error(block_fn, rng) -> float:
    """Eq. (3): stacking columns, vec(sum_a L_a h L_a^dagger) =
    (sum_a conj(L_a) (x) L_a) vec(h); checked for 1- and 2-qubit Kraus sets."""
    worst = 0.0
    for k in (1, 2):
        d = 1 << k
        kraus = synth.random_kraus_set(k, 3, rng)
        h = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        S = sum(np.kron(L.conj(), L) for L in kraus)
        lhs = block_fn(h, kraus).reshape(-1, order="F")
        rhs = S @ h.reshape(-1, order="F")
        worst = max(worst, rel(lhs, rhs))
    return worst


def hermiticity_error(kmap, n, rng) -> float:
    """Any Kraus map keeps H hermitian (Section III, argument before III-A)."""
    H = synth.random_hermitian_dense(n, rng)
    worst = 0.0
    for k in (1, 2):
        t = [int(v) for v in rng.choice(n, size=k, replace=False)]
        kraus = (rng.standard_normal((3, 1 << k, 1 << k)) + 1j * rng.standard_normal((3, 1 << k, 1 << k)))
        out = kmap(H, kraus, t)
        worst = max(worst, rel(out, out.conj().T))
    return worst


def trace_preservation_error(kmap, n, rng) -> float:
    """Trace-preserving sets keep tr rho: depolarising (Section IV-A), amplitude
    damping, dephasing, Haar unitaries, a random rank-4 two-qubit set."""
    rho = random_density(n, rng)
    sets = [
        (synth.depolarising_kraus(0.07), [int(rng.integers(n))]),
        (synth.amplitude_damping_kraus(0.3), [int(rng.integers(n))]),
        (synth.dephasing_kraus(0.2), [int(rng.integers(n))]),
        (synth.haar_unitary(2, rng)[None], [int(rng.integers(n))]),
        (synth.random_kraus_set(2, 4, rng), [int(v) for v in rng.choice(n, 2, replace=False)]),
    ]
    worst = 0.0
    for kraus, t in sets:
        worst = max(worst, abs(np.trace(kmap(rho, kraus, t)).real - 1.0))
    return worst


def depolarising_closed_form_error(kmap, n, rng, p=0.1) -> float:
    """Depolarising on qubit a (Section IV-A): entries whose row and column
    differ in bit a scale by 1 - 4p/3; entries with equal bit a become
    (1 - 2p/3) rho_ij + (2p/3) rho_{i^2^a, j^2^a}; I/N is a fixed point."""
    rho = synth.random_hermitian_dense(n, rng)
    N = 1 << n
    worst = 0.0
    for a in range(n):
        out = kmap(rho, synth.depolarising_kraus(p), [a])
        i = np.arange(N)[:, None]
        j = np.arange(N)[None, :]
        f = 1 << a
        differ = ((i ^ j) & f) != 0
        expect = np.where(differ, (1 - 4 * p / 3) * rho,
                          (1 - 2 * p / 3) * rho + (2 * p / 3) * rho[i ^ f, j ^ f])
        worst = max(worst, float(np.abs(out - expect).max()))
        mm = np.eye(N) / N
        worst = max(worst, float(np.abs(kmap(mm, synth.depolarising_kraus(p), [a]) - mm).max()))
    return worst


def amplitude_damping_error(kmap, n, rng, gamma=0.2, reps=3) -> float:
    """Amplitude damping on qubit a applied ``reps`` times: the bit-a=1
    population scales by (1-g)^reps, coherences between bit a = 0 and 1 by
    (1-g)^(reps/2), and the trace is kept."""
    rho = random_density(n, rng)
    a = int(rng.integers(n))
    out = rho
    for _ in range(reps):
        out = kmap(out, synth.amplitude_damping_kraus(gamma), [a])
    N = 1 << n
    idx = np.arange(N)
    one = (idx >> a) & 1 == 1
    p1_before = rho[one, one].real.sum()
    p1_after = out[one, one].real.sum()
    err = abs(p1_after - (1 - gamma) ** reps * p1_before)
    i = idx[:, None]
    j = idx[None, :]
    mask = (((i >> a) & 1) == 0) & (((j >> a) & 1) == 1)
    err = max(err, float(np.abs(out[mask] - (1 - gamma) ** (reps / 2) * rho[mask]).max()))
    err = max(err, abs(np.trace(out).real - 1.0))
    return float(err)


def dephasing_error(kmap, n, rng, p=0.15) -> float:
    """Dephasing on qubit a: entries with differing bit a scale by 1 - 2p, the
    others are unchanged."""
    rho = synth.random_hermitian_dense(n, rng)
    a = int(rng.integers(n))
    out = kmap(rho, synth.dephasing_kraus(p), [a])
    N = 1 << n
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    differ = ((i ^ j) >> a) & 1 == 1
    return float(np.abs(out - np.where(differ, (1 - 2 * p) * rho, rho)).max())


def duality_error(kmap, kmap_adj, n, rng) -> float:
    """tr(O Phi(rho)) = tr(Phi*(O) rho) (Section I and II-A), for a random
    non-unital two-qubit Kraus set; Phi*(I) = I for a trace-preserving set."""
    rho = random_density(n, rng)
    O = synth.random_hermitian_dense(n, rng)
    t = [int(v) for v in rng.choice(n, 2, replace=False)]
    kraus = synth.random_kraus_set(2, 3, rng)
    lhs = np.trace(O @ kmap(rho, kraus, t))
    rhs = np.trace(kmap_adj(O, kraus, t) @ rho)
    err = abs(lhs - rhs) / max(abs(lhs), 1e-12)
    I = np.eye(1 << n)
    err = max(err, float(np.abs(kmap_adj(I, kraus, t) - I).max()))
    return float(err)


def unitary_roundtrip_error(kmap, n, rng) -> float:
    """U followed by U^dagger returns H."""
    H = synth.random_hermitian_dense(n, rng)
    t = [int(v) for v in rng.choice(n, 2, replace=False)]
    U = synth.haar_unitary(4, rng)
    back = kmap(kmap(H, U[None], t), U.conj().T[None], t)
    return rel(back, H)


def positivity_error(kmap, n, rng) -> float:
    """A CP map keeps rho positive: the smallest eigenvalue stays >= 0."""
    rho = random_density(n, rng, rank=2)
    worst = 0.0
    for _ in range(4):
        t = [int(v) for v in rng.choice(n, 2, replace=False)]
        rho = kmap(rho, synth.random_kraus_set(2, 5, rng), t)
        rho = kmap(rho, synth.depolarising_kraus(0.05), [t[0]])
        worst = max(worst, max(0.0, -float(np.linalg.eigvalsh((rho + rho.conj().T) / 2).min())))
    return worst


def cnot_basis_error(kmap, n, rng) -> float:
    """CNOT on (control c, target t) maps the matrix unit E_ij to
    E_{f(i), f(j)} with f flipping bit t when bit c is set; this fixes which
    local bit belongs to which target without reference to any matrix
    convention.  Also: the quarter of entries with bit c clear in both row
    and column is left bitwise unchanged (Appendix, CNOT discussion)."""
    N = 1 << n
    c, t = (int(v) for v in rng.choice(n, 2, replace=False))
    f = lambda v: v ^ (1 << t) if (v >> c) & 1 else v
    err = 0.0
    for _ in range(6):
        i, j = (int(v) for v in rng.integers(0, N, size=2))
        E = np.zeros((N, N), dtype=np.complex128)
        E[i, j] = 1.0
        out = kmap(E, synth.cnot_matrix()[None], [c, t])
        ref = np.zeros_like(E)
        ref[f(i), f(j)] = 1.0
        err = max(err, float(np.abs(out - ref).max()))
    H = synth.random_hermitian_dense(n, rng)
    out = kmap(H, synth.cnot_matrix()[None], [c, t])
    idx = np.arange(N)
    zero = ((idx >> c) & 1) == 0
    q = np.ix_(zero, zero)
    if not np.array_equal(out[q], H[q]):
        err = max(err, 1.0)
    return err


def diagonal_gate_error(kmap, n, rng) -> float:
    """Diagonal gates leave the entries whose row and column share the target
    bit unchanged (Section II-B); with S and Z the result is exact."""
    H = synth.random_hermitian_dense(n, rng)
    N = 1 << n
    a = int(rng.integers(n))
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    same = (((i ^ j) >> a) & 1) == 0
    err = 0.0
    for g in ("S", "Z"):
        out = kmap(H, synth.named_gate(g)[None], [a])
        if not np.array_equal(out[same], H[same]):
            err = 1.0
    return err


def local_vs_dense_error(local_map, dense_map, n, rng) -> float:
    """The block form (Eq. (2)) and the Kronecker form (Eq. (1)) agree on
    every target set, in both pictures."""
    H = synth.random_hermitian_dense(n, rng)
    worst = 0.0
    targets = [[q] for q in range(n)] + [[a, b] for a in range(n) for b in range(n) if a != b]
    for t in targets:
        kraus = synth.random_kraus_set(len(t), 2, rng)
        worst = max(worst, rel(local_map(H, kraus, t), dense_map(H, kraus, t)))
    return worst
