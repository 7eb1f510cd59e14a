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


# ---------------------------------------------------------------- blocks --

def _digits_index(s, u, targets, n):
    """Index built digit by digit (little-endian): the digit at targets[l] is
    bit l of u, the remaining positions, in increasing order, take the bits of
    s in order.  Written without bit insertion, as a check of it."""
    k = len(targets)
    s_bits = [(s >> b) & 1 for b in range(n - k)]
    digits = []
    for q in range(n):
        if q in targets:
            digits.append((u >> list(targets).index(q)) & 1)
        else:
            digits.append(s_bits.pop(0))
    return sum(d << q for q, d in enumerate(digits))


def block_indices_error(block_indices, n, target_sets) -> int:
    """Eq. (2) and Subroutine 1: the 2^(n-k) invariant subspaces of a k-local
    op partition the index range, and member u of subspace s has its target
    bits spelling u (local bit l on targets[l], in the caller's order) and its
    other bits spelling s.  Returns the number of violations (0 = pinned)."""
    bad = 0
    N = 1 << n
    for targets in target_sets:
        k = len(targets)
        seen = np.zeros(N, dtype=np.int64)
        for s in range(1 << (n - k)):
            got = [int(v) for v in block_indices(s, targets)]
            want = [_digits_index(s, u, targets, n) for u in range(1 << k)]
            bad += sum(1 for a, b in zip(got, want) if a != b) + abs(len(got) - len(want))
            for g in got:
                if 0 <= g < N:
                    seen[g] += 1
                else:
                    bad += 1
        bad += int(np.count_nonzero(seen != 1))
    return bad


def block_form_consistency_error(block_indices, block_update, local_map, n, rng) -> float:
    """Eq. (2): gathering block h_{s,s'} (rows of subspace s, columns of s')
    after the whole-matrix map equals mapping the gathered block, for every
    pair (s, s'), both pictures, and unsorted target orders."""
    H = synth.random_hermitian_dense(n, rng)
    worst = 0.0
    for targets in ([2], [3, 1], [0, 4], [4, 2, 0] if n >= 5 else [2, 0, 1]):
        k = len(targets)
        kraus = synth.random_kraus_set(k, 2, rng) if k < 3 else synth.haar_unitary(8, rng)[None]
        for adjoint in (False, True):
            full = local_map(H, kraus, targets, adjoint=adjoint)
            idx = [block_indices(s, targets) for s in range(1 << (n - k))]
            for r in idx:
                for c in idx:
                    blk = block_update(H[np.ix_(r, c)], kraus, adjoint=adjoint)
                    worst = max(worst, float(np.abs(full[np.ix_(r, c)] - blk).max()))
    return worst


# ----------------------------------------------------------- pauli sums --

def _pauli_masks(codes_row):
    """x marks X/Y positions, z marks Y/Z positions, ny counts the Y's."""
    x = z = ny = 0
    for q, c in enumerate(int(v) for v in codes_row):
        if c in (1, 2):
            x |= 1 << q
        if c in (2, 3):
            z |= 1 << q
        ny += c == 2
    return x, z, ny


def _parity(v):
    return bin(int(v)).count("1") & 1


def pauli_sum_matrix_error(pauli_sum_matrix, n, rng, nterms=7) -> float:
    """Section I's observables as Pauli sums, entry by entry: a string with
    masks (x, z) and ny Y factors sends basis state j to
    i^ny (-1)^popcount(j & z) |j xor x> (X flips a bit, Z signs it, Y = iXZ
    does both), so O[j ^ x, j] gets c_t times that phase.  Random strings
    over all four letters, including I on some qubits."""
    N = 1 << n
    codes = rng.integers(0, 4, size=(nterms, n))
    codes[0, :] = 2  # an all-Y string: the phase i^n matters
    coeffs = rng.standard_normal(nterms)
    want = np.zeros((N, N), dtype=np.complex128)
    for row, c in zip(codes, coeffs):
        x, z, ny = _pauli_masks(row)
        for j in range(N):
            want[j ^ x, j] += c * (1j ** ny) * (-1.0 if _parity(j & z) else 1.0)
    got = np.asarray(pauli_sum_matrix(codes, coeffs))
    return float(np.abs(got - want).max())


def pauli_sum_expectation_error(pauli_sum_expectation, n, rng, nterms=9) -> float:
    """tr(rho O) for a Pauli sum from the masks alone: for each string,
    sum_j (-i)^ny (-1)^popcount(j & z) rho[j ^ x, j], weighted by c_t and
    summed (Section I).  Checked on a random density matrix."""
    N = 1 << n
    rho = random_density(n, rng)
    codes = rng.integers(0, 4, size=(nterms, n))
    codes[0, :] = 2
    codes[1, :] = 0
    codes[1, 0] = 2  # a single Y: the sign of (-i)^ny matters
    coeffs = rng.standard_normal(nterms)
    want = 0.0
    for row, c in zip(codes, coeffs):
        x, z, ny = _pauli_masks(row)
        tot = 0.0 + 0.0j
        for j in range(N):
            tot += ((-1j) ** ny) * (-1.0 if _parity(j & z) else 1.0) * rho[j ^ x, j]
        want += c * tot.real
    return abs(float(pauli_sum_expectation(rho, codes, coeffs)) - want)


# ------------------------------------------------------------- op order --

def op_order_error(apply_ops, n=3, q=1, gamma=0.3) -> float:
    """Section II-A: a circuit applies its maps one after the other.  X then
    amplitude damping on qubit q takes |0><0| to gamma|0><0| + (1-gamma)|e><e|
    (e = 2^q: X moves the population to bit q = 1, damping returns a fraction
    gamma); the other order leaves |e><e|.  In the Heisenberg picture with the
    ops given as [damping, X], the projector P1 on bit q = 1 goes to
    (1-gamma) P0 (damping's adjoint keeps P1 scaled by 1-gamma, X's swaps it to
    P0); the other order gives P1 + gamma P0.  Returns the largest deviation
    from these hand-derived results."""
    from types import SimpleNamespace

    N = 1 << n
    e = 1 << q
    X = synth.named_gate("X")[None]
    ad = synth.amplitude_damping_kraus(gamma)
    opX = SimpleNamespace(targets=[q], mats=X)
    opA = SimpleNamespace(targets=[q], mats=ad)
    E0 = np.zeros((N, N), dtype=np.complex128)
    E0[0, 0] = 1.0
    want = np.zeros_like(E0)
    want[0, 0] = gamma
    want[e, e] = 1.0 - gamma
    err = float(np.abs(apply_ops(E0, [opX, opA]) - want).max())
    idx = np.arange(N)
    P1 = np.diag(((idx >> q) & 1).astype(np.complex128))
    P0 = np.eye(N, dtype=np.complex128) - P1
    err = max(err, float(np.abs(apply_ops(P1, [opA, opX], adjoint=True) - (1.0 - gamma) * P0).max()))
    return err


# ------------------------------------------------------------- readouts --

def trace_error(trace, n, rng) -> float:
    """The trace is invariant under unitary similarity: tr(U diag(l) U^dagger)
    = sum l for a Haar U; and tr I = N."""
    N = 1 << n
    lam = rng.standard_normal(N)
    U = synth.haar_unitary(N, rng)
    A = (U * lam) @ U.conj().T
    err = abs(float(trace(A)) - float(lam.sum()))
    err = max(err, abs(float(trace(np.eye(N, dtype=np.complex128))) - N))
    return err


def density_from_factor_error(density_from_factor, n, rng) -> float:
    """rho = G G^dagger / tr: for a single column v the result is the
    projector on v (rho v = v, rho^2 = rho); for r orthonormal columns scaled
    by any c it is the projector on their span divided by r (eigenvalues 1/r,
    r times, and 0)."""
    N = 1 << n
    v = rng.standard_normal((N, 1)) + 1j * rng.standard_normal((N, 1))
    P = np.asarray(density_from_factor(v))
    err = float(np.abs(P @ v - v).max() / np.abs(v).max())
    err = max(err, float(np.abs(P @ P - P).max()))
    r = 3
    Q = synth.haar_unitary(N, rng)[:, :r] * (2.0 - 0.5j)
    R = np.asarray(density_from_factor(Q))
    ev = np.sort(np.linalg.eigvalsh((R + R.conj().T) / 2))
    want = np.concatenate([np.zeros(N - r), np.full(r, 1.0 / r)])
    err = max(err, float(np.abs(ev - want).max()), float(np.abs(R - R.conj().T).max()))
    return err
