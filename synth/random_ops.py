"""Seeded random inputs: state factors, gates, Kraus sets, Pauli sums."""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Sequence

import numpy as np


@dataclass(frozen=True)
class Op:
    """One k-local quantum operation of a circuit.

    kind:     "unitary" (one matrix, r = 1) or "channel" (Kraus set, r >= 1)
    targets:  qubits acted on; local bit ``l`` of ``mats`` <-> ``targets[l]``
    mats:     complex128 array of shape (r, 2^k, 2^k)
    label:    free-form name used in reports ("haar1", "cnot", "depol", ...)
    """

    kind: str
    targets: tuple
    mats: np.ndarray = field(repr=False)
    label: str = ""

    @property
    def k(self) -> int:
        return len(self.targets)

    @property
    def r(self) -> int:
        return int(self.mats.shape[0])


def make_rng(seed) -> np.random.Generator:
    """A numpy Generator from an integer seed or a SeedSequence."""
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))


def spawn_rngs(seed: int, count: int) -> list:
    """``count`` independent Generators derived from one base seed."""
    return [make_rng(s) for s in np.random.SeedSequence(int(seed)).spawn(count)]


def _complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Entries with independent N(0,1) real and imaginary parts."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def ginibre_factor(n: int, rank: int, rng: np.random.Generator) -> np.ndarray:
    """Ginibre matrix G of shape (2^n, rank), complex128.

    A density matrix is formed from it as G G^dagger / tr(G G^dagger); that
    product is left to each consumer.
    """
    return _complex_gaussian(rng, (1 << n, rank)).astype(np.complex128)


def random_hermitian_dense(n: int, rng: np.random.Generator) -> np.ndarray:
    """(G + G^dagger)/2 for a square Ginibre G: hermitian, neither positive nor
    normalised, the kind of operator the paper benchmarks on (Section IV-A)."""
    g = _complex_gaussian(rng, (1 << n, 1 << n))
    return ((g + g.conj().T) / 2).astype(np.complex128)


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed U(d): QR of a complex Ginibre matrix with the phases of
    diag(R) moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    z = _complex_gaussian(rng, (d, d)) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph[None, :]).astype(np.complex128)


def haar_special_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar U(d) rescaled to determinant one."""
    u = haar_unitary(d, rng)
    return (u / np.linalg.det(u) ** (1.0 / d)).astype(np.complex128)


_I2 = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def depolarising_kraus(p: float) -> np.ndarray:
    """Single-qubit depolarising channel with the four Kraus operators of
    Section IV-A: sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z."""
    a = np.sqrt(1.0 - p)
    b = np.sqrt(p / 3.0)
    return np.stack([a * _I2, b * _X, b * _Y, b * _Z]).astype(np.complex128)


def amplitude_damping_kraus(gamma: float) -> np.ndarray:
    """Textbook amplitude damping: [[1,0],[0,sqrt(1-g)]] and [[0,sqrt(g)],[0,0]]."""
    k0 = np.array([[1, 0], [0, np.sqrt(1.0 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0, np.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return np.stack([k0, k1])


def dephasing_kraus(p: float) -> np.ndarray:
    """Textbook dephasing: sqrt(1-p) I and sqrt(p) Z."""
    return np.stack([np.sqrt(1.0 - p) * _I2, np.sqrt(p) * _Z]).astype(np.complex128)


def named_gate(name: str, theta: float = 0.0) -> np.ndarray:
    """A few fixed single-qubit gates (complex128, 2x2)."""
    name = name.upper()
    if name == "I":
        return _I2.copy()
    if name == "X":
        return _X.copy()
    if name == "Y":
        return _Y.copy()
    if name == "Z":
        return _Z.copy()
    if name == "H":
        return (np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0))
    if name == "S":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "T":
        return np.diag([1, np.exp(1j * np.pi / 4)]).astype(np.complex128)
    if name == "RZ":
        return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)
    if name == "RY":
        c, s = np.cos(theta / 2), np.sin(theta / 2)
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    raise ValueError(f"unknown gate {name}")


def cnot_matrix() -> np.ndarray:
    """CNOT on targets (control, target): local bit 0 is the control, local
    bit 1 the target; the target bit flips when the control bit is one."""
    m = np.zeros((4, 4), dtype=np.complex128)
    for u in range(4):
        m[u ^ 2 if (u & 1) else u, u] = 1.0
    return m


def permutation_gate(name: str) -> np.ndarray:
    """Multi-qubit gates with one nonzero per row.  Local bit l belongs to
    targets[l]: CZ (phase -1 on |11>), SWAP, ISWAP (swap with phase i),
    TOFFOLI (bits 0, 1 control, bit 2 flips), CCZ (phase -1 on |111>),
    FREDKIN (bit 0 controls a swap of bits 1 and 2)."""
    name = name.upper()
    if name in ("CZ", "SWAP", "ISWAP"):
        d = 4
    elif name in ("TOFFOLI", "CCZ", "FREDKIN"):
        d = 8
    else:
        raise ValueError(f"unknown gate {name}")
    m = np.zeros((d, d), dtype=np.complex128)
    for u in range(d):
        b = [(u >> l) & 1 for l in range(3)]
        if name == "CZ":
            m[u, u] = -1.0 if u == 3 else 1.0
        elif name == "SWAP":
            m[(u & ~3) | (b[0] << 1) | b[1], u] = 1.0
        elif name == "ISWAP":
            m[(b[0] << 1) | b[1], u] = 1j if b[0] != b[1] else 1.0
        elif name == "TOFFOLI":
            m[u ^ 4 if (b[0] and b[1]) else u, u] = 1.0
        elif name == "CCZ":
            m[u, u] = -1.0 if u == 7 else 1.0
        else:  # FREDKIN
            v = (b[0] | (b[2] << 1) | (b[1] << 2)) if b[0] else u
            m[v, u] = 1.0
    return m


def random_monomial(k: int, rng: np.random.Generator, diagonal: bool = False) -> np.ndarray:
    """A 2^k x 2^k unitary with one nonzero per row: a uniformly random
    permutation (the identity when ``diagonal``) with uniform random phases."""
    d = 1 << k
    perm = np.arange(d) if diagonal else rng.permutation(d)
    m = np.zeros((d, d), dtype=np.complex128)
    m[np.arange(d), perm] = np.exp(2j * np.pi * rng.random(d))
    return m


def random_pauli_sum(n: int, nterms: int, rng: np.random.Generator):
    """``nterms`` Pauli strings uniform over {I,X,Y,Z}^n without the identity
    string, with N(0,1) real coefficients.  Returns (codes uint8 (nterms, n),
    coeffs float64 (nterms,))."""
    codes = np.zeros((nterms, n), dtype=np.uint8)
    for t in range(nterms):
        while True:
            row = rng.integers(0, 4, size=n, dtype=np.uint8)
            if row.any():
                break
        codes[t] = row
    coeffs = rng.standard_normal(nterms).astype(np.float64)
    return codes, coeffs


def random_kraus_set(k: int, r: int, rng: np.random.Generator) -> np.ndarray:
    """A random trace-preserving Kraus set of rank r on k qubits: the first r
    column blocks of a Haar isometry, so that sum_a L_a^dagger L_a = I."""
    d = 1 << k
    u = haar_unitary(d * r, rng)
    return np.stack([u[a * d:(a + 1) * d, :d] for a in range(r)]).astype(np.complex128)


def unitary_op(targets: Sequence[int], u: np.ndarray, label: str = "") -> Op:
    return Op("unitary", tuple(int(t) for t in targets), np.asarray(u, np.complex128)[None], label)


def channel_op(targets: Sequence[int], kraus: np.ndarray, label: str = "") -> Op:
    return Op("channel", tuple(int(t) for t in targets), np.asarray(kraus, np.complex128), label)
