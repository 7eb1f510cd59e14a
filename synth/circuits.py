"""Whole synthetic workloads: circuits shaped like the ones the library is
measured on.  Every function is deterministic in its seed."""

from __future__ import annotations

import math

import numpy as np

from .random_ops import (
    Op,
    amplitude_damping_kraus,
    channel_op,
    cnot_matrix,
    dephasing_kraus,
    depolarising_kraus,
    ginibre_factor,
    haar_special_unitary,
    haar_unitary,
    make_rng,
    random_pauli_sum,
    spawn_rngs,
    unitary_op,
)


def _random_mixed_op(n: int, rng: np.random.Generator, second_channel: str) -> Op:
    """One op of the mixed random workload: 50% Haar U(2) on a uniform qubit,
    30% Haar U(4) on a uniform ordered pair of distinct qubits, 20% a
    single-qubit channel (half depolarising, half ``second_channel``) with
    strength drawn from U(0, 0.1)."""
    c = rng.random()
    if c < 0.5 or n < 2:
        q = int(rng.integers(0, n))
        return unitary_op([q], haar_unitary(2, rng), "haar1")
    if c < 0.8:
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        return unitary_op([a, b], haar_unitary(4, rng), "haar2")
    q = int(rng.integers(0, n))
    s = float(rng.uniform(0.0, 0.1))
    if rng.random() < 0.5:
        return channel_op([q], depolarising_kraus(s), "depol")
    if second_channel == "amp":
        return channel_op([q], amplitude_damping_kraus(s), "ampdamp")
    return channel_op([q], dephasing_kraus(s), "dephase")


def circuit_plain_n8(seed: int = 1234, n: int = 8, nops: int = 200):
    """Small plain workload: full-rank Ginibre factor (2^n x 2^n) and ``nops``
    random ops (Haar 1q / Haar 2q / depolarising or amplitude damping)."""
    r_state, r_ops = spawn_rngs(seed, 2)
    g = ginibre_factor(n, 1 << n, r_state)
    ops = [_random_mixed_op(n, r_ops, "amp") for _ in range(nops)]
    return g, ops


def circuit_sweep(n: int = 14, seed: int = 1414, rank: int = 16, nterms: int = 64):
    """Sweep workload: every op class on every qubit position.

    * Haar U(2) on each qubit 0..n-1 (intra- and cross-tile targets);
    * CNOT and Haar SU(4) on adjacent pairs (q, q+1) and on distant pairs
      (q, n-1-q);
    * four-Kraus depolarising channel on each qubit, p ~ U(0, 0.1).

    Returns (G of shape (2^n, rank), ops, (pauli codes, coeffs)).
    """
    r_state, r_ops, r_obs = spawn_rngs(seed, 3)
    g = ginibre_factor(n, rank, r_state)
    ops = []
    for q in range(n):
        ops.append(unitary_op([q], haar_unitary(2, r_ops), f"haar1[{q}]"))
    pairs = [(q, q + 1) for q in range(n - 1)] + [(q, n - 1 - q) for q in range(n // 2)]
    for a, b in pairs:
        ops.append(unitary_op([a, b], cnot_matrix(), f"cnot[{a},{b}]"))
        ops.append(unitary_op([a, b], haar_special_unitary(4, r_ops), f"su4[{a},{b}]"))
    for q in range(n):
        ops.append(channel_op([q], depolarising_kraus(float(r_ops.uniform(0, 0.1))), f"depol[{q}]"))
    codes, coeffs = random_pauli_sum(n, nterms, r_obs)
    return g, ops, (codes, coeffs)


def layer_n16(layer: int, rng: np.random.Generator, n: int = 16, gamma: float = 0.01):
    """One layer of the layered workload: Haar U(2) on every qubit, a brickwork
    of Haar U(4) (pairs (0,1),(2,3),... on even layers, (1,2),(3,4),... on odd
    layers), then amplitude damping with strength ``gamma`` on every qubit."""
    ops = []
    for q in range(n):
        ops.append(unitary_op([q], haar_unitary(2, rng), "haar1"))
    start = 0 if layer % 2 == 0 else 1
    for a in range(start, n - 1, 2):
        ops.append(unitary_op([a, a + 1], haar_unitary(4, rng), "haar2"))
    kd = amplitude_damping_kraus(gamma)
    for q in range(n):
        ops.append(channel_op([q], kd, "ampdamp"))
    return ops


def circuit_layers(n: int = 16, layers: int = 100, seed: int = 1616, rank: int = 16):
    """Layered workload: rank-``rank`` Ginibre factor and ``layers`` layers of
    :func:`layer_n16` (returned as a list of per-layer op lists)."""
    r_state, r_ops = spawn_rngs(seed, 2)
    g = ginibre_factor(n, rank, r_state)
    return g, [layer_n16(l, r_ops, n) for l in range(layers)]


def batched_workload(count: int = 4096, seed: int = 4096, n_lo: int = 4, n_hi: int = 11,
                     ops_lo: int = 20, ops_hi: int = 64):
    """Many independent small operators: n ~ U{n_lo..n_hi}, a full-rank
    Ginibre factor each, and a random circuit of U{ops_lo..ops_hi} ops from the
    mixed workload with dephasing as the second channel.

    Returns a list of (n, G, ops)."""
    rngs = spawn_rngs(seed, count)
    out = []
    for rng in rngs:
        n = int(rng.integers(n_lo, n_hi + 1))
        g = ginibre_factor(n, 1 << n, rng)
        nops = int(rng.integers(ops_lo, ops_hi + 1))
        out.append((n, g, [_random_mixed_op(n, rng, "dephase") for _ in range(nops)]))
    return out


def serving_requests(count: int, rate: float, seed: int = 2000, n_lo: int = 6, n_hi: int = 16,
                     ops_lo: int = 10, ops_hi: int = 300, nterms: int = 64, rank: int = 16):
    """A Poisson request stream.  Each request: arrival time (s), n drawn
    log-uniformly in [n_lo, n_hi] (n = floor(exp(U(ln n_lo, ln(n_hi+1))))),
    dtype "c128" or "c64" with equal odds, a Ginibre factor of rank
    min(rank, 2^n), U{ops_lo..ops_hi} mixed ops, and with probability 1/2 a
    Pauli sum of ``nterms`` terms to take the expectation of (else None: the
    trace is returned)."""
    rng_t, *rngs = spawn_rngs(seed, count + 1)
    gaps = rng_t.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    out = []
    for i, rng in enumerate(rngs):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi + 1)))))
        n = max(n_lo, min(n_hi, n))
        dtype = "c128" if rng.random() < 0.5 else "c64"
        g = ginibre_factor(n, min(rank, 1 << n), rng)
        nops = int(rng.integers(ops_lo, ops_hi + 1))
        ops = [_random_mixed_op(n, rng, "dephase") for _ in range(nops)]
        obs = random_pauli_sum(n, nterms, rng) if rng.random() < 0.5 else None
        out.append(dict(arrival=float(t[i]), n=n, dtype=dtype, G=g, ops=ops, pauli=obs))
    return out


__all__ = [
    "circuit_plain_n8",
    "circuit_sweep",
    "layer_n16",
    "circuit_layers",
    "batched_workload",
    "serving_requests",
    "make_rng",
]
