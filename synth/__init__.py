"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only draws inputs: random factors for states and observables,
Haar-random gates, textbook Kraus sets, Pauli-sum descriptions and whole
circuits shaped like the workloads the library is measured on.  It holds none
of the method's arithmetic (no conjugation, no transfer matrix, no tiled
layout, no reductions), so that the oracle and the GPU path can both consume
it without sharing any of the computation they are compared on.

Conventions (Section II-A of the paper, with the readings documented in the
design notes):

* qubit ``q`` is bit ``q`` of a basis index (little-endian);
* a k-local operator ``L`` acting on ``targets`` is a ``2^k x 2^k`` matrix
  whose local index bit ``l`` corresponds to ``targets[l]`` (user order);
* a Kraus set is an array of shape ``(r, 2^k, 2^k)``;
* a Pauli string is a row of ``n`` codes, 0=I 1=X 2=Y 3=Z, column ``q``
  acting on qubit ``q``.
"""

from .random_ops import (
    Op,
    make_rng,
    spawn_rngs,
    ginibre_factor,
    random_hermitian_dense,
    haar_unitary,
    haar_special_unitary,
    depolarising_kraus,
    amplitude_damping_kraus,
    dephasing_kraus,
    named_gate,
    cnot_matrix,
    permutation_gate,
    random_monomial,
    random_pauli_sum,
    random_kraus_set,
)
from .circuits import (
    circuit_plain_n8,
    circuit_sweep,
    layer_n16,
    circuit_layers,
    batched_workload,
    serving_requests,
)

__all__ = [
    "Op",
    "make_rng",
    "spawn_rngs",
    "ginibre_factor",
    "random_hermitian_dense",
    "haar_unitary",
    "haar_special_unitary",
    "depolarising_kraus",
    "amplitude_damping_kraus",
    "dephasing_kraus",
    "named_gate",
    "cnot_matrix",
    "permutation_gate",
    "random_monomial",
    "random_pauli_sum",
    "random_kraus_set",
    "circuit_plain_n8",
    "circuit_sweep",
    "layer_n16",
    "circuit_layers",
    "batched_workload",
    "serving_requests",
]
