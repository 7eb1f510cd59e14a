"""CPU oracle for the k-local hermitian conjugation -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct complex128 implementation of
what the library's GPU path computes, written from the paper "Orkan:
cache-friendly simulation of quantum operations on hermitian operators"
(arXiv 2604.15765).  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the HIP path: the only
thing both sides use is the seeded input generators in ``synth``.

Contents
--------
dense       Eq. (1) with Kronecker-expanded Kraus operators (the paper's naive
            BLAS baseline of Section IV-A), Schroedinger and Heisenberg maps.
local_block Eq. (2): the same map as independent 2^k x 2^k block updates,
            both over a whole dense matrix (tensor contraction) and for single
            sampled blocks gathered with Subroutine 1 (insertBits).
readouts    trace, tr(rho O), Pauli strings and Pauli sums.
layout      the tiled lower-triangle format of Section III-B and Table I, the
            case analysis of Algorithm 3 and the tiled expectation formula.

Every function cites the passage of the paper it follows.  Readings of
passages that are silent or inconsistent are listed in the design notes; the
ones that matter here are: qubit q is bit q of an index (little-endian); local
bit l of a k-local matrix belongs to ``targets[l]``; the Heisenberg map is
sum_a L_a^dagger H L_a; the tiled expectation's off-diagonal sum is strict.
"""

from .dense import expand_local, kraus_map, kraus_map_adjoint, apply_ops
from .local_block import (
    insert_bits,
    local_block_map,
    block_update,
    block_indices,
    gather_block,
    scatter_block,
    apply_ops_local,
)
from .readouts import (
    trace,
    expectation,
    pauli_string_matrix,
    pauli_sum_matrix,
    pauli_sum_expectation,
    density_from_factor,
)
from . import layout

__all__ = [
    "expand_local",
    "kraus_map",
    "kraus_map_adjoint",
    "apply_ops",
    "insert_bits",
    "local_block_map",
    "block_update",
    "block_indices",
    "gather_block",
    "scatter_block",
    "apply_ops_local",
    "trace",
    "expectation",
    "pauli_string_matrix",
    "pauli_sum_matrix",
    "pauli_sum_expectation",
    "density_from_factor",
    "layout",
]
