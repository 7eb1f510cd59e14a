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

Every function cites the passage of the paper it follows, and every one is
pinned by a CPU test (``tests/test_oracle_pins.py``) to something other than
itself; ``tests/test_oracle_mutations.py`` plants a plausible mistake in each
and shows that a pin fails:

    expand_local           np.kron for single targets and adjacent pairs (both
                           orders); CNOT's action on matrix units
    kraus_map              closed forms of Pauli conjugation, depolarising,
                           amplitude damping, dephasing; hermiticity, trace
                           preservation, positivity; diagonal gates and CNOT
                           leave their fixed entries bitwise; 2x2 worked cases
    kraus_map_adjoint      duality tr(O Phi(rho)) = tr(Phi*(O) rho), unitality
    apply_ops(_local)      hand-derived results of two non-commuting ops
                           (X, amplitude damping) in both pictures
    insert_bits            digit-string construction, bijection
    block_indices          digit-string construction for unsorted targets;
                           the subspaces partition the index range
    block_update           the column-stacking identity behind Eq. (3)
    local_block_map        the Kronecker form on every target set; every
                           gathered block equals block_update of the block
    trace                  unitary invariance, tr I = N
    expectation            tr(rho I) = tr rho; single Pauli strings by masks
    pauli_string_matrix,   entry-by-entry phase/permutation closed form;
    pauli_sum_matrix,      tr(rho O) from the bit masks alone
    pauli_sum_expectation
    density_from_factor    projector for one column, P/r for r orthonormal
    layout                 Table I, round trip, Algorithm 3 case counts and
                           tile ownership, the strict tiled expectation  Readings of
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
    "apply_ops_local",
    "trace",
    "expectation",
    "pauli_string_matrix",
    "pauli_sum_matrix",
    "pauli_sum_expectation",
    "density_from_factor",
    "layout",
]
