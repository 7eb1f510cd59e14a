"""The Pauli-sum expectation entry point that allocates no device memory.

Called through the C ABI and checked against ht_expectation_pauli_sum on the
same operator: the two run the same kernels in the same term and summation
order, so the results must agree bit for bit.  Two calls in a row share the
fixed device array, the second on a smaller operator with fewer terms, so a
call that read anything the previous one left behind would show here.  The
result is also held to the oracle (Section I: tr(rho O) for a Pauli sum).
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ht():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_15765_amd as ht
    return ht


def _noalloc(ht, h, codes, coeffs):
    out = ctypes.c_double(12345.0)
    st = ht.lib.ht_expectation_pauli_sum_noalloc(
        h.handle, int(codes.shape[0]), ctypes.c_void_p(codes.ctypes.data), ctypes.c_void_p(coeffs.ctypes.data),
        ctypes.byref(out))
    return st, out.value


def _terms_with_repeated_masks(n, nterms, rng):
    """Random strings plus strings that share a flip mask (Z-only strings have
    mask 0; X and Y on the same qubits share one), so that the order of equal
    masks decides the summation order."""
    codes, coeffs = synth.random_pauli_sum(n, nterms, rng)
    extra = np.zeros((6, n), dtype=np.uint8)
    extra[0, 0] = 3
    extra[1, n - 1] = 3
    extra[2, :] = 3
    extra[3, 1] = 1
    extra[4, 1] = 2
    extra[5, 1] = 1
    extra[5, 0] = 3
    codes = np.ascontiguousarray(np.concatenate([extra, codes])[:nterms])
    coeffs = np.ascontiguousarray(coeffs[:nterms])
    return codes, coeffs


@pytest.mark.parametrize("order", ["noalloc_first", "allocating_first"])
def test_noalloc_pauli_sum_equals_the_allocating_entry_point(ht, order):
    rng = synth.make_rng(7070)
    # second call: smaller operator, fewer terms, other storage type
    for n, m, dtype, nterms in ((11, 5, "c128", 256), (6, 2, "c64", 9)):
        G = synth.ginibre_factor(n, 5, rng)
        h = ht.Herm(n, m, dtype)
        h.init_lowrank(G)
        h.scale(1.0 / h.trace())
        h.apply_unitary([n - 1, 0], synth.haar_unitary(4, rng))
        codes, coeffs = _terms_with_repeated_masks(n, nterms, rng)
        print(f"noalloc case n={n} m={m} {dtype} nterms={nterms} {order}", flush=True)
        if order == "noalloc_first":
            st, got = _noalloc(ht, h, codes, coeffs)
            want = h.expectation_pauli_sum(codes, coeffs)
        else:
            want = h.expectation_pauli_sum(codes, coeffs)
            st, got = _noalloc(ht, h, codes, coeffs)
        assert st == 0, ht.lib.ht_last_error().decode()
        assert got == want, (got, want)
        # and a repeat gives the same bits
        st2, again = _noalloc(ht, h, codes, coeffs)
        assert st2 == 0 and again == got
        rho = h.to_dense()
        ref = oracle.pauli_sum_expectation(rho, codes, coeffs)
        tol = 1e-12 * np.linalg.norm(rho) * np.abs(coeffs).sum()
        assert abs(got - ref) <= tol, (got, ref)
        h.close()


def test_noalloc_rejects_more_terms_than_the_array_holds(ht):
    rng = synth.make_rng(7071)
    n = 5
    h = ht.Herm(n, 2)
    h.init_identity(1.0 / (1 << n))
    codes, coeffs = synth.random_pauli_sum(n, 257, rng)
    st, out = _noalloc(ht, h, codes, coeffs)
    assert st == 1 and out == 12345.0
    assert "256" in ht.lib.ht_last_error().decode()
    st, out = _noalloc(ht, h, codes[:0], coeffs[:0])
    assert st == 1 and out == 12345.0
    # the binding's method reaches the same entry point
    assert h.expectation_pauli_sum_noalloc(codes[:40], coeffs[:40]) == h.expectation_pauli_sum(codes[:40], coeffs[:40])
    h.close()
