"""The conjugation pass's per-lane body, run on the CPU, against the oracle.

``_hostcheck.so`` compiles the same ``conj_group_lane`` the GPU kernel runs (from
csrc/ht_geom.h) for the host and drives it over every group, patch and lane
of a pass with a memory policy that rejects out-of-range accesses and counts
writes.  These tests establish, before anything runs on a GPU, that every
pass stays inside the storage, writes every stored entry exactly once, and
computes the oracle's result (decoded with the oracle's own model of the
tiled layout) -- for all tile edges, qubit positions, target orders, Kraus
ranks and both pictures at small n.
"""

import ctypes
import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import layout

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(os.path.dirname(HERE), "paper_2604_15765_amd", "_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(SO):
        pytest.skip("_hostcheck.so not built")
    lib = ctypes.CDLL(SO)
    f = lib.htc_emulate_conj
    vp = ctypes.c_void_p
    f.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp,
                  ctypes.c_int, vp, vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int, ctypes.c_char_p,
                  ctypes.c_size_t]
    f.restype = ctypes.c_int
    return f


def emulate(f, raw, n, m, targets, kraus, heis, order=0):
    raw = np.ascontiguousarray(raw, dtype=np.complex128).copy()
    kraus = np.ascontiguousarray(kraus, dtype=np.complex128)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    wc = np.zeros(raw.size, dtype=np.int32)
    lanes = ctypes.c_uint64()
    err = ctypes.create_string_buffer(256)
    rc = f(raw.ctypes.data, raw.size, n, m, len(targets), t.ctypes.data, kraus.shape[0], kraus.ctypes.data,
           int(heis), wc.ctypes.data, None, ctypes.byref(lanes), order, err, 256)
    assert rc == 0, err.value.decode()
    return raw, wc


def reference(H, kraus, targets, heis):
    return (oracle.kraus_map_adjoint if heis else oracle.kraus_map)(H, kraus, targets)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check(f, n, m, targets, kraus, heis, rng):
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    order = int(rng.integers(2))  # both work orders of the kernel
    out, wc = emulate(f, raw, n, m, targets, kraus, heis, order)
    assert np.all(wc == 1), f"write counts {np.unique(wc)} for n={n} m={m} t={targets}"
    got = layout.decode(out, n, m)
    ref = reference(H, kraus, targets, heis)
    e = rel(got, ref)
    assert e < 1e-13, (n, m, targets, kraus.shape[0], heis, e)
    return out


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_single_qubit_every_position(hc, m):
    rng = synth.make_rng(100 + m)
    for n in range(1, 7):
        for a in range(n):
            for heis in (False, True):
                check(hc, n, m, [a], synth.haar_unitary(2, rng)[None], heis, rng)          # direct form
                check(hc, n, m, [a], synth.random_kraus_set(1, 3, rng), heis, rng)        # transfer form


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_two_qubit_every_ordered_pair(hc, m):
    rng = synth.make_rng(200 + m)
    for n in range(2, 7):
        for a, b in itertools.permutations(range(n), 2):
            heis = bool(rng.integers(2))
            check(hc, n, m, [a, b], synth.haar_unitary(4, rng)[None], heis, rng)
            check(hc, n, m, [a, b], synth.random_kraus_set(2, 3, rng), heis, rng)


def test_complex_nonsymmetric_channel_orders(hc):
    """Transfer-matrix ordering is only visible with complex, non-symmetric
    Kraus operators (for real or depolarising sets both orders agree)."""
    rng = synth.make_rng(300)
    S, T = synth.named_gate("S"), synth.named_gate("T")
    ry = synth.named_gate("RY", 0.7) @ synth.named_gate("RZ", 0.3)
    kr = np.stack([np.sqrt(0.5) * S, np.sqrt(0.3) * T, np.sqrt(0.2) * ry])
    for m in (1, 2, 3):
        for a in range(5):
            check(hc, 5, m, [a], kr, False, rng)


def test_large_tile_edges_and_single_tile(hc):
    rng = synth.make_rng(400)
    for n, m in ((7, 6), (7, 7), (8, 8), (3, 8), (6, 3)):
        for t in ([0], [n - 1], [0, n - 1], [n - 1, 1 % n] if n > 1 else [0]):
            if len(set(t)) != len(t):
                continue
            check(hc, n, m, t, synth.haar_unitary(1 << len(t), rng)[None], False, rng)


def test_diagonal_tile_halves_consistent_after_cross_op(hc):
    """After an op whose targets select tiles, the stored upper halves of the
    diagonal tiles are rewritten as conjugates of the lower ones."""
    rng = synth.make_rng(500)
    n, m = 6, 2
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    for t in ([4], [2, 5], [5, 3]):
        raw, _ = emulate(hc, raw, n, m, t, synth.haar_unitary(1 << len(t), rng)[None], False)
        assert layout.diagonal_tile_asymmetry(raw, n, m) < 1e-14


def test_pauli_x_twice_is_bitwise_identity(hc):
    rng = synth.make_rng(600)
    n, m = 6, 3
    H = synth.random_hermitian_dense(n, rng)
    raw = layout.encode(H, m)
    X = synth.named_gate("X")[None]
    for a in range(n):
        once, _ = emulate(hc, raw, n, m, [a], X, False)
        twice, _ = emulate(hc, once, n, m, [a], X, False)
        assert np.array_equal(twice, raw)
