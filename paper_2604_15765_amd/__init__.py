"""hermtile: k-local quantum operations on tiled hermitian operators (MI355X).

Thin Python binding of the C-ABI in ``include/hermtile.h``: argument
marshalling only.  Every step of the computation runs in the HIP kernels of
``libhermtile.so``; PyTorch provides device memory and streams.  Importing the
package fails if the library has not been built (``__graft_entry__.build()``
or ``python paper_2604_15765_amd/build_ext.py``).
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # first: the library must bind to the HIP runtime torch has loaded

__all__ = ["Herm", "Batch", "Circuit", "Graph", "Server", "capture_begin", "capture_end", "lib", "SCHRODINGER",
           "HEISENBERG", "HermError", "storage_bytes", "effective_tile_log2", "prepare_op",
           "kernel_class_names", "set_tuning"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhermtile.so")

SCHRODINGER = 0
HEISENBERG = 1
_DTYPES = {"c128": 0, "c64": 1}
_STATUS = {0: "HT_OK", 1: "HT_EINVAL", 2: "HT_ENOMEM", 3: "HT_EDEVICE", 4: "HT_EUNSUPPORTED"}


class HermError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _hip_runtime_copies():
    """Paths of every libamdhip64 mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    copies = _hip_runtime_copies()
    if len(copies) > 1:
        raise ImportError(f"two HIP runtimes are loaded ({sorted(copies)}); import torch first")
    c_int, c_int64, c_double, c_size_t, vp = (ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                              ctypes.c_size_t, ctypes.c_void_p)
    P = ctypes.POINTER
    sig = {
        "ht_storage_bytes": (c_size_t, [c_int, c_int, c_int]),
        "ht_effective_tile_log2": (c_int, [c_int, c_int]),
        "ht_herm_create": (c_int, [c_int, c_int, c_int, vp, c_size_t, vp, P(vp)]),
        "ht_herm_destroy": (c_int, [vp]),
        "ht_herm_set_stream": (c_int, [vp, vp]),
        "ht_herm_info": (c_int, [vp, P(c_int), P(c_int), P(c_int), P(vp), P(c_size_t)]),
        "ht_herm_synchronize": (c_int, [vp]),
        "ht_herm_init_zero": (c_int, [vp]),
        "ht_herm_init_identity": (c_int, [vp, c_double]),
        "ht_herm_init_dense": (c_int, [vp, vp, c_int64, c_int]),
        "ht_herm_init_lowrank": (c_int, [vp, vp, c_int, c_int]),
        "ht_herm_init_pauli_sum": (c_int, [vp, c_int, vp, vp]),
        "ht_herm_to_dense": (c_int, [vp, vp, c_int64, c_int]),
        "ht_herm_get_entries": (c_int, [vp, c_int64, vp, vp, vp]),
        "ht_herm_read_raw": (c_int, [vp, c_size_t, c_size_t, vp]),
        "ht_herm_copy": (c_int, [vp, vp]),
        "ht_apply_unitary": (c_int, [vp, c_int, vp, vp, c_int]),
        "ht_apply_channel": (c_int, [vp, c_int, vp, c_int, vp, c_int]),
        "ht_trace": (c_int, [vp, P(c_double)]),
        "ht_expectation": (c_int, [vp, vp, P(c_double)]),
        "ht_expectation_pauli_sum": (c_int, [vp, c_int, vp, vp, P(c_double)]),
        "ht_expectation_pauli_sum_noalloc": (c_int, [vp, c_int, vp, vp, P(c_double)]),
        "ht_scale": (c_int, [vp, c_double]),
        "ht_last_error": (ctypes.c_char_p, []),
        "ht_profile_enable": (c_int, [vp, c_int]),
        "ht_profile_read": (c_int, [vp, c_int, P(c_int), vp, vp, vp]),
        "ht_profile_reset": (c_int, [vp]),
        "ht_kernel_class_name": (ctypes.c_char_p, [c_int]),
        "ht_prepare_op": (c_int, [c_int, c_int, c_int, vp, c_int, vp, c_int, vp, P(c_int), P(c_int), vp]),
        "ht_set_tuning": (c_int, [ctypes.c_char_p, c_int64]),
        "ht_tune_passes": (c_int, [vp, c_int, c_int, vp, P(c_int)]),
        "ht_set_pass_shape": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int]),
        "ht_batch_create": (c_int, [P(vp)]),
        "ht_batch_destroy": (c_int, [vp]),
        "ht_batch_set_param": (c_int, [vp, ctypes.c_char_p, c_int64]),
        "ht_batch_add_unitary": (c_int, [vp, vp, c_int, vp, vp, c_int]),
        "ht_batch_add_channel": (c_int, [vp, vp, c_int, vp, c_int, vp, c_int]),
        "ht_batch_size": (c_int, [vp, P(c_int64), P(c_int64)]),
        "ht_batch_run": (c_int, [vp, vp]),
        "ht_batch_clear": (c_int, [vp]),
        "ht_batch_autotune": (c_int, [vp, c_int, vp]),
        "ht_circuit_create": (c_int, [P(vp)]),
        "ht_circuit_destroy": (c_int, [vp]),
        "ht_circuit_add_unitary": (c_int, [vp, c_int, vp, vp]),
        "ht_circuit_add_channel": (c_int, [vp, c_int, vp, c_int, vp]),
        "ht_circuit_size": (c_int, [vp, P(c_int64)]),
        "ht_circuit_plan": (c_int, [vp, c_int, c_int, P(c_int64)]),
        "ht_circuit_pass_info": (c_int, [vp, c_int64, P(c_int), vp, P(c_int64), vp, vp]),
        "ht_circuit_apply": (c_int, [vp, vp]),
        "ht_capture_begin": (c_int, [vp]),
        "ht_capture_end": (c_int, [vp, P(vp)]),
        "ht_graph_launch": (c_int, [vp, vp]),
        "ht_graph_destroy": (c_int, [vp]),
        "ht_server_config_default": (None, [vp]),
        "ht_server_create": (c_int, [vp, P(vp)]),
        "ht_server_submit": (c_int, [vp, vp, P(c_int64)]),
        "ht_server_wait_idle": (c_int, [vp, c_double]),
        "ht_server_poll": (c_int, [vp, c_int64, vp, vp, vp, vp, vp, vp, P(c_int64)]),
        "ht_server_now": (c_int, [vp, P(c_double)]),
        "ht_server_last_error": (c_int, [vp, ctypes.c_char_p, c_size_t]),
        "ht_server_destroy": (c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int) -> None:
    if status != 0:
        raise HermError(status, lib.ht_last_error().decode())


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


# Shape checks.  The C side receives bare pointers and reads as many entries
# as the sizes imply, so every array is checked here before its address is
# passed on; a mismatch raises ValueError and nothing is called.

def _targets(targets) -> np.ndarray:
    t = np.ascontiguousarray(targets, dtype=np.int32)
    if t.ndim != 1 or not 1 <= t.shape[0] <= 3:
        raise ValueError(f"targets must be a sequence of 1 to 3 qubits, got shape {t.shape}")
    return t


def _unitary(U, k: int) -> np.ndarray:
    U = _c128(U)
    d = 1 << k
    if U.shape != (d, d):
        raise ValueError(f"a {k}-qubit matrix must be {d} x {d}, got shape {U.shape}")
    return U


def _kraus(kraus, k: int) -> np.ndarray:
    K = _c128(kraus)
    if K.ndim == 2:
        K = K[None]
    d = 1 << k
    if K.ndim != 3 or K.shape[1:] != (d, d) or K.shape[0] < 1:
        raise ValueError(f"{k}-qubit Kraus operators must have shape (r, {d}, {d}), got {K.shape}")
    return K


def _pauli(codes, coeffs, n: int):
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    if codes.ndim != 2 or codes.shape[1] != n or codes.shape[0] < 1:
        raise ValueError(f"Pauli codes must have shape (nterms, {n}), got {codes.shape}")
    if coeffs.shape != (codes.shape[0],):
        raise ValueError(f"Pauli coefficients must have shape ({codes.shape[0]},), got {coeffs.shape}")
    return codes, coeffs


def _factor(G, n: int):
    """(array or tensor, on_device) for a factor G of shape (2^n, rank)."""
    N = 1 << n
    if isinstance(G, torch.Tensor) and G.is_cuda:
        if G.dtype != torch.complex128:
            raise ValueError(f"a device factor must be complex128, got {G.dtype}")
        if G.dim() != 2 or G.shape[0] != N or G.shape[1] < 1:
            raise ValueError(f"the factor must have shape ({N}, rank), got {tuple(G.shape)}")
        return G.contiguous(), True
    G = _c128(G)
    if G.ndim != 2 or G.shape[0] != N or G.shape[1] < 1:
        raise ValueError(f"the factor must have shape ({N}, rank), got {G.shape}")
    return G, False


def storage_bytes(n: int, tile_log2: int, dtype: str = "c128") -> int:
    return int(lib.ht_storage_bytes(n, tile_log2, _DTYPES[dtype]))


def effective_tile_log2(n: int, tile_log2: int) -> int:
    return int(lib.ht_effective_tile_log2(n, tile_log2))


def kernel_class_names():
    out = []
    i = 0
    while True:
        s = lib.ht_kernel_class_name(i)
        if s is None:
            return out
        out.append(s.decode())
        i += 1


def set_tuning(name: str, value: int) -> None:
    _check(lib.ht_set_tuning(name.encode(), int(value)))


PASS_SHAPES = ("lane", "stage", "stage_3/4", "stage_5/8", "steps", "steps_3/4", "steps_5/8",
               "steps_quarter", "steps_quarter_3/4", "steps_quarter_5/8",
               "steps_quarter_alt", "steps_quarter_alt_3/4", "steps_quarter_alt_5/8",
               "stage_alt", "stage_alt_3/4", "stage_alt_5/8",
               "steps_quarter_4th", "steps_quarter_4th_3/4", "steps_quarter_4th_5/8",
               "stage_alt_256x2")


def set_pass_shape(dtype: str, n: int, tile_log2: int, row: dict) -> None:
    """ht_set_pass_shape for one record of Herm.tune_passes (row["shape"]
    None: back to the automatic choice)."""
    shape = -1 if row.get("shape") is None else PASS_SHAPES.index(row["shape"])
    _check(lib.ht_set_pass_shape(_DTYPES[dtype], int(n), int(tile_log2), int(row["k"]), int(row["cross"]),
                                 1 if row["form"] == "transfer" else 0, 1 if row["low_intra"] else 0,
                                 1 if row.get("far") else 0, shape))


def prepare_op(n: int, tile_log2: int, targets: Sequence[int], mats, picture: int = SCHRODINGER):
    """ht_prepare_op: returns (sorted_targets, ncross, form, coef complex array)."""
    mats = _c128(mats)
    if mats.ndim == 2:
        mats = mats[None]
    k = len(targets)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    st = np.zeros(3, dtype=np.int32)
    nc = ctypes.c_int()
    form = ctypes.c_int()
    coef = np.zeros(2 * 64 * 64, dtype=np.float64)
    _check(lib.ht_prepare_op(n, tile_log2, k, _ptr(t), mats.shape[0], _ptr(mats), picture,
                             _ptr(st), ctypes.byref(nc), ctypes.byref(form), _ptr(coef)))
    d = 1 << k
    if form.value == 3:  # k = 3 Kraus form: the operators themselves
        c = coef[:2 * mats.shape[0] * d * d].view(np.complex128)
        return (list(st[:k]), nc.value, form.value, c.reshape(mats.shape[0], d, d).copy())
    ne = d ** 4 if form.value == 1 else d * d
    c = coef[:2 * ne].view(np.complex128)
    side = d * d if form.value == 1 else d
    out = (list(st[:k]), nc.value, form.value, c.reshape(side, side).copy())
    if form.value == 2:  # native form: also the permutation
        return out + ([int(x) for x in coef[2 * ne:2 * ne + d]],)
    return out


class Herm:
    """One tiled hermitian operator on the GPU (an ``ht_herm`` handle).

    The tiled storage is a torch uint8 tensor owned by this object and lent to
    the library; calls are enqueued on ``stream`` (default: torch's current
    stream of ``device``)."""

    def __init__(self, n: int, tile_log2: int = 5, dtype: str = "c128",
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be one of {list(_DTYPES)}")
        self.n = int(n)
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = storage_bytes(n, tile_log2, dtype)
        if nbytes == 0:
            raise HermError(1, f"invalid n={n} or tile_log2={tile_log2}")
        with torch.cuda.device(self.device):
            self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if self.stream != torch.cuda.current_stream(self.device):
                # the buffer was allocated on the current stream: order the
                # handle's stream after it, and free it only after its work
                self.stream.wait_stream(torch.cuda.current_stream(self.device))
                self.buffer.record_stream(self.stream)
            h = ctypes.c_void_p()
            _check(lib.ht_herm_create(self.n, tile_log2, _DTYPES[dtype], ctypes.c_void_p(self.buffer.data_ptr()),
                                      nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.tile_log2 = effective_tile_log2(n, tile_log2)
        self.nbytes = nbytes

    # lifetime ----------------------------------------------------------
    def close(self) -> None:
        """Destroy the handle (after its stream has drained) and release the storage."""
        if getattr(self, "_h", None):
            _check(lib.ht_herm_destroy(self._h))
            self._h = None
            self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def set_stream(self, stream: torch.cuda.Stream) -> None:
        _check(lib.ht_herm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream
        self.buffer.record_stream(stream)

    def synchronize(self) -> None:
        _check(lib.ht_herm_synchronize(self._h))

    # init / IO ---------------------------------------------------------
    def init_zero(self) -> "Herm":
        _check(lib.ht_herm_init_zero(self._h))
        return self

    def init_identity(self, scale: float = 1.0) -> "Herm":
        _check(lib.ht_herm_init_identity(self._h, float(scale)))
        return self

    def _use_on_stream(self, t: torch.Tensor) -> None:
        """A device input read by work enqueued on the handle's stream: order
        that stream after the tensor's producer and keep the memory alive until
        the work has run."""
        cur = torch.cuda.current_stream(self.device)
        if self.stream != cur:
            self.stream.wait_stream(cur)
        t.record_stream(self.stream)

    def init_dense(self, A) -> "Herm":
        N = 1 << self.n
        if isinstance(A, torch.Tensor) and A.is_cuda:
            if A.dtype != torch.complex128:
                raise ValueError(f"a device matrix must be complex128, got {A.dtype}")
            if A.dim() != 2 or A.shape[0] != N or A.shape[1] < N:
                raise ValueError(f"the matrix must have shape ({N}, >= {N}), got {tuple(A.shape)}")
            A = A.contiguous()
            self._use_on_stream(A)
            _check(lib.ht_herm_init_dense(self._h, ctypes.c_void_p(A.data_ptr()), A.shape[1], 1))
            return self
        A = _c128(A)
        if A.ndim != 2 or A.shape[0] != N or A.shape[1] < N:
            raise ValueError(f"the matrix must have shape ({N}, >= {N}), got {A.shape}")
        _check(lib.ht_herm_init_dense(self._h, _ptr(A), A.shape[1], 0))
        return self

    def init_lowrank(self, G) -> "Herm":
        G, on_device = _factor(G, self.n)
        if on_device:
            self._use_on_stream(G)
            _check(lib.ht_herm_init_lowrank(self._h, ctypes.c_void_p(G.data_ptr()), G.shape[1], 1))
            return self
        _check(lib.ht_herm_init_lowrank(self._h, _ptr(G), G.shape[1], 0))
        return self

    def init_pauli_sum(self, codes, coeffs) -> "Herm":
        codes, coeffs = _pauli(codes, coeffs, self.n)
        _check(lib.ht_herm_init_pauli_sum(self._h, codes.shape[0], _ptr(codes), _ptr(coeffs)))
        return self

    def to_dense(self) -> np.ndarray:
        N = 1 << self.n
        out = np.empty((N, N), dtype=np.complex128)
        _check(lib.ht_herm_to_dense(self._h, _ptr(out), N, 0))
        return out

    def get_entries(self, rows, cols) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(rows.shape[0], dtype=np.complex128)
        _check(lib.ht_herm_get_entries(self._h, rows.shape[0], _ptr(rows), _ptr(cols), _ptr(out)))
        return out

    def read_raw(self, offset: int = 0, nbytes: Optional[int] = None) -> np.ndarray:
        if nbytes is None:
            nbytes = self.nbytes - offset
        out = np.empty(nbytes, dtype=np.uint8)
        _check(lib.ht_herm_read_raw(self._h, offset, nbytes, _ptr(out)))
        return out

    def raw_entries(self) -> np.ndarray:
        """The whole tiled storage as a complex128 array (c64 widened)."""
        raw = self.read_raw()
        if self.dtype == "c128":
            return raw.view(np.complex128).copy()
        return raw.view(np.complex64).astype(np.complex128)

    def copy_from(self, other: "Herm") -> "Herm":
        _check(lib.ht_herm_copy(self._h, other._h))
        return self

    # hot path ----------------------------------------------------------
    def apply_unitary(self, targets: Sequence[int], U, picture: int = SCHRODINGER) -> None:
        t = _targets(targets)
        U = _unitary(U, t.shape[0])
        _check(lib.ht_apply_unitary(self._h, t.shape[0], _ptr(t), _ptr(U), picture))

    def apply_channel(self, targets: Sequence[int], kraus, picture: int = SCHRODINGER) -> None:
        t = _targets(targets)
        K = _kraus(kraus, t.shape[0])
        _check(lib.ht_apply_channel(self._h, t.shape[0], _ptr(t), K.shape[0], _ptr(K), picture))

    def apply_op(self, op, picture: int = SCHRODINGER) -> None:
        """Apply an op with ``kind``, ``targets`` and ``mats`` (see ``synth.Op``)."""
        if op.kind == "unitary":
            self.apply_unitary(op.targets, op.mats[0], picture)
        else:
            self.apply_channel(op.targets, op.mats, picture)

    # reductions --------------------------------------------------------
    def trace(self) -> float:
        out = ctypes.c_double()
        _check(lib.ht_trace(self._h, ctypes.byref(out)))
        return out.value

    def expectation(self, other: "Herm") -> float:
        out = ctypes.c_double()
        _check(lib.ht_expectation(self._h, other._h, ctypes.byref(out)))
        return out.value

    def expectation_pauli_sum(self, codes, coeffs) -> float:
        codes, coeffs = _pauli(codes, coeffs, self.n)
        out = ctypes.c_double()
        _check(lib.ht_expectation_pauli_sum(self._h, codes.shape[0], _ptr(codes), _ptr(coeffs),
                                            ctypes.byref(out)))
        return out.value

    def expectation_pauli_sum_noalloc(self, codes, coeffs) -> float:
        """expectation_pauli_sum through the entry point that allocates no
        device memory (at most 256 terms; calls on one GPU must not overlap)."""
        codes, coeffs = _pauli(codes, coeffs, self.n)
        out = ctypes.c_double()
        _check(lib.ht_expectation_pauli_sum_noalloc(self._h, codes.shape[0], _ptr(codes), _ptr(coeffs),
                                                    ctypes.byref(out)))
        return out.value

    def tune_passes(self, reps: int = 2) -> list:
        """ht_tune_passes: time the launch shapes of every pass class on this
        operator (identity passes: the represented matrix is unchanged) and
        keep the fastest; returns one dict per class."""
        rows = np.zeros((64, 8), dtype=np.float64)
        nr = ctypes.c_int()
        _check(lib.ht_tune_passes(self._h, int(reps), 64, _ptr(rows), ctypes.byref(nr)))
        return [dict(k=int(r[0]), cross=int(r[1]), form="transfer" if r[2] else "direct", low_intra=bool(r[3]),
                     far=bool(r[4]), shape=PASS_SHAPES[int(r[5])], ms=float(r[6]), lane_ms=float(r[7]))
                for r in rows[:min(nr.value, 64)]]

    def scale(self, alpha: float) -> None:
        _check(lib.ht_scale(self._h, float(alpha)))

    # measurement -------------------------------------------------------
    def profile_enable(self, on: bool = True) -> None:
        _check(lib.ht_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self) -> None:
        _check(lib.ht_profile_reset(self._h))

    def profile_read(self) -> dict:
        nmax = 64
        nc = ctypes.c_int()
        launches = np.zeros(nmax, dtype=np.int64)
        ms = np.zeros(nmax, dtype=np.float64)
        by = np.zeros(nmax, dtype=np.float64)
        _check(lib.ht_profile_read(self._h, nmax, ctypes.byref(nc), _ptr(launches), _ptr(ms), _ptr(by)))
        names = kernel_class_names()
        return {names[i]: dict(launches=int(launches[i]), ms=float(ms[i]), bytes=float(by[i]))
                for i in range(nc.value) if launches[i] > 0}


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


MAX_QUBITS = 18  # HT_MAX_QUBITS


class BatchTuning(ctypes.Structure):
    """ht_batch_tuning (field order as in include/hermtile.h)."""

    _fields_ = [
        ("tile_log2", ctypes.c_int * (MAX_QUBITS + 1)),
        ("threads", ctypes.c_int),
        ("wg_per_cu", ctypes.c_int),
        ("lds_max_bytes", ctypes.c_int64),
        ("sample_operators", ctypes.c_int),
        ("configs_timed", ctypes.c_int),
        ("sample_seconds_before", ctypes.c_double),
        ("sample_seconds_after", ctypes.c_double),
        ("tuning_seconds", ctypes.c_double),
    ]


class Batch:
    """ht_batch: ops for many operators, executed in one persistent launch."""

    def __init__(self, **params):
        b = ctypes.c_void_p()
        _check(lib.ht_batch_create(ctypes.byref(b)))
        self._b = b
        self._keep = {}
        for k, v in params.items():
            self.set_param(k, v)

    def set_param(self, name: str, value: int) -> None:
        _check(lib.ht_batch_set_param(self._b, name.encode(), int(value)))

    def add_unitary(self, h: Herm, targets, U, picture: int = SCHRODINGER) -> None:
        t = _targets(targets)
        U = _unitary(U, t.shape[0])
        _check(lib.ht_batch_add_unitary(self._b, h.handle, t.shape[0], _ptr(t), _ptr(U), picture))
        self._keep[id(h)] = h

    def add_channel(self, h: Herm, targets, kraus, picture: int = SCHRODINGER) -> None:
        t = _targets(targets)
        K = _kraus(kraus, t.shape[0])
        _check(lib.ht_batch_add_channel(self._b, h.handle, t.shape[0], _ptr(t), K.shape[0], _ptr(K),
                                        picture))
        self._keep[id(h)] = h

    def add_op(self, h: Herm, op, picture: int = SCHRODINGER) -> None:
        if op.kind == "unitary":
            self.add_unitary(h, op.targets, op.mats[0], picture)
        else:
            self.add_channel(h, op.targets, op.mats, picture)

    def size(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.ht_batch_size(self._b, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def run(self, stream=None) -> None:
        _check(lib.ht_batch_run(self._b, _stream_ptr(stream)))

    def clear(self) -> None:
        _check(lib.ht_batch_clear(self._b))
        self._keep = {}

    def autotune(self, sample_operators: int = 0) -> dict:
        """ht_batch_autotune; returns the chosen tile exponent per qubit count
        ({n: tile_log2}) and launch shape, and the sample's timings."""
        t = BatchTuning()
        _check(lib.ht_batch_autotune(self._b, int(sample_operators), ctypes.addressof(t)))
        return {
            "tile_log2": {n: t.tile_log2[n] for n in range(MAX_QUBITS + 1) if t.tile_log2[n]},
            "threads": t.threads,
            "wg_per_cu": t.wg_per_cu,
            "lds_max_bytes": t.lds_max_bytes,
            "sample_operators": t.sample_operators,
            "configs_timed": t.configs_timed,
            "sample_seconds_before": t.sample_seconds_before,
            "sample_seconds_after": t.sample_seconds_after,
            "tuning_seconds": t.tuning_seconds,
        }

    def close(self) -> None:
        if getattr(self, "_b", None):
            _check(lib.ht_batch_destroy(self._b))
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Circuit:
    """ht_circuit: an op sequence applied with fusion of neighbouring ops."""

    def __init__(self, ops=()):
        c = ctypes.c_void_p()
        _check(lib.ht_circuit_create(ctypes.byref(c)))
        self._c = c
        for op in ops:
            self.add_op(op)

    def add_unitary(self, targets, U) -> None:
        t = _targets(targets)
        U = _unitary(U, t.shape[0])
        _check(lib.ht_circuit_add_unitary(self._c, t.shape[0], _ptr(t), _ptr(U)))

    def add_channel(self, targets, kraus) -> None:
        t = _targets(targets)
        K = _kraus(kraus, t.shape[0])
        _check(lib.ht_circuit_add_channel(self._c, t.shape[0], _ptr(t), K.shape[0], _ptr(K)))

    def add_op(self, op) -> None:
        if op.kind == "unitary":
            self.add_unitary(op.targets, op.mats[0])
        else:
            self.add_channel(op.targets, op.mats)

    def size(self) -> int:
        n = ctypes.c_int64()
        _check(lib.ht_circuit_size(self._c, ctypes.byref(n)))
        return n.value

    def plan(self, picture: int = SCHRODINGER, max_qubits: int = 2) -> int:
        n = ctypes.c_int64()
        _check(lib.ht_circuit_plan(self._c, picture, max_qubits, ctypes.byref(n)))
        return n.value

    def pass_info(self, i: int, transfer: bool = True) -> dict:
        """Pass i of the last plan: qubits, op indices, transfer matrix."""
        k = ctypes.c_int()
        t = np.zeros(3, dtype=np.int32)
        nops = ctypes.c_int64()
        _check(lib.ht_circuit_pass_info(self._c, i, ctypes.byref(k), _ptr(t), ctypes.byref(nops), None, None))
        idx = np.zeros(max(nops.value, 1), dtype=np.int64)
        S = None
        if transfer and k.value <= 2:
            d = 1 << (2 * k.value)
            S = np.zeros(2 * d * d, dtype=np.float64)
        _check(lib.ht_circuit_pass_info(self._c, i, None, None, None, _ptr(idx),
                                        _ptr(S) if S is not None else None))
        out = {"targets": [int(x) for x in t[:k.value]], "ops": [int(x) for x in idx[:nops.value]]}
        if S is not None:
            d = 1 << (2 * k.value)
            out["transfer"] = S.view(np.complex128).reshape(d, d).copy()
        return out

    def apply(self, h: "Herm") -> None:
        _check(lib.ht_circuit_apply(self._c, h.handle))

    def close(self) -> None:
        if getattr(self, "_c", None):
            _check(lib.ht_circuit_destroy(self._c))
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """ht_graph: a captured sequence of hot-path calls."""

    def __init__(self, handle: ctypes.c_void_p):
        self._g = handle

    def launch(self, stream=None) -> None:
        _check(lib.ht_graph_launch(self._g, _stream_ptr(stream)))

    def close(self) -> None:
        if getattr(self, "_g", None):
            _check(lib.ht_graph_destroy(self._g))
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture_begin(stream) -> None:
    _check(lib.ht_capture_begin(_stream_ptr(stream)))


def capture_end(stream) -> Graph:
    g = ctypes.c_void_p()
    _check(lib.ht_capture_end(_stream_ptr(stream), ctypes.byref(g)))
    return Graph(g)


class ServerConfig(ctypes.Structure):
    """ht_server_config."""
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int),
                ("batch_max_qubits", ctypes.c_int), ("chunk_ops", ctypes.c_int),
                ("large_chunk_ops", ctypes.c_int), ("tile_log2", ctypes.c_int), ("fifo", ctypes.c_int),
                ("batch_threads", ctypes.c_int), ("batch_wg_per_cu", ctypes.c_int),
                ("lds_max_bytes", ctypes.c_size_t), ("max_large_active", ctypes.c_int),
                ("medium_max_qubits", ctypes.c_int), ("max_medium_active", ctypes.c_int),
                ("fuse_qubits", ctypes.c_int)]


class _Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dtype", ctypes.c_int), ("rank", ctypes.c_int),
                ("G", ctypes.c_void_p), ("nops", ctypes.c_int), ("op_k", ctypes.c_void_p),
                ("op_targets", ctypes.c_void_p), ("op_r", ctypes.c_void_p), ("op_mats", ctypes.c_void_p),
                ("picture", ctypes.c_int), ("nterms", ctypes.c_int), ("codes", ctypes.c_void_p),
                ("coeffs", ctypes.c_void_p)]


class Server:
    """ht_server: continuous-batching request server on the current device."""

    def __init__(self, **cfg):
        c = ServerConfig()
        lib.ht_server_config_default(ctypes.byref(c))
        for k, v in cfg.items():
            if not hasattr(c, k):
                raise ValueError(f"unknown server option {k}")
            setattr(c, k, int(v))
        self.config = {f: getattr(c, f) for f, _ in ServerConfig._fields_}
        s = ctypes.c_void_p()
        _check(lib.ht_server_create(ctypes.byref(c), ctypes.byref(s)))
        self._s = s

    def submit(self, n: int, G, ops, pauli=None, dtype: str = "c128", picture: int = SCHRODINGER) -> int:
        """Queue a request: state G G^dagger / tr, ops (objects with targets and
        mats), readout tr(rho O) for pauli = (codes, coeffs) or the trace."""
        if isinstance(G, torch.Tensor):
            G = G.detach().cpu().numpy()
        G, _ = _factor(G, int(n))
        tg = np.zeros(2 * len(ops), dtype=np.int32)
        blocks = []
        for i, op in enumerate(ops):
            t = _targets(op.targets)
            if t.shape[0] > 2:
                raise ValueError(f"op {i}: served requests take 1- and 2-qubit ops, got {t.shape[0]} targets")
            tg[2 * i:2 * i + t.shape[0]] = t
            blocks.append(_kraus(op.mats, t.shape[0]))
        k = np.array([len(op.targets) for op in ops], dtype=np.int32)
        r = np.array([b.shape[0] for b in blocks], dtype=np.int32)
        mats = (np.ascontiguousarray(np.concatenate([b.reshape(-1) for b in blocks]))
                if ops else np.zeros(1, np.complex128))
        req = _Request(n=n, dtype=_DTYPES[dtype], rank=G.shape[1], G=G.ctypes.data, nops=len(ops),
                       op_k=k.ctypes.data, op_targets=tg.ctypes.data, op_r=r.ctypes.data,
                       op_mats=mats.ctypes.data, picture=picture, nterms=0, codes=None, coeffs=None)
        if pauli is not None:
            codes, coeffs = _pauli(pauli[0], pauli[1], int(n))
            req.nterms, req.codes, req.coeffs = codes.shape[0], codes.ctypes.data, coeffs.ctypes.data
        rid = ctypes.c_int64()
        _check(lib.ht_server_submit(self._s, ctypes.byref(req), ctypes.byref(rid)))
        return rid.value

    def wait_idle(self, timeout_s: float = 600.0) -> None:
        _check(lib.ht_server_wait_idle(self._s, float(timeout_s)))

    def poll(self, max_results: int = 1 << 16):
        ids = np.zeros(max_results, np.int64)
        st = np.zeros(max_results, np.int32)
        vals = np.zeros(max_results, np.float64)
        ts, ta, td = (np.zeros(max_results, np.float64) for _ in range(3))
        cnt = ctypes.c_int64()
        _check(lib.ht_server_poll(self._s, max_results, _ptr(ids), _ptr(st), _ptr(vals), _ptr(ts), _ptr(ta),
                                  _ptr(td), ctypes.byref(cnt)))
        c = cnt.value
        return [dict(id=int(ids[i]), status=int(st[i]), value=float(vals[i]), t_submit=float(ts[i]),
                     t_admit=float(ta[i]), t_done=float(td[i])) for i in range(c)]

    def now(self) -> float:
        t = ctypes.c_double()
        _check(lib.ht_server_now(self._s, ctypes.byref(t)))
        return t.value

    def last_error(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(lib.ht_server_last_error(self._s, buf, 512))
        return buf.value.decode()

    def close(self) -> None:
        if getattr(self, "_s", None):
            _check(lib.ht_server_destroy(self._s))
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
