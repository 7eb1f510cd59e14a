"""Measure what HBM delivers for the conjugation pass's access shapes.

    python -m paper_2604_15765_amd.stream_probe [--bytes N]

Runs the kernels of csrc/ht_probe.hip (``_probe.so``, built with the
library) on a buffer of the n = 16 complex128 operator's size and prints one
JSON line: read-only, write-only and copy bandwidth, and in-place
read-modify-write bandwidth for 1, 2, 4 and 16 concurrent far-apart streams,
with and without nontemporal hints, each the best over a few grid sizes.
Bandwidth counts bytes read plus bytes written.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--bytes", type=int, default=34376515584)
    p.add_argument("--reps", type=int, default=4)
    args = p.parse_args()
    lib = ctypes.CDLL(os.path.join(HERE, "_probe.so"))
    torch.cuda.set_device(0)
    nb = args.bytes // 4096 * 4096
    n16 = nb // 16
    a = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    grids = (1024, 2048, 4096)
    out = torch.empty(max(grids) * 256, dtype=torch.int32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = ctypes.c_void_p
    u64 = ctypes.c_uint64

    def best(fn, moved):
        res = 0.0
        for g in grids:
            assert fn(g) == 0
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.reps):
                fn(g)
            e1.record()
            torch.cuda.synchronize()
            res = max(res, moved / (e0.elapsed_time(e1) / args.reps * 1e-3) / 1e9)
        return res

    r = {"buffer_bytes": nb}
    r["read_GBps"] = best(lambda g: lib.htp_read(vp(a.data_ptr()), u64(n16), g, vp(out.data_ptr()), st), nb)
    r["write_GBps"] = best(lambda g: lib.htp_write(vp(b.data_ptr()), u64(n16), g, st), nb)
    r["copy_GBps"] = best(lambda g: lib.htp_copy(vp(b.data_ptr()), vp(a.data_ptr()), u64(n16), g, st), 2 * nb)
    for ns in (1, 2, 4, 16):
        per = 16 // ns
        items = (n16 // ns) // (per * 64)
        moved = 2 * 16 * ns * items * per * 64
        for nt in (0, 1):
            r[f"rmw_{ns}streams_{'nt' if nt else 'plain'}_GBps"] = best(
                lambda g, ns=ns, nt=nt: lib.htp_rmw(ns, nt, vp(a.data_ptr()), u64(n16), g, st), moved)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
