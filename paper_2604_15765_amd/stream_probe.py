"""Measure what HBM delivers for the conjugation pass's access shapes.

    python -m paper_2604_15765_amd.stream_probe [--bytes N]

Runs the kernels of csrc/ht_probe.hip (``_probe.so``, built with the
library) on a buffer of the n = 16 complex128 operator's size and prints one
JSON line: read-only, write-only and copy bandwidth, and in-place
read-modify-write bandwidth for 1, 2, 4 and 16 concurrent far-apart streams,
with and without nontemporal hints, and in-place tile-by-tile streams of
16 KiB tiles with contiguous and with 8 x 8-patch instructions, each the best
over a few grid sizes; workgroup read and write bursts; and "colourings", in
which the 1 KiB runs that a workgroup step moves share a few address bits.
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
    p.add_argument("--summary", help="also write a text summary to this file")
    args = p.parse_args()
    lib = ctypes.CDLL(os.path.join(HERE, "_probe.so"))
    torch.cuda.set_device(0)
    nb = args.bytes // 4096 * 4096
    n16 = nb // 16
    a = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    grids = (1024, 2048, 4096, 8192)
    out = torch.empty(max(grids) * 256, dtype=torch.int32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = ctypes.c_void_p
    u64 = ctypes.c_uint64

    def best(fn, moved):
        return best_of(fn, moved, grids)

    def best_of(fn, moved, grid_list):
        res = 0.0
        for g in grid_list:
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
    ntiles = nb // 16384
    for pat, name in ((0, "contiguous"), (1, "patch8x8")):
        r[f"tile_rmw_{name}_nt_GBps"] = best(
            lambda g, pat=pat: lib.htp_tile(pat, vp(a.data_ptr()), u64(ntiles), g, st), 2 * ntiles * 16384)
    # workgroup bursts (reads of a step complete before its writes)
    for ns, w, x in ((1, 4, 0), (1, 8, 0), (1, 16, 0), (1, 4, 1), (1, 8, 1), (4, 4, 0), (4, 16, 0), (16, 16, 0)):
        wpr = w // ns
        steps = (n16 // ns) // (1024 * wpr)
        moved = 2 * 16 * ns * steps * wpr * 1024
        name = f"wg_{ns}regions_{w}waves{'_lds' if x else ''}_GBps"
        r[name] = best_of(lambda g, ns=ns, w=w, x=x: lib.htp_wg(ns, w, x, vp(a.data_ptr()), u64(n16), g, st),
                          moved, (256, 192))
    for ns in (1, 2, 4):
        steps = (n16 // ns) // (8192 // ns)
        moved = 2 * steps * 8192 * 16
        for g in (256, 192):
            r[f"xstage_{ns}regions_grid{g}_GBps"] = best_of(
                lambda g_, ns=ns: lib.htp_xstage(ns, vp(a.data_ptr()), u64(n16), g_, st), moved, (g,))
    # colourings of 1 KiB units (every unit moved once; 256 workgroups)
    nunits = (nb // 1024) // (64 << 10) * (64 << 10)
    sink = torch.empty(256 * 256 * 16, dtype=torch.uint8, device="cuda")
    for name, g, cb, sel in (("contiguous", 0, 0, 0), ("bits10-12", 0, 3, 0), ("bits11-13", 1, 3, 0),
                             ("bits12-14", 2, 3, 0), ("bits12-14_not_by_xcd", 2, 3, 3), ("bits13-15", 3, 3, 0),
                             ("bits14-16", 4, 3, 0), ("bits12-13", 2, 2, 0), ("bit14", 4, 1, 0),
                             ("bit15", 5, 1, 0)):
        for mode, tag, moved in ((0, "rmw", 2 * nunits * 1024), (1, "read", nunits * 1024)):
            r[f"colour_{name}_{tag}_GBps"] = best_of(
                lambda g_, mode=mode, g=g, cb=cb, sel=sel: lib.htp_colour(
                    mode, vp(a.data_ptr()), u64(nunits), g, cb, sel, g_, vp(sink.data_ptr()), st),
                moved, (256,))
    print(json.dumps(r), flush=True)
    if args.summary:
        write_summary(r, args.summary)


def write_summary(r: dict, path: str) -> None:
    lines = [
        f"# HBM streaming ceilings on MI355X (gfx950), one {r['buffer_bytes']:,}-byte buffer "
        "(the n = 16 c128 operator)",
        "# command: python3 -m paper_2604_15765_amd.stream_probe --summary "
        "profiles/hbm_stream_probe_n16_c128.txt   (kernels: paper_2604_15765_amd/csrc/ht_probe.hip)",
        "# bandwidth = (bytes read + bytes written) / kernel time (torch events), best of grids "
        "1024/2048/4096/8192 x 256 threads",
        "# rmw_<S>streams: in-place read-modify-write of S far-apart regions in lockstep, 16 x 16 B loads "
        "per lane in flight",
        "#   (an intra-tile pass is one stream; a cross-tile pass groups 4 tiles from different parts of "
        "the buffer, a two-tile-bit pass 16); nt = nontemporal loads and stores",
        "# tile_rmw: one 16 KiB tile (32 x 32 entries) per wave and step, nontemporal; contiguous = 1 KiB "
        "per load instruction,",
        "#   patch8x8 = the conjugation pass's lane patch (8 rows x 128 B at a 512-byte stride per "
        "instruction)",
        "# wg_<S>regions_<W>waves: W waves of a workgroup move 16 KiB each per step from S far-apart regions, "
        "all loads before any store (barrier);",
        "#   _lds: through LDS; best of grids 256/192 workgroups",
        "# xstage_<S>regions_grid<G>: 512 threads move 128 KiB per step through LDS in S runs, next step "
        "prefetched; G workgroups",
        "# colour_<bits>_<rmw|read>: 256 workgroups, each step 64 units of 1 KiB whose unit-index bits equal "
        "bits of the workgroup index (the XCD's, unless not_by_xcd):",
        "#   the named address bits are then equal across a workgroup step; contiguous = 64 KiB per step",
        "",
    ]
    for k, v in r.items():
        if k.endswith("_GBps"):
            lines.append(f"{k:34s} {v / 1000:6.3f} TB/s   ({100 * v / 8000:5.1f}% of the 8 TB/s spec)")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
