"""Summarise rocprofv3 output of the benchmark into a short text file.

    python -m paper_2604_15765_amd.profile_summary \\
        --stats DIR --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --command "..." --out profiles/NAME.txt

Inputs are rocprofv3 CSV output directories: a --kernel-trace --stats run of
bench.py, one --pmc FETCH_SIZE and one --pmc WRITE_SIZE run of bench.py, and
the same two counters for ``bench.py --copy-only`` (a plain copy kernel over
buffers of the operator's size, whose bytes are known).  The copy kernel
calibrates the counters: factor = known bytes / counter bytes, per counter.
The summary lists, per conjugation kernel class, the average duration, the
calibrated HBM bytes read and written per launch, and a fingerprint of the
kernel sources the counters were taken with (bench.py reports the traffic
only while the sources still match it).
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/ht_geom.h", "csrc/ht_conj.hip")


def source_fingerprint() -> str:
    """Hash of the kernel sources without their comments and blank lines
    (an edit of a comment leaves the profiled kernels as they were)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def kernel_class(name: str):
    """'conj_kernel<double, 1, 1, 0, 0>' -> 'c128_k1_c1_direct' (also the
    workgroup-step kernels conj_sync_kernel and conj_pipe_kernel),
    'stage_kernel<double, 2, 1, 512, true>' -> 'c128_k2_c0_transfer' (also
    with the granule-order flag, 'stage_kernel<double, 2, 1, 512, true, true>'),
    'native_kernel<float, 3, 2, 0, 16, 0>' -> 'c64_k3_c2_native',
    'k3_kernel<double, 1, 3>' -> 'c128_k3_c1_kraus',
    'pair_kernel<1, 1, 0, 3, 2>' -> 'c64_k1_c1_direct' (complex64 only; also
    the step form 'pair_sync_kernel<1, 1, 0, 3, 2, 1024>'), and the pair
    passes' diagonal-group launch 'pair_diag_kernel<2, 2, 0, 3>' ->
    'c64_k2_c2_direct_diag'; None otherwise."""
    m = re.search(r"conj_(?:sync_|pipe_)?kernel<(double|float), (\d), (\d), (\d), (\d)", name)
    if m:
        dt = "c128" if m.group(1) == "double" else "c64"
        return f"{dt}_k{m.group(2)}_c{m.group(3)}_{'direct' if m.group(4) == '0' else 'transfer'}"
    m = re.search(r"stage_kernel<(double|float), (\d), (\d), \d+, (?:true|false)(?:, (?:true|false))?>", name)
    if m:
        dt = "c128" if m.group(1) == "double" else "c64"
        return f"{dt}_k{m.group(2)}_c0_{'direct' if m.group(3) == '0' else 'transfer'}"
    m = re.search(r"native_kernel<(double|float), (\d), (\d), (\d)", name)
    if m:
        dt = "c128" if m.group(1) == "double" else "c64"
        return f"{dt}_k{m.group(2)}_c{m.group(3)}_native"
    m = re.search(r"k3_kernel<(double|float), (\d), (\d)>", name)
    if m:
        dt = "c128" if m.group(1) == "double" else "c64"
        return f"{dt}_k3_c{m.group(2)}_kraus"
    m = re.search(r"pair_(?:sync_)?kernel<(\d), (\d), (\d), (\d), (\d)(?:, \d+)?>", name)
    if m:
        return f"c64_k{m.group(1)}_c{m.group(2)}_{'direct' if m.group(3) == '0' else 'transfer'}"
    m = re.search(r"pair_diag_kernel<(\d), (\d), (\d), (\d)>", name)
    if m:
        return f"c64_k{m.group(1)}_c{m.group(2)}_{'direct' if m.group(3) == '0' else 'transfer'}_diag"
    return None


def _counter_avg(rows, counter, select):
    vals = [float(r["Counter_Value"]) * 1024.0 for r in rows
            if r["Counter_Name"] == counter and select(r["Kernel_Name"])]
    return sum(vals) / len(vals) if vals else None


def main():
    p = argparse.ArgumentParser()
    for a in ("stats", "fetch", "write", "copy-fetch", "copy-write", "command", "out"):
        p.add_argument("--" + a, required=True)
    p.add_argument("--copy-bytes", type=float, default=34376515584.0,
                   help="bytes the copy kernel reads (and writes) per launch")
    p.add_argument("--title", default="conjugation passes of the n = 16 complex128 layered benchmark",
                   help="what the profiled command ran")
    args = p.parse_args()

    stats = _csv(args.stats, "kernel_stats.csv")
    fetch = _csv(args.fetch, "counter_collection.csv")
    write = _csv(args.write, "counter_collection.csv")
    cfetch = _csv(args.copy_fetch, "counter_collection.csv")
    cwrite = _csv(args.copy_write, "counter_collection.csv")
    is_copy = lambda n: "copy_kernel" in n
    f_copy = _counter_avg(cfetch, "FETCH_SIZE", is_copy)
    w_copy = _counter_avg(cwrite, "WRITE_SIZE", is_copy)
    kf = args.copy_bytes / f_copy
    kw = args.copy_bytes / w_copy

    lines = [
        f"# rocprofv3 summary: {args.title}",
        f"# kernel source fingerprint: {source_fingerprint()}",
        "# commands (from the repository root; rocprofv3 run from /tmp with absolute paths):",
    ]
    lines += [f"#   {c.strip()}" for c in args.command.split(";") if c.strip()]
    lines += [
        "",
        "## kernel trace statistics (--kernel-trace --stats)",
        f"{'kernel':70s} {'calls':>6s} {'avg_ms':>9s} {'share_%':>8s}",
    ]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        cls = kernel_class(r["Name"])
        label = f"{name} [{cls}]" if cls else name
        lines.append(f"{label[:70]:70s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:9.3f} "
                     f"{float(r['Percentage']):8.2f}")
    lines += [
        "",
        "## HBM byte counters (--pmc FETCH_SIZE, --pmc WRITE_SIZE; KiB per dispatch x 1024)",
        f"copy-kernel calibration ({args.copy_bytes:.0f} B read and written per launch): "
        f"FETCH_SIZE reads {f_copy:.4e} B -> factor {kf:.4f}; WRITE_SIZE reads {w_copy:.4e} B -> factor {kw:.4f}",
        f"{'class':22s} {'launches':>8s} {'read_GB':>9s} {'write_GB':>9s} {'traffic_GB':>10s}",
    ]
    classes = sorted({kernel_class(r["Kernel_Name"]) for r in fetch} - {None})
    for cls in classes:
        sel = lambda n, cls=cls: kernel_class(n) == cls
        f = _counter_avg(fetch, "FETCH_SIZE", sel)
        w = _counter_avg(write, "WRITE_SIZE", sel)
        nl = sum(1 for r in fetch if sel(r["Kernel_Name"]))
        if f is None or w is None:
            continue
        lines.append(f"{cls:22s} {nl:8d} {f * kf / 1e9:9.3f} {w * kw / 1e9:9.3f} {(f * kf + w * kw) / 1e9:10.3f}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(path: str):
    """{class: traffic bytes per launch} from a summary whose fingerprint
    matches the current kernel sources, else None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    m = re.search(r"kernel source fingerprint: (\w+)", text)
    if not m or m.group(1) != source_fingerprint():
        return None
    out = {}
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 5 and re.match(r"c(128|64)_k\d_c\d_(direct|transfer|native|kraus)$", parts[0]):
            out[parts[0]] = float(parts[4]) * 1e9
    return out


if __name__ == "__main__":
    main()
