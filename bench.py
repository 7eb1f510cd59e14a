"""Benchmark: gate-conjugations per second on an n = 16 complex128 operator.

Workload (one GPU): a rank-16 Ginibre density matrix on n = 16 qubits
(65536 x 65536, 34.4 GB of c128 tiles at tile edge 32) evolved by layers of
    Haar U(2) on every qubit, a brickwork of Haar U(4) (alternating even/odd
    pairs) and amplitude damping (gamma = 0.01) on every qubit,
i.e. 39 or 40 conjugation passes per layer.  One step = one layer plus the
trace and a 64-term Pauli-sum expectation of the evolved state, so every
stage of the hot path runs in each step: host op preparation, intra-tile,
cross-tile and two-tile-bit passes, and the FP64 reductions.

Output: one JSON line (rank 0).  ``value`` = conjugation passes per second
over the K timed steps; ``roofline`` = algorithmic bytes (every stored entry
read and written once per pass) / measured time of the kernel class that takes
the most time, against MI355X's 8 TB/s; ``cpu_baseline`` = the CPU oracle
(Eq. (2) block form, numpy) on a bounded sample, see ``cpu_baseline()``;
``complex64`` = the same steps from the same state in complex64 storage
(FP64 arithmetic), see ``c64_run()``; ``fused`` = the same steps from the
same state with each layer run as a fused circuit (ops grouped into 2-qubit
passes), see ``fused_run()``.
``value`` is the op-by-op figure: one pass per op, as the method defines.
``serving`` = the metric's served half: circuits/s and p50/p99 latency of a
Poisson request stream under continuous batching (and with each request's
ops fused) against the plain one-at-a-time baseline, see ``serve_run()``.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 16] [--tile-log2 5]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0
METRIC = "n=16 c128 gate conj/s & HBM GB/s; served circuits/s + p99 vs plain"


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=8)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=16)
    p.add_argument("--tile-log2", type=int, default=5)
    p.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    p.add_argument("--seed", type=int, default=1616)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fused", action="store_true", help="skip the fused-circuit run of the same steps")
    p.add_argument("--no-c64", action="store_true",
                   help="skip the complex64-storage run of the same steps (run only with --dtype c128)")
    p.add_argument("--no-serve", action="store_true", help="skip the served-requests run")
    p.add_argument("--serve-count", type=int, default=48, help="requests of the served-requests run")
    p.add_argument("--serve-rate", type=float, default=1000.0, help="Poisson arrival rate (/s) of that run")
    p.add_argument("--cpu-sample-n", type=int, default=12,
                   help="qubits of the dense sub-operator the CPU oracle is timed on")
    p.add_argument("--tune", action="append", default=[], metavar="NAME=VALUE",
                   help="launch tuning passed to ht_set_tuning (repeatable)")
    p.add_argument("--copy-only", action="store_true",
                   help="only run the plain copy kernel on a buffer of the operator's size "
                        "(calibration of hardware byte counters)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(n_full: int, n_sample: int, seed: int) -> dict:
    """Time the CPU oracle on a bounded sample of the workload.

    Sample: the 2^s x 2^s sub-operator (s = n_sample) that fixing the top
    n_full - s qubits selects, evolved by two layers of the same op mix on its s
    qubits (a k-local op on those qubits maps that sub-operator to itself), with
    the oracle's Eq. (2) block form over the dense matrix.  The oracle's cost is
    proportional to the number of entries, so the per-op time is scaled by
    4^(n_full - s) to the full operator.  Reported as conjugation passes/s."""
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    rng = synth.make_rng(seed)
    G = synth.ginibre_factor(n_sample, 16, rng)
    rho = oracle.density_from_factor(G)
    ops = synth.layer_n16(0, rng, n=n_sample) + synth.layer_n16(1, rng, n=n_sample)
    t0 = time.perf_counter()
    done = 0
    for op in ops:
        rho = oracle.local_block_map(rho, op.mats, op.targets)
        done += 1
        if time.perf_counter() - t0 > 25.0:
            break
    dt = time.perf_counter() - t0
    per_op_sample = dt / done
    per_op_full = per_op_sample * 4.0 ** (n_full - n_sample)
    return {
        "value": 1.0 / per_op_full,
        "unit": "gate-conj/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"oracle Eq.(2) block form (numpy complex128) on the {1 << n_sample}x{1 << n_sample} "
                   f"sub-operator of the n={n_full} state with the top {n_full - n_sample} qubits fixed, "
                   f"{done} ops of two layers of the same mix on its {n_sample} qubits in {dt:.1f} s; "
                   f"per-op time scaled by 4^{n_full - n_sample} to n={n_full}"),
        "seconds": dt,
    }


def c64_run(ht, G, layers, args, codes, coeffs, tr_c128, ev_c128) -> dict:
    """The same steps from the same initial state in complex64 storage (FP64
    arithmetic and reductions, the pair layout where it applies): its own
    passes/s and HBM rate, and how far its readouts are from the complex128
    run's after the same steps."""
    import torch
    h = ht.Herm(args.n, args.tile_log2, "c64")
    h.init_lowrank(G)
    h.scale(1.0 / h.trace())
    for l in range(args.warmup):
        for op in layers[l]:
            h.apply_op(op)
    h.profile_reset()
    h.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nops = 0
    for l in range(args.warmup, args.warmup + args.steps):
        for op in layers[l]:
            h.apply_op(op)
        nops += len(layers[l])
        tr, ev = h.trace(), h.expectation_pauli_sum(codes, coeffs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = h.profile_read()
    h.profile_enable(False)
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    out = {
        "value": nops / elapsed,
        "unit": "gate-conj/s",
        "ms_per_step": elapsed / args.steps * 1e3,
        "storage_bytes": h.nbytes,
        "hbm_GBps": nops * 2.0 * h.nbytes / elapsed / 1e9,
        "dominant_class": dom_name,
        "dominant_GBps": dom["bytes"] / (dom["ms"] * 1e-3) / 1e9,
        "trace_diff_vs_c128": abs(tr - tr_c128),
        "pauli_expectation_diff_vs_c128": abs(ev - ev_c128),
    }
    h.close()
    log(f"[bench] complex64: {out['value']:.1f} gate-conj/s, {out['hbm_GBps']:.0f} GB/s")
    return out


def fused_run(ht, h, G, layers, args, codes, coeffs, tr_plain, ev_plain) -> dict:
    """The same steps from the same initial state with each layer applied as
    a fused circuit (neighbouring ops composed on the host into 2-qubit
    passes; planning and composition inside the timed region).  Reports its
    throughput in the same unit and how far its readouts are from the
    op-by-op run's."""
    import torch
    h.init_lowrank(G)
    h.scale(1.0 / h.trace())
    circuits = []

    def step(ops):
        c = ht.Circuit(ops)
        npass = c.plan(ht.SCHRODINGER, 2)
        c.apply(h)
        circuits.append(c)
        return npass, h.trace(), h.expectation_pauli_sum(codes, coeffs)

    for l in range(args.warmup):
        step(layers[l])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nops = npasses = 0
    tr = ev = None
    for l in range(args.warmup, args.warmup + args.steps):
        npass, tr, ev = step(layers[l])
        nops += len(layers[l])
        npasses += npass
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] fused: {nops / elapsed:.1f} gate-conj/s, {npasses / args.steps:.1f} passes per step")
    for c in circuits:
        c.close()
    return {
        "value": nops / elapsed,
        "unit": "gate-conj/s",
        "ms_per_step": elapsed / args.steps * 1e3,
        "passes_per_step": npasses / args.steps,
        "ops_per_step": nops / args.steps,
        "trace_diff_vs_op_by_op": abs(tr - tr_plain),
        "pauli_expectation_diff_vs_op_by_op": abs(ev - ev_plain),
        "note": "each layer as one ht_circuit: neighbouring ops composed in FP64 into passes on at most "
                "2 qubits (ops on disjoint qubits reordered), one streaming pass per group",
    }


def serve_run(ht, count: int, rate: float, seed: int) -> dict:
    """The served half of the metric: a Poisson stream of `count` requests
    (n log-uniform in 6..16, 10..300 mixed ops, c128/c64, half with a 64-term
    Pauli-sum readout; the stream `bench_ext.py serve` sweeps) served by the
    continuous-batching server and by the plain one-at-a-time baseline on the
    same requests: circuits/s and p50/p99 latency (arrival to result)."""
    import synth
    reqs = synth.serving_requests(count, rate, seed=seed)

    def stream(**cfg):
        srv = ht.Server(**cfg)
        t_start = srv.now()
        ids = []
        for r in reqs:
            while srv.now() - t_start < r["arrival"]:
                time.sleep(min(0.001, max(0.0, r["arrival"] - (srv.now() - t_start))))
            ids.append(srv.submit(r["n"], r["G"], r["ops"], r["pauli"], r["dtype"]))
        srv.wait_idle(1800)
        res = {d["id"]: d for d in srv.poll()}
        srv.close()
        recs = [res[i] for i in ids]
        lat = np.array([d["t_done"] - d["t_submit"] for d in recs])
        span = max(d["t_done"] for d in recs) - min(d["t_submit"] for d in recs)
        return ({"circuits_per_s": len(recs) / span, "p50_s": float(np.percentile(lat, 50)),
                 "p99_s": float(np.percentile(lat, 99)),
                 "failed": sum(1 for d in recs if d["status"] != 0)}, [d["value"] for d in recs])

    cont, v_cont = stream()
    log(f"[bench] served (continuous batching): {cont}")
    fused, v_fused = stream(fuse_qubits=2)
    log(f"[bench] served (continuous batching, each request's ops fused into 2-qubit passes): {fused}")
    fifo, v_fifo = stream(fifo=1)
    log(f"[bench] served (one at a time): {fifo}")
    return {
        "requests": count, "rate_per_s": rate, "ops": sum(len(r["ops"]) for r in reqs),
        "unit": "circuits/s", "continuous": cont, "continuous_fused": fused, "plain_fifo": fifo,
        "throughput_ratio": cont["circuits_per_s"] / fifo["circuits_per_s"],
        "p99_ratio": fifo["p99_s"] / cont["p99_s"],
        "p50_ratio": fifo["p50_s"] / cont["p50_s"],
        "fused_throughput_ratio": fused["circuits_per_s"] / fifo["circuits_per_s"],
        "fused_p99_ratio": fifo["p99_s"] / fused["p99_s"],
        "results_bitwise_equal": v_cont == v_fifo,
        "fused_max_rel_dev": max(abs(a - b) / max(1.0, abs(b)) for a, b in zip(v_fused, v_fifo)),
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the build this measures is single-GPU "
              "(multi-GPU sharding is a design note, not implemented); use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_15765_amd as ht
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n, m = args.n, args.tile_log2
    tuning = {}
    for t in args.tune:
        name, value = t.split("=")
        ht.set_tuning(name, int(value))
        tuning[name] = int(value)

    if args.copy_only:
        a = ht.Herm(n, m, args.dtype)
        b = ht.Herm(n, m, args.dtype)
        a.init_zero()
        b.init_zero()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            b.copy_from(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        print(json.dumps({"copy_bytes_each_way": a.nbytes, "ms": dt * 1e3,
                          "GBps_read_plus_write": 2 * a.nbytes / dt / 1e9}), flush=True)
        return

    # ---------------------------------------------------------------- setup
    r_state, r_ops, r_obs = synth.spawn_rngs(args.seed, 3)
    G = synth.ginibre_factor(n, 16, r_state)
    layers = [synth.layer_n16(l, r_ops, n=n) for l in range(args.warmup + args.steps)]
    codes, coeffs = synth.random_pauli_sum(n, 64, r_obs)

    h = ht.Herm(n, m, args.dtype, device=dev)
    log(f"[bench] n={n} tile_edge={1 << h.tile_log2} dtype={args.dtype} storage={h.nbytes / 1e9:.2f} GB")
    h.init_lowrank(G)
    h.scale(1.0 / h.trace())
    torch.cuda.synchronize()

    def step(ops):
        for op in ops:
            h.apply_op(op)
        tr = h.trace()
        ev = h.expectation_pauli_sum(codes, coeffs)
        return tr, ev

    for l in range(args.warmup):
        step(layers[l])
        log(f"[bench] warmup step {l + 1}/{args.warmup} done")

    h.profile_reset()
    h.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nops = 0
    tr = ev = None
    for l in range(args.warmup, args.warmup + args.steps):
        tr, ev = step(layers[l])
        nops += len(layers[l])
        log(f"[bench] step {l - args.warmup + 1}/{args.steps}: trace={tr:.15f} <O>={ev:+.6e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = h.profile_read()
    h.profile_enable(False)

    # --------------------------------------------------------------- report
    per_op_bytes = 2.0 * h.nbytes
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    dom_avg_ms = dom["ms"] / dom["launches"]
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    classes = {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"],
                   "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in sorted(prof.items())}
    kernel_ms = sum(v["ms"] for v in prof.values())
    # HBM bytes per launch of the dominant class from the committed rocprofv3
    # counter summary, if it was taken with the current kernel sources
    from paper_2604_15765_amd.profile_summary import read_traffic
    counted = read_traffic(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                        f"conj_n{n}_{args.dtype}_counters.txt"))
    traffic = counted.get(dom_name) if counted else None
    out = {
        "metric": METRIC,
        "value": nops / elapsed,
        "unit": "gate-conj/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"n{n}_{args.dtype}_layers: rank-16 Ginibre state, n={n}, tile edge "
                         f"{1 << h.tile_log2}, per step one layer (Haar U(2) on all qubits, brickwork "
                         f"Haar U(4), amplitude damping 0.01 on all qubits) + trace + 64-term Pauli sum"),
            "n": n, "tile_edge": 1 << h.tile_log2, "storage": args.dtype,
            "ops_per_step": nops / args.steps, "storage_bytes": h.nbytes, "tuning": tuning,
        },
        "hbm_GBps": nops * per_op_bytes / elapsed / 1e9,
        # the paper's effective bandwidth: stored bytes / time per op (one direction)
        "logical_GiBps": nops * h.nbytes / elapsed / 2 ** 30,
        "hbm_frac": nops * per_op_bytes / elapsed / 1e9 / HBM_PEAK_GBPS,
        "kernel_time_frac": kernel_ms * 1e-3 / elapsed,
        "roofline": {
            "bound": "hbm",
            "kernel": dom_name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "avg_launch_ms": dom_avg_ms,
            "bytes_per_launch": per_op_bytes,
        },
        "kernel_classes": classes,
        "final_trace": tr,
        "final_pauli_expectation": ev,
    }
    if args.dtype == "c128" and not args.no_c64:
        out["complex64"] = c64_run(ht, G, layers, args, codes, coeffs, tr, ev)
    if not args.no_fused:
        out["fused"] = fused_run(ht, h, G, layers, args, codes, coeffs, tr, ev)
    if not args.no_serve:
        h.close()
        torch.cuda.empty_cache()
        out["serving"] = serve_run(ht, args.serve_count, args.serve_rate, args.seed)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(n, min(args.cpu_sample_n, n), args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
