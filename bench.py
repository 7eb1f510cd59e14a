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
    p.add_argument("--no-tune", action="store_true",
                   help="skip the launch-shape tuning of the passes (ht_tune_passes) before timing")
    p.add_argument("--tuned-shapes-out", help="write the tuned pass shapes (JSON) to this file")
    p.add_argument("--tuned-shapes-in",
                   help="apply the pass shapes of this file (written by --tuned-shapes-out) instead of tuning")
    p.add_argument("--tune-only", action="store_true", help="stop after tuning (with --tuned-shapes-out)")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-operators run")
    p.add_argument("--batched-count", type=int, default=4096, help="operators of the batched run")
    p.add_argument("--batched-per-n", type=int, default=32,
                   help="operators per n of the batched run checked against the oracle")
    p.add_argument("--serve-count", type=int, default=256, help="requests per rate of the served-requests run")
    p.add_argument("--serve-rates", default="100,1000", help="Poisson arrival rates (/s) of that run")
    p.add_argument("--tune", action="append", default=[], metavar="NAME=VALUE",
                   help="launch tuning passed to ht_set_tuning (repeatable)")
    p.add_argument("--copy-only", action="store_true",
                   help="only run the plain copy kernel on a buffer of the operator's size "
                        "(calibration of hardware byte counters)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _oracle_per_op(n_full: int, n_sample: int, seed: int, budget_s: float) -> dict:
    """Per-op time of the CPU oracle (Eq. (2) block form, numpy complex128)
    on the 2^s x 2^s sub-operator (s = n_sample) that fixing the top
    n_full - s qubits selects -- a k-local op on the low s qubits maps it to
    itself -- over ops drawn in random order from two layers of the benchmark's
    op mix on those s qubits, until `budget_s` seconds have passed."""
    import oracle
    import synth
    rng = synth.make_rng(seed)
    G = synth.ginibre_factor(n_sample, 16, rng)
    rho = oracle.density_from_factor(G)
    ops = synth.layer_n16(0, rng, n=n_sample) + synth.layer_n16(1, rng, n=n_sample)
    order = rng.permutation(len(ops))
    t0 = time.perf_counter()
    done = 0
    for i in order:
        op = ops[int(i)]
        rho = oracle.local_block_map(rho, op.mats, op.targets)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"n_sample": n_sample, "ops": done, "seconds": dt, "per_op_s": dt / done,
            "gate_conj_per_s_at_sample_size": done / dt}


def cpu_baseline(n_full: int, seed: int) -> dict:
    """Time the CPU oracle on a bounded sample of the workload.

    Measured at n = 14 (the largest size whose dense 4 GiB matrix the oracle
    handles on a host in seconds per op): the per-op time there, scaled by
    4^(n_full - 14) to the full operator (the oracle's cost is proportional to
    the number of entries), gives the reported passes/s.  A second sample at
    n = 12, scaled by 4^(n_full - 12), is reported beside it."""
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    main_n = min(14, n_full)
    m = _oracle_per_op(n_full, main_n, seed, 25.0)
    sec = _oracle_per_op(n_full, min(12, n_full), seed + 1, 8.0)
    scale = 4.0 ** (n_full - main_n)
    return {
        "value": 1.0 / (m["per_op_s"] * scale),
        "unit": "gate-conj/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"oracle Eq.(2) block form (numpy complex128) on the {1 << main_n}x{1 << main_n} "
                   f"sub-operator of the n={n_full} state with the top {n_full - main_n} qubits fixed, "
                   f"{m['ops']} ops drawn at random from two layers of the same mix on its {main_n} qubits "
                   f"in {m['seconds']:.1f} s ({m['per_op_s']:.2f} s per op); per-op time scaled by "
                   f"4^{n_full - main_n} to n={n_full}"),
        "seconds": m["seconds"],
        "measured": m,
        "secondary_n12": {**sec, "scaled_gate_conj_per_s": 1.0 / (sec["per_op_s"] * 4.0 ** (n_full - sec["n_sample"]))},
        "host_cores": len(os.sched_getaffinity(0)),
    }


def copy_ceiling(ht, h, reps: int = 5) -> dict:
    """The library's copy kernel over a second buffer of h's size: read
    plus write bytes per second, the practical streaming ceiling that the
    pass's in-place read-modify-write compares with."""
    import torch
    b = ht.Herm(h.n, h.tile_log2, h.dtype)
    try:
        b.copy_from(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.copy_from(h)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    finally:
        b.close()
    gbps = 2 * h.nbytes / dt / 1e9
    return {"GBps": gbps, "frac_of_peak": gbps / HBM_PEAK_GBPS, "bytes_per_launch": 2 * h.nbytes,
            "note": "out-of-place copy of an operator-sized buffer, host-timed over 5 launches"}


def c64_run(ht, G, layers, args, codes, coeffs, tr_c128, ev_c128, h128) -> dict:
    """The same steps from the same initial state in complex64 storage (FP64
    arithmetic and reductions, the pair layout where it applies): its own
    passes/s and HBM rate; how far its readouts and 200,000 sampled entries
    are from the complex128 run's after the same steps (the parity-tested
    FP64 state); and both storage types against the CPU oracle after two
    layers of the same mix at n = 11, with the complex64 bound."""
    import torch
    import oracle
    import synth
    h = ht.Herm(args.n, args.tile_log2, "c64")
    h.init_lowrank(G)
    h.scale(1.0 / h.trace())
    if args.tuned_shapes_in:
        with open(args.tuned_shapes_in) as fh:
            for r in json.load(fh).get("c64", []):
                ht.set_pass_shape("c64", args.n, args.tile_log2, r)
    elif not args.no_tune:
        h.tune_passes(2)
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
    rng = synth.make_rng(args.seed + 7)
    rows = rng.integers(0, 1 << args.n, size=200000)
    cols = rng.integers(0, 1 << args.n, size=200000)
    e128 = h128.get_entries(rows, cols)
    e64 = h.get_entries(rows, cols)
    passes = nops + sum(len(layers[l]) for l in range(args.warmup))
    # both storage types against the oracle on the same mix at n = 11
    n11 = 11
    r11 = synth.make_rng(args.seed + 11)
    G11 = synth.ginibre_factor(n11, 16, r11)
    ops11 = synth.layer_n16(0, r11, n=n11) + synth.layer_n16(1, r11, n=n11)
    ref11 = oracle.apply_ops_local(oracle.density_from_factor(G11), ops11)
    err11 = {}
    for dt in ("c128", "c64"):
        g = ht.Herm(n11, args.tile_log2, dt).init_lowrank(G11)
        g.scale(1.0 / g.trace())
        for op in ops11:
            g.apply_op(op)
        err11[dt] = float(np.linalg.norm(g.to_dense() - ref11) / np.linalg.norm(ref11))
        g.close()
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
        "sampled_rel_frobenius_vs_c128": float(np.linalg.norm(e64 - e128) / np.linalg.norm(e128)),
        "sampled_entries": int(rows.size),
        "passes": passes,
        "bound_rel_frobenius": (passes + 1) * 2.0 ** -24,
        "n11_vs_oracle": {"passes": len(ops11), "rel_frobenius": err11,
                          "bound_c64": (len(ops11) + 1) * 2.0 ** -24, "tolerance_c128": 1e-12},
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


def batched_run(ht, count: int, per_n: int, seed: int) -> dict:
    """The batched extension on its own workload: `count` independent
    operators, n ~ U{4..11}, each a normalised Ginibre state of rank
    min(2^n, 64) under its own U{20..64}-op random noisy circuit (Haar 1q/2q,
    depolarising/dephasing), evolved (1) with one launch per op, (2) in one
    persistent batched launch, (3) in one batched launch with the launch
    shape and tile edge per n picked by the autotuner, and (4) the same with
    each operator's ops fused into 2-qubit passes.  Final states: (2) and (3)
    bitwise against one launch per op at the same tile edges, (4) against (3);
    a stratified sample (`per_n` operators per n) against the CPU oracle's
    block form, whose time on the host's cores is reported as its rate."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import synth

    rngs = synth.spawn_rngs(seed, count)
    work = []
    for rng in rngs:
        n = int(rng.integers(4, 12))
        G = synth.ginibre_factor(n, min(1 << n, 64), rng)
        ops = [synth.circuits._random_mixed_op(n, rng, "dephase") for _ in range(int(rng.integers(20, 65)))]
        work.append((n, G, ops))
    nops = sum(len(w[2]) for w in work)
    G_dev = [torch.from_numpy(G).to("cuda") for _, G, _ in work]
    default_edges = {n: 5 for n in range(4, 12)}

    def fresh(edges):
        hs = []
        for (n, _, _), g in zip(work, G_dev):
            h = ht.Herm(n, edges[n]).init_lowrank(g)
            h.scale(1.0 / h.trace())
            hs.append(h)
        torch.cuda.synchronize()
        return hs

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def run_plain(hs):
        for h, (_, _, ops) in zip(hs, work):
            for op in ops:
                h.apply_op(op)

    def queue(hs, **params):
        b = ht.Batch(**params)
        for h, (_, _, ops) in zip(hs, work):
            for op in ops:
                b.add_op(h, op)
        return b

    plain = fresh(default_edges)
    t_plain = timed(lambda: run_plain(plain))
    batched = fresh(default_edges)
    b = queue(batched, threads=256, wg_per_cu=2)
    t_batch = timed(b.run)
    same_batch = all(torch.equal(x.buffer, y.buffer) for x, y in zip(plain, batched))
    del plain
    log(f"[bench] batched: plain {t_plain:.3f} s, one batched launch {t_batch:.3f} s")
    cfg = b.autotune(512)
    b.close()
    edges = dict(default_edges)
    edges.update(cfg["tile_log2"])
    tplain = fresh(edges)
    t_tplain = timed(lambda: run_plain(tplain))
    tuned = fresh(edges)
    tb = queue(tuned, threads=cfg["threads"], wg_per_cu=cfg["wg_per_cu"], lds_max_bytes=cfg["lds_max_bytes"])
    t_tuned = timed(tb.run)
    tb.close()
    same_tuned = all(torch.equal(x.buffer, y.buffer) for x, y in zip(tplain, tuned))
    del tplain
    fused = fresh(edges)
    fb = queue(fused, threads=cfg["threads"], wg_per_cu=cfg["wg_per_cu"], lds_max_bytes=cfg["lds_max_bytes"],
               fuse_qubits=2)
    t_fused_plan = timed(fb.run)  # host planning and composition of every operator's passes, then the launch
    fused_dev = max(float(np.linalg.norm(x.to_dense() - y.to_dense()) / np.linalg.norm(y.to_dense()))
                    for x, y, (n, _, _) in zip(fused, tuned, work) if n <= 8)
    # oracle on the stratified sample, operators spread over the host's cores
    sample, seen = [], {}
    for i, (n, _, _) in enumerate(work):
        if seen.get(n, 0) < per_n:
            seen[n] = seen.get(n, 0) + 1
            sample.append(i)
    cores = len(os.sched_getaffinity(0))

    def ref(i):
        n, G, ops = work[i]
        return oracle.apply_ops_local(oracle.density_from_factor(G), ops)

    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)
    except Exception:
        limit = None
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        refs = list(ex.map(ref, sample))
    t_oracle = time.perf_counter() - t0
    if limit is not None:
        limit.restore_original_limits()
    worst = {"batched": 0.0, "tuned": 0.0, "fused": 0.0}
    for i, r in zip(sample, refs):
        nr = np.linalg.norm(r)
        for name, hs in (("batched", batched), ("tuned", tuned), ("fused", fused)):
            worst[name] = max(worst[name], float(np.linalg.norm(hs[i].to_dense() - r) / nr))
    # the same fused batch again: plans cached, device time plus table upload
    # (the operators now hold the circuits applied twice; nothing is compared after this)
    t_fused = timed(fb.run)
    fb.close()
    log(f"[bench] batched: tuned {t_tuned:.3f} s (plain at the tuned edges {t_tplain:.3f} s), "
        f"fused {t_fused:.3f} s ({t_fused_plan:.3f} s with planning)")
    oracle_ops = sum(len(work[i][2]) for i in sample)
    log(f"[bench] batched: oracle on {len(sample)} operators in {t_oracle:.1f} s, max errors {worst}")
    for hs in (batched, tuned, fused):
        for h in hs:
            h.close()
    return {
        "operators": count, "ops": nops, "unit": "circuits/s",
        "workload": "n ~ U{4..11}, Ginibre rank min(2^n, 64), U{20..64} ops each: 50% Haar 1q, 30% Haar 2q, "
                    "20% 1q depolarising/dephasing p ~ U(0, 0.1)",
        "plain_launches": {"s": t_plain, "circuits_per_s": count / t_plain, "gate_conj_per_s": nops / t_plain},
        "batched_launch": {"s": t_batch, "circuits_per_s": count / t_batch, "gate_conj_per_s": nops / t_batch,
                           "speedup_vs_plain": t_plain / t_batch, "bitwise_equal_to_plain": same_batch},
        "autotuned": {"s": t_tuned, "circuits_per_s": count / t_tuned, "config": cfg,
                      "plain_launches_same_edges_s": t_tplain, "speedup_vs_plain": t_plain / t_tuned,
                      "bitwise_equal_to_plain_same_edges": same_tuned},
        "fused": {"s": t_fused, "s_with_host_planning": t_fused_plan,
                  "circuits_per_s": count / t_fused, "speedup_vs_plain": t_plain / t_fused,
                  "max_rel_frobenius_vs_unfused_n_le_8": fused_dev},
        "oracle_check": {"operators": len(sample), "per_n": per_n, "max_rel_frobenius": worst,
                         "tolerance": 1e-12, "oracle_s": t_oracle, "oracle_threads": cores,
                         "oracle_circuits_per_s": len(sample) / t_oracle,
                         "oracle_gate_conj_per_s": oracle_ops / t_oracle},
    }


def serve_run(ht, count: int, rates, seed: int) -> dict:
    """The served half of the metric: Poisson streams of `count` requests
    (n log-uniform in 6..16, 10..300 mixed ops, c128/c64, half with a 64-term
    Pauli-sum readout) at each arrival rate, served four ways on the same
    requests -- one at a time (the plain baseline), with continuous batching,
    and both again with each request's ops fused into 2-qubit passes -- so
    that batching and fusion are measured apart: circuits/s and p50/p99
    latency (arrival to result)."""
    import synth

    def stream(reqs, **cfg):
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
        busy = np.array([d["t_done"] - d["t_admit"] for d in recs])
        big = np.array([r["n"] >= 14 for r in reqs])
        return ({"circuits_per_s": len(recs) / span, "p50_s": float(np.percentile(lat, 50)),
                 "p99_s": float(np.percentile(lat, 99)), "makespan_s": span,
                 "failed": sum(1 for d in recs if d["status"] != 0),
                 # one at a time, a request's admit-to-done time is its service time
                 "service_share_n_ge_14": float(busy[big].sum() / busy.sum())},
                [d["value"] for d in recs])

    out = {"requests_per_rate": count, "unit": "circuits/s", "rates": {}}
    for rate in rates:
        reqs = synth.serving_requests(count, rate, seed=seed)
        legs, vals = {}, {}
        for name, cfg in (("plain_fifo", {"fifo": 1}), ("continuous", {}),
                          ("fused_fifo", {"fifo": 1, "fuse_qubits": 2}), ("continuous_fused", {"fuse_qubits": 2})):
            legs[name], vals[name] = stream(reqs, **cfg)
            if name.startswith("continuous"):
                legs[name].pop("service_share_n_ge_14")
            log(f"[bench] served at {rate:g}/s, {name}: {legs[name]}")
        f, c, ff, cf = legs["plain_fifo"], legs["continuous"], legs["fused_fifo"], legs["continuous_fused"]
        out["rates"][f"{rate:g}"] = {
            "ops": sum(len(r["ops"]) for r in reqs),
            "n_ge_14_requests": sum(1 for r in reqs if r["n"] >= 14),
            **legs,
            # batching alone: continuous vs one at a time, unfused and fused
            "batching_throughput_ratio": c["circuits_per_s"] / f["circuits_per_s"],
            "batching_p99_ratio": f["p99_s"] / c["p99_s"],
            "batching_p50_ratio": f["p50_s"] / c["p50_s"],
            "batching_throughput_ratio_fused": cf["circuits_per_s"] / ff["circuits_per_s"],
            "batching_p99_ratio_fused": ff["p99_s"] / cf["p99_s"],
            "batching_p50_ratio_fused": ff["p50_s"] / cf["p50_s"],
            # fusion alone, one at a time; and both against the plain baseline
            "fusion_throughput_ratio": ff["circuits_per_s"] / f["circuits_per_s"],
            "combined_throughput_ratio": cf["circuits_per_s"] / f["circuits_per_s"],
            "combined_p99_ratio": f["p99_s"] / cf["p99_s"],
            "results_bitwise_equal_continuous_vs_fifo": vals["continuous"] == vals["plain_fifo"],
            "results_bitwise_equal_fused_continuous_vs_fused_fifo":
                vals["continuous_fused"] == vals["fused_fifo"],
            "fused_max_rel_dev_vs_plain": max(abs(a - b) / max(1.0, abs(b))
                                              for a, b in zip(vals["continuous_fused"], vals["plain_fifo"])),
        }
    return out


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
    # launch shapes per pass class timed on this operator (identity passes:
    # the state is unchanged), outside the timed region
    t0 = time.perf_counter()
    if args.tuned_shapes_in:
        with open(args.tuned_shapes_in) as fh:
            tuned = json.load(fh)[args.dtype]
        for r in tuned:
            ht.set_pass_shape(args.dtype, n, m, r)
    else:
        tuned = [] if args.no_tune else h.tune_passes(2)
    tune_s = time.perf_counter() - t0
    for r in tuned:
        log(f"[bench] pass shape {r}")
    if args.tuned_shapes_out:
        shapes = {args.dtype: tuned}
        if args.dtype == "c128" and not args.no_c64:
            h64 = ht.Herm(n, m, "c64")
            h64.init_lowrank(G)
            shapes["c64"] = h64.tune_passes(2)
            h64.close()
        with open(args.tuned_shapes_out, "w") as fh:
            json.dump(shapes, fh, indent=1)
    if args.tune_only:
        return

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
            "tuned_shapes": {f"k{r['k']}_c{r['cross']}_{r['form']}{'_low' if r['low_intra'] else ''}"
                             f"{'_far' if r.get('far') else ''}": r["shape"]
                             for r in tuned},
            "tune_s": tune_s,
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
            "copy_kernel": copy_ceiling(ht, h),
        },
        "kernel_classes": classes,
        "final_trace": tr,
        "final_pauli_expectation": ev,
    }
    if args.dtype == "c128" and not args.no_c64:
        out["complex64"] = c64_run(ht, G, layers, args, codes, coeffs, tr, ev, h)
    if not args.no_fused:
        out["fused"] = fused_run(ht, h, G, layers, args, codes, coeffs, tr, ev)
    if not args.no_serve or not args.no_batched:
        h.close()
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_run(ht, args.batched_count, args.batched_per_n, 4096)
        torch.cuda.empty_cache()
    if not args.no_serve:
        out["serving"] = serve_run(ht, args.serve_count, [float(x) for x in args.serve_rates.split(",")],
                                   args.seed)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(n, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
