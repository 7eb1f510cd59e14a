"""Benchmarks of the extensions: batched launches, serving, complex64 storage.

    python bench_ext.py batched   [--count 4096]
    python bench_ext.py serve     [--rates 10,100,1000] [--count 48]
    python bench_ext.py precision [--layers 4]
    python bench_ext.py native    [--reps 5]
    python bench_ext.py paper     [--ns 6,8,10,12,14,16]

Each prints one JSON line.  All inputs are seeded and synthetic (see synth/).

batched:   many independent operators (n ~ U{4..11}, U{20..64} mixed ops
           each: Haar 1q/2q, depolarising/dephasing) evolved three ways --
           one launch per op, replayed HIP graphs (one per operator), one
           persistent batched launch -- with the final states compared
           bitwise on the device and a stratified sample checked against
           the CPU oracle.
serve:     Poisson request streams (n log-uniform in 6..16, 10..300 mixed
           ops, c128/c64, half with a 64-term Pauli-sum readout) served by the
           continuous-batching server and by the one-at-a-time baseline on
           the same requests: circuits/s, p50/p99 latency, equal results.
paper:     the paper's experiment shapes: one op type (depolarising, H, X,
           Haar 1q, CNOT, Haar 2q) at every qubit position for n = 6..16
           with the paper's logical bandwidth (median and 95 % CI of repeated
           intervals); the n = 8 circuit on the GPU and the CPU oracle; the
           n = 14 sweep circuit per class, in both pictures (duality), and
           its whole evolved state against the CPU oracle.
native:    permutation-and-phase gates (X, Z, T, dephasing, CNOT, CZ, SWAP,
           Toffoli, CCZ, Fredkin) at n = 16 with the native pass and with
           the generic pass: time per pass and algorithmic bytes moved.
precision: the n = 16 layered workload in complex64 storage (FP64
           arithmetic and reductions) next to complex128: passes/s, and the
           complex64 error against the complex128 GPU state on sampled
           entries and against the CPU oracle at n = 11.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ batched

def run_batched(args):
    import torch
    import oracle
    import paper_2604_15765_amd as ht
    import synth

    torch.cuda.set_device(0)
    rngs = synth.spawn_rngs(args.seed, args.count)
    work = []
    for rng in rngs:
        n = int(rng.integers(4, 12))
        G = synth.ginibre_factor(n, min(1 << n, 64), rng)
        ops = [synth.circuits._random_mixed_op(n, rng, "dephase") for _ in range(int(rng.integers(20, 65)))]
        work.append((n, G, ops))
    nops = sum(len(w[2]) for w in work)
    tile = {n: args.tile_log2 for n in range(1, 12)}
    log(f"[batched] {args.count} operators, {nops} ops, "
        f"{sum(ht.storage_bytes(w[0], tile[w[0]]) for w in work) / 1e9:.1f} GB per copy")

    G_dev = [torch.from_numpy(G).to("cuda") for _, G, _ in work]

    def fresh(edges=tile):
        hs = []
        for (n, _, _), g in zip(work, G_dev):
            h = ht.Herm(n, edges[n]).init_lowrank(g)
            h.scale(1.0 / h.trace())
            hs.append(h)
        torch.cuda.synchronize()
        return hs

    # 1. one launch per op
    plain = fresh()
    t0 = time.perf_counter()
    for h, (_, _, ops) in zip(plain, work):
        for op in ops:
            h.apply_op(op)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"[batched] plain launches: {t_plain:.3f} s")

    # 2. captured graphs, one per operator
    s = torch.cuda.Stream()
    graphed = fresh()
    t0 = time.perf_counter()
    graphs = []
    for h, (_, _, ops) in zip(graphed, work):
        h.set_stream(s)
        ht.capture_begin(s)
        for op in ops:
            h.apply_op(op)
        graphs.append(ht.capture_end(s))
    t_capture = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in graphs:
        g.launch(s)
    s.synchronize()
    t_graph = time.perf_counter() - t0
    log(f"[batched] graphs: capture {t_capture:.3f} s, replay {t_graph:.3f} s")

    # 3. one persistent batched launch
    batched = fresh()
    batch = ht.Batch(threads=args.threads, wg_per_cu=args.wg_per_cu)
    t0 = time.perf_counter()
    for h, (_, _, ops) in zip(batched, work):
        for op in ops:
            batch.add_op(h, op)
    t_build = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.run()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"[batched] batch: build {t_build:.3f} s, run {t_batch:.3f} s")

    same_graph = all(torch.equal(a.buffer, b.buffer) for a, b in zip(plain, graphed))
    same_batch = all(torch.equal(a.buffer, b.buffer) for a, b in zip(plain, batched))
    del graphs, graphed

    # 4. autotuned: tile edge per n and launch shape picked on a sample of the
    # queued batch, operators created with the chosen edges; then the same
    # with each operator's ops fused into 2-qubit passes
    tuned_cfg = batch.autotune(args.tune_sample)
    log(f"[batched] autotune: {tuned_cfg}")
    edges = dict(tile)
    edges.update(tuned_cfg["tile_log2"])
    del plain
    tplain = fresh(edges)
    t0 = time.perf_counter()
    for h, (_, _, ops) in zip(tplain, work):
        for op in ops:
            h.apply_op(op)
    torch.cuda.synchronize()
    t_tplain = time.perf_counter() - t0
    tuned = fresh(edges)
    tbatch = ht.Batch(threads=tuned_cfg["threads"], wg_per_cu=tuned_cfg["wg_per_cu"],
                      lds_max_bytes=tuned_cfg["lds_max_bytes"])
    for h, (_, _, ops) in zip(tuned, work):
        for op in ops:
            tbatch.add_op(h, op)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tbatch.run()
    torch.cuda.synchronize()
    t_tuned = time.perf_counter() - t0
    log(f"[batched] tuned edges, plain launches: {t_tplain:.3f} s; tuned batch: {t_tuned:.3f} s")
    same_tuned = all(torch.equal(a.buffer, b.buffer) for a, b in zip(tplain, tuned))
    del tplain
    fused = fresh(edges)
    fbatch = ht.Batch(threads=tuned_cfg["threads"], wg_per_cu=tuned_cfg["wg_per_cu"],
                      lds_max_bytes=tuned_cfg["lds_max_bytes"], fuse_qubits=2)
    for h, (_, _, ops) in zip(fused, work):
        for op in ops:
            fbatch.add_op(h, op)
    fbatch.run()  # plans and composes every operator's passes (host), then runs
    torch.cuda.synchronize()
    fused2 = fresh(edges)
    fbatch.clear()
    for h, (_, _, ops) in zip(fused2, work):
        for op in ops:
            fbatch.add_op(h, op)
    t0 = time.perf_counter()
    fbatch.run()
    torch.cuda.synchronize()
    t_fused_total = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fbatch.run()  # fused lists cached: device time plus table upload
    torch.cuda.synchronize()
    t_fused = time.perf_counter() - t0
    log(f"[batched] fused batch: {t_fused:.3f} s (with planning {t_fused_total:.3f} s)")
    devs = []
    for a, b, (n, _, _) in zip(fused, tuned, work):
        if n <= 8 and len(devs) < 256:
            da, db = a.to_dense(), b.to_dense()
            devs.append(float(np.linalg.norm(da - db) / np.linalg.norm(db)))
    fused_dev = max(devs)
    npasses = 0
    for (_, _, ops) in work:
        c = ht.Circuit(ops)
        npasses += c.plan(ht.SCHRODINGER, 2)
        c.close()
    log(f"[batched] fused: {npasses} passes for {nops} ops; max deviation from unfused {fused_dev:.2e}")

    # oracle on a stratified sample: the first `per_n` operators of each n
    # (32 per n: 256 operators), timed on the host as the CPU rate
    worst = 0.0
    checked = 0
    oracle_s = 0.0
    oracle_ops = 0
    seen = {}
    for h, ht_, (n, G, ops) in zip(batched, tuned, work):
        if seen.get(n, 0) >= args.per_n:
            continue
        seen[n] = seen.get(n, 0) + 1
        t0 = time.perf_counter()
        ref = oracle.apply_ops_local(oracle.density_from_factor(G), ops)
        oracle_s += time.perf_counter() - t0
        oracle_ops += len(ops)
        for x in (h, ht_):
            worst = max(worst, float(np.linalg.norm(x.to_dense() - ref) / np.linalg.norm(ref)))
        checked += 1
        if checked % 16 == 0:
            log(f"[batched] oracle: {checked} operators checked, {oracle_s:.1f} s so far")
    log(f"[batched] oracle: {checked} operators, {oracle_ops} ops in {oracle_s:.1f} s, max error {worst:.2e}")
    out = {
        "bench": "batched",
        "operators": args.count, "ops": nops,
        "tile_log2": args.tile_log2,
        "plain": {"s": t_plain, "circuits_per_s": args.count / t_plain, "gate_conj_per_s": nops / t_plain},
        "graph": {"s": t_graph, "capture_s": t_capture, "circuits_per_s": args.count / t_graph,
                  "gate_conj_per_s": nops / t_graph},
        "batched": {"s": t_batch, "build_s": t_build, "circuits_per_s": args.count / t_batch,
                    "gate_conj_per_s": nops / t_batch, "threads": args.threads, "wg_per_cu": args.wg_per_cu},
        "tuned": {"s": t_tuned, "plain_s": t_tplain, "circuits_per_s": args.count / t_tuned,
                  "gate_conj_per_s": nops / t_tuned, "autotune": tuned_cfg,
                  "speedup_vs_plain_same_edges": t_tplain / t_tuned,
                  "speedup_vs_plain_default_edges": t_plain / t_tuned},
        "fused": {"s": t_fused, "s_with_planning": t_fused_total, "circuits_per_s": args.count / t_fused,
                  "gate_conj_per_s": nops / t_fused, "speedup_vs_plain_default_edges": t_plain / t_fused,
                  "passes": npasses, "max_rel_frobenius_vs_unfused_n_le_8": fused_dev},
        "speedup_vs_plain": t_plain / t_batch, "speedup_vs_graph": t_graph / t_batch,
        "bitwise_equal": {"graph": same_graph, "batched": same_batch, "tuned_vs_plain": same_tuned},
        "oracle_check": {"operators": checked, "max_rel_frobenius": worst, "tolerance": 1e-12,
                         "oracle_s": oracle_s, "oracle_circuits_per_s": checked / oracle_s,
                         "oracle_gate_conj_per_s": oracle_ops / oracle_s,
                         "host_threads": len(os.sched_getaffinity(0))},
        "state": "Ginibre factor of rank min(2^n, 64), normalised",
    }
    print(json.dumps(out), flush=True)


# -------------------------------------------------------------------- serve

def _serve_stream(ht, reqs, rate_hint, **cfg):
    srv = ht.Server(**cfg)
    t_start = srv.now()
    ids = []
    for r in reqs:
        while srv.now() - t_start < r["arrival"]:
            time.sleep(min(0.001, max(0.0, r["arrival"] - (srv.now() - t_start))))
        ids.append(srv.submit(r["n"], r["G"], r["ops"], r["pauli"], r["dtype"]))
    srv.wait_idle(1800)
    res = {d["id"]: d for d in srv.poll()}
    err = srv.last_error()
    srv.close()
    recs = [res[i] for i in ids]
    lat = np.array([d["t_done"] - d["t_submit"] for d in recs])
    span = max(d["t_done"] for d in recs) - min(d["t_submit"] for d in recs)
    return {
        "circuits_per_s": len(recs) / span,
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()), "makespan_s": span, "errors": err,
        "failed": sum(1 for d in recs if d["status"] != 0),
    }, [d["value"] for d in recs]


def run_serve(args):
    import torch
    import paper_2604_15765_amd as ht
    import synth

    torch.cuda.set_device(0)
    rates = [float(x) for x in args.rates.split(",")]
    results = []
    for rate in rates:
        reqs = synth.serving_requests(args.count, rate, seed=args.seed)
        nops = sum(len(r["ops"]) for r in reqs)
        log(f"[serve] rate {rate}/s: {len(reqs)} requests, {nops} ops, n: "
            f"{sorted(r['n'] for r in reqs)}")
        cont, v_cont = _serve_stream(ht, reqs, rate, budget_bytes=args.budget_gb << 30,
                                     max_active=args.max_active, batch_max_qubits=args.batch_max_qubits,
                                     medium_max_qubits=args.medium_max_qubits,
                                     max_medium_active=args.max_medium_active,
                                     chunk_ops=args.chunk_ops, large_chunk_ops=args.large_chunk_ops)
        log(f"[serve]   continuous: {cont}")
        fused, v_fused = _serve_stream(ht, reqs, rate, budget_bytes=args.budget_gb << 30,
                                       max_active=args.max_active, batch_max_qubits=args.batch_max_qubits,
                                       medium_max_qubits=args.medium_max_qubits,
                                       max_medium_active=args.max_medium_active,
                                       chunk_ops=args.chunk_ops, large_chunk_ops=args.large_chunk_ops,
                                       fuse_qubits=2)
        log(f"[serve]   continuous, fused: {fused}")
        fifo, v_fifo = _serve_stream(ht, reqs, rate, budget_bytes=args.budget_gb << 30, fifo=1)
        log(f"[serve]   one at a time: {fifo}")
        dev = max(abs(a - b) / max(1.0, abs(b)) for a, b, r in zip(v_fused, v_fifo, reqs))
        results.append({"rate": rate, "requests": len(reqs), "ops": nops, "continuous": cont,
                        "continuous_fused": fused, "plain_fifo": fifo, "equal_results": v_cont == v_fifo,
                        "fused_max_rel_dev": dev,
                        "throughput_ratio": cont["circuits_per_s"] / fifo["circuits_per_s"],
                        "p99_ratio": fifo["p99_s"] / cont["p99_s"],
                        "fused_throughput_ratio": fused["circuits_per_s"] / fifo["circuits_per_s"],
                        "fused_p99_ratio": fifo["p99_s"] / fused["p99_s"]})
    print(json.dumps({"bench": "serve", "results": results,
                      "workload": "Poisson arrivals; n = floor(exp(U(ln 6, ln 17))); 10..300 mixed ops; "
                                  "c128/c64 50/50; half with a 64-term Pauli-sum readout"}), flush=True)


# ------------------------------------------------------------------- native

def run_native(args):
    """Permutation-and-phase gates at n = 16, c128, tile edge 32: each gate
    at intra and tile-selecting positions, timed with the native pass and
    with the generic pass (native off; for k = 3 the Kraus form), on the
    same operator; and general three-qubit unitaries and channels (Kraus
    form)."""
    import torch
    import paper_2604_15765_amd as ht
    import synth

    torch.cuda.set_device(0)
    n = 16
    rng = synth.make_rng(args.seed)
    h = ht.Herm(n, 5).init_lowrank(synth.ginibre_factor(n, 16, rng))
    h.scale(1.0 / h.trace())
    cases = [
        ("X", [3], synth.named_gate("X")), ("X", [12], synth.named_gate("X")),
        ("Z", [4], synth.named_gate("Z")), ("Z", [12], synth.named_gate("Z")),
        ("T", [12], synth.named_gate("T")),
        ("dephasing", [12], synth.dephasing_kraus(0.1)),
        ("CNOT", [3, 4], synth.cnot_matrix()), ("CNOT", [8, 12], synth.cnot_matrix()),
        ("CZ", [9, 13], synth.permutation_gate("CZ")), ("SWAP", [6, 11], synth.permutation_gate("SWAP")),
        ("TOFFOLI", [3, 4, 12], synth.permutation_gate("TOFFOLI")),
        ("TOFFOLI", [8, 10, 14], synth.permutation_gate("TOFFOLI")),
        ("CCZ", [7, 9, 15], synth.permutation_gate("CCZ")),
        ("FREDKIN", [5, 11, 13], synth.permutation_gate("FREDKIN")),
    ]
    # general three-qubit ops (no native form): the Kraus-form pass
    kraus3 = [
        ("haar8", [2, 3, 4], synth.haar_unitary(8, rng)), ("haar8", [0, 1, 2], synth.haar_unitary(8, rng)),
        ("haar8", [3, 4, 12], synth.haar_unitary(8, rng)), ("haar8", [5, 10, 15], synth.haar_unitary(8, rng)),
        ("kraus3_r2", [3, 8, 12], synth.random_kraus_set(3, 2, rng)),
        ("kraus3_r4", [3, 8, 12], synth.random_kraus_set(3, 4, rng)),
        ("kraus3_r8", [3, 8, 12], synth.random_kraus_set(3, 8, rng)),
    ]
    results = []
    for name, t, g in cases + kraus3:
        kraus = g if g.ndim == 3 else g[None]
        row = {"gate": name, "targets": t}
        for native in ((1,) if name.startswith(("haar8", "kraus3")) else (1, 0)):
            # native 0: the generic pass (k <= 2) or the Kraus form (k = 3)
            ht.set_tuning("native", native)
            for _ in range(2):
                h.apply_channel(t, kraus)
            h.profile_reset()
            h.profile_enable(True)
            for _ in range(args.reps):
                h.apply_channel(t, kraus)
            prof = h.profile_read()
            h.profile_enable(False)
            (cls, v), = prof.items()
            key = "native" if native and cls.endswith("native") else "generic"
            row[key] = {"class": cls, "avg_ms": v["ms"] / v["launches"],
                        "bytes_per_launch": v["bytes"] / v["launches"],
                        "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
        ht.set_tuning("native", 1)
        if "generic" in row and "native" in row:
            row["speedup"] = row["generic"]["avg_ms"] / row["native"]["avg_ms"]
        log(f"[native] {row}")
        results.append(row)
    print(json.dumps({"bench": "native", "n": n, "tile_edge": 32, "storage": "c128",
                      "storage_bytes": h.nbytes, "results": results}), flush=True)


# -------------------------------------------------------------------- paper

def median_ci95(samples):
    """Median of the samples and a distribution-free 95 % confidence interval
    for it from order statistics: [x_(j), x_(n+1-j)] with j the largest index
    for which P(Binomial(n, 1/2) < j) <= 2.5 % (n = 10: the 2nd and 9th of
    the sorted samples, coverage 97.9 %)."""
    x = sorted(samples)
    n = len(x)
    j, acc = 0, 0.0
    for i in range(n + 1):
        acc += math.comb(n, i) / 2.0 ** n  # P(B <= i)
        if acc > 0.025:
            break
        j = i + 1
    j = max(j, 1)
    return float(np.median(x)), x[j - 1], x[n - j]


def run_paper(args):
    """The paper's own experiment shapes, on the GPU: one op type applied at
    every qubit position for n = 6..16 (time per op, read+write GB/s, and
    the paper's logical bandwidth = stored bytes / time per op, in GiB/s);
    the n = 8 200-op circuit on the GPU and on the CPU oracle; the n = 14
    sweep circuit with per-class rates and the oracle's per-op time.

    Timing follows the paper's protocol (Section IV): per n, op type and
    qubit position, one timing interval covers L consecutive applications
    to the continuously evolving operator (L chosen per n so an interval
    moves about 2 GB); after a warm-up the interval is repeated --reps
    times and the median with a 95 % confidence interval is reported.
    Intervals are timed with HIP events on the operator's stream.  The
    operator is the paper's random (G + G^dagger)/2 (not PSD, not
    normalised) for n <= 12 and a rank-4 Ginibre density above (a dense
    host matrix would not fit); the values do not change the time."""
    import torch
    import oracle
    import paper_2604_15765_amd as ht
    import synth

    torch.cuda.set_device(0)
    rng = synth.make_rng(args.seed)
    H1 = synth.named_gate("H")
    X1 = synth.named_gate("X")
    depol = synth.depolarising_kraus(0.1)
    out = {"bench": "paper", "reps": args.reps, "sweep": [], "positions": []}
    for n in [int(x) for x in args.ns.split(",")]:
        if n <= 12:
            h = ht.Herm(n, 5).init_dense(synth.random_hermitian_dense(n, rng))
        else:
            h = ht.Herm(n, 5).init_lowrank(torch.from_numpy(synth.ginibre_factor(n, 4, rng)).to("cuda"))
            h.scale(1.0 / h.trace())
        if n >= 12 and not args.no_tune:
            h.tune_passes(2)  # launch shapes per pass class (identity passes: the operator is unchanged)
        stream = h.stream
        U1 = synth.haar_unitary(2, rng)
        U2 = synth.haar_unitary(4, rng)
        kinds = [("depolarising", 1, depol), ("H", 1, H1[None]), ("X", 1, X1[None]), ("haar1", 1, U1[None]),
                 ("cnot", 2, synth.cnot_matrix()[None]), ("haar2", 2, U2[None])]
        L = max(1, min(50, int(2e9 / (2 * h.nbytes))))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.reps)]
        for name, k, mats in kinds:
            positions = [[a] for a in range(n)] if k == 1 else [[a, a + 1] for a in range(n - 1)]
            per_pos = []
            for t in positions:
                for _ in range(min(L, 3)):  # warm-up
                    h.apply_channel(t, mats)
                for r in range(args.reps):
                    ev[2 * r].record(stream)
                    for _ in range(L):
                        h.apply_channel(t, mats)
                    ev[2 * r + 1].record(stream)
                stream.synchronize()
                us = [ev[2 * r].elapsed_time(ev[2 * r + 1]) * 1e3 / L for r in range(args.reps)]
                med, lo, hi = median_ci95(us)
                row = {"n": n, "op": name, "targets": t, "ops_per_interval": L, "us_per_op": med,
                       "us_ci95": [lo, hi], "rw_GBps": 2 * h.nbytes / med / 1e3,
                       "logical_GiBps": h.nbytes / (med * 1e-6) / 2 ** 30}
                out["positions"].append(row)
                per_pos.append(med)
            mean_us = float(np.mean(per_pos))
            row = {"n": n, "op": name, "positions": len(positions), "us_per_op": mean_us,
                   "us_per_op_range": [float(min(per_pos)), float(max(per_pos))],
                   "rw_GBps": 2 * h.nbytes / mean_us / 1e3,
                   "logical_GiBps": h.nbytes / (mean_us * 1e-6) / 2 ** 30}
            out["sweep"].append(row)
            log(f"[paper] n={n} {name}: {mean_us:.1f} us/op (positions {min(per_pos):.1f}..{max(per_pos):.1f}), "
                f"logical {row['logical_GiBps']:.0f} GiB/s")
        h.close()
        torch.cuda.empty_cache()

    # n = 8, 200 ops: GPU (launch-bound) and the dense CPU oracle
    G, ops = synth.circuit_plain_n8(seed=1234)
    h = ht.Herm(8, 5).init_lowrank(torch.from_numpy(G).to("cuda"))
    h.scale(1.0 / h.trace())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op in ops:
        h.apply_op(op)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    rho = oracle.density_from_factor(G)
    t0 = time.perf_counter()
    ref = oracle.apply_ops(rho, ops)
    t_cpu = time.perf_counter() - t0
    out["n8_circuit"] = {"ops": len(ops), "gpu_s": t_gpu, "oracle_s": t_cpu,
                         "rel_frobenius": float(np.linalg.norm(h.to_dense() - ref) / np.linalg.norm(ref))}
    log(f"[paper] n=8 circuit: GPU {t_gpu * 1e3:.1f} ms, oracle {t_cpu:.1f} s")

    # n = 14 sweep circuit: every class at every position.  Schroedinger on
    # the state, Heisenberg on a 64-term Pauli sum through the adjoint circuit
    # in reverse order; duality tr(O Phi(rho)) = tr(Phi*(O) rho) on the GPU,
    # and the whole evolved state against the oracle's local-block form
    G, ops, (codes, coeffs) = synth.circuit_sweep(n=14)
    h = ht.Herm(14, 5).init_lowrank(torch.from_numpy(G).to("cuda"))
    h.scale(1.0 / h.trace())
    if not args.no_tune:
        h.tune_passes(2)
    h.profile_reset()
    h.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op in ops:
        h.apply_op(op)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    prof = h.profile_read()
    h.profile_enable(False)
    classes = {c: {"launches": v["launches"], "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
               for c, v in sorted(prof.items())}
    O = ht.Herm(14, 5).init_pauli_sum(codes, coeffs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op in reversed(ops):
        O.apply_op(op, ht.HEISENBERG)
    torch.cuda.synchronize()
    t_heis = time.perf_counter() - t0
    rho0 = ht.Herm(14, 5).init_lowrank(torch.from_numpy(G).to("cuda"))
    rho0.scale(1.0 / rho0.trace())
    e_s = h.expectation_pauli_sum(codes, coeffs)
    e_h = O.expectation(rho0)
    O.close()
    rho0.close()
    res = {"ops": len(ops), "gate_conj_per_s": len(ops) / t_gpu, "classes": classes,
           "heisenberg_gate_conj_per_s": len(ops) / t_heis,
           "expectation_schroedinger": e_s, "expectation_heisenberg": e_h,
           "duality_abs_diff": abs(e_s - e_h)}
    log(f"[paper] n=14 sweep: {len(ops) / t_gpu:.0f} gate-conj/s (Heisenberg {len(ops) / t_heis:.0f}); "
        f"duality |{e_s:.6e} - {e_h:.6e}| = {abs(e_s - e_h):.1e}")
    if args.n14_oracle:
        got = h.to_dense()
        h.close()
        torch.cuda.empty_cache()
        rho = oracle.density_from_factor(G)
        t_cpu = 0.0
        for i, op in enumerate(ops):
            t0 = time.perf_counter()
            rho = oracle.local_block_map(rho, op.mats, op.targets)
            t_cpu += time.perf_counter() - t0
            if (i + 1) % 8 == 0:
                log(f"[paper] n=14 oracle: {i + 1}/{len(ops)} ops, {t_cpu:.0f} s")
        res["oracle_s_per_op"] = t_cpu / len(ops)
        res["oracle_ops_timed"] = len(ops)
        res["rel_frobenius_vs_oracle"] = float(np.linalg.norm(got - rho) / np.linalg.norm(rho))
        res["host_threads"] = len(os.sched_getaffinity(0))
        log(f"[paper] n=14 vs oracle (whole state, {len(ops)} ops): {res['rel_frobenius_vs_oracle']:.2e}, "
            f"oracle {res['oracle_s_per_op']:.2f} s per op")
    out["n14_sweep"] = res
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- precision

def run_precision(args):
    import torch
    import oracle
    import paper_2604_15765_amd as ht
    import synth

    torch.cuda.set_device(0)
    out = {"bench": "precision"}
    # n = 16: throughput and the c64 error against the c128 GPU state
    n = 16
    r_state, r_ops, r_obs = synth.spawn_rngs(args.seed, 3)
    G = synth.ginibre_factor(n, 16, r_state)
    layers = [synth.layer_n16(l, r_ops, n=n) for l in range(args.layers)]
    codes, coeffs = synth.random_pauli_sum(n, 64, r_obs)
    states = {}
    for dtype in ("c128", "c64"):
        h = ht.Herm(n, 5, dtype).init_lowrank(G)
        h.scale(1.0 / h.trace())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cnt = 0
        for ops in layers:
            for op in ops:
                h.apply_op(op)
            cnt += len(ops)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[dtype] = {"gate_conj_per_s": cnt / dt, "GBps": cnt * 2 * h.nbytes / dt / 1e9,
                      "trace": h.trace(), "pauli_expectation": h.expectation_pauli_sum(codes, coeffs)}
        states[dtype] = h
        log(f"[precision] n=16 {dtype}: {out[dtype]}")
    rng = synth.make_rng(args.seed + 1)
    rows = rng.integers(0, 1 << n, size=200000)
    cols = rng.integers(0, 1 << n, size=200000)
    a = states["c128"].get_entries(rows, cols)
    b = states["c64"].get_entries(rows, cols)
    out["n16_c64_vs_c128"] = {
        "sampled_entries": int(rows.size),
        "rel_frobenius_sampled": float(np.linalg.norm(a - b) / np.linalg.norm(a)),
        "trace_diff": abs(out["c128"]["trace"] - out["c64"]["trace"]),
        "pauli_expectation_diff": abs(out["c128"]["pauli_expectation"] - out["c64"]["pauli_expectation"]),
        "passes": sum(len(l) for l in layers),
        "bound_rel_frobenius": (sum(len(l) for l in layers) + 1) * 2.0 ** -24,
    }
    del states
    torch.cuda.empty_cache()
    # smaller n: both storage types against the CPU oracle
    n = args.check_n
    G = synth.ginibre_factor(n, 16, r_state)
    lay = [synth.layer_n16(l, r_ops, n=n) for l in range(args.layers)]
    ops = [op for l in lay for op in l]
    ref = oracle.apply_ops_local(oracle.density_from_factor(G), ops)
    errs = {}
    for dtype in ("c128", "c64"):
        h = ht.Herm(n, 5, dtype).init_lowrank(G)
        h.scale(1.0 / h.trace())
        for op in ops:
            h.apply_op(op)
        errs[dtype] = float(np.linalg.norm(h.to_dense() - ref) / np.linalg.norm(ref))
    out[f"n{n}_vs_oracle"] = {"passes": len(ops), "rel_frobenius": errs,
                            "bound_c64": (len(ops) + 1) * 2.0 ** -24, "tolerance_c128": 1e-12}
    out["speedup_c64_over_c128"] = out["c64"]["gate_conj_per_s"] / out["c128"]["gate_conj_per_s"]
    print(json.dumps(out), flush=True)


def main():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = p.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("batched")
    b.add_argument("--count", type=int, default=4096)
    b.add_argument("--seed", type=int, default=4096)
    b.add_argument("--tile-log2", type=int, default=5)
    b.add_argument("--threads", type=int, default=256)
    b.add_argument("--wg-per-cu", type=int, default=2)
    b.add_argument("--per-n", type=int, default=32, help="operators per n checked against the oracle")
    b.add_argument("--tune-sample", type=int, default=512, help="operators the autotuner times")
    s = sub.add_parser("serve")
    s.add_argument("--rates", default="10,100,1000")
    s.add_argument("--count", type=int, default=48)
    s.add_argument("--seed", type=int, default=2000)
    s.add_argument("--budget-gb", type=int, default=200)
    s.add_argument("--max-active", type=int, default=32)
    s.add_argument("--batch-max-qubits", type=int, default=8)
    s.add_argument("--medium-max-qubits", type=int, default=12)
    s.add_argument("--max-medium-active", type=int, default=4)
    s.add_argument("--chunk-ops", type=int, default=64)
    s.add_argument("--large-chunk-ops", type=int, default=4)
    r = sub.add_parser("precision")
    r.add_argument("--layers", type=int, default=4)
    r.add_argument("--check-n", type=int, default=11, help="qubits of the oracle-checked run")
    r.add_argument("--seed", type=int, default=1616)
    v = sub.add_parser("native")
    v.add_argument("--seed", type=int, default=1616)
    v.add_argument("--reps", type=int, default=5)
    q = sub.add_parser("paper")
    q.add_argument("--seed", type=int, default=530)
    q.add_argument("--ns", default="6,8,10,12,14,16")
    q.add_argument("--reps", type=int, default=10, help="timing intervals per (n, op, position)")
    q.add_argument("--no-tune", action="store_true", help="skip the pass tuner (ht_tune_passes) for n >= 12")
    q.add_argument("--no-n14-oracle", dest="n14_oracle", action="store_false",
                   help="skip the whole-state oracle run of the n = 14 sweep circuit (minutes on the host)")
    args = p.parse_args()
    {"batched": run_batched, "serve": run_serve, "precision": run_precision,
     "native": run_native, "paper": run_paper}[args.cmd](args)


if __name__ == "__main__":
    main()
