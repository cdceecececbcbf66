#!/usr/bin/env python3
"""Benchmark: (alpha,beta)-core peeling on one MI355X.

Workload: seeded Chung-Lu bipartite graph with |U| = 1,000,000,
|L| = 500,000, 20,000,000 distinct edges, degree-distribution exponent 2.1 on
both layers, expected degrees capped at 50,000; query (alpha,beta) = (10,10).
One step = one index-free GCC query (Algorithm 1: scan, peel, bitmask) on
the resident CSR.  The same query on the build's degree-rank copy, cold-cache
runs of both, GCC+ (Algorithm 2) with its core-number preprocessing, the
billion-edge sweep, the batch and the serving loop are reported as extra
fields; preprocessing is timed apart from queries, as in Table II.

Metric: edges peeled per second = (m - |E(core)|) / step time, with the
numerator taken from the CPU oracle so it does not depend on the GPU code.
Roofline: the query's algorithmic bytes, computed from the oracle's counts
(8 B per vertex, n/8, 16 B + 4 B per entry of each removed vertex, 8 B per
peeled edge), over the step's device time (HIP events), against 8 TB/s.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def _cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor()


# The sources of the GCC step's kernels, their launches and the data layout
# they read (the core-number, component, vertex-set and serving sources are
# not part of the step).
STEP_SOURCES = ("abcore_internal.h", "api.hip", "build.hip", "peel.hip", "prim.h", "wave.h")


def _kernel_source_hash() -> str:
    """SHA-256 over the GCC step's sources, sorted by name (name, then
    content)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(STEP_SOURCES):
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2606_07148_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


PROFILE = os.path.join(ROOT, "profiles", "gcc_chung_lu_1M_500k_20M_a10_b10.md")


def _counter_traffic_step(mode: str):
    """HBM bytes of one step of `mode` ("index_free" or "rank_order") from
    the committed hardware-counter summary (FETCH_SIZE and WRITE_SIZE of
    every kernel of the step, scaled by a plain copy's readings), or None
    when the kernel sources changed since the counters were taken."""
    try:
        text = open(PROFILE).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != _kernel_source_hash():
        return None
    return rec.get("steps", {}).get(mode)


def bench_batch(args, pkg, torch, np, bigraph_gen) -> dict:
    """Batched queries: Chung-Lu |U|=10M |L|=5M m=200M gamma=2.1 cap 50k,
    256 (alpha,beta) pairs log-uniform in [1,256]^2, one abcore_compute_batch
    call (captured HIP graph, nested queries) against 256 sequential
    abcore_compute calls on the same GPU; answers compared bit for bit."""
    spec = bigraph_gen.CONFIGS[4]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    print(f"# batch graph generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    deu = torch.from_numpy(eu).cuda()
    dev = torch.from_numpy(ev).cuda()
    pkg.abcore_device_memory(reset_peak=True)
    g = pkg.abcore_build_csr(nU, nL, deu, dev)
    del deu, dev, eu, ev
    a, b = bigraph_gen.loguniform_pairs(256, 1, 256, spec["seed"] + 1000)
    alphas, betas = [int(x) for x in a], [int(x) for x in b]
    q = len(alphas)
    words = g.nwords
    out = torch.empty((q, words), dtype=torch.int32, device="cuda")
    seq = torch.empty((q, words), dtype=torch.int32, device="cuda")
    # sequential: one query at a time
    for i in range(min(4, q)):
        pkg.abcore_compute(g, alphas[i], betas[i], pkg.ABCORE_GCC, out=seq[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(q):
        pkg.abcore_compute(g, alphas[i], betas[i], pkg.ABCORE_GCC, out=seq[i])
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    # batched: the first call plans and captures, later calls replay
    t0 = time.perf_counter()
    pkg.abcore_compute_batch(g, alphas, betas, out=out)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    reps = max(1, args.batch_reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        pkg.abcore_compute_batch(g, alphas, betas, out=out)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / reps
    parity = bool(torch.equal(out, seq))
    parent, _, states = pkg.abcore_batch_plan(alphas, betas)
    _, peak = pkg.abcore_device_memory()
    n = nU + nL
    gold = _golden("c4")
    extra = {}
    if gold is not None and len(gold["queries"]) == q:
        gq = gold["queries"]
        extra["parity_vs_oracle_digests"] = all(
            _sha_words(out[i][: (n + 31) // 32]) == gq[i]["bitmask_sha256"] for i in range(q))
        seq_bytes = sum(_gcc_bytes(n, x) for x in gq)
        # a nested query scans n vertices and peels only the difference
        # between its parent's core and its own; a repeated query copies a
        # bitmask
        nested = 0
        for i in range(q):
            p = parent[i]
            if p >= 0 and (alphas[p], betas[p]) == (alphas[i], betas[i]):
                nested += 2 * (n // 8)
            elif p >= 0:
                nested += 8 * n + n // 8 + sum(
                    c * (gq[i][k] - gq[p][k]) for c, k in
                    ((16, "removed"), (4, "removed_degree_sum"), (8, "m_peeled")))
            else:
                nested += _gcc_bytes(n, gq[i])
        extra.update(sequential_algorithmic_bytes=seq_bytes,
                     sequential_frac=seq_bytes / seq_s / 1e9 / HBM_PEAK_GBS,
                     batch_algorithmic_bytes=nested,
                     batch_frac=nested / batch_s / 1e9 / HBM_PEAK_GBS,
                     batch_frac_of_sequential_bytes=seq_bytes / batch_s / 1e9 / HBM_PEAK_GBS)
    g.destroy()
    return {
        "workload": "chung-lu |U|=10,000,000 |L|=5,000,000 m=200,000,000 gamma=2.1/2.1 "
                    "cap=50,000; 256 (alpha,beta) log-uniform in [1,256]^2 (seed 1004)",
        "queries": q,
        "batched_queries_per_s": q / batch_s,
        "batch_ms": batch_s * 1e3,
        "first_call_ms": first_s * 1e3,
        "sequential_queries_per_s": q / seq_s,
        "sequential_ms": seq_s * 1e3,
        "speedup_vs_sequential": seq_s / batch_s,
        "parity_vs_sequential": parity,
        "roots": sum(1 for p in parent if p < 0),
        "state_buffers": states,
        "replays": reps,
        "device_memory_library_peak_bytes": peak,
        **extra,
    }


def _pct(values, q):
    import numpy as np
    return float(np.percentile(np.asarray(values, np.float64), q)) if len(values) else None


def _drive(pkg, g, ups, lo, hi, sched_ns=None):
    """Submits requests lo..hi-1 of the stream in order (at their scheduled
    steady-clock times when given, else as fast as admission allows) and
    polls them; returns (results in order, submit times, wall seconds)."""
    n = hi - lo
    res = [None] * n
    t_sub = [0] * n
    waiting = []
    i = 0
    t0 = time.monotonic_ns()
    while i < n or waiting:
        if i < n and (sched_ns is None or time.monotonic_ns() >= sched_ns[i]):
            k = lo + i
            t = pkg.abcore_try_submit(g, ups["u"][k], ups["v"][k], ups["op"][k],
                                      ups["alpha"][k], ups["beta"][k])
            if t is not None:
                t_sub[i] = time.monotonic_ns()
                waiting.append((i, t))
                i += 1
                continue
        still = []
        for j, t in waiting:
            r = pkg.abcore_poll(g, t)
            if r is None:
                still.append((j, t))
            else:
                res[j] = r
        waiting = still
    return res, t_sub, (time.monotonic_ns() - t0) / 1e9


def bench_serve(args, pkg, torch, np, bigraph_gen) -> dict:
    """Serving on-the-fly queries: Chung-Lu |U|=20M |L|=10M m=500M gamma=2.1
    cap 50k; a stream of edge updates (70% insertions of new edges, 30%
    deletions of present ones), each asking (alpha,beta)-membership with
    alpha, beta log-uniform in [2,64].  Sequential abcore_query (one at a
    time) against the serving loop, closed loop (as fast as admitted) and
    open loop (Poisson arrivals at fractions of the closed-loop rate);
    latency = completion - scheduled arrival.  Every served answer is
    compared with the sequential answer of the same request."""
    spec = bigraph_gen.CONFIGS[5]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, args.serve_requests, spec["seed"] + 1000)
    print(f"# serving graph and stream generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    handles = []
    pkg.abcore_device_memory(reset_peak=True)
    for _ in range(3 if args.serve_prune else 2):
        deu = torch.from_numpy(eu).cuda()
        dev = torch.from_numpy(ev).cuda()
        handles.append(pkg.abcore_build_csr(nU, nL, deu, dev))
        del deu, dev
    del eu, ev
    torch.cuda.empty_cache()
    g_seq, g_srv = handles[:2]
    pkg.abcore_components(g_seq)
    total = len(ups["u"])
    # sequential: one abcore_query at a time
    seq = []
    t_seq = []
    for k in range(total):
        t1 = time.perf_counter()
        try:
            a, b = pkg.abcore_query(g_seq, ups["u"][k], ups["v"][k], ups["op"][k],
                                    ups["alpha"][k], ups["beta"][k])
            seq.append(("OK", a, b))
        except pkg.AbcoreError as e:
            seq.append((e.name, None, None))
        t_seq.append(time.perf_counter() - t1)
    seq_qps = total / sum(t_seq)
    if args.serve_pull:
        pkg.abcore_set_option(g_srv, pkg.ABCORE_OPT_PULL, args.serve_pull)
    pkg.abcore_serve_start(g_srv, args.serve_inflight, args.serve_slots, 0)
    phases = []
    served = []
    # closed loop: the first part of the stream as fast as admission allows
    n_closed = total // 3
    res, t_sub, wall = _drive(pkg, g_srv, ups, 0, n_closed)
    lat = [(r["t_done_ns"] - s) / 1e6 for r, s in zip(res, t_sub)]
    closed_qps = n_closed / wall
    phases.append({"mode": "closed", "requests": n_closed, "queries_per_s": closed_qps,
                   "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99)})
    served += res
    # open loop at fractions of the closed-loop rate: Poisson arrivals
    lo = n_closed
    fracs = [0.25, 0.5, 0.8, 0.95]
    per = (total - n_closed) // len(fracs)
    for f in fracs:
        hi = lo + per
        lam = f * closed_qps
        gaps = np.asarray(ups["gap"][lo:hi], np.float64) / lam
        start = time.monotonic_ns() + 1_000_000
        sched = (start + np.cumsum(gaps) * 1e9).astype(np.int64).tolist()
        res, t_sub, wall = _drive(pkg, g_srv, ups, lo, hi, sched)
        lat = [(r["t_done_ns"] - s) / 1e6 for r, s in zip(res, sched)]
        phases.append({"mode": "open", "rate_fraction": f, "offered_per_s": lam,
                       "requests": hi - lo, "queries_per_s": (hi - lo) / wall,
                       "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99)})
        served += res
        lo = hi
    _, peak = pkg.abcore_device_memory()
    counters = pkg.abcore_serve_stop(g_srv)
    pruned = None
    if args.serve_prune:
        # the same requests, closed loop, with stale core-number pruning: a
        # snapshot of the core numbers at start and after every
        # serve_prune applied updates (its time included)
        g_pr = handles[2]
        pkg.abcore_set_option(g_pr, pkg.ABCORE_OPT_SERVE_PRUNE, args.serve_prune)
        if args.serve_pull:
            pkg.abcore_set_option(g_pr, pkg.ABCORE_OPT_PULL, args.serve_pull)
        t0 = time.perf_counter()
        pkg.abcore_serve_start(g_pr, args.serve_inflight, args.serve_slots, 0)
        start_s = time.perf_counter() - t0
        res, t_sub, wall = _drive(pkg, g_pr, ups, 0, total)
        pc = pkg.abcore_serve_counters(g_pr)
        pkg.abcore_serve_stop(g_pr)
        lat = [(r["t_done_ns"] - s0) / 1e6 for r, s0 in zip(res, t_sub)]
        pmis = sum(1 for r, w in zip(res, seq) if r["status"] != w[0] or
                   (w[0] == "OK" and (r["answer"], r["bits"]) != (w[1], w[2])))
        pruned = {"requests": total, "refresh_every": args.serve_prune,
                  "queries_per_s": total / wall, "speedup_vs_sequential": (total / wall) / seq_qps,
                  "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                  "decided_without_peel": pc["decided_without_peel"],
                  "core_snapshots": pc["core_snapshots"], "snapshot_ms": pc["snapshot_ms"],
                  "first_snapshot_in_serve_start_s": start_s,
                  "answers_equal_sequential": pmis == 0, "mismatches": pmis}
    n_cmp = len(served)
    mismatch = 0
    for r, w in zip(served, seq[:n_cmp]):
        if r["status"] != w[0] or (w[0] == "OK" and (r["answer"], r["bits"]) != (w[1], w[2])):
            mismatch += 1
    for h in handles:
        h.destroy()
    return {
        "workload": "chung-lu |U|=20,000,000 |L|=10,000,000 m=500,000,000 gamma=2.1/2.1 "
                    "cap=50,000; update stream 70% insertions / 30% deletions, "
                    "(alpha,beta) log-uniform in [2,64] (seed 1005), prefix of "
                    f"{total} requests",
        "requests": total,
        "sequential_queries_per_s": seq_qps,
        "sequential_p50_ms": _pct([t * 1e3 for t in t_seq], 50),
        "sequential_p99_ms": _pct([t * 1e3 for t in t_seq], 99),
        "served_closed_loop_queries_per_s": closed_qps,
        # the closed loop serves the first third of the stream: compared with
        # the sequential rate over the same requests
        "sequential_queries_per_s_same_requests": n_closed / sum(t_seq[:n_closed]),
        "speedup_vs_sequential": closed_qps / (n_closed / sum(t_seq[:n_closed])),
        "phases": phases,
        "device_slots": args.serve_slots,
        "max_inflight": args.serve_inflight,
        "windows": counters["windows"],
        "device_memory_library_peak_bytes_two_handles": peak,
        "stale_core_pruning": pruned,
        "answers_equal_sequential": mismatch == 0 and (pruned is None or
                                                        pruned["answers_equal_sequential"]),
        "mismatches": mismatch,
    }


def _golden(name: str):
    """Oracle digests of a large workload (tests/golden/<name>_oracle.json,
    written offline from the oracle alone), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def _gcc_bytes(n: int, q: dict) -> int:
    """Algorithmic bytes of one GCC query from the oracle's counts: deg0
    read and deg written (8 B per vertex), the bitmask (n/8), offsets and
    row of every removed vertex (16 B + 4 B per entry), one 4-byte
    read-modify-write atomic per peeled edge (8 B)."""
    return 8 * n + n // 8 + 16 * q["removed"] + 4 * q["removed_degree_sum"] + 8 * q["m_peeled"]


def _core_split(report) -> dict:
    """Where a core decomposition spent its time: the levels peeled before
    the switch to the h-index fixpoint, and that fixpoint (host wall clock
    of each phase, both zero when the levels finished the job alone)."""
    return {"levels_ms": report["core_levels_ms"], "hindex_ms": report["core_top_ms"],
            "hindex": report["core_top"]}


def _core_warm(pkg, torch, g):
    """The core decomposition again on the same handle (the switch option
    set to its default drops the cached numbers): the first call also pays
    for the first use of its temporaries' memory, this one does not."""
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pkg.abcore_core_numbers(g)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    return ms, _core_split(pkg.abcore_graph_report(g))


def _sha_words(t) -> str:
    import hashlib
    return hashlib.sha256(t.cpu().numpy().astype("<u4").tobytes()).hexdigest()


def bench_sweep(args, pkg, torch, np, bigraph_gen) -> dict:
    """The billion-edge GCC+ sweep: Chung-Lu |U|=50M |L|=20M m=10^9, degree
    exponents 2.0 / 2.3, cap 50k; core numbers once, then alpha = beta in
    {1, 2, 4, ..., 256} with GCC+ (each a pack of the core numbers) and, for
    comparison, with index-free GCC (each a full peel).  Every bitmask is
    compared with the oracle's digest; GCC's rate and roofline use the
    oracle's counts of each query."""
    spec = bigraph_gen.CONFIGS[3]
    nU, nL = spec["n_upper"], spec["n_lower"]
    n = nU + nL
    gold = _golden("c3")
    gq = {} if gold is None else {(q["alpha"], q["beta"]): q for q in gold["queries"]}
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    print(f"# sweep graph generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    m = len(eu)
    deu = torch.from_numpy(eu).cuda()
    dev = torch.from_numpy(ev).cuda()
    del eu, ev
    pkg.abcore_device_memory(reset_peak=True)
    g = pkg.abcore_build_csr(nU, nL, deu, dev)
    del deu, dev
    torch.cuda.empty_cache()
    report = pkg.abcore_graph_report(g)
    resident, _ = pkg.abcore_device_memory()
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, max_core = pkg.abcore_core_numbers(g)
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - t0) * 1e3
    split = _core_split(pkg.abcore_graph_report(g))
    warm_ms, warm_split = _core_warm(pkg, torch, g)
    out = torch.empty(g.nwords, dtype=torch.int32, device="cuda")
    ref = torch.empty(g.nwords, dtype=torch.int32, device="cuda")
    rows = []
    parity = True
    oracle_parity = gold is not None
    pack_bytes = 4 * n + n // 8
    for k in [1, 2, 4, 8, 16, 32, 64, 128, 256]:
        times = {}
        for algo, name in ((pkg.ABCORE_GCC, "gcc"), (pkg.ABCORE_GCC_PLUS, "gcc_plus")):
            dst = ref if algo == pkg.ABCORE_GCC else out
            pkg.abcore_compute(g, k, k, algo, out=dst)
            torch.cuda.synchronize()
            reps = 5
            t0 = time.perf_counter()
            for _ in range(reps):
                pkg.abcore_compute(g, k, k, algo, out=dst)
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) * 1e3 / reps
        parity = parity and bool(torch.equal(out, ref))
        row = {"alpha": k, "beta": k, "gcc_plus_ms": times["gcc_plus"],
               "gcc_plus_pack_frac": pack_bytes / (times["gcc_plus"] / 1e3) / 1e9 / HBM_PEAK_GBS,
               "gcc_ms": times["gcc"]}
        q = gq.get((k, k))
        if q is not None:
            B = _gcc_bytes(n, q)
            row.update(gcc_edges_peeled_per_s=q["m_peeled"] / (times["gcc"] / 1e3),
                       gcc_algorithmic_bytes=B,
                       gcc_frac=B / (times["gcc"] / 1e3) / 1e9 / HBM_PEAK_GBS)
            oracle_parity = oracle_parity and _sha_words(ref[: (n + 31) // 32]) == \
                q["bitmask_sha256"]
        rows.append(row)
    _, peak = pkg.abcore_device_memory()
    g.destroy()
    total_plus = sum(r["gcc_plus_ms"] for r in rows)
    return {
        "workload": "chung-lu |U|=50,000,000 |L|=20,000,000 m=1,000,000,000 "
                    "gamma=2.0/2.3 cap=50,000; alpha=beta in {1,2,4,...,256}",
        "m": m, "core_preprocessing_ms": prep_ms,
        "core_preprocessing_edges_per_s": m / (prep_ms / 1e3),
        "core_preprocessing_frac": (20 * n + 16 * m) / (prep_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "max_core": max_core, "core_split": split,
        "core_preprocessing_warm_ms": warm_ms, "core_split_warm": warm_split,
        "core_preprocessing_warm_frac":
            (20 * n + 16 * m) / (warm_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "queries": rows, "gcc_plus_total_ms": total_plus,
        "gcc_total_ms": sum(r["gcc_ms"] for r in rows),
        "gcc_plus_pack_bytes": pack_bytes,
        "parity_gcc_plus_vs_gcc": parity,
        "parity_vs_oracle_digests": oracle_parity,
        "build": report,
        "device_memory_library_peak_bytes": peak,
        "device_memory_library_resident_after_build_bytes": resident,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate CPU time spent on the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--peel-mode", type=int, default=0)
    ap.add_argument("--gcc-only", action="store_true",
                    help="skip GCC+ and its core-number preprocessing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-query section")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the billion-edge GCC+ sweep section")
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-inflight", type=int, default=64)
    ap.add_argument("--serve-prune", type=int, default=256,
                    help="ABCORE_OPT_SERVE_PRUNE of a third, pruned served run (0 = none)")
    ap.add_argument("--serve-pull", type=int, default=0,
                    help="ABCORE_OPT_PULL of the served handle (0 = default)")
    ap.add_argument("--step-mode", choices=["both", "index_free", "rank_order"], default="both",
                    help="GCC step variants to run (one alone for per-kernel hardware counters)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device copy of MIB MiB (hardware-counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design notes); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import bigraph_gen
    import paper_2606_07148_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    pkg.load()

    spec = bigraph_gen.CONFIGS[2]
    alpha = beta = 10
    nU, nL = spec["n_upper"], spec["n_lower"]
    n = nU + nL
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    gen_s = time.perf_counter() - t0
    print(f"# generated {len(eu)} edges in {gen_s:.1f}s", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # give the scale between counted and moved bytes
        words = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(words, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    deu = torch.from_numpy(eu).cuda()
    dev = torch.from_numpy(ev).cuda()
    torch.cuda.synchronize()
    pkg.abcore_device_memory(reset_peak=True)
    t0 = time.perf_counter()
    g = pkg.abcore_build_csr(nU, nL, deu, dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    resident_c2, _ = pkg.abcore_device_memory()
    del deu, dev
    if args.peel_mode:
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, args.peel_mode)

    # --- oracle: numerators of the metric and the CPU baseline ------------
    import oracle
    ref = oracle.Graph(nU, nL, eu, ev)
    deg = ref.degrees()
    reps, cpu_t = 0, 0.0
    stats_o = None
    member = None
    while True:
        t0 = time.perf_counter()
        member, stats_o = oracle.peel(ref, alpha, beta)
        cpu_t += time.perf_counter() - t0
        reps += 1
        if args.no_cpu_baseline or cpu_t >= args.cpu_seconds:
            break
    m_peeled = stats_o["m_peeled"]
    removed = stats_o["removed"]
    sum_deg_removed = stats_o["removed_degree_sum"]
    want = oracle.pack(member)

    # --- GPU: GCC steps ---------------------------------------------------
    # Algorithmic bytes of one GCC query, from the oracle's counts alone
    # (independent of the implementation): deg0 read and deg written (8 B
    # per vertex), the bitmask (n/8), offsets and row of every removed
    # vertex (16 B + 4 B per entry), one 4-byte read-modify-write atomic per
    # peeled edge (8 B).
    B = 8 * n + n // 8 + 16 * removed + 4 * sum_deg_removed + 8 * m_peeled
    out = torch.empty(max(1, g.nwords), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    flush = torch.empty(1 << 28, dtype=torch.int32, device="cuda")  # 1 GiB

    def run_steps(rank_mode: int, cold: bool = False, steps: int = args.steps) -> dict:
        """Warm-up, parity, then `steps` wall-clock-timed steps and `steps`
        steps each bracketed by a HIP event pair on the kernels' stream; a
        cold step first writes 1 GiB (evicting L2 and the 256 MB Infinity
        Cache) outside its events."""
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, rank_mode)
        for _ in range(args.warmup):
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
        torch.cuda.synchronize()
        ok = bool(np.array_equal(out.cpu().numpy().view(np.uint32)[: len(want)], want))
        _, st = pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out, stats=True)
        torch.cuda.synchronize()
        wall = None
        if not cold:
            t0 = time.perf_counter()
            for _ in range(steps):
                pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3 / steps
        evs = []
        for k in range(steps):
            if cold:
                flush.fill_(k)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ok = ok and bool(np.array_equal(out.cpu().numpy().view(np.uint32)[: len(want)], want))
        durs = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
        ev_ms = float(durs.mean())
        return {"ms_per_step": wall, "event_ms_mean": ev_ms,
                "event_ms_p50": float(np.percentile(durs, 50)),
                "event_ms_p90": float(np.percentile(durs, 90)),
                "algorithmic_GBs": B / (ev_ms / 1e3) / 1e9,
                "frac": B / (ev_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                "parity": ok, "stats": st}

    def kernel_split(rank_mode: int) -> dict:
        """Per-kernel device time of the step (an event pair around every
        launch, recorded by the library on the launch stream)."""
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, rank_mode)
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_TIMING, 1)
        for kind in range(5):
            pkg.abcore_kernel_timing(g, kind, reset=True)
        for _ in range(args.steps):
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
        torch.cuda.synchronize()
        kt = {kind: pkg.abcore_kernel_timing(g, kind, reset=True) for kind in range(5)}
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_TIMING, 0)
        names = {0: "peel", 1: "pull", 2: "scan", 3: "pack", 4: "fixup"}
        return {names[k]: {"avg_launch_us": ms * 1e3 / cnt, "launches_per_step": cnt / args.steps}
                for k, (ms, cnt) in kt.items() if cnt > 0}

    modes = {"index_free": 2, "rank_order": 1}
    runs = {}
    for name, mode in modes.items():
        if args.step_mode not in ("both", name):
            continue
        runs[name] = run_steps(mode)
        runs[name]["kernels"] = kernel_split(mode)
        if args.step_mode == "both":
            runs[name + "_cold"] = run_steps(mode, cold=True)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, 2)
    parity = all(r["parity"] for r in runs.values())
    # the headline is the index-free step (Algorithm 1 on the CSR alone)
    free = runs.get("index_free") or runs["rank_order"]
    ranked = runs.get("rank_order")
    free_cold = runs.get("index_free_cold")
    ranked_cold = runs.get("rank_order_cold")
    gst = free["stats"]
    ms_per_step = free["ms_per_step"]
    value = m_peeled / (ms_per_step / 1e3)
    report = pkg.abcore_graph_report(g)
    traffic = _counter_traffic_step("index_free" if "index_free" in runs else "rank_order")
    ranked_traffic = _counter_traffic_step("rank_order")

    # --- GCC+ (Algorithm 2): preprocessing + query ------------------------
    gcc_plus = None
    plus_parity = True
    if not args.gcc_only:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, max_core = pkg.abcore_core_numbers(g)
        torch.cuda.synchronize()
        prep_ms = (time.perf_counter() - t0) * 1e3
        split = _core_split(pkg.abcore_graph_report(g))
        warm_ms, warm_split = _core_warm(pkg, torch, g)
        for _ in range(args.warmup):
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC_PLUS, out=out)
        torch.cuda.synchronize()
        plus_parity = bool(np.array_equal(out.cpu().numpy().view(np.uint32)[: len(want)], want))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC_PLUS, out=out)
        torch.cuda.synchronize()
        plus_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        # alpha = beta: Lemma 1 leaves no uncertain vertex, so the query is a
        # pack of the cached core numbers (4 B read per vertex, n/8 written)
        pack_bytes = 4 * n + n // 8
        gcc_plus = {"ms_per_query": plus_ms, "parity": plus_parity,
                    "query_is_pack_of_core_numbers": True,
                    "pack_GBs": pack_bytes / (plus_ms / 1e3) / 1e9,
                    "pack_frac": pack_bytes / (plus_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                    "core_preprocessing_ms": prep_ms, "max_core": max_core,
                    "core_split": split,
                    "core_preprocessing_warm_ms": warm_ms, "core_split_warm": warm_split,
                    "edges_peeled_per_s_incl_preprocessing":
                        m_peeled / ((prep_ms + plus_ms) / 1e3)}
        # Algorithm 2 with alpha != beta (uncertain vertices are peeled),
        # against GCC on the same pairs; both results must agree bit for bit
        asym = []
        for (pa, pb) in ((5, 20), (40, 8)):
            row = {"alpha": pa, "beta": pb}
            res = {}
            for name, algo in (("gcc", pkg.ABCORE_GCC), ("gcc_plus", pkg.ABCORE_GCC_PLUS)):
                for _ in range(args.warmup):
                    pkg.abcore_compute(g, pa, pb, algo, out=out)
                torch.cuda.synchronize()
                res[name] = out.clone()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    pkg.abcore_compute(g, pa, pb, algo, out=out)
                torch.cuda.synchronize()
                row[name + "_ms"] = (time.perf_counter() - t0) * 1e3 / args.steps
            row["equal"] = bool(torch.equal(res["gcc"], res["gcc_plus"]))
            plus_parity = plus_parity and row["equal"]
            asym.append(row)
        gcc_plus["asymmetric_index_free"] = asym
    _, peak_c2 = pkg.abcore_device_memory()
    c2_torch_peak = torch.cuda.max_memory_allocated()
    del flush
    torch.cuda.empty_cache()

    batch = None
    if not args.no_batch:
        batch = bench_batch(args, pkg, torch, np, bigraph_gen)

    serve = None
    if not args.no_serve:
        serve = bench_serve(args, pkg, torch, np, bigraph_gen)
    sweep = None
    if not args.no_sweep:
        sweep = bench_sweep(args, pkg, torch, np, bigraph_gen)

    result = {
        "metric": "edges peeled/sec",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic: seeded Chung-Lu bipartite graph (bigraph_gen config 2)",
        "config": {
            "workload": "chung-lu |U|=1,000,000 |L|=500,000 m=20,000,000 gamma=2.1/2.1 "
                        "cap=50,000; (alpha,beta)=(10,10); GCC, index-free (vertex order, "
                        "CSR only)",
            "n_upper": nU, "n_lower": nL, "m": int(ref.m), "alpha": alpha, "beta": beta,
            "algo": "GCC", "seed": spec["seed"],
            "edge_sha256": bigraph_gen.edge_hash(eu, ev),
        },
        "roofline": {
            "bound": "hbm",
            "scope": "one GCC query (scan, pull round, asynchronous peel)",
            "achieved": free["algorithmic_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": free["frac"],
            "traffic": None if traffic is None else traffic["bytes"],
            "algorithmic_bytes": B,
            "step_event_us": free["event_ms_mean"] * 1e3,
            "traffic_ratio": None if traffic is None else traffic["bytes"] / B,
        },
        "index_free": {k: v for k, v in free.items() if k != "stats"},
        "rank_order": None if ranked is None else dict(
            {k: v for k, v in ranked.items() if k != "stats"},
            preprocessing_ms=report["ranks_ms"], extra_device_bytes=report["ranks_bytes"],
            traffic=None if ranked_traffic is None else ranked_traffic["bytes"],
            edges_peeled_per_s=m_peeled / (ranked["ms_per_step"] / 1e3)),
        "cold_cache": None if free_cold is None else {
            "index_free": {k: v for k, v in free_cold.items() if k not in ("stats", "ms_per_step")},
            "rank_order": {k: v for k, v in ranked_cold.items()
                           if k not in ("stats", "ms_per_step")},
            "flush": "1 GiB written before each step, outside its events"},
        "build": report,
        "device_memory": {"library_peak_bytes": peak_c2,
                          "library_resident_after_build_bytes": resident_c2,
                          "torch_peak_bytes": c2_torch_peak},
        "gpu_stats": gst,
        "parity": parity,
        "m_peeled": m_peeled,
        "removed": removed,
        "removed_degree_sum": sum_deg_removed,
        "rounds": stats_o["rounds"],
        "input_edges_per_s": ref.m / (ms_per_step / 1e3),
        "gcc_plus": gcc_plus,
        "batch": batch,
        "serve": serve,
        "sweep": sweep,
        "build_s": build_s,
    }
    if not args.no_cpu_baseline:
        # the same query on every host thread (multithreaded CPU peel)
        import cpu_peel
        threads = cpu_peel.max_threads()
        preps, pt, par_ok = 0, 0.0, True
        while preps < 3 or pt < args.cpu_seconds / 2:
            t0 = time.perf_counter()
            pm, _ = cpu_peel.peel(nU, nL, ref.off, ref.cols, alpha, beta, threads)
            pt += time.perf_counter() - t0
            preps += 1
            par_ok = par_ok and bool(np.array_equal(pm, member))
        pper = pt / preps
        result["cpu_parallel"] = {
            "value": m_peeled / pper, "unit": "edges/s", "cores": threads,
            "kind": "multithreaded CPU peel (OpenMP rounds, atomic decrements)",
            "sample": f"{preps} peels of the full config-2 graph at (10,10), "
                      f"{pper * 1e3:.2f} ms each on {threads} threads (CSR build excluded)",
            "parity_vs_oracle": par_ok}
        per = cpu_t / reps
        result["cpu_baseline"] = {
            "value": m_peeled / per, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} single-threaded oracle peels of the full config-2 graph at "
                      f"(10,10), {per * 1e3:.1f} ms each (CSR build excluded)",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(),
        }
    print(json.dumps(result), flush=True)
    g.destroy()
    ok = (parity and plus_parity and result.get("cpu_parallel", {}).get("parity_vs_oracle", True)
          and (batch is None or batch["parity_vs_sequential"])
          and (batch is None or batch.get("parity_vs_oracle_digests", True))
          and (serve is None or serve["answers_equal_sequential"])
          and (sweep is None or (sweep["parity_gcc_plus_vs_gcc"]
                                 and sweep["parity_vs_oracle_digests"])))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
