#!/usr/bin/env python3
"""Benchmark: (alpha,beta)-core peeling on one MI355X.

Workload: seeded Chung-Lu bipartite graph with |U| = 1,000,000,
|L| = 500,000, 20,000,000 distinct edges, degree-distribution exponent 2.1 on
both layers, expected degrees capped at 50,000; query (alpha,beta) = (10,10).
One step = one GCC query (Algorithm 1: scan, peel rounds, bitmask pack) on
the resident graph.  GCC+ (Algorithm 2) on the same query and its core-number
preprocessing are timed separately and reported as extra fields, like the
paper's Table II separates preprocessing from query time.

Metric: edges peeled per second = (m - |E(core)|) / step time, with the
numerator taken from the CPU oracle so it does not depend on the GPU code.
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


def _kernel_source_hash() -> str:
    """SHA-256 over the kernel sources, sorted by name (name, then content)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_2606_07148_amd", "csrc", "*"))):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed hardware-counter
    summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "gcc_chung_lu_1M_500k_20M_a10_b10.md")
    try:
        text = open(path).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != _kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes"]


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
    for _ in range(2):
        deu = torch.from_numpy(eu).cuda()
        dev = torch.from_numpy(ev).cuda()
        handles.append(pkg.abcore_build_csr(nU, nL, deu, dev))
        del deu, dev
    del eu, ev
    torch.cuda.empty_cache()
    g_seq, g_srv = handles
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
    counters = pkg.abcore_serve_stop(g_srv)
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
        "speedup_vs_sequential": closed_qps / seq_qps,
        "phases": phases,
        "device_slots": args.serve_slots,
        "max_inflight": args.serve_inflight,
        "windows": counters["windows"],
        "answers_equal_sequential": mismatch == 0,
        "mismatches": mismatch,
    }


def bench_sweep(args, pkg, torch, np, bigraph_gen) -> dict:
    """The billion-edge GCC+ sweep: Chung-Lu |U|=50M |L|=20M m=10^9, degree
    exponents 2.0 / 2.3, cap 50k; core numbers once, then alpha = beta in
    {1, 2, 4, ..., 256} with GCC+ (each a scan of the core numbers) and, for
    comparison, with GCC.  Results compared bit for bit."""
    spec = bigraph_gen.CONFIGS[3]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    print(f"# sweep graph generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    m = len(eu)
    deu = torch.from_numpy(eu).cuda()
    dev = torch.from_numpy(ev).cuda()
    del eu, ev
    g = pkg.abcore_build_csr(nU, nL, deu, dev)
    del deu, dev
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, max_core = pkg.abcore_core_numbers(g)
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty(g.nwords, dtype=torch.int32, device="cuda")
    ref = torch.empty(g.nwords, dtype=torch.int32, device="cuda")
    rows = []
    parity = True
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
        rows.append({"alpha": k, "beta": k, "gcc_plus_ms": times["gcc_plus"],
                     "gcc_ms": times["gcc"]})
    g.destroy()
    total_plus = sum(r["gcc_plus_ms"] for r in rows)
    return {
        "workload": "chung-lu |U|=50,000,000 |L|=20,000,000 m=1,000,000,000 "
                    "gamma=2.0/2.3 cap=50,000; alpha=beta in {1,2,4,...,256}",
        "m": m, "core_preprocessing_ms": prep_ms, "max_core": max_core,
        "queries": rows, "gcc_plus_total_ms": total_plus,
        "gcc_total_ms": sum(r["gcc_ms"] for r in rows),
        "gcc_plus_input_edges_per_s": m * len(rows) / (total_plus / 1e3),
        "parity_gcc_plus_vs_gcc": parity,
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
    ap.add_argument("--serve-pull", type=int, default=0,
                    help="ABCORE_OPT_PULL of the served handle (0 = default)")
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
    t0 = time.perf_counter()
    g = pkg.abcore_build_csr(nU, nL, deu, dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
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

    # --- GPU: GCC timed region -------------------------------------------
    out = torch.empty(max(1, g.nwords), dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)[: len(want)]
    parity = bool(np.array_equal(got, want))
    _, gst = pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out, stats=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    # per-kernel durations: the same steps again with an event pair around
    # every launch, on the stream the kernels run on
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_TIMING, 1)
    for kind in range(5):
        pkg.abcore_kernel_timing(g, kind, reset=True)
    for _ in range(args.steps):
        pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC, out=out)
    torch.cuda.synchronize()
    ktime = {kind: pkg.abcore_kernel_timing(g, kind, reset=True) for kind in range(5)}
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_TIMING, 0)
    value = m_peeled / (ms_per_step / 1e3)

    # algorithmic bytes per query of each kernel, from the oracle's sets:
    # F0 = scan frontier, A1 = its complement, R = removed vertices
    thr = np.where(np.arange(n) < nU, alpha, beta)
    f0 = deg < thr
    removed_mask = ~member
    lower = nU + ev.astype(np.int64)
    upper = eu.astype(np.int64)
    pulled = bool(gst["pulled"])
    if pulled:
        a1 = ~f0
        r2 = removed_mask & a1
        touch_r2 = r2[upper] | r2[lower]
        touch_f0 = f0[upper] | f0[lower]
        m2 = int(np.count_nonzero(touch_r2 & ~touch_f0))
        push_bytes = 16 * int(r2.sum()) + 4 * int(deg[r2].sum()) + 8 * m2
        pull_bytes = 20 * int(a1.sum()) + 4 * int(deg[a1].sum()) + n // 8
    else:
        push_bytes = 16 * removed + 4 * sum_deg_removed + 8 * m_peeled
        pull_bytes = 0
    # the asynchronous mode scans and resets the workspace in one kernel
    # that does not queue the frontier: it returns the previous query's
    # queued items to empty, and a pushed first round queues the frontier
    # from the bitmap in the pull kernel instead
    fused_scan = args.peel_mode in (0, 3)
    rank_order = bool(gst.get("rank_order", 0))
    n_f0 = int(f0.sum())
    if rank_order:
        # the query runs on the degree-rank relabelling, without a scan
        # launch: the pull round reads a light row's offsets (8 B) and
        # entries and writes its degree (4 B), searches a split row, and
        # writes the survivor bitmap into the result (deg0 read, n/8
        # written); the peel maps each survivor it removes to its vertex
        # (4 B) and clears its bit in the result (an 8 B read-modify-write),
        # so no pack pass follows, and after termination returns its queued
        # items to empty (4 B each) and zeroes the next query's 4096 x 10
        # partial sums
        a1 = ~f0
        light = a1 & (deg <= 64)
        heavy = a1 & (deg > 64)
        r2n = removed - n_f0
        scan_bytes = 0
        pull_bytes = (12 * int(light.sum()) + 4 * int(deg[light].sum())
                      + (24 + 4 * 16 * 4) * int(heavy.sum()) + 4 * n + n // 8)
    elif fused_scan:
        queued = removed - n_f0 if pulled else removed
        scan_bytes = 8 * n + n // 8 + 4 * queued
        if not pulled:
            pull_bytes = n // 8 + 4 * n_f0
        else:
            # on an unchanged graph the pull round counts on the degree-rank
            # copy: a row of at most 64 entries is read whole, a split row is
            # searched (16 probes of 4 B in about four steps) and completed
            # at once; the survivor bits are read, no bitmap is staged
            light = a1 & (deg <= 64)
            heavy = a1 & (deg > 64)
            pull_bytes = (20 * int(light.sum()) + 4 * int(deg[light].sum())
                          + (24 + 4 * 16 * 4) * int(heavy.sum()) + n // 8)
    else:
        scan_bytes = 8 * n + 4 * n_f0 + (n // 8 if pulled else 0)
    pack_bytes = (12 * (removed - n_f0) + 4 * (removed - n_f0) + 8 * 4096 * 10 if rank_order
                  else 4 * n + n // 8)
    kinfo = {}
    peel_name = {1: "peel_round_kernel<0>", 2: "peel_persistent_kernel<0>"}.get(
        args.peel_mode, "peel_async_kernel<0>")  # <0> = the GCC instantiation
    # the degree-rank pull round stages no bitmap: the kLds = false build
    names = {0: peel_name, 1: "pull_round_kernel<false>" if (fused_scan and pulled)
             else "pull_round_kernel<true>",
             2: "scan_reset_gcc_kernel" if fused_scan else "scan_gcc_kernel", 3: "pack_kernel",
             4: "pull_fixup_kernel"}
    # fixup: split rows (more than 64 entries): row id, deg0 and deg read
    # (none after a degree-rank pull round, which completes them itself)
    fixup_bytes = 12 * int(np.count_nonzero(deg > 64)) if pulled and not fused_scan else 0
    kbytes = {0: push_bytes, 1: pull_bytes, 2: scan_bytes, 3: pack_bytes, 4: fixup_bytes}
    # the asynchronous peel runs the pack and the pull round's completion
    # itself (no separate launches): its bytes include theirs
    if ktime[3][1] == 0:
        kbytes[0] += pack_bytes
    if ktime[4][1] == 0:
        kbytes[0] += fixup_bytes
    for kind, (ms, launches) in ktime.items():
        if launches == 0:
            continue
        per_launch_s = ms / 1e3 / launches
        bpl = kbytes[kind] * args.steps / launches
        kinfo[names[kind]] = {"avg_launch_us": per_launch_s * 1e6, "launches_per_step":
                              launches / args.steps, "bytes_per_launch": bpl,
                              "achieved_GBs": bpl / per_launch_s / 1e9 if per_launch_s > 0 else 0}
    dom = max(kinfo, key=lambda k: kinfo[k]["avg_launch_us"] * kinfo[k]["launches_per_step"])
    step_bytes = scan_bytes + pull_bytes + push_bytes + pack_bytes + fixup_bytes

    # --- GCC+ (Algorithm 2): preprocessing + query ------------------------
    gcc_plus = None
    plus_parity = True
    if not args.gcc_only:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, max_core = pkg.abcore_core_numbers(g)
        torch.cuda.synchronize()
        prep_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC_PLUS, out=out)
        torch.cuda.synchronize()
        plus_parity = bool(np.array_equal(out.cpu().numpy().view(np.uint32)[: len(want)], want))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pkg.abcore_compute(g, alpha, beta, pkg.ABCORE_GCC_PLUS, out=out)
        torch.cuda.synchronize()
        plus_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        gcc_plus = {"ms_per_query": plus_ms, "parity": plus_parity,
                    "edges_peeled_per_s": m_peeled / (plus_ms / 1e3),
                    "core_preprocessing_ms": prep_ms, "max_core": max_core}
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
        gcc_plus["asymmetric"] = asym

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
                        "cap=50,000; (alpha,beta)=(10,10); GCC",
            "n_upper": nU, "n_lower": nL, "m": int(ref.m), "alpha": alpha, "beta": beta,
            "algo": "GCC", "seed": spec["seed"],
            "edge_sha256": bigraph_gen.edge_hash(eu, ev),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": kinfo[dom]["achieved_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": kinfo[dom]["achieved_GBs"] / HBM_PEAK_GBS,
            "traffic": _counter_traffic(dom),
            "bytes_per_launch": kinfo[dom]["bytes_per_launch"],
            "avg_launch_us": kinfo[dom]["avg_launch_us"],
        },
        "kernels": kinfo,
        "gpu_stats": gst,
        "parity": parity,
        "m_peeled": m_peeled,
        "removed": removed,
        "rounds": stats_o["rounds"],
        "step_algorithmic_bytes": step_bytes,
        "step_gbs": step_bytes / (ms_per_step / 1e3) / 1e9,
        "input_edges_per_s": ref.m / (ms_per_step / 1e3),
        "gcc_plus": gcc_plus,
        "batch": batch,
        "serve": serve,
        "sweep": sweep,
        "build_s": build_s,
    }
    if not args.no_cpu_baseline:
        per = cpu_t / reps
        result["cpu_baseline"] = {
            "value": m_peeled / per, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} single-threaded oracle peels of the full config-2 graph at "
                      f"(10,10), {per * 1e3:.1f} ms each (CSR build excluded)",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(),
        }
    print(json.dumps(result), flush=True)
    g.destroy()
    ok = (parity and plus_parity and (batch is None or batch["parity_vs_sequential"])
          and (serve is None or serve["answers_equal_sequential"])
          and (sweep is None or sweep["parity_gcc_plus_vs_gcc"]))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
