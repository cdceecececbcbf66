"""Writes the oracle's digests of the two largest workloads, for the GPU tests
that run them at full size.  Calls only ``bigraph_gen`` (the seeded inputs)
and ``oracle`` (the sequential CPU oracle); nothing here touches the device
library.  Run on a CPU host with about 48 GB of memory:

    python tests/golden/make_large_golden.py c3   # -> c3_oracle.json
    python tests/golden/make_large_golden.py c4   # -> c4_oracle.json
    python tests/golden/make_large_golden.py c5   # -> c5_oracle.json

c3: Chung-Lu |U| = 5e7, |L| = 2e7, m = 1e9, degree exponents 2.0 / 2.3,
    cap 50,000 (seed 3).  Digests: the edge list, the CSR (Sec. III storage,
    unified ids of Sec. IV-A), the core numbers (Definition 2) and, for the
    GCC+ sweep alpha = beta in {1, 2, ..., 256} and three asymmetric pairs,
    the (alpha,beta)-core's bitmask (Definition 1) with the peel's counts.
c4: Chung-Lu |U| = 1e7, |L| = 5e6, m = 2e8, exponent 2.1, cap 50,000 (seed 4)
    and its 256 queries, log-uniform in [1,256]^2 (seed 1004): each query's
    bitmask digest and peel counts.
c5: Chung-Lu |U| = 2e7, |L| = 1e7, m = 5e8, exponent 2.1, cap 50,000
    (seed 5) and its update stream (seed 1005).  Answers of sampled updates
    of a prefix (Problem 2 of Sec. III, by recomputation on the updated
    graph as Sec. V requires), and the digest of the graph after the prefix.

Digests are SHA-256 of little-endian arrays: the edge list as interleaved
int32 (u, v) pairs sorted by (u, v); ``off`` as int64; ``cols`` as int32;
core numbers as int32; bitmasks as uint32 words (bit x % 32 of word x // 32).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import bigraph_gen  # noqa: E402
import oracle  # noqa: E402
from tests.digests import sha_array, sha_edges  # noqa: E402

C3_SWEEP = [1, 2, 4, 8, 16, 32, 64, 128, 256]
C3_ASYM = [(3, 17), (40, 6), (100, 2)]
C5_PREFIX = 2000
C5_SAMPLES = [0, 1, 2, 3, 7, 50, 199, 400, 777, 1000, 1333, 1666, 1999]


def log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def query_record(g, a, b):
    member, st = oracle.peel(g, a, b)
    bits = oracle.pack(member)
    return dict(alpha=a, beta=b, members=int(member.sum()), bitmask_sha256=sha_array(bits, "<u4"),
                removed=st["removed"], removed_degree_sum=st["removed_degree_sum"],
                m_peeled=st["m_peeled"], rounds=st["rounds"])


def c3():
    spec = bigraph_gen.CONFIGS[3]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.time()
    eu, ev = bigraph_gen.make_graph(spec)
    log(f"c3: generated {len(eu)} edges in {time.time() - t0:.0f}s")
    out = dict(config=3, spec={k: spec[k] for k in spec}, n_upper=nU, n_lower=nL)
    out["edge_sha256"] = sha_edges(eu, ev)
    log("c3: edge digest done")
    g = oracle.Graph(nU, nL, eu, ev)
    del eu, ev
    log(f"c3: oracle CSR, m = {g.m}")
    out["m"] = g.m
    out["off_sha256"] = sha_array(g.off, "<i8")
    out["cols_sha256"] = sha_array(g.cols, "<i4")
    deg = np.diff(g.off)
    out["max_degree_upper"] = int(deg[:nU].max())
    out["max_degree_lower"] = int(deg[nU:].max())
    out["isolated"] = int((deg == 0).sum())
    del deg
    log("c3: CSR digests done")
    t0 = time.time()
    core = oracle.core_numbers(g)
    out["core_seconds"] = round(time.time() - t0, 1)
    out["core_sha256"] = sha_array(core, "<i4")
    out["max_core"] = int(core.max())
    out["core_at_least"] = {str(k): int((core >= k).sum()) for k in C3_SWEEP}
    del core
    log(f"c3: core numbers, max {out['max_core']}")
    out["queries"] = []
    for k in C3_SWEEP:
        out["queries"].append(query_record(g, k, k))
        log(f"c3: ({k},{k}) members {out['queries'][-1]['members']}")
    for a, b in C3_ASYM:
        out["queries"].append(query_record(g, a, b))
        log(f"c3: ({a},{b}) members {out['queries'][-1]['members']}")
    path = os.path.join(HERE, "c3_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log("wrote", path)


def c4():
    spec = bigraph_gen.CONFIGS[4]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.time()
    eu, ev = bigraph_gen.make_graph(spec)
    log(f"c4: generated {len(eu)} edges in {time.time() - t0:.0f}s")
    a, b = bigraph_gen.loguniform_pairs(256, 1, 256, spec["seed"] + 1000)
    out = dict(config=4, spec={k: spec[k] for k in spec}, n_upper=nU, n_lower=nL,
               query_seed=spec["seed"] + 1000)
    out["edge_sha256"] = sha_edges(eu, ev)
    g = oracle.Graph(nU, nL, eu, ev)
    del eu, ev
    out["m"] = g.m
    out["off_sha256"] = sha_array(g.off, "<i8")
    out["cols_sha256"] = sha_array(g.cols, "<i4")
    out["queries"] = []
    for i, (x, y) in enumerate(zip(a.tolist(), b.tolist())):
        out["queries"].append(query_record(g, int(x), int(y)))
        if i % 32 == 31:
            log(f"c4: {i + 1} queries")
    path = os.path.join(HERE, "c4_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log("wrote", path)


def c5():
    spec = bigraph_gen.CONFIGS[5]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.time()
    eu, ev = bigraph_gen.make_graph(spec)
    log(f"c5: generated {len(eu)} edges in {time.time() - t0:.0f}s")
    upd = bigraph_gen.update_stream(spec, eu, ev, C5_PREFIX, spec["seed"] + 1000)
    out = dict(config=5, spec={k: spec[k] for k in spec}, n_upper=nU, n_lower=nL,
               prefix=C5_PREFIX, stream_seed=spec["seed"] + 1000)
    out["edge_sha256"] = sha_edges(eu, ev)
    h = hashlib.sha256()
    for k in ("u", "v", "op", "alpha", "beta"):
        h.update(np.ascontiguousarray(upd[k], "<i4").tobytes())
    out["stream_sha256"] = h.hexdigest()
    last = max(C5_SAMPLES)

    def on_graph(i, g):
        if i == last:
            out["final_m"] = g.m
            out["final_off_sha256"] = sha_array(g.off, "<i8")
            out["final_cols_sha256"] = sha_array(g.cols, "<i4")
        log(f"c5: update {i} answered (m = {g.m})")

    res = oracle.gfq_stream_sampled(nU, nL, eu, ev, upd, C5_SAMPLES, on_graph=on_graph)
    out["samples"] = [dict(index=i, u=int(upd["u"][i]), v=int(upd["v"][i]), op=int(upd["op"][i]),
                           alpha=int(upd["alpha"][i]), beta=int(upd["beta"][i]),
                           status=res[i][0], answer=res[i][1], bits=res[i][2])
                      for i in C5_SAMPLES]
    path = os.path.join(HERE, "c5_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log("wrote", path)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c4", "c5"]
    for w in which:
        {"c3": c3, "c4": c4, "c5": c5}[w]()
