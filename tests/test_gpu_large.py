"""The billion-edge workload: Chung-Lu |U| = 50M, |L| = 20M, 10^9 edges,
degree exponents 2.0 / 2.3, expected degrees capped at 50,000; the GCC+
sweep alpha = beta in {1, 2, 4, ..., 256} and three asymmetric queries.

At full size the device results are compared with the oracle's digests in
``tests/golden/c3_oracle.json`` (written offline by
``tests/golden/make_large_golden.py`` from the oracle alone): the edge
list, the CSR the device built (Sec. III storage, unified ids of Sec.
IV-A), the core numbers (Definition 2) and every query's bitmask
(Definition 1), for GCC (Algorithm 1) and GCC+ (Algorithm 2).  A 1/50-scale
graph with the same exponents is compared element by element with the
oracle run live."""
import json
import os
import time

import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.digests import sha_array, sha_edges
from tests.gpu_util import bits_np, ensure_built, say, serve_all, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle.json")


def test_billion_edge_graph_matches_oracle_digests():
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    gold = json.load(open(GOLDEN))
    spec = bigraph_gen.CONFIGS[3]
    nU, nL = spec["n_upper"], spec["n_lower"]
    n = nU + nL
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    say(f"large: generated {len(eu)} edges in {time.perf_counter() - t0:.1f}s")
    assert sha_edges(eu, ev) == gold["edge_sha256"], "the generated edge list differs"
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    del eu, ev
    torch.cuda.empty_cache()
    assert g.m == gold["m"]
    off, cols = pkg.abcore_export_csr(g)
    torch.cuda.synchronize()
    assert sha_array(off.cpu().numpy(), "<i8") == gold["off_sha256"], "CSR offsets differ"
    del off
    assert sha_array(cols.cpu().numpy(), "<i4") == gold["cols_sha256"], "CSR columns differ"
    del cols
    torch.cuda.empty_cache()
    say("large: CSR equals the oracle's")
    core, max_core = pkg.abcore_core_numbers(g)
    assert max_core == gold["max_core"]
    assert sha_array(core.cpu().numpy(), "<i4") == gold["core_sha256"], "core numbers differ"
    for k, cnt in gold["core_at_least"].items():
        assert int((core >= int(k)).sum()) == cnt
    say(f"large: core numbers equal the oracle's (max {max_core})")
    for q in gold["queries"]:
        a, b = q["alpha"], q["beta"]
        for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
            bits, st = pkg.abcore_compute(g, a, b, algo, stats=True)
            words = bits_np(bits)[: (n + 31) // 32]
            assert sha_array(words, "<u4") == q["bitmask_sha256"], (a, b, algo)
            assert st["removed"] == q["removed"], (a, b, algo)
        say(f"large: ({a},{b}) equals the oracle ({q['members']} members)")
    g.destroy()


def test_billion_edge_shape_at_one_fiftieth_elementwise():
    """Same exponents and cap at 1/50 scale (|U| = 1M, |L| = 400k, m = 20M):
    every bitmask word and every core number equals the oracle's."""
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    spec = bigraph_gen.scaled(3, 1 / 50)
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ref = oracle.Graph(nU, nL, eu, ev)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    core, _ = pkg.abcore_core_numbers(g)
    assert np.array_equal(core.cpu().numpy(), oracle.core_numbers(ref))
    for (a, b) in [(k, k) for k in (1, 2, 4, 8, 16, 32, 64, 128, 256)] + \
            [(3, 17), (40, 6), (100, 2)]:
        want = oracle.pack(oracle.compute(ref, a, b))
        for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
            got = bits_np(pkg.abcore_compute(g, a, b, algo))[: len(want)]
            assert np.array_equal(got, want), (a, b, algo)
    say("large/50: all queries and core numbers equal the oracle's")
    g.destroy()


GOLDEN5 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle.json")


def test_update_stream_at_full_size_matches_oracle_samples():
    """The 5e8-edge serving workload (Chung-Lu |U| = 20M, |L| = 10M, exponent
    2.1) and a prefix of its update stream, one request at a time
    (abcore_query) and through the serving engine: at the sampled indices
    both answers equal the oracle's recomputation on the updated graph
    (Problem 2 of Sec. III, Sec. V), every served result equals the
    sequential one, and the graph after the prefix equals the oracle's."""
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    gold = json.load(open(GOLDEN5))
    spec = bigraph_gen.CONFIGS[5]
    nU, nL = spec["n_upper"], spec["n_lower"]
    t0 = time.perf_counter()
    eu, ev = bigraph_gen.make_graph(spec)
    say(f"c5: generated {len(eu)} edges in {time.perf_counter() - t0:.1f}s")
    assert sha_edges(eu, ev) == gold["edge_sha256"]
    ups = bigraph_gen.update_stream(spec, eu, ev, gold["prefix"], gold["stream_seed"])
    import hashlib
    h = hashlib.sha256()
    for k in ("u", "v", "op", "alpha", "beta"):
        h.update(np.ascontiguousarray(ups[k], "<i4").tobytes())
    assert h.hexdigest() == gold["stream_sha256"]
    samples = {s["index"]: s for s in gold["samples"]}

    def final_graph_matches(g):
        off, cols = pkg.abcore_export_csr(g)
        torch.cuda.synchronize()
        assert cols.numel() == 2 * gold["final_m"]
        assert sha_array(off.cpu().numpy(), "<i8") == gold["final_off_sha256"]
        assert sha_array(cols.cpu().numpy(), "<i4") == gold["final_cols_sha256"]

    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    seq = []
    t0 = time.perf_counter()
    for i in range(gold["prefix"]):
        try:
            ans, bits = pkg.abcore_query(g, ups["u"][i], ups["v"][i], ups["op"][i],
                                         ups["alpha"][i], ups["beta"][i])
            seq.append(("OK", ans, bits))
        except pkg.AbcoreError as e:
            seq.append((e.name, None, None))
        if i in samples:
            s = samples[i]
            assert seq[-1] == (s["status"], s["answer"], s["bits"]), (i, seq[-1], s)
    say(f"c5: {gold['prefix']} sequential queries in {time.perf_counter() - t0:.1f}s, "
        f"{len(samples)} equal the oracle")
    final_graph_matches(g)
    g.destroy()
    torch.cuda.empty_cache()
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    del eu, ev
    pkg.abcore_serve_start(g, 64, 0, 0)
    t0 = time.perf_counter()
    served = serve_all(g, ups, 64)
    pkg.abcore_serve_stop(g)
    say(f"c5: {gold['prefix']} served queries in {time.perf_counter() - t0:.1f}s")
    for i, r in enumerate(served):
        got = (r["status"], r["answer"] if r["status"] == "OK" else None,
               r["bits"] if r["status"] == "OK" else None)
        assert got == seq[i], (i, got, seq[i])
    final_graph_matches(g)
    g.destroy()
