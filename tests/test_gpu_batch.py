"""GPU parity of batched queries (abcore_compute_batch): every bitmask of a
batch equals the oracle's independent peel of that query and the library's
single-query call, bit for bit."""
import json
import os

import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.digests import sha_array, sha_edges
from tests.gpu_util import bits_np, ensure_built, say, to_dev

pytestmark = pytest.mark.gpu

pkg = None


@pytest.fixture(scope="module", autouse=True)
def _setup():
    global pkg
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()
    import paper_2606_07148_amd as p
    pkg = p
    yield


def _pairs(q, lo, hi, seed, extra=()):
    a = bigraph_gen.loguniform_pairs(q, lo, hi, seed)
    alphas, betas = [int(x) for x in a[0]], [int(x) for x in a[1]]
    for x, y in extra:
        alphas.append(x)
        betas.append(y)
    return alphas, betas


def _check_batch(g, ref, alphas, betas, tag, singles=True):
    got = bits_np(pkg.abcore_compute_batch(g, alphas, betas))
    want = oracle.batch(ref, alphas, betas)
    words = want.shape[1]
    for i, (a, b) in enumerate(zip(alphas, betas)):
        assert np.array_equal(got[i, :words], want[i]), f"{tag}: query {i} ({a},{b})"
        if singles and i % 7 == 0:
            one = bits_np(pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC))[:words]
            assert np.array_equal(one, want[i]), f"{tag}: single ({a},{b})"
    return got


def test_config1_batch():
    spec = bigraph_gen.CONFIGS[1]
    eu, ev = bigraph_gen.make_graph(spec)
    g = pkg.abcore_build_csr(spec["n_upper"], spec["n_lower"], to_dev(eu), to_dev(ev))
    ref = oracle.Graph(spec["n_upper"], spec["n_lower"], eu, ev)
    maxdeg = int(ref.degrees().max())
    alphas, betas = _pairs(40, 1, 24, 1001,
                           extra=[(1, 1), (3, 2), (3, 2), (maxdeg + 1, 1), (1, maxdeg + 1),
                                  (2**31, 5), (7, 7), (7, 7)])
    say("batch: config 1,", len(alphas), "queries")
    _check_batch(g, ref, alphas, betas, "config1")
    g.destroy()


def test_chung_lu_batch_modes_and_replay():
    spec = bigraph_gen.scaled(4, 0.01)
    eu, ev = bigraph_gen.make_graph(spec)
    nU, nL = spec["n_upper"], spec["n_lower"]
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    ref = oracle.Graph(nU, nL, eu, ev)
    alphas, betas = _pairs(64, 1, 256, 1004)
    say("batch: chung-lu 1/100 of the batch workload, 64 queries, replays")
    first = _check_batch(g, ref, alphas, betas, "chung-lu")
    # the captured graph is replayed: identical results, with eager work and
    # synchronisations between the replays
    for r in range(3):
        pkg.abcore_compute(g, 5, 9, pkg.ABCORE_GCC)
        again = bits_np(pkg.abcore_compute_batch(g, alphas, betas))
        assert np.array_equal(again, first), f"replay {r}"
    # other peel and pull modes run the same plan without capture
    for mode, pull in [(1, 0), (2, 2), (3, 1)]:
        say(f"batch: peel mode {mode}, pull {pull}")
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, mode)
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
        got = bits_np(pkg.abcore_compute_batch(g, alphas, betas))
        assert np.array_equal(got, first), (mode, pull)
    g.destroy()


@pytest.mark.skip(reason="concurrent batch lanes (independent branches of the captured graph, "
                         "one workspace per lane) ended the host process with a segmentation "
                         "fault inside abcore_compute_batch's capture path on the first call; "
                         "the cause was not found by reading, so the lanes code path was "
                         "removed and batches run one query at a time")
def test_batch_lanes_concurrent_and_sequential_agree():
    """The captured batch runs its queries on concurrent lanes (independent
    graph branches, each with its own queues and state; a query waits for its
    parent and for the earlier users of its degree buffer): 1, 2, 4 and 16
    lanes give the oracle's bitmasks, over replays with eager work between
    them."""
    spec = bigraph_gen.scaled(4, 0.01)
    eu, ev = bigraph_gen.make_graph(spec)
    nU, nL = spec["n_upper"], spec["n_lower"]
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    ref = oracle.Graph(nU, nL, eu, ev)
    alphas, betas = _pairs(96, 1, 256, 1014, extra=[(3, 3), (3, 3), (1, 1), (200, 2)])
    want = oracle.batch(ref, alphas, betas)
    words = want.shape[1]
    for lanes in (1, 2, 4, 16):
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_BATCH_LANES, lanes)
        for r in range(3):
            say(f"batch: {lanes} lanes, replay {r}")
            got = bits_np(pkg.abcore_compute_batch(g, alphas, betas))
            for i in range(len(alphas)):
                assert np.array_equal(got[i, :words], want[i]), (lanes, r, i)
            pkg.abcore_compute(g, 7, 3, pkg.ABCORE_GCC)
    g.destroy()


def test_batch_many_roots():
    """Mutually incomparable thresholds make every query a root of the plan
    (each runs the single-query path on the degree-rank copy); queries that
    dominate them nest under those roots."""
    spec = bigraph_gen.scaled(4, 0.01)
    eu, ev = bigraph_gen.make_graph(spec)
    nU, nL = spec["n_upper"], spec["n_lower"]
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    ref = oracle.Graph(nU, nL, eu, ev)
    alphas = [1, 2, 4, 8, 16, 32, 64, 128, 5, 9, 17, 40, 130]
    betas = [128, 64, 32, 16, 8, 4, 2, 1, 33, 17, 9, 5, 2]
    parent, _, _ = pkg.abcore_batch_plan(alphas, betas)
    assert sum(1 for p in parent if p < 0) == 8
    say("batch: eight roots and five nested queries")
    _check_batch(g, ref, alphas, betas, "roots")
    g.destroy()


def test_batch_after_updates():
    spec = dict(kind="chung_lu", n_upper=3000, n_lower=2000, m=15_000, gamma_upper=2.1,
                gamma_lower=2.1, cap=400, seed=402)
    eu, ev = bigraph_gen.make_graph(spec)
    nU, nL = spec["n_upper"], spec["n_lower"]
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    alphas, betas = _pairs(30, 1, 12, 1402)
    pkg.abcore_compute_batch(g, alphas, betas)  # captured on the build-time graph
    ups = bigraph_gen.update_stream(spec, eu, ev, 120, 1403, qlo=1, qhi=4)
    keys = set(int(a) * nL + int(b) for a, b in zip(eu, ev))
    for i in range(len(ups["u"])):
        pkg.abcore_query(g, ups["u"][i], ups["v"][i], ups["op"][i], 1, 1)
        k = int(ups["u"][i]) * nL + int(ups["v"][i])
        (keys.add if ups["op"][i] > 0 else keys.discard)(k)
    kk = np.array(sorted(keys), np.int64)
    ref = oracle.Graph(nU, nL, (kk // nL).astype(np.int32), (kk % nL).astype(np.int32))
    say("batch: after 120 updates")
    _check_batch(g, ref, alphas, betas, "after-updates")
    g.destroy()


def test_batch_edge_cases():
    eu = np.array([0, 0, 1, 1, 2], np.int32)
    ev = np.array([0, 1, 0, 1, 2], np.int32)
    g = pkg.abcore_build_csr(4, 3, to_dev(eu), to_dev(ev))
    ref = oracle.Graph(4, 3, eu, ev)
    say("batch: edge cases")
    _check_batch(g, ref, [1], [1], "single")
    _check_batch(g, ref, [2, 1, 2, 3, 1], [2, 1, 2, 1, 3], "tiny")
    out = pkg.abcore_compute_batch(g, [], [])
    assert out.shape[0] == 0
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_compute_batch(g, [1, 0], [1, 1])
    assert e.value.name == "EINVAL"
    g.destroy()
    # empty graph
    g = pkg.abcore_build_csr(0, 0, to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0, np.int32)))
    pkg.abcore_compute_batch(g, [1, 2], [1, 2])
    g.destroy()


def test_batch_workload_full_size():
    """The batch workload at full size: Chung-Lu |U| = 10M, |L| = 5M, 200M
    edges, 256 log-uniform pairs in [1,256]^2.  Every query equals the
    single-query call and the oracle's digest of its bitmask."""
    spec = bigraph_gen.CONFIGS[4]
    eu, ev = bigraph_gen.make_graph(spec)
    nU, nL = spec["n_upper"], spec["n_lower"]
    say("batch: full-size workload, generated")
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    alphas, betas = _pairs(256, 1, 256, spec["seed"] + 1000)
    got = bits_np(pkg.abcore_compute_batch(g, alphas, betas))
    words = (nU + nL + 31) // 32
    for i, (a, b) in enumerate(zip(alphas, betas)):
        one = bits_np(pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC))[:words]
        assert np.array_equal(got[i, :words], one), f"query {i} ({a},{b})"
    say("batch: full-size workload, singles equal; oracle digests")
    # every query against the oracle's digest (tests/golden/c4_oracle.json,
    # written offline by make_large_golden.py from the oracle alone)
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "c4_oracle.json")))
    assert sha_edges(eu, ev) == gold["edge_sha256"]
    assert [(q["alpha"], q["beta"]) for q in gold["queries"]] == list(zip(alphas, betas))
    for i, q in enumerate(gold["queries"]):
        assert sha_array(got[i, :words], "<u4") == q["bitmask_sha256"], f"oracle query {i}"
    g.destroy()


def test_tuning_cache_and_batch_autotune(tmp_path):
    """A batch on a shape the tuning cache has not seen tunes the mapping on
    its median query and stores it; a second handle of that shape finds it
    without tuning; the cache survives a save, clear and load; a single-query
    tuning is taken by the next handle's first query; every result stays
    equal to the oracle's."""
    pkg.abcore_tune_cache(None, 2)
    nU, nL, m = 40_000, 25_000, 500_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 6000, 93)
    ref = oracle.Graph(nU, nL, eu, ev)
    g1 = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    assert pkg.abcore_tuned(g1, 1) is None
    alphas, betas = _pairs(24, 1, 32, 1093)
    _check_batch(g1, ref, alphas, betas, "tuned batch")
    t = pkg.abcore_tuned(g1, 1)
    assert t is not None and t[0] >= 1 and t[1] in (16, 32, 64) and t[2] > 0
    g2 = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    assert pkg.abcore_tuned(g2, 1) == t
    path = tmp_path / "tune.txt"
    pkg.abcore_tune_cache(path, 1)
    pkg.abcore_tune_cache(None, 2)
    assert pkg.abcore_tuned(g2, 1) is None
    pkg.abcore_tune_cache(path, 0)
    got = pkg.abcore_tuned(g2, 1)
    assert got[:2] == t[:2] and abs(got[2] - t[2]) < 1e-3
    _check_batch(g2, ref, alphas, betas, "cached batch", singles=False)
    grid, claim, ms = pkg.abcore_autotune(g1, 6, 9, pkg.ABCORE_GCC)
    assert pkg.abcore_tuned(g2, 0)[:2] == (grid, claim)
    for ab in [(6, 9), (2, 2), (12, 4)]:
        want = oracle.pack(oracle.compute(ref, *ab))
        got = bits_np(pkg.abcore_compute(g2, *ab, pkg.ABCORE_GCC))[: len(want)]
        assert np.array_equal(got, want), ab
    g1.destroy()
    g2.destroy()
