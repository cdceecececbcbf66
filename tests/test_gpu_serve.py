"""GPU parity of the serving loop (abcore_submit / abcore_poll): every served
result equals the one-at-a-time abcore_query result (alone) and the oracle's
recomputation on the updated graph, whatever the concurrency (in the mix)."""
import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.gpu_util import ensure_built, say, serve_all, to_dev

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


def _with_invalid(ups, every=23):
    """Adds rejected requests: a repeated insertion and a repeated deletion."""
    out = {k: [] for k in ("u", "v", "op", "alpha", "beta")}
    for i in range(len(ups["u"])):
        for k in out:
            out[k].append(int(ups[k][i]))
        if i % every == every - 1:
            for k in out:
                out[k].append(int(ups[k][i]))  # the same update again: rejected
    return {k: np.array(v, np.int32) for k, v in out.items()}


def _sequential(nU, nL, eu, ev, ups):
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    out = []
    for i in range(len(ups["u"])):
        try:
            ans, bits = pkg.abcore_query(g, ups["u"][i], ups["v"][i], ups["op"][i],
                                         ups["alpha"][i], ups["beta"][i])
            out.append(("OK", ans, bits))
        except pkg.AbcoreError as e:
            out.append((e.name, None, None))
    return g, out


def _compare(served, want, tag):
    for i, (r, w) in enumerate(zip(served, want)):
        if w[0] != "OK":
            assert r["status"] == w[0], f"{tag} request {i}: {r} vs {w}"
        else:
            assert r["status"] == "OK", f"{tag} request {i}: {r}"
            assert (r["answer"], r["bits"]) == (w[1], w[2]), f"{tag} request {i}: {r} vs {w}"


@pytest.mark.parametrize("slots,window,inflight,pull",
                         [(8, 64, 256, 0), (3, 5, 7, 0), (1, 1, 1, 0), (8, 64, 256, 2),
                          (4, 16, 32, 1)])
def test_served_stream_equals_alone_and_oracle(slots, window, inflight, pull):
    spec = dict(kind="chung_lu", n_upper=3000, n_lower=2000, m=12_000, gamma_upper=2.1,
                gamma_lower=2.1, cap=400, seed=501)
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = _with_invalid(bigraph_gen.update_stream(spec, eu, ev, 400, 1501, qlo=1, qhi=6))
    say(f"serve: {len(ups['u'])} requests, slots {slots}, window {window}, "
        f"inflight {inflight}, pull {pull}")
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
    pkg.abcore_serve_start(g, inflight, slots, window)
    served = serve_all(g, ups, inflight)
    counters = pkg.abcore_serve_stop(g)
    assert counters["answered"] + counters["rejected"] == len(ups["u"])
    want = oracle.gfq_stream(nU, nL, eu, ev, ups)
    _compare(served, want, "oracle")
    g2, alone = _sequential(nU, nL, eu, ev, ups)
    _compare(served, alone, "alone")
    # the served graph equals the one-at-a-time graph afterwards
    o1, c1 = pkg.abcore_export_csr(g)
    o2, c2 = pkg.abcore_export_csr(g2)
    assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    # and the handle works normally after serving
    for a, b in [(2, 2), (1, 3)]:
        x1 = pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC).cpu().numpy()
        x2 = pkg.abcore_compute(g2, a, b, pkg.ABCORE_GCC).cpu().numpy()
        assert np.array_equal(x1, x2)
    # one-at-a-time queries continue identically on both handles
    for (u, v, op) in [(int(eu[0]), int(ev[0]), -1), (int(eu[0]), int(ev[0]), 1), (5, 7, 1)]:
        r = []
        for h in (g, g2):
            try:
                r.append(pkg.abcore_query(h, u, v, op, 2, 2))
            except pkg.AbcoreError as e:
                r.append(e.name)
        assert r[0] == r[1], (u, v, op, r)
    g.destroy()
    g2.destroy()


def test_serving_blocks_other_calls_and_restarts():
    eu = np.array([0, 0, 1, 1, 2], np.int32)
    ev = np.array([0, 1, 0, 1, 2], np.int32)
    g = pkg.abcore_build_csr(4, 3, to_dev(eu), to_dev(ev))
    pkg.abcore_serve_start(g, 4, 2, 2)
    say("serve: busy handle")
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_compute(g, 1, 1)
    assert e.value.name == "EBUSY"
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_submit(g, 9, 0, 1, 1, 1)
    assert e.value.name == "EINVAL"
    t = pkg.abcore_submit(g, 3, 2, 1, 1, 1)   # insert (3,2): u3 and v2 in the (1,1)-core
    t2 = pkg.abcore_submit(g, 3, 2, 1, 1, 1)  # again: rejected
    t3 = pkg.abcore_submit(g, 0, 0, -1, 2, 2)  # delete (0,0): the (2,2)-core loses u0, v0
    res = {}
    while len(res) < 3:
        for x in (t, t2, t3):
            if x not in res:
                r = pkg.abcore_poll(g, x)
                if r is not None:
                    res[x] = r
    assert res[t]["status"] == "OK" and res[t]["answer"] and res[t]["bits"] == 3
    assert res[t2]["status"] == "EEXIST"
    assert res[t3]["status"] == "OK" and not res[t3]["answer"] and res[t3]["bits"] == 0
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_poll(g, 1000)
    assert e.value.name == "EINVAL"
    pkg.abcore_serve_stop(g)
    # restart and serve again on the same handle
    t4 = pkg.abcore_submit(g, 0, 0, 1, 2, 2)  # re-insert (0,0): the 4-cycle is back
    while (r := pkg.abcore_poll(g, t4)) is None:
        pass
    assert r["status"] == "OK" and r["answer"]
    pkg.abcore_serve_stop(g)
    bits = pkg.abcore_compute(g, 2, 2).cpu().numpy().view(np.uint32)
    assert int(bits[0]) == 0b0011 | (0b011 << 4)  # u0,u1 and v0,v1 (ids 4,5)
    g.destroy()


def test_served_stream_power_law():
    """A 1/100 scale of the serving workload (Chung-Lu, 300k vertices, 5M
    edges), alpha and beta log-uniform in [2,64]: served in the mix equals one
    at a time; the oracle checks sampled requests."""
    spec = bigraph_gen.scaled(5, 0.01)
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 240, spec["seed"] + 1000)
    say("serve: power-law 1/100 scale, 240 requests, pull always")
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, 2)
    pkg.abcore_serve_start(g, 64, 8, 64)
    served = serve_all(g, ups, 64)
    pkg.abcore_serve_stop(g)
    g2, alone = _sequential(nU, nL, eu, ev, ups)
    _compare(served, alone, "alone")
    sample = {0, 1, 2, 57, 120, 239}
    want = oracle.gfq_stream(nU, nL, eu, ev, ups, check_only=sample)
    _compare([served[i] for i in sorted(sample)], [want[i] for i in sorted(sample)], "oracle")
    g.destroy()
    g2.destroy()


@pytest.mark.parametrize("pull", [1, 2])
def test_served_versions_of_vertex_zero_edges(pull):
    """Queries in a window see edges of vertex 0 deleted later in the same
    window (a deleted entry to vertex 0 is stored as ~0 = -1)."""
    eu = np.array([0, 0, 1, 1, 3, 3, 4], np.int32)
    ev = np.array([0, 1, 0, 1, 3, 4, 3], np.int32)
    nU = nL = 6
    cycle = [(2, 0, 1, 2, 2), (0, 0, -1, 2, 2), (0, 0, 1, 2, 2), (2, 0, -1, 1, 1),
             (0, 1, -1, 2, 2), (0, 1, 1, 1, 2)]
    reqs = cycle * 40
    ups = {k: np.array([r[i] for r in reqs], np.int32)
           for i, k in enumerate(("u", "v", "op", "alpha", "beta"))}
    say("serve: vertex-0 versions, pull", pull)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
    pkg.abcore_serve_start(g, 64, 8, 64)
    served = serve_all(g, ups, 64)
    counters = pkg.abcore_serve_stop(g)
    g2, alone = _sequential(nU, nL, eu, ev, ups)
    _compare(served, alone, "alone")
    want = oracle.gfq_stream(nU, nL, eu, ev, ups)
    _compare(served, want, "oracle")
    assert counters["windows"] < len(reqs)  # several requests shared windows
    g.destroy()
    g2.destroy()


@pytest.mark.parametrize("prune,slots,window", [(1, 4, 16), (7, 3, 5), (64, 8, 64), (2, 1, 1)])
def test_served_stream_with_stale_core_pruning(prune, slots, window):
    """Stale core-number pruning (ABCORE_OPT_SERVE_PRUNE): requests decided
    from the snapshot's intervals skip the peel, every answer and endpoint
    bit still equals the oracle's recomputation and the one-at-a-time
    result, snapshots are retaken every `prune` updates (prune >= 2), and
    the final graph equals the one-at-a-time graph."""
    spec = dict(kind="chung_lu", n_upper=3000, n_lower=2000, m=12_000, gamma_upper=2.1,
                gamma_lower=2.1, cap=400, seed=502)
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = _with_invalid(bigraph_gen.update_stream(spec, eu, ev, 300, 1502, qlo=1, qhi=12))
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_SERVE_PRUNE, prune)
    pkg.abcore_serve_start(g, 64, slots, window)
    served = serve_all(g, ups, 64)
    c = pkg.abcore_serve_counters(g)
    pkg.abcore_serve_stop(g)
    say(f"serve prune {prune}: decided {c['decided_without_peel']} of {c['answered']}, "
        f"snapshots {c['core_snapshots']} ({c['snapshot_ms']:.1f} ms)")
    assert c["decided_without_peel"] > 0
    valid = c["answered"]
    if prune >= 2:
        # a snapshot is retaken at the end of the window in which the count
        # of updates since the last one reaches `prune`
        again = c["core_snapshots"] - 1
        assert valid // (prune + window - 1) - 1 <= again <= valid // prune
    else:
        assert c["core_snapshots"] == 1
    want = oracle.gfq_stream(nU, nL, eu, ev, ups)
    _compare(served, want, "oracle")
    g2, alone = _sequential(nU, nL, eu, ev, ups)
    _compare(served, alone, "alone")
    o1, c1 = pkg.abcore_export_csr(g)
    o2, c2 = pkg.abcore_export_csr(g2)
    assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    g.destroy()
    g2.destroy()
