"""Failure handling forced from the host, with every kernel ending normally:
a fake device-memory budget (abcore_set_memory_budget) makes builds and
computations fail with ENOMEM and change nothing, and makes the serving
engine admit with fewer device working sets (back-pressure: the rest of the
stream waits, EBUSY at max_inflight); a per-request deadline
(ABCORE_OPT_SERVE_DEADLINE_US) makes served requests report ETIMEDOUT while
their updates still apply in order (the final graph equals the oracle's)."""
import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.gpu_util import bits_np, ensure_built, say, serve_all, to_dev

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
    p.abcore_set_memory_budget(0)


def _spec():
    return dict(kind="chung_lu", n_upper=3000, n_lower=2000, m=12_000, gamma_upper=2.1,
                gamma_lower=2.1, cap=400, seed=601)


def _final_graph(nU, nL, eu, ev, ups):
    keys = set(int(a) * nL + int(b) for a, b in zip(eu, ev))
    for i in range(len(ups["u"])):
        k = int(ups["u"][i]) * nL + int(ups["v"][i])
        (keys.add if ups["op"][i] > 0 else keys.discard)(k)
    kk = np.array(sorted(keys), np.int64)
    return oracle.Graph(nU, nL, (kk // nL).astype(np.int32), (kk % nL).astype(np.int32))


def test_budget_makes_build_and_computation_fail_cleanly():
    spec = _spec()
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ref = oracle.Graph(nU, nL, eu, ev)
    deu, dev = to_dev(eu), to_dev(ev)
    before, _ = pkg.abcore_device_memory()
    try:
        # a build that cannot fit: ENOMEM, no handle, nothing left allocated
        say("budget: build under a budget of 1 KiB above current")
        pkg.abcore_set_memory_budget(before + 1024)
        with pytest.raises(pkg.AbcoreError) as e:
            pkg.abcore_build_csr(nU, nL, deu, dev)
        assert e.value.name == "ENOMEM"
        assert pkg.abcore_device_memory()[0] == before
        pkg.abcore_set_memory_budget(0)
        g = pkg.abcore_build_csr(nU, nL, deu, dev)
        built, _ = pkg.abcore_device_memory()
        want = oracle.pack(oracle.compute(ref, 3, 2))
        got = bits_np(pkg.abcore_compute(g, 3, 2, pkg.ABCORE_GCC))[: len(want)]
        assert np.array_equal(got, want)
        # the core numbers allocate on first use: ENOMEM under a tight budget,
        # and the handle is unchanged (GCC still exact, GCC+ exact later)
        say("budget: core numbers under a budget at the current footprint")
        pkg.abcore_set_memory_budget(pkg.abcore_device_memory()[0] + 1)
        with pytest.raises(pkg.AbcoreError) as e:
            pkg.abcore_core_numbers(g)
        assert e.value.name == "ENOMEM"
        with pytest.raises(pkg.AbcoreError) as e:
            pkg.abcore_compute(g, 3, 5, pkg.ABCORE_GCC_PLUS)
        assert e.value.name == "ENOMEM"
        got = bits_np(pkg.abcore_compute(g, 3, 2, pkg.ABCORE_GCC))[: len(want)]
        assert np.array_equal(got, want)
        pkg.abcore_set_memory_budget(0)
        core, mx = pkg.abcore_core_numbers(g)
        assert np.array_equal(core.cpu().numpy(), oracle.core_numbers(ref))
        for a, b in [(3, 5), (2, 2)]:
            w = oracle.pack(oracle.compute(ref, a, b))
            got = bits_np(pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC_PLUS))[: len(w)]
            assert np.array_equal(got, w), (a, b)
        g.destroy()
        assert pkg.abcore_device_memory()[0] == before
        assert built > before
    finally:
        pkg.abcore_set_memory_budget(0)


def test_budget_admits_with_fewer_working_sets():
    spec = _spec()
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 200, 1601, qlo=1, qhi=6)
    want = oracle.gfq_stream(nU, nL, eu, ev, ups)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    try:
        # the footprint of serving with one and with two working sets
        pkg.abcore_serve_start(g, 64, 1, 8)
        one, _ = pkg.abcore_device_memory()
        pkg.abcore_serve_stop(g)
        pkg.abcore_serve_start(g, 64, 2, 8)
        two, _ = pkg.abcore_device_memory()
        pkg.abcore_serve_stop(g)
        slot = two - one
        assert slot > 0
        say(f"budget: one working set is {slot} bytes")
        # room for one working set and a half: 4 requested, 1 created
        pkg.abcore_set_memory_budget(one + slot // 2)
        pkg.abcore_serve_start(g, 16, 4, 8)
        assert pkg.abcore_serve_counters(g)["device_slots"] == 1
        served = serve_all(g, ups, 16)
        pkg.abcore_serve_stop(g)
        for i, r in enumerate(served):
            st, wans, wbits = want[i]
            assert r["status"] == st, i
            if st == "OK":
                assert (r["answer"], r["bits"]) == (wans, wbits), i
        # no room for any working set: ENOMEM, the handle keeps working
        pkg.abcore_set_memory_budget(one - slot // 2)
        with pytest.raises(pkg.AbcoreError) as e:
            pkg.abcore_serve_start(g, 16, 4, 8)
        assert e.value.name == "ENOMEM"
        pkg.abcore_set_memory_budget(0)
        ref = _final_graph(nU, nL, eu, ev, ups)
        w = oracle.pack(oracle.compute(ref, 2, 3))
        assert np.array_equal(bits_np(pkg.abcore_compute(g, 2, 3, pkg.ABCORE_GCC))[: len(w)], w)
    finally:
        pkg.abcore_set_memory_budget(0)
        g.destroy()


def test_admission_back_pressure_returns_ebusy():
    spec = _spec()
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 64, 1602, qlo=1, qhi=6)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    pkg.abcore_serve_start(g, 2, 1, 1)
    tickets, busy = [], 0
    for i in range(len(ups["u"])):
        t = pkg.abcore_try_submit(g, ups["u"][i], ups["v"][i], ups["op"][i], ups["alpha"][i],
                                  ups["beta"][i])
        if t is None:
            busy += 1
            break
        tickets.append(t)
    # two admitted at most before the first EBUSY (the engine may finish some
    # meanwhile, so more can be admitted in total, never more than 2 at once)
    assert busy == 1 and len(tickets) >= 2
    pkg.abcore_serve_stop(g)
    g.destroy()


@pytest.mark.parametrize("deadline_us", [1, 3_600_000_000])
def test_deadline_drops_queries_but_applies_updates(deadline_us):
    spec = _spec()
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 150, 1603, qlo=1, qhi=6)
    want = oracle.gfq_stream(nU, nL, eu, ev, ups)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_SERVE_DEADLINE_US, deadline_us)
    pkg.abcore_serve_start(g, 32, 2, 8)
    say(f"deadline {deadline_us} us: {len(ups['u'])} requests")
    served = serve_all(g, ups, 32)
    counters = pkg.abcore_serve_counters(g)
    pkg.abcore_serve_stop(g)
    for i, r in enumerate(served):
        st, wans, wbits = want[i]
        if st != "OK":
            assert r["status"] == st, i  # a rejected update stays rejected
        elif deadline_us == 1:
            assert r["status"] == "ETIMEDOUT", (i, r)
        else:
            assert r["status"] == "OK" and (r["answer"], r["bits"]) == (wans, wbits), i
    valid = sum(1 for w in want if w[0] == "OK")
    assert counters["timed_out"] == (valid if deadline_us == 1 else 0)
    # the updates were applied in order either way
    ref = _final_graph(nU, nL, eu, ev, ups)
    off, cols = pkg.abcore_export_csr(g)
    assert np.array_equal(off.cpu().numpy(), ref.off)
    assert np.array_equal(cols.cpu().numpy(), ref.cols)
    g.destroy()


def test_core_numbers_without_room_for_the_hindex_phase():
    """The h-index phase of the core decomposition needs buffers of the deep
    core's size, which the handle keeps for later decompositions; under a
    budget that leaves room for the per-vertex arrays only, the level peel
    finishes the decomposition instead and the core numbers still equal the
    oracle's (Definition 2).  Later, without the budget, the phase runs on
    the updated graph and agrees with the oracle again."""
    spec = bigraph_gen.scaled(2, 0.05)
    nU, nL = spec["n_upper"], spec["n_lower"]
    n = nU + nL
    eu, ev = bigraph_gen.make_graph(spec)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    try:
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, 1 << 30)
        # core numbers, two alive lists and the removed bitmap (the arrays
        # every decomposition allocates on first use), and 1 KiB more
        arrays = 3 * 4 * n + 4 * ((n + 31) // 32)
        now, _ = pkg.abcore_device_memory()
        pkg.abcore_set_memory_budget(now + arrays + 1024)
        say("budget: core numbers with room for the per-vertex arrays only")
        core, mx = pkg.abcore_core_numbers(g)
        pkg.abcore_set_memory_budget(0)
        assert pkg.abcore_graph_report(g)["core_top"]["vertices"] == 0
        want = oracle.core_numbers(oracle.Graph(nU, nL, eu, ev))
        assert np.array_equal(core.cpu().numpy(), want)
        assert mx == int(want.max())
        # an update changes the graph, so the next call decomposes again,
        # now with the h-index phase
        u, v = 0, 0
        present = set(zip(eu.tolist(), ev.tolist()))
        while (u, v) in present:
            v += 1
        pkg.abcore_query(g, u, v, 1, 2, 2)
        present.add((u, v))
        core, mx = pkg.abcore_core_numbers(g)
        assert pkg.abcore_graph_report(g)["core_top"]["vertices"] > 0
        pe = np.array(sorted(present), np.int32)
        want = oracle.core_numbers(oracle.Graph(nU, nL, pe[:, 0], pe[:, 1]))
        assert np.array_equal(core.cpu().numpy(), want)
        assert mx == int(want.max())
    finally:
        pkg.abcore_set_memory_budget(0)
        g.destroy()
