"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Every comparison is exact (integer membership); inputs are seeded synthetic
graphs from bigraph_gen.
"""
import numpy as np
import pytest

import bigraph_gen
import oracle
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


def _make(nU, nL, eu, ev):
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    ref = oracle.Graph(nU, nL, eu, ev)
    return g, ref


def _check_core(g, ref, a, b, algo, tag="", tombstones=False):
    bits, st = pkg.abcore_compute(g, a, b, algo, stats=True)
    mem, ost = oracle.peel(ref, a, b)
    want = oracle.pack(mem)
    got = bits_np(bits)[: len(want)]
    assert np.array_equal(got, want), f"{tag} ({a},{b}) algo={algo}: bitmask differs"
    if algo == pkg.ABCORE_GCC:
        assert st["removed"] == ost["removed"], (tag, a, b)
        if st["rounds"] >= 0:  # the asynchronous peel has no rounds
            assert st["rounds"] == ost["rounds"], (tag, a, b)
        # a push peel reads exactly the rows of removed vertices; a pull first
        # round reads the surviving rows instead; after deletions the peel
        # also reads tombstoned entries
        if st["pulled"]:
            pass
        elif tombstones:
            assert st["entries_read"] >= ost["removed_degree_sum"], (tag, a, b)
        else:
            assert st["entries_read"] == ost["removed_degree_sum"], (tag, a, b)
    return st, ost


# (peel mode, pull mode): 3 asynchronous worklist, 2 cooperative rounds,
# 1 one kernel per round; pull 0 auto, 1 never, 2 always
MODES = [(3, 0), (3, 1), (3, 2), (2, 0), (2, 2), (1, 1), (1, 2)]


def _set_mode(g, peel, pull):
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, peel)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)


# ------------------------------------------------------------------ build --


def test_build_matches_oracle_csr():
    spec = bigraph_gen.CONFIGS[1]
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    rng = np.random.default_rng(0)
    dup = rng.choice(len(eu), 5000, replace=False)
    eu2 = np.concatenate([eu, eu[dup]])
    ev2 = np.concatenate([ev, ev[dup]])
    perm = rng.permutation(len(eu2))
    eu2, ev2 = eu2[perm], ev2[perm]
    say("build: config 1 shuffled with 5000 duplicates")
    g, ref = _make(nU, nL, eu2, ev2)
    assert g.m == ref.m == len(eu)
    off, cols = pkg.abcore_export_csr(g)
    assert np.array_equal(off.cpu().numpy(), ref.off)
    assert np.array_equal(cols.cpu().numpy(), ref.cols)
    g.destroy()


def test_build_rejects_out_of_range():
    say("build: out-of-range endpoint")
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_build_csr(4, 4, to_dev([0, 4]), to_dev([0, 1]))
    assert e.value.name == "EINVAL"


# ------------------------------------------------------------ computation --


@pytest.mark.parametrize("peel,pull", MODES)
def test_config1_gcc_and_gccplus(peel, pull):
    spec = bigraph_gen.CONFIGS[1]
    eu, ev = bigraph_gen.make_graph(spec)
    g, ref = _make(spec["n_upper"], spec["n_lower"], eu, ev)
    _set_mode(g, peel, pull)
    say("config 1: (3,2) GCC / GCC+, mode", peel, pull)
    st, _ = _check_core(g, ref, 3, 2, pkg.ABCORE_GCC, "c1")
    assert st["pulled"] == (1 if pull == 2 else 0) or pull == 0
    _check_core(g, ref, 3, 2, pkg.ABCORE_GCC_PLUS, "c1")
    for a, b in [(1, 1), (2, 2), (5, 3), (3, 5), (10, 14), (14, 10), (13, 27), (40, 40)]:
        say("config 1:", a, b)
        _check_core(g, ref, a, b, pkg.ABCORE_GCC, "c1")
        _check_core(g, ref, a, b, pkg.ABCORE_GCC_PLUS, "c1")
    g.destroy()


@pytest.mark.parametrize("seed,peel,pull", [(101, 3, 0), (102, 3, 2), (103, 3, 1),
                                            (104, 2, 0), (105, 2, 2), (106, 1, 1),
                                            (107, 1, 2)])
def test_chung_lu_small_grid(seed, peel, pull):
    nU, nL, m = 30_000, 20_000, 400_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 5000, seed)
    g, ref = _make(nU, nL, eu, ev)
    _set_mode(g, peel, pull)
    for a, b in [(1, 1), (2, 3), (3, 2), (5, 5), (4, 9), (9, 4), (12, 30), (30, 12), (64, 64),
                 (1000, 1)]:
        say("chung-lu", seed, a, b, "mode", peel, pull)
        for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
            _check_core(g, ref, a, b, algo, f"cl{seed}")
    g.destroy()


def test_rank_order_queries():
    """GCC queries on an unchanged graph run on its degree-rank relabelling
    (survivors of the scan = the vertices of degree >= threshold, a prefix of
    each layer's rank order); after an update they run in vertex order.  Both
    equal the oracle; the first frontier counts the scan's frontier."""
    nU, nL, m = 30_000, 20_000, 400_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 5000, 111)
    g, ref = _make(nU, nL, eu, ev)
    deg = ref.degrees()
    pairs = [(1, 1), (2, 3), (5, 5), (4, 9), (9, 4), (12, 30), (64, 64), (1000, 1),
             (int(deg[:nU].max()), 2), (int(deg[:nU].max()) + 1, 1),
             (3, int(deg[nU:].max()) + 1), (2**31 - 1, 2**31 - 1)]
    for pull in (2, 0):
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
        for a, b in pairs:
            say("rank order: pull", pull, a, b)
            st, _ = _check_core(g, ref, a, b, pkg.ABCORE_GCC, f"rank pull{pull}")
            thr = np.where(np.arange(nU + nL) < nU, a, b)
            if pull == 2:
                assert st["rank_order"] == 1 and st["pulled"] == 1, (a, b)
            if st["rank_order"]:
                assert st["initial"] == int(np.count_nonzero(deg < thr)), (a, b)
    # an inserted edge: vertex order from then on
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, 2)
    u, v = 0, 0
    have = set(zip(eu.tolist(), ev.tolist()))
    while (u, v) in have:
        v += 1
    pkg.abcore_query(g, u, v, 1, 1, 1)
    ref = oracle.Graph(nU, nL, np.append(eu, np.int32(u)), np.append(ev, np.int32(v)))
    for a, b in [(2, 3), (5, 5), (12, 30)]:
        st, _ = _check_core(g, ref, a, b, pkg.ABCORE_GCC, "after insert")
        assert st["rank_order"] == 0
    g.destroy()


def test_rank_order_interleaved_with_other_work():
    """Queries in rank order alternate between two workspace states, each
    leaving the other ready; batches (captured and replayed), GCC+, core
    numbers and vertex-order queries in between must not disturb them."""
    nU, nL, m = 20_000, 15_000, 250_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 3000, 112)
    g, ref = _make(nU, nL, eu, ev)
    want = {}

    def check(a, b, tag):
        if (a, b) not in want:
            want[(a, b)] = oracle.pack(oracle.peel(ref, a, b)[0])
        w = want[(a, b)]
        got = bits_np(pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC))[: len(w)]
        assert np.array_equal(got, w), (tag, a, b)

    seq = [(10, 10), (5, 20), (40, 8), (2, 3), (10, 10)]
    for i, ab in enumerate(seq):
        check(*ab, f"run {i}")
    alphas, betas = [3, 5, 9, 12], [4, 4, 10, 2]
    for rep in range(3):
        got = bits_np(pkg.abcore_compute_batch(g, alphas, betas))
        for i, ab in enumerate(zip(alphas, betas)):
            if ab not in want:
                want[ab] = oracle.pack(oracle.peel(ref, *ab)[0])
            assert np.array_equal(got[i, : len(want[ab])], want[ab]), ("batch", rep, ab)
        for k in range(rep + 1):  # an odd, then an even number of exchanges
            check(*seq[k], f"after batch {rep}")
    pkg.abcore_compute(g, 4, 9, pkg.ABCORE_GCC_PLUS)
    check(7, 7, "after GCC+")
    pkg.abcore_core_numbers(g)
    check(7, 7, "after core numbers")
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, 2)
    check(6, 11, "vertex order")
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, 1)
    check(6, 11, "rank order again")
    _, st = pkg.abcore_compute(g, 6, 11, pkg.ABCORE_GCC, stats=True)
    assert st["rank_order"] == 1
    check(6, 11, "after stats")
    g.destroy()


def test_repeat_runs_identical():
    eu, ev = bigraph_gen.chung_lu(50_000, 30_000, 600_000, 2.1, 2.1, 8000, 7)
    g = pkg.abcore_build_csr(50_000, 30_000, to_dev(eu), to_dev(ev))
    say("repeatability (6,6) x 5")
    first = bits_np(pkg.abcore_compute(g, 6, 6)).copy()
    for _ in range(4):
        assert np.array_equal(bits_np(pkg.abcore_compute(g, 6, 6)), first)
    g.destroy()


@pytest.mark.parametrize("grid", [1, 3, 17])
def test_async_small_grids(grid):
    """The asynchronous peel with fewer workgroups than sub-queues: items of
    sub-queues without a workgroup of their own are taken by stealing."""
    nU, nL, m = 30_000, 20_000, 400_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 5000, 77 + grid)
    g, ref = _make(nU, nL, eu, ev)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_GRID, grid)
    say("async peel, grid", grid)
    for (a, b) in [(4, 4), (9, 3), (2, 12)]:
        for pull in (1, 2):
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
            _check_core(g, ref, a, b, pkg.ABCORE_GCC, f"grid{grid}")
        _check_core(g, ref, a, b, pkg.ABCORE_GCC_PLUS, f"grid{grid}")
    g.destroy()


def test_autotune_keeps_results_exact():
    nU, nL, m = 40_000, 25_000, 500_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 6000, 91)
    g, ref = _make(nU, nL, eu, ev)
    say("autotune")
    for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
        grid, claim, ms = pkg.abcore_autotune(g, 6, 9, algo)
        assert grid >= 1 and claim in (16, 32, 64) and ms > 0
        for ab in [(6, 9), (2, 2), (12, 4)]:
            _check_core(g, ref, *ab, algo, f"tuned grid{grid} claim{claim}")
    g.destroy()


@pytest.mark.parametrize("peel,pull", [(3, 0), (3, 1), (3, 2), (2, 2), (1, 1)])
def test_shared_queue_capacity_overflow(peel, pull):
    """The 16 frontier sub-queues share one capacity bound (a 16th of
    2n + pieces + 256 each, plus 4,096 slots).  With every append sent to
    sub-queue 0 first, it fills and later appends overflow into the others
    (the rest of a full sub-queue is filled with skip slots): results stay
    exact for GCC, GCC+, core numbers and GFQ updates in every peel mode."""
    nU, nL, m = 30_000, 20_000, 400_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 5000, 108)
    g, ref = _make(nU, nL, eu, ev)
    _set_mode(g, peel, pull)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_APPEND_SUBQUEUE, 1)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, 1)  # every level queued
    for a, b in [(1, 1), (2, 3), (5, 5), (9, 4), (12, 30), (64, 64)]:
        say("shared capacity: mode", peel, pull, "query", a, b)
        for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
            _check_core(g, ref, a, b, algo, "overflow")
    say("shared capacity: core numbers")
    core, mx = pkg.abcore_core_numbers(g)
    want = oracle.core_numbers(ref)
    assert np.array_equal(core.cpu().numpy(), want)
    assert mx == int(want.max())
    spec = dict(kind="chung_lu", n_upper=nU, n_lower=nL, m=m, gamma_upper=2.1,
                gamma_lower=2.1, cap=5000, seed=108)
    ups = bigraph_gen.update_stream(spec, eu, ev, 40, 1108, qlo=1, qhi=16)
    want = oracle.gfq_stream(nU, nL, eu, ev, ups)
    say("shared capacity: 40 GFQ updates")
    for i in range(len(ups["u"])):
        ans, bits = pkg.abcore_query(g, ups["u"][i], ups["v"][i], ups["op"][i],
                                     ups["alpha"][i], ups["beta"][i])
        st, wans, wbits = want[i]
        assert st == "OK"
        assert (ans, bits) == (wans, wbits), f"update {i}"
    g.destroy()


# ----------------------------------------------------------- core numbers --


@pytest.mark.parametrize("seed,peel", [(201, 3), (202, 1), (203, 2)])
def test_core_numbers(seed, peel):
    nU, nL, m = 40_000, 25_000, 500_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.3, 6000, seed)
    g, ref = _make(nU, nL, eu, ev)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, peel)
    say("core numbers", seed, "mode", peel)
    core, mx = pkg.abcore_core_numbers(g)
    want = oracle.core_numbers(ref)
    assert np.array_equal(core.cpu().numpy(), want)
    assert mx == int(want.max())
    g.destroy()


def test_components():
    nU, nL, m = 20_000, 20_000, 15_000  # sparse: many components
    eu, ev = bigraph_gen.uniform(nU, nL, m, 301)
    g, ref = _make(nU, nL, eu, ev)
    say("components")
    comp = pkg.abcore_components(g).cpu().numpy()
    assert np.array_equal(comp, oracle.components(ref))
    g.destroy()


# ------------------------------------------------------------- edge cases --


def test_edge_cases():
    # no edges: nothing survives for alpha, beta >= 1
    say("edge: empty edge set")
    g = pkg.abcore_build_csr(5, 7, to_dev([]), to_dev([]))
    assert g.m == 0
    assert not bits_np(pkg.abcore_compute(g, 1, 1)).any()
    assert not bits_np(pkg.abcore_compute(g, 2, 1, pkg.ABCORE_GCC_PLUS)).any()
    core, mx = pkg.abcore_core_numbers(g)
    assert mx == 0 and not core.cpu().numpy().any()
    g.destroy()
    # a star with a 50,000-degree hub plus a K_{3,3}
    say("edge: 50k hub star")
    hub_v = np.arange(50_000, dtype=np.int32)
    eu = np.concatenate([np.zeros(50_000, np.int32), np.repeat(np.arange(1, 4), 3)])
    ev = np.concatenate([hub_v, np.tile(np.arange(50_000, 50_003), 3)])
    g, ref = _make(4, 50_003, eu, ev)
    for a, b in [(1, 1), (2, 1), (1, 2), (3, 3), (4, 1), (50_000, 1), (50_001, 1)]:
        for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
            _check_core(g, ref, a, b, algo, "star")
    g.destroy()
    # complete bipartite K_{40,70}
    say("edge: K_{40,70}")
    eu = np.repeat(np.arange(40, dtype=np.int32), 70)
    ev = np.tile(np.arange(70, dtype=np.int32), 40)
    g, ref = _make(40, 70, eu, ev)
    for a, b in [(70, 40), (71, 40), (70, 41), (1, 1), (35, 20)]:
        for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
            _check_core(g, ref, a, b, algo, "K")
    g.destroy()
    # a hub that crosses its threshold during the rounds (its row is split
    # into pieces when queued): 100 private degree-1 neighbours, 100 shared
    # with a second upper vertex
    say("edge: hub crossing in a later round")
    eu = np.concatenate([np.zeros(200, np.int32), np.ones(100, np.int32)])
    ev = np.concatenate([np.arange(200), np.arange(100, 200)]).astype(np.int32)
    g, ref = _make(2, 200, eu, ev)
    for peel, pull in MODES:
        _set_mode(g, peel, pull)
        for a, b in [(101, 2), (150, 2), (1, 2), (100, 2), (2, 2)]:
            _check_core(g, ref, a, b, pkg.ABCORE_GCC, "hub")
            _check_core(g, ref, a, b, pkg.ABCORE_GCC_PLUS, "hub")
    g.destroy()
    # a long path: one vertex per end per round
    say("edge: path of 3001 vertices")
    L = 3001
    pos = np.arange(L - 1)
    u = np.where(pos % 2 == 0, pos // 2, (pos + 1) // 2).astype(np.int32)
    v = np.where(pos % 2 == 0, pos // 2, pos // 2).astype(np.int32)
    g, ref = _make((L + 1) // 2, L // 2, u, v)
    for peel in (3, 2, 1):
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, peel)
        st, ost = _check_core(g, ref, 2, 2, pkg.ABCORE_GCC, "path")
        assert st["rounds"] in (-1, (L + 1) // 2)
    g.destroy()


# -------------------------------------------------------------------- GFQ --


@pytest.mark.parametrize("pull", [0, 2, 1])
def test_gfq_stream_matches_recomputation(pull):
    spec = dict(kind="chung_lu", n_upper=3000, n_lower=2000, m=12_000, gamma_upper=2.1,
                gamma_lower=2.1, cap=400, seed=401)
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 300, 1401, qlo=1, qhi=6)
    g = pkg.abcore_build_csr(spec["n_upper"], spec["n_lower"], to_dev(eu), to_dev(ev))
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
    want = oracle.gfq_stream(spec["n_upper"], spec["n_lower"], eu, ev, ups)
    say("gfq: 300 updates, pull mode", pull)
    for i in range(len(ups["u"])):
        ans, bits = pkg.abcore_query(g, ups["u"][i], ups["v"][i], ups["op"][i],
                                     ups["alpha"][i], ups["beta"][i])
        st, wans, wbits = want[i]
        assert st == "OK"
        assert (ans, bits) == (wans, wbits), f"update {i}"
    # the graph after the stream equals the oracle's final graph
    off, cols = pkg.abcore_export_csr(g)
    nL = spec["n_lower"]
    keys = set((int(a) * nL + int(b)) for a, b in zip(eu, ev))
    for i in range(len(ups["u"])):
        k = int(ups["u"][i]) * nL + int(ups["v"][i])
        (keys.add if ups["op"][i] > 0 else keys.discard)(k)
    kk = np.array(sorted(keys), np.int64)
    ref = oracle.Graph(spec["n_upper"], nL, (kk // nL).astype(np.int32),
                       (kk % nL).astype(np.int32))
    assert np.array_equal(off.cpu().numpy(), ref.off)
    assert np.array_equal(cols.cpu().numpy(), ref.cols)
    # components and the whole-graph computation on the updated graph
    assert np.array_equal(pkg.abcore_components(g).cpu().numpy(), oracle.components(ref))
    for algo in (pkg.ABCORE_GCC, pkg.ABCORE_GCC_PLUS):
        _check_core(g, ref, 2, 3, algo, "after-stream", tombstones=True)
    for pull in (1, 2, 0):  # pull form over tombstones and inserted edges too
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
        for ab in [(2, 3), (3, 2), (1, 1), (4, 4)]:
            _check_core(g, ref, *ab, pkg.ABCORE_GCC, f"after-stream pull{pull}", tombstones=True)
    core, _ = pkg.abcore_core_numbers(g)
    assert np.array_equal(core.cpu().numpy(), oracle.core_numbers(ref))
    g.destroy()


def test_gfq_errors_leave_graph_unchanged():
    eu = np.array([0, 0, 1], np.int32)
    ev = np.array([0, 1, 1], np.int32)
    g = pkg.abcore_build_csr(3, 3, to_dev(eu), to_dev(ev))
    say("gfq: error statuses")
    off0, cols0 = [t.cpu().numpy() for t in pkg.abcore_export_csr(g)]
    for (u, v, op, name) in [(0, 0, 1, "EEXIST"), (2, 2, -1, "ENOENT"), (3, 0, 1, "EINVAL"),
                             (0, 0, 2, "EINVAL")]:
        with pytest.raises(pkg.AbcoreError) as e:
            pkg.abcore_query(g, u, v, op, 1, 1)
        assert e.value.name == name
        off1, cols1 = [t.cpu().numpy() for t in pkg.abcore_export_csr(g)]
        assert np.array_equal(off0, off1) and np.array_equal(cols0, cols1)
    # insert, delete, re-insert the same pair (CSR edge and inserted edge)
    assert pkg.abcore_query(g, 0, 0, -1, 1, 1) == (False, 1)  # (0,0) gone; v0 isolated
    assert pkg.abcore_query(g, 0, 0, 1, 1, 1) == (True, 3)
    assert pkg.abcore_query(g, 2, 2, 1, 1, 1) == (True, 3)
    assert pkg.abcore_query(g, 2, 2, -1, 1, 1) == (False, 0)
    assert pkg.abcore_query(g, 2, 2, 1, 1, 1) == (True, 3)
    g.destroy()


# ------------------------------------------------------- full-size config 2 --


def test_config2_full_size():
    spec = bigraph_gen.CONFIGS[2]
    nU, nL = spec["n_upper"], spec["n_lower"]
    say("config 2: generating 20M edges")
    eu, ev = bigraph_gen.make_graph(spec)
    g, ref = _make(nU, nL, eu, ev)
    for a, b in [(10, 10), (5, 20), (20, 5), (2, 2)]:
        say("config 2:", a, b)
        _check_core(g, ref, a, b, pkg.ABCORE_GCC, "c2")
        _check_core(g, ref, a, b, pkg.ABCORE_GCC_PLUS, "c2")
    core, mx = pkg.abcore_core_numbers(g)
    assert np.array_equal(core.cpu().numpy(), oracle.core_numbers(ref))
    # rank order against vertex order over a spread of thresholds (the same
    # graph, both on the device; the four pairs above also against the oracle)
    alphas, betas = bigraph_gen.loguniform_pairs(24, 1, 300, 2002)
    say("config 2: rank order against vertex order, 24 pairs")
    for a, b in zip(alphas.tolist(), betas.tolist()):
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, 2)
        want, sv = pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC, stats=True)
        want = bits_np(want)
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, 1)
        got, sr = pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC, stats=True)
        assert sv["rank_order"] == 0
        assert np.array_equal(bits_np(got), want), (a, b)
        assert sr["removed"] == sv["removed"], (a, b)
    g.destroy()


@pytest.mark.parametrize("switch", [0, 1, 2, 8, 1 << 20])
def test_core_numbers_level_and_hindex_phases(switch):
    """Core numbers (Definition 2) equal the oracle's Batagelj-Zaversnik
    values whichever share of the levels the h-index fixpoint finishes: the
    default switch, levels only (1, 2, 8 live vertices: never reached before
    the end), and from the first check (2^20 live vertices), on two
    power-law graphs and the uniform one, and after updates (tombstones and
    inserted edges in the rows)."""
    specs = [bigraph_gen.scaled(2, 0.05), bigraph_gen.scaled(3, 1 / 400), bigraph_gen.CONFIGS[1]]
    for spec in specs:
        nU, nL = spec["n_upper"], spec["n_lower"]
        eu, ev = bigraph_gen.make_graph(spec)
        g, ref = _make(nU, nL, eu, ev)
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, switch)
        core, mx = pkg.abcore_core_numbers(g)
        want = oracle.core_numbers(ref)
        assert np.array_equal(core.cpu().numpy(), want), (spec, switch)
        assert mx == int(want.max())
        # after updates: the rows hold tombstones and inserted edges
        ups = bigraph_gen.update_stream(spec, eu, ev, 30, 2024)
        present = set(zip(eu.tolist(), ev.tolist()))
        for i in range(len(ups["u"])):
            u, v, op = int(ups["u"][i]), int(ups["v"][i]), int(ups["op"][i])
            if (op > 0) == ((u, v) in present):
                continue
            pkg.abcore_query(g, u, v, op, 2, 2)
            (present.add if op > 0 else present.discard)((u, v))
        pe = np.array(sorted(present), np.int32)
        ref2 = oracle.Graph(nU, nL, pe[:, 0], pe[:, 1])
        core, mx = pkg.abcore_core_numbers(g)
        want = oracle.core_numbers(ref2)
        assert np.array_equal(core.cpu().numpy(), want), (spec, switch, "after updates")
        say(f"core numbers switch {switch}: n={nU + nL}, max {mx}")
        g.destroy()


def test_core_numbers_hindex_layers_past_the_lds_cache():
    """The h-index phase keeps the first 63,488 values of the layer a half
    reads in LDS and reads the rest from memory: started at the first check
    on the 2x10^7-edge graph (about a million live vertices), both layers of
    the deep core exceed that, long rows need more than one binned pass, and
    the result still equals the oracle's core numbers (Definition 2)."""
    spec = bigraph_gen.CONFIGS[2]
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    g, ref = _make(nU, nL, eu, ev)
    want = oracle.core_numbers(ref)
    pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, 1 << 22)
    core, mx = pkg.abcore_core_numbers(g)
    top = pkg.abcore_graph_report(g)["core_top"]
    say(f"config 2 core numbers from the first check: {top}")
    assert top["vertices"] > 2 * 63488, top
    assert np.array_equal(core.cpu().numpy(), want)
    assert mx == int(want.max())
    g.destroy()


def test_core_numbers_hindex_buffers_kept_and_grown():
    """The handle keeps the h-index phase's buffers between decompositions:
    switch points that give a small, a large, a small and again a large
    deep core make them grow once and then serve smaller and equal deep
    cores as they are.  Every decomposition equals the oracle's core numbers
    (Definition 2), and destroying the handle returns every byte."""
    spec = bigraph_gen.scaled(2, 0.05)
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    before, _ = pkg.abcore_device_memory()
    g, ref = _make(nU, nL, eu, ev)
    want = oracle.core_numbers(ref)
    sizes = []
    try:
        for switch in (1 << 13, 1 << 30, 1 << 13, 1 << 30):
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, switch)
            core, mx = pkg.abcore_core_numbers(g)
            top = pkg.abcore_graph_report(g)["core_top"]
            say(f"kept buffers, switch {switch}: {top}, {pkg.abcore_device_memory()[0]} bytes")
            assert np.array_equal(core.cpu().numpy(), want), switch
            assert mx == int(want.max())
            sizes.append((top["vertices"], pkg.abcore_device_memory()[0]))
        assert 0 < sizes[0][0] < sizes[1][0], sizes
        # the small deep core again fits the grown buffers: no allocation
        assert sizes[2][1] == sizes[1][1] == sizes[3][1], sizes
    finally:
        g.destroy()
    assert pkg.abcore_device_memory()[0] == before


def test_core_numbers_hindex_long_rows_by_id_ranges():
    """A dense graph whose deep core's rows average over 512 entries: on a
    graph unchanged since the build the h-index phase fills those rows by
    id ranges of the other layer, one range per XCD (ranges of 160 ids here,
    the last ones ragged or empty, rows appended in any order).  Core
    numbers equal the oracle's (Definition 2); after an update the same
    graph takes the one-walk-per-row fill and agrees again."""
    nU, nL = 1201, 1187
    m = int(0.45 * nU * nL)
    eu, ev = bigraph_gen.make_graph(dict(kind="uniform", n_upper=nU, n_lower=nL, m=m, seed=91))
    g, ref = _make(nU, nL, eu, ev)
    try:
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, 1 << 30)
        core, mx = pkg.abcore_core_numbers(g)
        top = pkg.abcore_graph_report(g)["core_top"]
        say(f"long rows: {top}, max core {mx}")
        assert top["vertices"] > 0 and top["entries"] >= 512 * top["vertices"], top
        want = oracle.core_numbers(ref)
        assert np.array_equal(core.cpu().numpy(), want)
        assert mx == int(want.max())
        present = set(zip(eu.tolist(), ev.tolist()))
        u, v = 0, 0
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
        g.destroy()


def test_core_numbers_hindex_wide_ranges():
    """Rows whose value range exceeds 16 bits in the h-index phase: ten
    lower vertices adjacent to 80,000 upper vertices (degree 80,000, core
    10) start at their degree, so their search spans [k0, 80,000]: more than
    two binned passes, long rows walked by a whole workgroup, and values
    past the LDS cache's 16-bit offsets (those rows read every value from
    memory).  Random edges around them give the other vertices varied cores.
    Core numbers equal the oracle's (Definition 2) with the h-index phase
    from the first check and with levels only."""
    rng = np.random.default_rng(77)
    nU, nL = 100_000, 1_010
    hub_u = np.repeat(np.arange(80_000, dtype=np.int32), 10)
    hub_v = np.tile(np.arange(10, dtype=np.int32), 80_000)
    ru = rng.integers(80_000, nU, 300_000, dtype=np.int32)
    rv = rng.integers(10, nL, 300_000, dtype=np.int32)
    pairs = np.unique(np.stack([np.concatenate([hub_u, ru]), np.concatenate([hub_v, rv])], 1), axis=0)
    eu, ev = pairs[:, 0].copy(), pairs[:, 1].copy()
    g, ref = _make(nU, nL, eu, ev)
    want = oracle.core_numbers(ref)
    for switch in (1 << 30, 1):
        pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, switch)
        core, mx = pkg.abcore_core_numbers(g)
        top = pkg.abcore_graph_report(g)["core_top"]
        say(f"wide ranges, switch {switch}: {top}, max core {mx}")
        assert (top["vertices"] > 0) == (switch > 1), top
        assert np.array_equal(core.cpu().numpy(), want), switch
        assert mx == int(want.max())
        # a changed option drops the cached core numbers only with the graph;
        # rebuild for the second switch
        g.destroy()
        g, _ = _make(nU, nL, eu, ev)
    g.destroy()
