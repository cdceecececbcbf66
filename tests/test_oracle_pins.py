"""Pins for the CPU oracle: checks against the paper's stated facts, brute
force from the definitions, closed forms, library routines and invariants.
None of these call the oracle twice to agree with itself."""
import itertools
import json
import os

import networkx as nx
import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.bruteforce import core_by_enumeration, core_numbers_by_enumeration

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _name_to_id(name, n_upper):
    return int(name[1:]) if name[0] == "u" else n_upper + int(name[1:])


def _random_tiny(rng, max_n=12):
    nU = int(rng.integers(1, 7))
    nL = int(rng.integers(1, max(2, max_n - nU + 1)))
    nL = min(nL, max_n - nU)
    pairs = [(u, v) for u in range(nU) for v in range(nL)]
    p = rng.uniform(0.15, 0.85)
    edges = [e for e in pairs if rng.random() < p]
    return nU, nL, edges


def _graph(nU, nL, edges):
    eu = np.array([e[0] for e in edges], np.int32)
    ev = np.array([e[1] for e in edges], np.int32)
    return oracle.Graph(nU, nL, eu, ev)


def _nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for x in range(g.n):
        for j in range(g.off[x], g.off[x + 1]):
            G.add_edge(x, int(g.cols[j]))
    return G


# ---------------------------------------------------------------- worked example


def test_worked_example_facts():
    fx = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    nU, nL = fx["n_upper"], fx["n_lower"]
    g = _graph(nU, nL, fx["edges"])
    for fact in fx["facts"]:
        k = fact["kind"]
        if k == "size":
            assert g.n == fact["n"] and g.m == fact["m"], fact["cite"]
        elif k == "core":
            mem = oracle.compute(g, fact["alpha"], fact["beta"])
            want = {_name_to_id(s, nU) for s in fact["members"]}
            assert set(np.flatnonzero(mem).tolist()) == want, fact["cite"]
        elif k == "first_round":
            deg = g.degrees()
            thr = np.where(np.arange(g.n) < nU, fact["alpha"], fact["beta"])
            want = {_name_to_id(s, nU) for s in fact["removed"]}
            assert set(np.flatnonzero(deg < thr).tolist()) == want, fact["cite"]
        elif k == "core_numbers":
            core = oracle.core_numbers(g)
            for name, val in fact["values"].items():
                assert core[_name_to_id(name, nU)] == val, (fact["cite"], name)
        elif k == "degree":
            assert g.degrees()[_name_to_id(fact["vertex"], nU)] == fact["degree"], fact["cite"]
        elif k == "query":
            up = fact["update"]
            upd = {key: np.array([val]) for key, val in up.items()}
            upd["alpha"] = np.array([fact["alpha"]])
            upd["beta"] = np.array([fact["beta"]])
            eu, ev = g.edges()
            res = oracle.gfq_stream(nU, nL, eu, ev, upd)
            assert res[0][0] == "OK" and res[0][1] == fact["answer"], fact["cite"]
            g2 = _graph(nU, nL, fx["edges"] + [[up["u"], up["v"]]])
            assert g2.degrees()[nU + up["v"]] == fact["degree_after"], fact["cite"]
        else:
            raise AssertionError(k)


def test_counterexample_literal_alg2():
    """Reading of Algorithm 2: uncertain vertices must count only neighbours
    with core number >= delta_l.  The literal procedure (whole-graph degrees)
    is reproduced here to show it disagrees with Definition 1."""
    fx = json.load(open(os.path.join(GOLDEN, "counterexample_alg2.json")))
    nU, nL = fx["n_upper"], fx["n_lower"]
    g = _graph(nU, nL, fx["edges"])
    a, b = fx["alpha"], fx["beta"]
    assert oracle.core_numbers(g).tolist() == fx["core_numbers"]
    mem = oracle.compute(g, a, b)
    assert np.flatnonzero(mem).tolist() == fx["core_members"]
    assert core_by_enumeration(nU, nL, [tuple(e) for e in fx["edges"]], a, b) == [False] * g.n
    # literal Algorithm 2 (for contrast): whole-graph degrees for uncertain vertices
    assert _literal_alg2(g, a, b) == fx["literal_alg2_members"]
    assert _restricted_alg2(g, a, b) == fx["core_members"]


def _literal_alg2(g, a, b):
    core = oracle.core_numbers(g)
    lo, hi = min(a, b), max(a, b)
    deg = g.degrees().astype(int).copy()
    thr = [a if x < g.n_upper else b for x in range(g.n)]
    unc = [lo <= core[x] < hi for x in range(g.n)]
    removed = [False] * g.n
    queue = [x for x in range(g.n) if unc[x] and deg[x] < thr[x]]
    for x in queue:
        removed[x] = True
    while queue:
        x = queue.pop()
        for j in range(g.off[x], g.off[x + 1]):
            w = int(g.cols[j])
            if unc[w] and not removed[w]:
                deg[w] -= 1
                if deg[w] < thr[w]:
                    removed[w] = True
                    queue.append(w)
    return [x for x in range(g.n) if core[x] >= lo and not removed[x]]


def _restricted_alg2(g, a, b):
    """Algorithm 2 inside G[{core >= delta_l}] (the reading the library uses)."""
    core = oracle.core_numbers(g)
    lo, hi = min(a, b), max(a, b)
    thr = [a if x < g.n_upper else b for x in range(g.n)]
    unc = [lo <= core[x] < hi for x in range(g.n)]
    deg = [sum(1 for j in range(g.off[x], g.off[x + 1]) if core[g.cols[j]] >= lo)
           for x in range(g.n)]
    removed = [False] * g.n
    queue = [x for x in range(g.n) if unc[x] and deg[x] < thr[x]]
    for x in queue:
        removed[x] = True
    while queue:
        x = queue.pop()
        for j in range(g.off[x], g.off[x + 1]):
            w = int(g.cols[j])
            if unc[w] and not removed[w]:
                deg[w] -= 1
                if deg[w] < thr[w]:
                    removed[w] = True
                    queue.append(w)
    return [x for x in range(g.n) if core[x] >= hi or (unc[x] and not removed[x])]


def test_restricted_alg2_matches_definition_on_random_graphs():
    rng = np.random.default_rng(7)
    for _ in range(150):
        nU, nL, edges = _random_tiny(rng, 11)
        g = _graph(nU, nL, edges)
        for a, b in [(1, 2), (2, 1), (2, 3), (3, 2), (1, 3), (3, 3)]:
            mem = oracle.compute(g, a, b)
            assert _restricted_alg2(g, a, b) == np.flatnonzero(mem).tolist()


# ---------------------------------------------------------------- brute force


def test_peel_equals_enumeration_tiny():
    rng = np.random.default_rng(1)
    for _ in range(120):
        nU, nL, edges = _random_tiny(rng, 12)
        g = _graph(nU, nL, edges)
        for a, b in [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (1, 3), (2, 3), (3, 2), (4, 2)]:
            want = core_by_enumeration(nU, nL, edges, a, b)
            got = oracle.compute(g, a, b).tolist()
            assert got == want, (nU, nL, edges, a, b)


def test_core_numbers_equal_enumeration_tiny():
    rng = np.random.default_rng(2)
    for _ in range(60):
        nU, nL, edges = _random_tiny(rng, 11)
        g = _graph(nU, nL, edges)
        assert oracle.core_numbers(g).tolist() == core_numbers_by_enumeration(nU, nL, edges)


# ---------------------------------------------------------------- closed forms


def _medium_graph(seed, nU=300, nL=200, m=1500):
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 120, seed)
    return oracle.Graph(nU, nL, eu, ev)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_closed_forms(seed):
    g = _medium_graph(seed)
    deg = g.degrees()
    nU = g.n_upper
    # (1,1)-core = the non-isolated vertices
    assert (oracle.compute(g, 1, 1) == (deg > 0)).all()
    for a in [2, 3, 5, 9]:
        # (a,1)-core = {u: deg(u) >= a} plus every lower neighbour of such u
        want = np.zeros(g.n, bool)
        big = np.flatnonzero(deg[:nU] >= a)
        want[big] = True
        for u in big:
            want[g.cols[g.off[u]:g.off[u + 1]]] = True
        assert (oracle.compute(g, a, 1) == want).all()
        # (1,b)-core symmetric
        want = np.zeros(g.n, bool)
        big = nU + np.flatnonzero(deg[nU:] >= a)
        want[big] = True
        for v in big:
            want[g.cols[g.off[v]:g.off[v + 1]]] = True
        assert (oracle.compute(g, 1, a) == want).all()
    # alpha above the largest upper degree empties the core (beta >= 1)
    assert not oracle.compute(g, int(deg[:nU].max()) + 1, 1).any()
    assert not oracle.compute(g, 1, int(deg[nU:].max()) + 1).any()


@pytest.mark.parametrize("seed", [21, 22])
def test_kk_core_and_core_numbers_match_networkx(seed):
    g = _medium_graph(seed, 400, 300, 2500)
    G = _nx_graph(g)
    cn = nx.core_number(G)
    core = oracle.core_numbers(g)
    assert all(core[x] == cn[x] for x in range(g.n))
    for k in range(1, max(cn.values()) + 2):
        want = set(nx.k_core(G, k).nodes)
        got = set(np.flatnonzero(oracle.compute(g, k, k)).tolist())
        assert got == want, k
        # {core >= k} is the (k,k)-core
        assert set(np.flatnonzero(core >= k).tolist()) == want


def test_components_match_networkx():
    g = _medium_graph(31, 500, 500, 700)  # sparse: many components
    comp = oracle.components(g)
    G = _nx_graph(g)
    parts = list(nx.connected_components(G))
    assert len(parts) > 5
    for part in parts:
        lab = min(part)
        assert all(comp[x] == lab for x in part)


# ---------------------------------------------------------------- invariants


@pytest.mark.parametrize("seed", [41, 42])
def test_feasibility_nesting_and_lemma1(seed):
    g = _medium_graph(seed, 600, 400, 5000)
    nU = g.n_upper
    core = oracle.core_numbers(g)
    prev = {}
    for a in range(1, 9):
        for b in range(1, 9):
            mem, st = oracle.peel(g, a, b)
            # feasibility: every survivor meets its threshold among survivors
            for x in np.flatnonzero(mem):
                nb = g.cols[g.off[x]:g.off[x + 1]]
                assert mem[nb].sum() >= (a if x < nU else b)
            # nested property: raising alpha or beta can only shrink the core
            if (a - 1, b) in prev:
                assert not (mem & ~prev[(a - 1, b)]).any()
            if (a, b - 1) in prev:
                assert not (mem & ~prev[(a, b - 1)]).any()
            prev[(a, b)] = mem
            # Lemma 1 (Sec. IV-B)
            lo, hi = min(a, b), max(a, b)
            assert not mem[core < lo].any()
            assert mem[core >= hi].all()
            # stats: removed count, degree sum of removed, peeled edges
            deg = g.degrees()
            assert st["removed"] == int((~mem).sum())
            assert st["removed_degree_sum"] == int(deg[~mem].sum())
            eu, ev = g.edges()
            inside = mem[eu] & mem[nU + ev]
            assert st["m_peeled"] == g.m - int(inside.sum())


def test_rounds_on_path():
    """A path u0-v0-u1-v1-...: under (2,2) the two ends peel inwards one vertex
    per side per round, so a path of L vertices takes ceil(L / 2) rounds."""
    for L in [2, 3, 7, 10, 31]:
        nU = (L + 1) // 2
        nL = L // 2
        edges = []
        for i in range(L - 1):
            a, b = i, i + 1  # path positions; even = upper, odd = lower
            u = (a if a % 2 == 0 else b) // 2
            v = (b if b % 2 == 1 else a) // 2
            edges.append((u, v))
        g = _graph(nU, nL, edges)
        mem, st = oracle.peel(g, 2, 2)
        assert not mem.any()
        assert st["rounds"] == (L + 1) // 2


# ---------------------------------------------------------------- CSR, bitmask


def test_csr_against_set_construction():
    rng = np.random.default_rng(5)
    nU, nL = 37, 53
    eu = rng.integers(0, nU, 900).astype(np.int32)
    ev = rng.integers(0, nL, 900).astype(np.int32)  # with duplicates, unsorted
    g = oracle.Graph(nU, nL, eu, ev)
    pairs = sorted(set(zip(eu.tolist(), ev.tolist())))
    assert g.m == len(pairs)
    for u in range(nU):
        row = g.cols[g.off[u]:g.off[u + 1]].tolist()
        assert row == sorted(nU + v for (a, v) in pairs if a == u)
    for v in range(nL):
        row = g.cols[g.off[nU + v]:g.off[nU + v + 1]].tolist()
        assert row == sorted(a for (a, b) in pairs if b == v)
    with pytest.raises(ValueError):
        oracle.Graph(nU, nL, np.array([nU], np.int32), np.array([0], np.int32))


def test_pack_layout():
    rng = np.random.default_rng(3)
    for n in [0, 1, 31, 32, 33, 95, 1000]:
        mem = rng.random(n) < 0.4
        words = oracle.pack(mem)
        assert len(words) == (n + 31) // 32
        for x in range(len(words) * 32):
            bit = (int(words[x // 32]) >> (x % 32)) & 1
            assert bit == (int(mem[x]) if x < n else 0)
        assert (oracle.unpack(words, n) == mem).all()


# ---------------------------------------------------------------- GFQ oracle


def test_gfq_stream_against_enumeration_and_monotonicity():
    rng = np.random.default_rng(9)
    for trial in range(25):
        nU, nL, edges = _random_tiny(rng, 11)
        present = set(edges)
        ups = {k: [] for k in ("u", "v", "op", "alpha", "beta")}
        cur = set(present)
        for _ in range(8):
            u = int(rng.integers(0, nU))
            v = int(rng.integers(0, nL))
            op = -1 if (u, v) in cur and rng.random() < 0.5 else 1
            if op == 1 and (u, v) in cur:
                op = -1
            (cur.discard if op < 0 else cur.add)((u, v))
            for k, val in zip(ups, (u, v, op, int(rng.integers(1, 4)), int(rng.integers(1, 4)))):
                ups[k].append(val)
        ups = {k: np.array(v) for k, v in ups.items()}
        eu = np.array([e[0] for e in edges], np.int32)
        ev = np.array([e[1] for e in edges], np.int32)
        res = oracle.gfq_stream(nU, nL, eu, ev, ups)
        cur = set(present)
        for i, (status, ans, bits) in enumerate(res):
            u, v, op = int(ups["u"][i]), int(ups["v"][i]), int(ups["op"][i])
            a, b = int(ups["alpha"][i]), int(ups["beta"][i])
            assert status == "OK"
            before = core_by_enumeration(nU, nL, sorted(cur), a, b)
            (cur.discard if op < 0 else cur.add)((u, v))
            after = core_by_enumeration(nU, nL, sorted(cur), a, b)
            assert ans == (after[u] and after[nU + v])
            assert bits == int(after[u]) | (int(after[nU + v]) << 1)
            # an insertion can only grow the core, a deletion only shrink it
            if op > 0:
                assert all(y or not x for x, y in zip(before, after))
            else:
                assert all(x or not y for x, y in zip(before, after))


def test_gfq_rejects_duplicate_insert_and_absent_delete():
    eu = np.array([0, 1], np.int32)
    ev = np.array([0, 0], np.int32)
    ups = dict(u=np.array([0, 0, 1]), v=np.array([0, 1, 1]), op=np.array([1, -1, 1]),
               alpha=np.array([1, 1, 1]), beta=np.array([1, 1, 1]))
    res = oracle.gfq_stream(2, 2, eu, ev, ups)
    assert [r[0] for r in res] == ["EEXIST", "ENOENT", "OK"]


def test_component_decomposition():
    """The core of G is the union of the cores of its connected components."""
    g = _medium_graph(51, 800, 800, 1200)
    comp = oracle.components(g)
    eu, ev = g.edges()
    for a, b in [(2, 2), (1, 3), (3, 1)]:
        whole = oracle.compute(g, a, b)
        union = np.zeros(g.n, bool)
        for c in np.unique(comp):
            keep = comp[eu] == c
            if not keep.any():
                continue
            sub = oracle.Graph(g.n_upper, g.n_lower, eu[keep], ev[keep])
            mem = oracle.compute(sub, a, b)
            union |= mem & (comp == c)
        assert (union == whole).all()


def _certify(g, mem, order, a, b):
    """Definition 1 certificate, computed here from the CSR alone: the
    survivors form an (a,b)-subgraph (feasibility), and the removed vertices,
    taken in the peel's order, each had fewer than its threshold of
    neighbours not removed before it -- so by induction along the order no
    removed vertex belongs to any (a,b)-subgraph, and the survivors are the
    maximal one."""
    n, nU = g.n, g.n_upper
    thr = np.where(np.arange(n) < nU, a, b)
    deg = g.degrees()
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = g.cols.astype(np.int64)
    assert len(order) == int((~mem).sum())
    assert len(np.unique(order)) == len(order)
    assert not mem[order].any()
    pos = np.full(n, np.iinfo(np.int64).max, np.int64)
    pos[order] = np.arange(len(order))
    later = pos[cols] > pos[rows]
    left = np.bincount(rows[later], minlength=n)
    removed = ~mem
    assert (left[removed] < thr[removed]).all(), "a removed vertex kept its threshold"
    inside = np.bincount(rows[mem[cols] & mem[rows]], minlength=n)
    assert (inside[mem] >= thr[mem]).all(), "a survivor lacks its threshold"


@pytest.mark.parametrize("which", ["uniform", "chung_lu_2", "chung_lu_3"])
def test_removal_order_certificate(which):
    """Maximality pinned in O(m): the oracle's removal order certifies its
    result on medium graphs of each workload shape, over a grid of queries
    including asymmetric ones and an empty core."""
    if which == "uniform":
        spec = bigraph_gen.CONFIGS[1]
    elif which == "chung_lu_2":
        spec = bigraph_gen.scaled(2, 0.01)
    else:
        spec = bigraph_gen.scaled(3, 1 / 2000)
    eu, ev = bigraph_gen.make_graph(spec)
    g = oracle.Graph(spec["n_upper"], spec["n_lower"], eu, ev)
    for a, b in [(1, 1), (3, 2), (2, 7), (10, 10), (40, 6), (100, 2), (10 ** 6, 1)]:
        mem, st, order = oracle.peel_order(g, a, b)
        assert np.array_equal(mem, oracle.compute(g, a, b))
        _certify(g, mem, order, a, b)


def test_certificate_rejects_planted_mistakes():
    """The certificate catches a wrong result: a dropped removal (a vertex
    kept that lacks support), an extra removal (a vertex removed that kept
    its threshold), and a swapped order."""
    spec = bigraph_gen.scaled(2, 0.01)
    eu, ev = bigraph_gen.make_graph(spec)
    g = oracle.Graph(spec["n_upper"], spec["n_lower"], eu, ev)
    a, b = 10, 10
    mem, st, order = oracle.peel_order(g, a, b)
    assert st["rounds"] >= 3  # the last removals had their threshold at the start
    _certify(g, mem, order, a, b)
    # the last removal undone: that vertex is kept without its support
    bad = mem.copy()
    bad[order[-1]] = True
    with pytest.raises(AssertionError):
        _certify(g, bad, order[:-1], a, b)
    # a survivor with neighbours inside removed first: it kept its threshold
    x = int(np.flatnonzero(mem)[0])
    bad = mem.copy()
    bad[x] = False
    with pytest.raises(AssertionError):
        _certify(g, bad, np.concatenate([[x], order]), a, b)
    # the first and last removals exchanged: a late vertex removed too early
    rev = order[::-1].copy()
    with pytest.raises(AssertionError):
        _certify(g, mem, rev, a, b)


def test_community_equals_enumeration_tiny():
    """Localized community search (Remark of Sec. V), both readings, against
    enumeration on tiny graphs: the connected reading is the maximal
    connected (alpha,beta)-subgraph containing q (brute force over vertex
    sets); the component reading is Definition 1's core (brute force)
    inside q's connected component (networkx)."""
    from tests.bruteforce import connected_core_by_enumeration
    rng = np.random.default_rng(77)
    checked = 0
    for _ in range(120):
        nU, nL, edges = _random_tiny(rng, max_n=11)
        g = _graph(nU, nL, edges)
        a, b = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        core = np.array(core_by_enumeration(nU, nL, edges, a, b))
        comps = list(nx.connected_components(_nx_graph(g)))
        for q in range(g.n):
            want_conn = connected_core_by_enumeration(nU, nL, edges, a, b, q)
            got_conn = oracle.community(g, q, a, b, connected=True)
            assert set(np.flatnonzero(got_conn).tolist()) == want_conn
            cq = next(c for c in comps if q in c)
            want_comp = {x for x in cq if core[x]}
            got_comp = oracle.community(g, q, a, b, connected=False)
            assert set(np.flatnonzero(got_comp).tolist()) == want_comp
            checked += len(want_conn) > 0
    assert checked > 50


def test_community_on_worked_example():
    """The worked example's (1,3)-core is {u0..u7, v0, v1, v2, v4}.  The
    fixture has two components (the K_{4,3} block and the rest), so the
    component reading splits the core between them, and the (2,3)-core
    K_{4,3} is one connected community."""
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "worked_example.json")))
    nU = fx["n_upper"]
    g = _graph(nU, fx["n_lower"], [tuple(e) for e in fx["edges"]])
    cores = {(f["alpha"], f["beta"]): {_name_to_id(s, nU) for s in f["members"]}
             for f in fx["facts"] if f["kind"] == "core"}
    want13 = cores[(1, 3)]
    block = {_name_to_id(s, nU) for s in ("u0", "u1", "u2", "u3", "v0", "v1", "v2")}
    a = set(np.flatnonzero(oracle.community(g, 0, 1, 3, connected=False)).tolist())
    b = set(np.flatnonzero(oracle.community(g, _name_to_id("u4", nU), 1, 3,
                                            connected=False)).tolist())
    assert a == want13 & block and b == want13 - block and a | b == want13
    want23 = cores[(2, 3)]
    for q in want23:
        got = oracle.community(g, q, 2, 3, connected=True)
        assert set(np.flatnonzero(got).tolist()) == want23
    # a vertex outside the core has an empty connected community
    assert not oracle.community(g, _name_to_id("u7", nU), 2, 3, connected=True).any()


def test_gfq_set_equals_community_after_update():
    """The GFQ set variant after each update equals the community search on
    the updated graph around its endpoints (both readings), and its endpoint
    membership equals gfq_stream's answer bits."""
    spec = bigraph_gen.CONFIGS[1]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 12, 4242)
    nU, nL = spec["n_upper"], spec["n_lower"]
    for connected in (False, True):
        res = oracle.gfq_set_stream(nU, nL, eu, ev, ups, connected)
        ans = oracle.gfq_stream(nU, nL, eu, ev, ups)
        present = set(zip(eu.tolist(), ev.tolist()))
        for i, ((st, mem), (st2, a, bits)) in enumerate(zip(res, ans)):
            assert st == st2
            u, v, op = int(ups["u"][i]), int(ups["v"][i]), int(ups["op"][i])
            if op > 0:
                present.add((u, v))
            else:
                present.discard((u, v))
            if st != "OK":
                continue
            assert bool(mem[u]) == bool(bits & 1) and bool(mem[nU + v]) == bool(bits >> 1 & 1)
            if i % 4 == 0:
                pe = np.array(sorted(present), np.int32)
                g = oracle.Graph(nU, nL, pe[:, 0], pe[:, 1])
                al, be = int(ups["alpha"][i]), int(ups["beta"][i])
                want = (oracle.community(g, u, al, be, connected) |
                        oracle.community(g, nU + v, al, be, connected))
                assert np.array_equal(mem, want)


def test_offsets_and_delta_equal_enumeration_tiny():
    """alpha_offset (Sec. VI-B) and delta (Table I) against Definition 1 by
    enumeration: the largest beta whose brute-force core is non-empty, and
    the largest symmetric one; delta also equals the maximum core number
    (Definition 2)."""
    rng = np.random.default_rng(91)
    for _ in range(60):
        nU, nL, edges = _random_tiny(rng, max_n=10)
        g = _graph(nU, nL, edges)
        for a in (1, 2, 3):
            want = 0
            for b in range(1, nU + 2):
                if any(core_by_enumeration(nU, nL, edges, a, b)):
                    want = b
            assert oracle.alpha_offset(g, a) == want
        want_d = max([d for d in range(1, nU + nL + 1)
                      if any(core_by_enumeration(nU, nL, edges, d, d))] or [0])
        assert oracle.delta(g) == want_d
        assert want_d == (int(oracle.core_numbers(g).max()) if g.n else 0)


def test_default_query_on_worked_example():
    """On the worked example delta = 3 (the K_{4,3} block's core number), so
    alpha = floor(1.2) = 1; the (1,beta)-core is non-empty up to beta = 4
    (u0..u3 keep v0..v2 at degree 4, and the star around v4 has degree 4),
    so alpha_offset(1) = 4 and beta = floor(2.4) = 2.  In K_{4,3} each upper
    vertex has degree 3 and each lower vertex 4, so alpha_offset(3) = 4; no
    upper vertex has degree 4, so alpha_offset(4) = 0."""
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "worked_example.json")))
    g = _graph(fx["n_upper"], fx["n_lower"], [tuple(e) for e in fx["edges"]])
    assert oracle.delta(g) == 3
    assert oracle.alpha_offset(g, 1) == 4
    assert oracle.alpha_offset(g, 3) == 4
    assert oracle.alpha_offset(g, 4) == 0
    assert oracle.default_query(g) == (1, 2)


def test_core_maintenance_property_on_streams():
    """The fact behind stale core-number pruning in serving (beyond the
    paper; the k-core maintenance property of Li, Yu and Mao, and Sariyuce et
    al.): inserting or deleting edge (u, v) changes only core numbers equal
    to K = min(core(u), core(v)) before the update, each by exactly one, up
    for an insertion and down for a deletion.  Checked with the oracle's
    core numbers (Definition 2) before and after every update of streams on
    power-law and uniform graphs."""
    for spec in (bigraph_gen.scaled(2, 0.002), bigraph_gen.CONFIGS[1]):
        nU, nL = spec["n_upper"], spec["n_lower"]
        eu, ev = bigraph_gen.make_graph(spec)
        ups = bigraph_gen.update_stream(spec, eu, ev, 60, 777)
        present = set(zip(eu.tolist(), ev.tolist()))
        g = oracle.Graph(nU, nL, eu, ev)
        before = oracle.core_numbers(g)
        changed_any = 0
        for i in range(len(ups["u"])):
            u, v, op = int(ups["u"][i]), int(ups["v"][i]), int(ups["op"][i])
            if (op > 0) == ((u, v) in present):
                continue  # rejected update
            k = min(int(before[u]), int(before[nU + v]))
            (present.add if op > 0 else present.discard)((u, v))
            pe = np.array(sorted(present), np.int32)
            after = oracle.core_numbers(oracle.Graph(nU, nL, pe[:, 0], pe[:, 1]))
            diff = after.astype(np.int64) - before
            moved = np.flatnonzero(diff)
            assert (before[moved] == k).all(), (i, k)
            assert (diff[moved] == (1 if op > 0 else -1)).all(), i
            changed_any += len(moved)
            before = after
        assert changed_any > 0
