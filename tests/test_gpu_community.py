"""GPU parity of the vertex-set variants of the Remark of Sec. V: localized
community search (abcore_community) and GFQ returning the core's vertex set
(abcore_query_set), both readings (the members in the query's component, and
the members connected to the query through members), against the oracle bit
for bit, on a graph of many small components, on the uniform workload and
on a power-law graph."""
import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.gpu_util import bits_np, ensure_built, say, to_dev

pytestmark = pytest.mark.gpu


def _graphs():
    yield "sparse", dict(kind="uniform", n_upper=3000, n_lower=2000, m=4200, seed=901)
    yield "uniform", bigraph_gen.CONFIGS[1]
    yield "power-law", bigraph_gen.scaled(2, 0.01)


@pytest.mark.parametrize("name,spec", list(_graphs()))
def test_community_matches_oracle(name, spec):
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ref = oracle.Graph(nU, nL, eu, ev)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    rng = np.random.default_rng(5)
    comp = oracle.components(ref)
    for (a, b) in [(1, 1), (2, 2), (3, 2), (2, 5)]:
        member = oracle.compute(ref, a, b)
        ins = np.flatnonzero(member)
        outs = np.flatnonzero(~member)
        qs = list(rng.choice(ins, min(4, len(ins)), replace=False)) if len(ins) else []
        qs += list(rng.choice(outs, min(2, len(outs)), replace=False)) if len(outs) else []
        for q in qs:
            for connected in (False, True):
                want = oracle.pack(oracle.community(ref, int(q), a, b, connected))
                bits, cnt = pkg.abcore_community(g, int(q), a, b, connected)
                got = bits_np(bits)[: len(want)]
                assert np.array_equal(got, want), (name, a, b, int(q), connected)
                assert cnt == int(oracle.unpack(want, ref.n).sum())
        say(f"community {name} ({a},{b}): {len(qs)} query vertices, "
            f"{len(np.unique(comp))} components")
    g.destroy()


@pytest.mark.parametrize("connected", [False, True])
def test_query_set_matches_oracle_stream(connected):
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    spec = dict(kind="uniform", n_upper=3000, n_lower=2000, m=4200, seed=901)
    nU, nL = spec["n_upper"], spec["n_lower"]
    eu, ev = bigraph_gen.make_graph(spec)
    ups = bigraph_gen.update_stream(spec, eu, ev, 40, 1901, qlo=1, qhi=3)
    want = oracle.gfq_set_stream(nU, nL, eu, ev, ups, connected)
    ans = oracle.gfq_stream(nU, nL, eu, ev, ups)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    for i in range(len(ups["u"])):
        try:
            a, bits, out, cnt = pkg.abcore_query_set(
                g, ups["u"][i], ups["v"][i], ups["op"][i], ups["alpha"][i], ups["beta"][i],
                connected)
        except pkg.AbcoreError as e:
            assert want[i][0] == e.name
            continue
        assert want[i][0] == "OK"
        assert (a, bits) == (ans[i][1], ans[i][2]), i
        w = oracle.pack(want[i][1])
        assert np.array_equal(bits_np(out)[: len(w)], w), i
        assert cnt == int(want[i][1].sum())
    # a static search after the updates sees the inserted edges and tombstones
    off, cols = pkg.abcore_export_csr(g)
    offn, colsn = off.cpu().numpy(), cols.cpu().numpy()
    uu = np.repeat(np.arange(nU, dtype=np.int32), np.diff(offn[: nU + 1]))
    vv = (colsn[: offn[nU]] - nU).astype(np.int32)
    ref = oracle.Graph(nU, nL, uu, vv)
    for q in (int(ups["u"][-1]), nU + int(ups["v"][-1]), 0):
        w = oracle.pack(oracle.community(ref, q, 2, 1, connected))
        bits, _ = pkg.abcore_community(g, q, 2, 1, connected)
        assert np.array_equal(bits_np(bits)[: len(w)], w), q
    g.destroy()


@pytest.mark.parametrize("which", ["uniform", "power-law", "worked"])
def test_offsets_delta_and_default_query_match_oracle(which):
    """alpha_offset, delta and the default query of Sec. VI-B against the
    oracle's plain sweeps."""
    import json
    import os
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    if which == "worked":
        fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                         "worked_example.json")))
        nU, nL = fx["n_upper"], fx["n_lower"]
        eu = np.array([e[0] for e in fx["edges"]], np.int32)
        ev = np.array([e[1] for e in fx["edges"]], np.int32)
    else:
        spec = bigraph_gen.CONFIGS[1] if which == "uniform" else bigraph_gen.scaled(2, 0.005)
        nU, nL = spec["n_upper"], spec["n_lower"]
        eu, ev = bigraph_gen.make_graph(spec)
    ref = oracle.Graph(nU, nL, eu, ev)
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    delta = oracle.delta(ref)
    alphas = sorted({1, 2, 3, max(1, delta // 2), delta, delta + 1, delta + 5})
    offs, d = pkg.abcore_alpha_offsets(g, alphas)
    assert d == delta
    assert offs == [oracle.alpha_offset(ref, a) for a in alphas], (alphas, offs)
    assert pkg.abcore_default_query(g) == oracle.default_query(ref)
    say(f"offsets {which}: delta {delta}, alphas {alphas} -> {offs}")
    g.destroy()
