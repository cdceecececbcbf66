"""The allocation-free entry point (abcore_compute_static) against
abcore_compute: the same GCC bitmask bit for bit, and both equal to the
oracle (Definition 1), on two calls in a row with the second graph smaller
than the first (the static working set keeps the last call's contents, so
the second call must start from a clean one), then again on the first graph.
A graph whose working set exceeds the static array is rejected."""
import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.gpu_util import bits_np, ensure_built, say, to_dev

pytestmark = pytest.mark.gpu


def test_static_matches_compute_and_oracle():
    import torch
    assert torch.cuda.is_available()
    ensure_built()
    import paper_2606_07148_amd as pkg
    graphs = []
    for f in (1.0, 0.05):
        spec = bigraph_gen.scaled(2, f)
        nU, nL = spec["n_upper"], spec["n_lower"]
        eu, ev = bigraph_gen.make_graph(spec)
        graphs.append((pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev)),
                       oracle.Graph(nU, nL, eu, ev)))
    queries = [(10, 10), (3, 17), (1, 1), (40, 6)]
    for rnd in range(2):
        for gi, (g, ref) in enumerate(graphs):
            for (a, b) in queries:
                say(f"no-alloc: round {rnd} graph {gi} (n={g.n}) ({a},{b})")
                want = oracle.pack(oracle.compute(ref, a, b))
                base = bits_np(pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC))[: len(want)]
                out = torch.full((g.nwords,), -1, dtype=torch.int32, device="cuda")
                pkg.abcore_compute_static(g, a, b, out)
                torch.cuda.synchronize()
                got = bits_np(out)[: len(want)]
                assert np.array_equal(got, base), f"static differs from compute ({a},{b})"
                assert np.array_equal(got, want), f"static differs from the oracle ({a},{b})"
    for g, _ in graphs:
        g.destroy()
    # too large for the static array (6,000,000 vertices): rejected, nothing
    # written
    spec = bigraph_gen.scaled(2, 4.0)
    eu, ev = bigraph_gen.make_graph(spec)
    g = pkg.abcore_build_csr(spec["n_upper"], spec["n_lower"], to_dev(eu), to_dev(ev))
    out = torch.full((g.nwords,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_compute_static(g, 10, 10, out)
    assert e.value.name == "EINVAL"
    torch.cuda.synchronize()
    assert bool((out == 7).all())
    g.destroy()
