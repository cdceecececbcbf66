"""The multithreaded CPU peel (the host comparison point) equals the oracle
bit for bit, with one and with several threads, and its round count equals
the oracle's FIFO generations (both peel the same frontiers)."""
import numpy as np
import pytest

import bigraph_gen
import cpu_peel
import oracle


@pytest.mark.parametrize("spec", [bigraph_gen.CONFIGS[1], bigraph_gen.scaled(2, 0.01),
                                  bigraph_gen.scaled(3, 1 / 2000)])
def test_cpu_peel_equals_oracle(spec):
    eu, ev = bigraph_gen.make_graph(spec)
    g = oracle.Graph(spec["n_upper"], spec["n_lower"], eu, ev)
    for a, b in [(1, 1), (3, 2), (2, 7), (10, 10), (40, 6), (10 ** 6, 1)]:
        want, st = oracle.peel(g, a, b)
        for threads in (1, 4, 0):
            got, rounds = cpu_peel.peel(g.n_upper, g.n_lower, g.off, g.cols, a, b, threads)
            assert np.array_equal(got, want), (a, b, threads)
            assert rounds == st["rounds"], (a, b, threads)
