"""Debug build (libabcore_debug.so, per-vertex enqueue counters): every
vertex that Algorithm 1's peel removes passes through the frontier queues,
and the crossing rule (a vertex is queued when the decrement of its degree
returns exactly its threshold) queues it once.  Checked against the oracle's
removed set and scan frontier in every peel mode, with the first round pushed
and pulled, in vertex and rank order, with appends forced to overflow into
other sub-queues, and for the level peel of the core decomposition
(Definition 2), which queues every vertex exactly once.  Round counts are
logged.  Exceptions that the design allows, for rows split into 64-entry
pieces only: the round modes queue such a row that a cascade removes as its
pieces (no vertex item), and after a pull round it may be queued twice (by
its last decrement and by the start phase's test of its count; the second
copy walks nothing).  GCC+ queues a vertex at most twice."""
import numpy as np
import pytest

import bigraph_gen
import oracle
from tests.gpu_util import bits_np, ensure_built, say, to_dev

pytestmark = pytest.mark.gpu

SPLIT = 64  # entries per row piece: longer rows are split


def _graph():
    nU, nL, m = 30_000, 20_000, 400_000
    eu, ev = bigraph_gen.chung_lu(nU, nL, m, 2.1, 2.1, 5000, 110)
    return nU, nL, eu, ev


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()
    import paper_2606_07148_amd as p
    return p


def _by_vertex(cnt_by_rank, deg0, nU):
    n = len(deg0)
    ids = np.arange(n)
    rank_vtx = np.concatenate([
        np.lexsort((ids[:nU], -deg0[:nU])),
        nU + np.lexsort((ids[nU:] - nU, -deg0[nU:]))])
    out = np.zeros(n, cnt_by_rank.dtype)
    out[rank_vtx] = cnt_by_rank
    return out


def _gcc_counts_ok(pkg, g, ref, deg0, nU, a, b, tag):
    pkg.abcore_debug_enqueue_counts(g, reset=True)
    bits, st = pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC, stats=True)
    cnt = pkg.abcore_debug_enqueue_counts(g, reset=True).cpu().numpy()
    if st["rank_order"]:
        # queries in rank order queue global degree ranks (within a layer:
        # decreasing degree, then id; the lower layer's ranks follow nU)
        cnt = _by_vertex(cnt, deg0, nU)
    mem, ost = oracle.peel(ref, a, b)
    mem = np.asarray(mem, bool)
    want = oracle.pack(mem)
    assert np.array_equal(bits_np(bits)[: len(want)], want), f"{tag} ({a},{b}) bitmask"
    thr = np.where(np.arange(len(deg0)) < nU, a, b)
    f0 = deg0 < thr
    split = deg0 > SPLIT
    removed = ~mem
    say(f"debug {tag} ({a},{b}): rounds {st['rounds']} (oracle {ost['rounds']}), "
        f"pulled {st['pulled']}, queued {int(cnt.sum())}, removed {int(removed.sum())}")
    assert not cnt[mem].any(), f"{tag} ({a},{b}): a member was queued"
    # every later removal of a row that is not split: queued exactly once
    later = removed & ~f0 & ~split
    assert (cnt[later] == 1).all(), f"{tag} ({a},{b}): counts {np.bincount(cnt[later])}"
    # the scan frontier: queued by the scan, except when the asynchronous
    # peel's pull round counts it out of the surviving rows instead
    f0_want = 0 if (st["pulled"] and st["rounds"] < 0) else 1
    assert (cnt[f0] == f0_want).all(), f"{tag} ({a},{b}): scan frontier"
    # a split row that crosses later: as its pieces (round modes, 0), as a
    # vertex (1), or twice after a pull round (the second copy walks nothing)
    assert (cnt[split & removed & ~f0] <= 2).all(), f"{tag} ({a},{b}): split row"
    if not st["pulled"]:
        assert (cnt[split & removed & ~f0] <= 1).all(), f"{tag} ({a},{b}): pushed split row"


@pytest.mark.parametrize("peel,pull,rank,overflow", [
    (3, 1, 2, False), (3, 2, 2, False), (3, 0, 1, False), (2, 0, 2, False),
    (1, 1, 2, False), (1, 2, 2, False), (3, 2, 2, True), (3, 1, 2, True)])
def test_gcc_queues_each_removal_once(pkg, peel, pull, rank, overflow):
    nU, nL, eu, ev = _graph()
    ref = oracle.Graph(nU, nL, eu, ev)
    deg0 = np.diff(np.asarray(ref.off, np.int64))
    with pkg.debug_library():
        g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
        try:
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, peel)
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_PULL, pull)
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_RANK_ORDER, rank)
            if overflow:
                pkg.abcore_set_option(g, pkg.ABCORE_OPT_APPEND_SUBQUEUE, 1)
            tag = f"peel {peel} pull {pull} rank {rank}" + (" overflow" if overflow else "")
            for a, b in [(2, 2), (5, 5), (3, 9), (9, 3), (20, 20), (64, 64)]:
                _gcc_counts_ok(pkg, g, ref, deg0, nU, a, b, tag)
            # GCC+: at most twice (uncertain list, then frontier); its core
            # numbers first (the level peel queues every vertex once more)
            pkg.abcore_core_numbers(g)
            for a, b in [(3, 9), (9, 3), (5, 20)]:
                pkg.abcore_debug_enqueue_counts(g, reset=True)
                pkg.abcore_compute(g, a, b, pkg.ABCORE_GCC_PLUS)
                cnt = pkg.abcore_debug_enqueue_counts(g, reset=True).cpu().numpy()
                assert (cnt <= 2).all(), f"{tag} GCC+ ({a},{b})"
        finally:
            g.destroy()


@pytest.mark.parametrize("peel", [3, 1, 2])
def test_level_peel_queues_every_vertex_once(pkg, peel):
    nU, nL, eu, ev = _graph()
    ref = oracle.Graph(nU, nL, eu, ev)
    with pkg.debug_library():
        g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
        try:
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_PEEL_MODE, peel)
            pkg.abcore_set_option(g, pkg.ABCORE_OPT_KCORE_SWITCH, 1)  # levels only
            pkg.abcore_debug_enqueue_counts(g, reset=True)
            core, mx = pkg.abcore_core_numbers(g)
            cnt = pkg.abcore_debug_enqueue_counts(g, reset=True).cpu().numpy()
            assert np.array_equal(core.cpu().numpy(), oracle.core_numbers(ref))
            say(f"debug core numbers, peel mode {peel}: max core {mx}, queued {int(cnt.sum())}")
            # every vertex exactly once, except that the round modes queue a
            # split row that a cascade removes as its pieces only
            deg0 = np.diff(np.asarray(ref.off, np.int64))
            split = deg0 > SPLIT
            assert (cnt[~split] == 1).all(), f"peel mode {peel}: counts {np.bincount(cnt)}"
            assert (cnt[split] == 1).all() if peel == 3 else (cnt[split] <= 1).all()
        finally:
            g.destroy()


def test_release_library_keeps_no_counts(pkg):
    nU, nL, eu, ev = _graph()
    g = pkg.abcore_build_csr(nU, nL, to_dev(eu), to_dev(ev))
    with pytest.raises(pkg.AbcoreError) as e:
        pkg.abcore_debug_enqueue_counts(g)
    assert e.value.name == "EINVAL"
    g.destroy()
