"""Host logic of batched queries: the plan that abcore_compute_batch follows
(no device call).  Checked against the dominance order it must respect and
against brute-force parent choices."""
import ctypes
import random

import pytest

import paper_2606_07148_amd as pkg

EINVAL = 1


@pytest.fixture(scope="module", autouse=True)
def _lib():
    pkg.load()


def _check_plan(alphas, betas):
    q = len(alphas)
    parent, order, states = pkg.abcore_batch_plan(alphas, betas)
    assert sorted(order) == list(range(q))
    pos = {i: k for k, i in enumerate(order)}
    distinct = {(a, b) for a, b in zip(alphas, betas)}
    for i in range(q):
        p = parent[i]
        if p < 0:
            # a root dominates no other distinct query's thresholds from below
            assert not any(alphas[j] <= alphas[i] and betas[j] <= betas[i]
                           and (alphas[j], betas[j]) != (alphas[i], betas[i])
                           for j in range(q)), i
            continue
        assert pos[p] < pos[i], "parent runs first"
        assert alphas[p] <= alphas[i] and betas[p] <= betas[i], "parent is dominated"
        if (alphas[p], betas[p]) != (alphas[i], betas[i]):
            # the dominated distinct query with the largest alpha + beta
            best = max(alphas[j] + betas[j] for j in range(q)
                       if alphas[j] <= alphas[i] and betas[j] <= betas[i]
                       and (alphas[j], betas[j]) != (alphas[i], betas[i]))
            assert alphas[p] + betas[p] == best
        else:
            # equal queries copy the first of them, which itself is no copy
            assert parent[p] < 0 or (alphas[parent[p]], betas[parent[p]]) != (alphas[p], betas[p])
    assert 1 <= states <= len(distinct)
    return parent, order, states


def test_chain_needs_one_buffer():
    a = list(range(1, 33))
    parent, order, states = _check_plan(a, a)
    assert states == 1
    assert order == list(range(32))
    assert parent == [-1] + list(range(31))


def test_star_and_duplicates():
    alphas = [5, 1, 9, 1, 30, 9]
    betas = [5, 1, 2, 1, 1, 2]
    parent, order, states = _check_plan(alphas, betas)
    assert parent[3] == 1  # duplicate of (1,1)
    assert parent[5] == 2  # duplicate of (9,2)
    assert parent[1] == -1
    assert states == 2


def test_random_batches():
    rng = random.Random(7)
    for trial in range(30):
        q = rng.randint(1, 80)
        alphas = [int(2 ** rng.uniform(0, 8)) for _ in range(q)]
        betas = [int(2 ** rng.uniform(0, 8)) for _ in range(q)]
        if trial % 3 == 0:  # heavy duplication
            alphas = [x % 4 + 1 for x in alphas]
            betas = [x % 3 + 1 for x in betas]
        _check_plan(alphas, betas)


def test_incomparable_queries_are_roots():
    alphas = [1, 2, 3, 4]
    betas = [4, 3, 2, 1]
    parent, _, states = _check_plan(alphas, betas)
    assert parent == [-1, -1, -1, -1]
    assert states == 1  # each chain ends at once and frees its buffer


def test_plan_rejects_bad_arguments():
    lib = pkg.load()
    a = (ctypes.c_uint32 * 2)(1, 0)
    b = (ctypes.c_uint32 * 2)(1, 1)
    assert lib.abcore_batch_plan(a, b, 2, None, None, None) == EINVAL
    assert lib.abcore_batch_plan(a, b, -1, None, None, None) == EINVAL
    assert lib.abcore_batch_plan(None, b, 1, None, None, None) == EINVAL
    assert lib.abcore_batch_plan(a, b, 0, None, None, None) == 0
    assert lib.abcore_compute_batch(None, a, b, 1, None, None) == EINVAL
