"""Brute-force definitions used to pin the oracle on tiny graphs.

These enumerate vertex subsets directly from Definition 1 and Definition 2 of
the paper; they are exponential and only run for n <= 14.
"""
from __future__ import annotations


def adjacency_masks(n_upper, n_lower, edges):
    n = n_upper + n_lower
    adj = [0] * n
    for u, v in edges:
        adj[u] |= 1 << (n_upper + v)
        adj[n_upper + v] |= 1 << u
    return adj


def feasible(S, adj, n_upper, alpha, beta):
    """Every upper member has >= alpha neighbours in S, lower >= beta."""
    x = S
    while x:
        low = x & -x
        i = low.bit_length() - 1
        thr = alpha if i < n_upper else beta
        if bin(adj[i] & S).count("1") < thr:
            return False
        x ^= low
    return True


def core_by_enumeration(n_upper, n_lower, edges, alpha, beta):
    """Definition 1: the union of all feasible vertex subsets (feasibility is
    closed under union, so the union is the unique maximal one)."""
    n = n_upper + n_lower
    adj = adjacency_masks(n_upper, n_lower, edges)
    union = 0
    for S in range(1, 1 << n):
        if S | union == union:
            continue  # adds nothing new
        if feasible(S, adj, n_upper, alpha, beta):
            union |= S
    return [bool(union >> i & 1) for i in range(n)]


def core_numbers_by_enumeration(n_upper, n_lower, edges):
    """Definition 2: largest delta with the vertex in the (delta,delta)-core."""
    n = n_upper + n_lower
    core = [0] * n
    delta = 1
    while True:
        mem = core_by_enumeration(n_upper, n_lower, edges, delta, delta)
        if not any(mem):
            return core
        for i in range(n):
            if mem[i]:
                core[i] = delta
        delta += 1


def connected_core_by_enumeration(n_upper, n_lower, edges, alpha, beta, q):
    """Union of every vertex set S that contains q, induces a connected
    subgraph and gives each upper vertex >= alpha and each lower vertex >=
    beta neighbours inside S.  The union of such sets is itself one (it is
    connected through q and keeps every degree), so it is the maximal
    connected (alpha,beta)-subgraph containing q (empty if there is none)."""
    import itertools
    n = n_upper + n_lower
    adj = [set() for _ in range(n)]
    for u, v in edges:
        adj[u].add(n_upper + v)
        adj[n_upper + v].add(u)
    best = set()
    others = [x for x in range(n) if x != q]
    for r in range(len(others) + 1):
        for comb in itertools.combinations(others, r):
            S = set(comb) | {q}
            if any(len(adj[x] & S) < (alpha if x < n_upper else beta) for x in S):
                continue
            seen, stack = {q}, [q]
            while stack:
                x = stack.pop()
                for w in adj[x] & S:
                    if w not in seen:
                        seen.add(w)
                        stack.append(w)
            if seen == S:
                best |= S
    return best
