"""CPU oracle for the (alpha,beta)-core method -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never calls it.

The arithmetic lives in ``abcore_oracle.c`` (plain sequential C, no shared
code with the device library); this module marshals arrays and adds the
compositions the paper defines in terms of those routines:

* ``compute``      -- Problem 1 (Sec. III): vertex set of the (alpha,beta)-core.
* ``core_numbers`` -- Definition 2.
* ``components``   -- connected components (Sec. V preprocessing).
* ``gfq_stream``   -- Problem 2 (Sec. III) / GFQ (Sec. V): after each edge
  update, membership of the updated edge's endpoints in the core of the
  updated graph, by full recomputation on that graph.
* ``community``    -- localized community search (Remark of Sec. V): the
  core around a query vertex.
* ``gfq_set_stream`` -- GFQ returning the core's vertex set around the updated
  edge (Remark of Sec. V), by recomputation.
* ``alpha_offset``, ``delta``, ``default_query`` -- the query parameters of
  Sec. VI-B (largest beta with a non-empty (alpha,beta)-core, largest
  non-empty symmetric core, and the default alpha = 0.4 delta, beta = 0.6
  alpha_offset).
* ``peel_order``   -- ``compute`` plus the sequential removal order (the
  certificate of maximality).
* ``gfq_stream_sampled`` -- ``gfq_stream`` at sampled indices of a stream on
  a graph too large for a Python edge set.
* ``pack``         -- the membership bitmask layout (bit x of word x // 32,
  least significant bit first; unified ids, lower vertex v is nU + v).

Every function here has a pin in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile ``abcore_oracle.c`` into ``liboracle.so`` (always recompiles)."""
    global _lib
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                    os.path.join(_HERE, "abcore_oracle.c"), "-o", tmp], check=True)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ABC_ORACLE_LIB: another build of the same source (the sanitizer test loads
    # one compiled with AddressSanitizer and UndefinedBehaviorSanitizer)
    path = os.environ.get("ABC_ORACLE_LIB", _LIB_PATH)
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.or_build_csr.restype = ctypes.c_int64
    lib.or_build_csr.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp]
    lib.or_peel.restype = ctypes.c_int
    lib.or_peel.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64,
                            ctypes.c_int64, vp, vp]
    lib.or_peel_order.restype = ctypes.c_int
    lib.or_peel_order.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64,
                                  ctypes.c_int64, vp, vp, vp]
    lib.or_core_numbers.restype = ctypes.c_int
    lib.or_core_numbers.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    lib.or_components.restype = ctypes.c_int
    lib.or_components.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Graph:
    """Host CSR of a bipartite graph in unified ids (upper first)."""

    def __init__(self, n_upper: int, n_lower: int, eu, ev):
        eu = np.ascontiguousarray(eu, np.int32)
        ev = np.ascontiguousarray(ev, np.int32)
        self.n_upper = int(n_upper)
        self.n_lower = int(n_lower)
        self.n = self.n_upper + self.n_lower
        self.off = np.zeros(self.n + 1, np.int64)
        cols = np.zeros(max(1, 2 * len(eu)), np.int32)
        md = _load().or_build_csr(self.n_upper, self.n_lower, len(eu), _ptr(eu), _ptr(ev),
                                  _ptr(self.off), _ptr(cols))
        if md < 0:
            raise ValueError("edge id out of range")
        self.m = int(md)
        self.cols = cols[: 2 * self.m].copy()

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)

    def edges(self):
        """Distinct edges as (upper index, lower index), sorted."""
        u = np.repeat(np.arange(self.n_upper, dtype=np.int32),
                      np.diff(self.off[: self.n_upper + 1]))
        v = self.cols[: self.m] - self.n_upper
        return u, v.astype(np.int32)


def peel(g: Graph, alpha: int, beta: int):
    """(alpha,beta)-core membership (bool per unified id) and peel stats."""
    member = np.zeros(max(1, g.n), np.uint8)
    st = np.zeros(4, np.int64)
    rc = _load().or_peel(g.n_upper, g.n_lower, _ptr(g.off), _ptr(g.cols), int(alpha),
                         int(beta), _ptr(member), _ptr(st))
    if rc != 0:
        raise MemoryError("oracle peel failed")
    stats = dict(removed=int(st[0]), removed_degree_sum=int(st[1]), m_peeled=int(st[2]),
                 rounds=int(st[3]))
    return member[: g.n].astype(bool), stats


def compute(g: Graph, alpha: int, beta: int) -> np.ndarray:
    return peel(g, alpha, beta)[0]


def peel_order(g: Graph, alpha: int, beta: int):
    """Like ``peel``, plus the removed vertices in the order the sequential
    peel marked them (int64[|R|]).  Each of them had fewer than its threshold
    of neighbours outside the earlier-removed ones when it was marked, which
    is what makes the result maximal (Definition 1)."""
    member = np.zeros(max(1, g.n), np.uint8)
    st = np.zeros(4, np.int64)
    order = np.zeros(max(1, g.n), np.int64)
    rc = _load().or_peel_order(g.n_upper, g.n_lower, _ptr(g.off), _ptr(g.cols), int(alpha),
                               int(beta), _ptr(member), _ptr(st), _ptr(order))
    if rc != 0:
        raise MemoryError("oracle peel failed")
    stats = dict(removed=int(st[0]), removed_degree_sum=int(st[1]), m_peeled=int(st[2]),
                 rounds=int(st[3]))
    return member[: g.n].astype(bool), stats, order[: stats["removed"]].copy()


def batch(g: Graph, alphas, betas) -> np.ndarray:
    """Bitmasks of several queries: one independent peel per query (the
    batch must equal the queries computed one at a time)."""
    return np.stack([pack(compute(g, a, b)) for a, b in zip(alphas, betas)])


def core_numbers(g: Graph) -> np.ndarray:
    core = np.zeros(max(1, g.n), np.int32)
    if _load().or_core_numbers(g.n_upper, g.n_lower, _ptr(g.off), _ptr(g.cols),
                               _ptr(core)) != 0:
        raise MemoryError("oracle core numbers failed")
    return core[: g.n]


def components(g: Graph) -> np.ndarray:
    comp = np.zeros(max(1, g.n), np.int32)
    if _load().or_components(g.n_upper, g.n_lower, _ptr(g.off), _ptr(g.cols),
                             _ptr(comp)) != 0:
        raise MemoryError("oracle components failed")
    return comp[: g.n]


def pack(member: np.ndarray) -> np.ndarray:
    """Membership bitmask: bit (x % 32) of word x // 32, LSB first, padding 0."""
    member = np.asarray(member, bool)
    nwords = (len(member) + 31) // 32
    bits = np.zeros(nwords * 32, np.uint8)
    bits[: len(member)] = member
    return np.packbits(bits, bitorder="little").view("<u4").astype(np.uint32)


def unpack(words: np.ndarray, n: int) -> np.ndarray:
    b = np.unpackbits(np.asarray(words, "<u4").view(np.uint8), bitorder="little")
    return b[:n].astype(bool)


def gfq_stream(n_upper: int, n_lower: int, eu, ev, updates, check_only=None):
    """GFQ by recomputation (Problem 2 of Sec. III; procedure of Sec. V).

    ``updates`` holds arrays u, v, op (+1 insert, -1 delete), alpha, beta.
    Updates are cumulative: query i is answered on the graph after updates
    0..i.  An insertion of a present edge or a deletion of an absent edge is
    rejected and leaves the graph unchanged (status 'EEXIST' / 'ENOENT').
    Returns per-update (status, answer, endpoint_bits) where answer is
    member(u) and member(nU + v) in the (alpha,beta)-core of the updated graph
    and endpoint_bits = member(u) | member(nU + v) << 1.
    ``check_only`` (optional set of indices) limits the recomputations to those
    updates; the others are applied without a peel and reported as None.
    """
    nL = int(n_lower)
    present = set((int(a) * nL + int(b)) for a, b in zip(np.asarray(eu), np.asarray(ev)))
    out = []
    for i in range(len(updates["u"])):
        u, v, op = int(updates["u"][i]), int(updates["v"][i]), int(updates["op"][i])
        key = u * nL + v
        if op > 0:
            if key in present:
                out.append(("EEXIST", None, None))
                continue
            present.add(key)
        else:
            if key not in present:
                out.append(("ENOENT", None, None))
                continue
            present.discard(key)
        if check_only is not None and i not in check_only:
            out.append(("OK", None, None))
            continue
        keys = np.fromiter(present, np.int64, len(present))
        g = Graph(n_upper, n_lower, (keys // nL).astype(np.int32), (keys % nL).astype(np.int32))
        member = compute(g, int(updates["alpha"][i]), int(updates["beta"][i]))
        bu, bv = bool(member[u]), bool(member[n_upper + v])
        out.append(("OK", bu and bv, int(bu) | (int(bv) << 1)))
    return out


def _connected_from(g: Graph, member: np.ndarray, seeds) -> np.ndarray:
    """Vertices reachable from the member seeds through member vertices
    only (breadth-first search over the induced subgraph of the members)."""
    out = np.zeros(g.n, bool)
    queue = [int(s) for s in seeds if member[int(s)] and not out[int(s)]]
    for s in queue:
        out[s] = True
    head = 0
    while head < len(queue):
        x = queue[head]
        head += 1
        for w in g.cols[g.off[x]:g.off[x + 1]]:
            w = int(w)
            if member[w] and not out[w]:
                out[w] = True
                queue.append(w)
    return out


def community(g: Graph, q: int, alpha: int, beta: int, connected: bool) -> np.ndarray:
    """Localized community search (Remark of Sec. V): the (alpha,beta)-core
    members in the connected component of G holding vertex q -- what peeling
    only that component leaves, since peeling never crosses components -- or,
    with ``connected``, the members connected to q through members (the
    connected part of the core containing q; empty when q is not a member)."""
    member = compute(g, alpha, beta)
    if connected:
        return _connected_from(g, member, [q])
    comp = components(g)
    return member & (comp == comp[int(q)])


def alpha_offset(g: Graph, alpha: int) -> int:
    """The largest beta >= 1 with a non-empty (alpha,beta)-core (alpha_offset
    of the default query rule in Sec. VI-B), 0 when even the (alpha,1)-core is
    empty: a plain sweep beta = 1, 2, ... of full peels."""
    beta = 0
    while compute(g, alpha, beta + 1).any():
        beta += 1
    return beta


def delta(g: Graph) -> int:
    """The largest delta with a non-empty (delta,delta)-core (the delta of
    Table I): a plain sweep of symmetric peels."""
    d = 0
    while compute(g, d + 1, d + 1).any():
        d += 1
    return d


def default_query(g: Graph):
    """The default (alpha,beta) of Sec. VI-B: alpha = 0.4 delta and beta =
    0.6 alpha_offset(alpha), each rounded down and at least 1."""
    a = max(1, (4 * delta(g)) // 10)
    return a, max(1, (6 * alpha_offset(g, a)) // 10)


def gfq_set_stream(n_upper: int, n_lower: int, eu, ev, updates, connected: bool):
    """GFQ returning the vertex set (Remark of Sec. V), by recomputation:
    after each cumulative update (u, v, op), the core members in the
    component(s) of u and nU + v in the updated graph, or with ``connected``
    the members connected to u or nU + v through members.  Rejected updates
    (present insertion, absent deletion) give (status, None).  Returns
    [(status, member bool array or None)]."""
    nL = int(n_lower)
    present = set((int(a) * nL + int(b)) for a, b in zip(np.asarray(eu), np.asarray(ev)))
    out = []
    for i in range(len(updates["u"])):
        u, v, op = int(updates["u"][i]), int(updates["v"][i]), int(updates["op"][i])
        key = u * nL + v
        if op > 0:
            if key in present:
                out.append(("EEXIST", None))
                continue
            present.add(key)
        else:
            if key not in present:
                out.append(("ENOENT", None))
                continue
            present.discard(key)
        keys = np.fromiter(present, np.int64, len(present))
        g = Graph(n_upper, n_lower, (keys // nL).astype(np.int32), (keys % nL).astype(np.int32))
        member = compute(g, int(updates["alpha"][i]), int(updates["beta"][i]))
        x, y = u, n_upper + v
        if connected:
            res = _connected_from(g, member, [x, y])
        else:
            comp = components(g)
            res = member & ((comp == comp[x]) | (comp == comp[y]))
        out.append(("OK", res))
    return out


def gfq_stream_sampled(n_upper: int, n_lower: int, eu, ev, updates, indices, on_graph=None):
    """``gfq_stream`` for graphs too large for a Python edge set: the same
    cumulative semantics (Problem 2 of Sec. III, recomputation per Sec. V),
    with the base edges kept as one sorted key array and the updates as two
    small sets (inserted keys, deleted base keys).  Only the updates listed in
    ``indices`` are answered (a full peel of the graph after that update);
    the stream is applied up to the largest of them.  Returns
    {index: (status, answer, endpoint_bits)} for those indices; a rejected
    update reports (status, None, None).  ``on_graph(i, graph)``, if given, is
    called with each oracle graph built for an answered index."""
    nL = int(n_lower)
    want = sorted(set(int(i) for i in indices))
    if not want:
        return {}
    base = np.unique(np.asarray(eu, np.int64) * nL + np.asarray(ev, np.int64))
    inserted, deleted = set(), set()

    def in_base(key):
        j = int(np.searchsorted(base, key))
        return j < len(base) and int(base[j]) == key

    out = {}
    wanted = set(want)
    for i in range(want[-1] + 1):
        u, v, op = int(updates["u"][i]), int(updates["v"][i]), int(updates["op"][i])
        key = u * nL + v
        b = in_base(key)
        present = key in inserted or (b and key not in deleted)
        if op > 0:
            if present:
                if i in wanted:
                    out[i] = ("EEXIST", None, None)
                continue
            if b:
                deleted.discard(key)
            else:
                inserted.add(key)
        else:
            if not present:
                if i in wanted:
                    out[i] = ("ENOENT", None, None)
                continue
            if key in inserted:
                inserted.discard(key)
            else:
                deleted.add(key)
        if i not in wanted:
            continue
        keep = np.ones(len(base), bool)
        if deleted:
            keep[np.searchsorted(base, np.fromiter(deleted, np.int64, len(deleted)))] = False
        keys = np.concatenate([base[keep], np.fromiter(inserted, np.int64, len(inserted))])
        del keep
        g = Graph(n_upper, n_lower, (keys // nL).astype(np.int32), (keys % nL).astype(np.int32))
        del keys
        member = compute(g, int(updates["alpha"][i]), int(updates["beta"][i]))
        bu, bv = bool(member[u]), bool(member[n_upper + v])
        out[i] = ("OK", bu and bv, int(bu) | (int(bv) << 1))
        if on_graph is not None:
            on_graph(i, g)
        del g
    return out


def timed_peel(g: Graph, alpha: int, beta: int):
    """Wall-clock seconds of one oracle peel (single thread) and its stats."""
    t0 = time.perf_counter()
    _, stats = peel(g, alpha, beta)
    return time.perf_counter() - t0, stats
