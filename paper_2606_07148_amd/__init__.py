"""Python binding of libabcore: (alpha,beta)-core computation (GCC, GCC+) and
on-the-fly edge queries (GFQ) on MI355X.

Argument marshalling only: every step runs in the HIP kernels of
``libabcore.so`` (built by ``paper_2606_07148_amd.build``).  Device buffers
are torch CUDA tensors; the stream is torch's current stream unless given.
Importing this package does not require a GPU, but every call does, and the
package raises ``ImportError`` when the library has not been built.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
# ABCORE_LIBRARY: another build of the same sources (the sanitizer test
# loads one whose host code is compiled with AddressSanitizer)
LIB_PATH = os.environ.get("ABCORE_LIBRARY", os.path.join(_HERE, "libabcore.so"))
DEBUG_LIB_PATH = os.path.join(_HERE, "libabcore_debug.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "abcore.h")

ABCORE_GCC = 0
ABCORE_GCC_PLUS = 1
ABCORE_OPT_PEEL_MODE = 1
ABCORE_OPT_GRID = 2
ABCORE_OPT_ROUNDS_PER_SYNC = 3
ABCORE_OPT_TIMING = 4
ABCORE_OPT_PULL = 5
ABCORE_OPT_CLAIM = 6
ABCORE_OPT_RANK_ORDER = 7
ABCORE_OPT_SPIN_LIMIT = 8
ABCORE_OPT_AUTOTUNE = 9
ABCORE_OPT_SERVE_PRUNE = 10
ABCORE_OPT_KCORE_SWITCH = 11
ABCORE_OPT_APPEND_SUBQUEUE = 12
ABCORE_OPT_SERVE_DEADLINE_US = 13

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOENT", 5: "EEXIST",
          6: "EBUSY", 7: "EAGAIN", 8: "ETIMEDOUT"}


class AbcoreError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class abcore_stats(ctypes.Structure):
    _fields_ = [("removed", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("entries_read", ctypes.c_int64), ("initial", ctypes.c_int64),
                ("uncertain", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("pulled", ctypes.c_int64), ("rank_order", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class abcore_report(ctypes.Structure):
    _fields_ = [("build_ms", ctypes.c_double), ("csr_ms", ctypes.c_double),
                ("pieces_ms", ctypes.c_double), ("ranks_ms", ctypes.c_double),
                ("graph_bytes", ctypes.c_int64), ("ranks_bytes", ctypes.c_int64),
                ("queue_bytes", ctypes.c_int64), ("core_top", ctypes.c_int64 * 4),
                ("core_levels_ms", ctypes.c_double), ("core_top_ms", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "core_top"}
        d["core_top"] = dict(zip(("k0", "vertices", "entries", "half_sweeps"), list(self.core_top)))
        return d


class abcore_edge_update(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int32), ("v", ctypes.c_int32), ("op", ctypes.c_int32)]


_lib = None
_libs = {}


def load():
    """The loaded library; ImportError if it has not been built."""
    global _lib
    if _lib is None:
        _lib = _open(LIB_PATH)
    return _lib


@contextlib.contextmanager
def debug_library():
    """Within the block every call goes to libabcore_debug.so, the same
    sources built with per-vertex enqueue counters (ABC_DEBUG_ENQUEUE).
    Handles made inside the block belong to that library; destroy them
    before leaving it (a Graph keeps the library that made it)."""
    global _lib
    prev = load()
    _lib = _open(DEBUG_LIB_PATH)
    try:
        yield _lib
    finally:
        _lib = prev


def _open(path):
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise ImportError(f"{os.path.basename(path)} not built ({path}); run "
                          "`python -m paper_2606_07148_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    P = ctypes.POINTER
    sig = {
        "abcore_last_error": (ctypes.c_char_p, []),
        "abcore_build_csr": (i32, [i32, i32, vp, vp, i64, vp, P(vp), P(i64)]),
        "abcore_destroy": (i32, [vp]),
        "abcore_debug_enqueue_counts": (i32, [vp, vp, i32, vp]),
        "abcore_graph_info": (i32, [vp, P(i32), P(i32), P(i64)]),
        "abcore_export_csr": (i32, [vp, vp, vp, P(i64), vp]),
        "abcore_compute": (i32, [vp, u32, u32, i32, vp, P(abcore_stats), vp]),
        "abcore_compute_static": (i32, [vp, u32, u32, vp, vp]),
        "abcore_core_numbers": (i32, [vp, vp, P(i32), vp]),
        "abcore_components": (i32, [vp, vp, vp]),
        "abcore_query": (i32, [vp, abcore_edge_update, u32, u32, P(i32), P(u32), vp]),
        "abcore_query_set": (i32, [vp, abcore_edge_update, u32, u32, i32, P(i32), P(u32), vp,
                                   P(i64), vp]),
        "abcore_community": (i32, [vp, i32, u32, u32, i32, vp, P(i64), vp]),
        "abcore_alpha_offsets": (i32, [vp, P(u32), i32, P(u32), P(i32), vp]),
        "abcore_default_query": (i32, [vp, P(u32), P(u32), vp]),
        "abcore_set_option": (i32, [vp, i32, i64]),
        "abcore_kernel_timing": (i32, [vp, i32, P(ctypes.c_double), P(i64), i32]),
        "abcore_compute_batch": (i32, [vp, P(u32), P(u32), i32, vp, vp]),
        "abcore_batch_plan": (i32, [P(u32), P(u32), i32, P(i32), P(i32), P(i32)]),
        "abcore_serve_start": (i32, [vp, i64, i32, i32]),
        "abcore_submit": (i32, [vp, abcore_edge_update, u32, u32, P(ctypes.c_uint64)]),
        "abcore_poll": (i32, [vp, ctypes.c_uint64, P(i32), P(u32), P(ctypes.c_uint64)]),
        "abcore_serve_stop": (i32, [vp, P(i64)]),
        "abcore_serve_counters": (i32, [vp, P(i64), i32]),
        "abcore_graph_report": (i32, [vp, P(abcore_report)]),
        "abcore_device_memory": (i32, [P(i64), P(i64), i32]),
        "abcore_set_memory_budget": (i32, [i64]),
        "abcore_tuned": (i32, [vp, i32, P(i32), P(i32), P(ctypes.c_double), P(i32)]),
        "abcore_tune_cache": (i32, [ctypes.c_char_p, i32]),
        "abcore_autotune": (i32, [vp, u32, u32, i32, P(i32), P(i32), P(ctypes.c_double), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _libs[path] = lib
    return lib


def declared_symbols() -> list:
    """Function names declared in include/abcore.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(abcore_[a-z_]+)\s*\(", text)))


def _check(status: int):
    if status != 0:
        msg = load().abcore_last_error().decode(errors="replace")
        raise AbcoreError(status, msg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


class Graph:
    """Owns one abcore_graph handle."""

    def __init__(self, handle, n_upper, n_lower, m):
        self._h = handle
        self._lib = load()
        self.n_upper = n_upper
        self.n_lower = n_lower
        self.n = n_upper + n_lower
        self.m = m

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph destroyed")
        return self._h

    @property
    def nwords(self) -> int:
        return (self.n + 31) // 32

    def destroy(self):
        if self._h is not None:
            self._lib.abcore_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def refresh(self):
        nu, nl, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(load().abcore_graph_info(self.handle, ctypes.byref(nu), ctypes.byref(nl),
                                        ctypes.byref(m)))
        self.m = int(m.value)
        return self


def abcore_build_csr(n_upper: int, n_lower: int, eu, ev, stream=None) -> Graph:
    """Build the device CSR from int32 CUDA tensors of endpoints."""
    import torch
    assert eu.dtype == torch.int32 and ev.dtype == torch.int32
    assert eu.is_cuda and ev.is_cuda and eu.numel() == ev.numel()
    eu = eu.contiguous()
    ev = ev.contiguous()
    h = ctypes.c_void_p()
    md = ctypes.c_int64()
    _check(load().abcore_build_csr(int(n_upper), int(n_lower), _ptr(eu), _ptr(ev),
                                   int(eu.numel()), _stream(stream), ctypes.byref(h),
                                   ctypes.byref(md)))
    return Graph(h, int(n_upper), int(n_lower), int(md.value))


def abcore_graph_report(g: Graph) -> dict:
    """Build phase times (ms) and byte counts of a handle."""
    r = abcore_report()
    _check(load().abcore_graph_report(g.handle, ctypes.byref(r)))
    return r.as_dict()


def abcore_device_memory(reset_peak: bool = False):
    """(current, peak) device bytes held by the library."""
    cur, peak = ctypes.c_int64(), ctypes.c_int64()
    _check(load().abcore_device_memory(ctypes.byref(cur), ctypes.byref(peak), int(reset_peak)))
    return int(cur.value), int(peak.value)


def abcore_debug_enqueue_counts(g: Graph, reset: bool = False, stream=None):
    """Per-vertex counts of appends to the frontier queues since the last
    reset (debug library only; EINVAL from the release library)."""
    import torch
    out = torch.zeros(max(g.n, 1), dtype=torch.int32, device="cuda")
    _check(load().abcore_debug_enqueue_counts(g.handle, _ptr(out), int(bool(reset)),
                                              _stream(stream)))
    return out[: g.n]


def abcore_set_memory_budget(nbytes: int) -> None:
    """Process-wide cap on the library's device bytes (0 = none)."""
    _check(load().abcore_set_memory_budget(int(nbytes)))


def abcore_destroy(g: Graph) -> None:
    g.destroy()


def abcore_set_option(g: Graph, option: int, value: int) -> None:
    _check(load().abcore_set_option(g.handle, int(option), int(value)))


ABCORE_KERNEL_PEEL = 0
ABCORE_KERNEL_PULL = 1
ABCORE_KERNEL_SCAN = 2
ABCORE_KERNEL_PACK = 3
ABCORE_KERNEL_FIXUP = 4


def abcore_kernel_timing(g: Graph, kernel: int, reset: bool = True):
    """(GPU milliseconds, launches) of one kernel kind recorded with
    ABCORE_OPT_TIMING on."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().abcore_kernel_timing(g.handle, int(kernel), ctypes.byref(ms), ctypes.byref(n),
                                       int(reset)))
    return float(ms.value), int(n.value)


def abcore_export_csr(g: Graph, stream=None):
    """(off int64[n+1], cols int32[2m]) CUDA tensors of the current graph."""
    import torch
    ent = ctypes.c_int64()
    _check(load().abcore_export_csr(g.handle, None, None, ctypes.byref(ent), None))
    off = torch.empty(g.n + 1, dtype=torch.int64, device="cuda")
    cols = torch.empty(max(1, int(ent.value)), dtype=torch.int32, device="cuda")
    _check(load().abcore_export_csr(g.handle, _ptr(off), _ptr(cols), ctypes.byref(ent),
                                    _stream(stream)))
    return off, cols[: int(ent.value)]


def abcore_compute(g: Graph, alpha: int, beta: int, algo: int = ABCORE_GCC, out=None,
                   stats: bool = False, stream=None):
    """Membership bitmask (int32 CUDA tensor of ceil(n/32) words, bit order
    LSB-first) of the (alpha,beta)-core; with stats=True also the counters."""
    import torch
    if out is None:
        out = torch.empty(max(1, g.nwords), dtype=torch.int32, device="cuda")
    st = abcore_stats() if stats else None
    _check(load().abcore_compute(g.handle, int(alpha), int(beta), int(algo), _ptr(out),
                                 ctypes.byref(st) if st is not None else None,
                                 _stream(stream)))
    return (out, st.as_dict()) if stats else out


def abcore_compute_static(g: Graph, alpha: int, beta: int, out, stream=None):
    """The GCC bitmask of abcore_compute, computed with no allocation (the
    working set lives in the library's static device array); ``out`` is a
    caller-allocated int32 CUDA tensor of ceil(n/32) words."""
    _check(load().abcore_compute_static(g.handle, int(alpha), int(beta), _ptr(out),
                                        _stream(stream)))
    return out


def _u32_array(values):
    vals = [int(x) for x in values]
    return (ctypes.c_uint32 * max(1, len(vals)))(*vals), len(vals)


def abcore_compute_batch(g: Graph, alphas, betas, out=None, stream=None):
    """Bitmasks of q queries: int32 CUDA tensor (q, ceil(n/32)); row i is the
    (alphas[i], betas[i])-core."""
    import torch
    a, q = _u32_array(alphas)
    b, qb = _u32_array(betas)
    if q != qb:
        raise ValueError("alphas and betas differ in length")
    if out is None:
        out = torch.empty((q, max(1, g.nwords)), dtype=torch.int32, device="cuda")
    _check(load().abcore_compute_batch(g.handle, a, b, q, _ptr(out), _stream(stream)))
    return out


def abcore_batch_plan(alphas, betas):
    """(parent list, execution order, degree buffers needed) of a batch."""
    a, q = _u32_array(alphas)
    b, qb = _u32_array(betas)
    if q != qb:
        raise ValueError("alphas and betas differ in length")
    parent = (ctypes.c_int32 * max(1, q))()
    order = (ctypes.c_int32 * max(1, q))()
    states = ctypes.c_int32()
    _check(load().abcore_batch_plan(a, b, q, parent, order, ctypes.byref(states)))
    return list(parent)[:q], list(order)[:q], int(states.value)


def abcore_autotune(g: Graph, alpha: int, beta: int, algo: int = ABCORE_GCC, stream=None):
    """Picks and sets the asynchronous-peel grid and claim size for this
    graph; returns (grid, claim, best ms)."""
    gr, cl, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load().abcore_autotune(g.handle, int(alpha), int(beta), int(algo), ctypes.byref(gr),
                                  ctypes.byref(cl), ctypes.byref(ms), _stream(stream)))
    return int(gr.value), int(cl.value), float(ms.value)


def abcore_serve_start(g: Graph, max_inflight: int = 0, device_slots: int = 0,
                       window: int = 0):
    """Starts the serving engine of the handle (0 = library defaults)."""
    _check(load().abcore_serve_start(g.handle, int(max_inflight), int(device_slots),
                                     int(window)))


def abcore_submit(g: Graph, u: int, v: int, op: int, alpha: int, beta: int) -> int:
    """Admits one request; returns its ticket.  AbcoreError EBUSY when the
    admission limit is reached."""
    t = ctypes.c_uint64()
    _check(load().abcore_submit(g.handle, abcore_edge_update(int(u), int(v), int(op)),
                                int(alpha), int(beta), ctypes.byref(t)))
    return int(t.value)


def abcore_try_submit(g: Graph, u: int, v: int, op: int, alpha: int, beta: int):
    """Like abcore_submit, but None instead of an EBUSY error."""
    t = ctypes.c_uint64()
    st = load().abcore_submit(g.handle, abcore_edge_update(int(u), int(v), int(op)),
                              int(alpha), int(beta), ctypes.byref(t))
    if st == 6:
        return None
    _check(st)
    return int(t.value)


def abcore_poll(g: Graph, ticket: int):
    """None while the request runs; else a dict with status ("OK", "EEXIST",
    "ENOENT", "ETIMEDOUT", ...), answer, bits and t_done_ns (time.monotonic_ns
    clock)."""
    ans = ctypes.c_int32()
    bits = ctypes.c_uint32()
    t = ctypes.c_uint64()
    st = load().abcore_poll(g.handle, int(ticket), ctypes.byref(ans), ctypes.byref(bits),
                            ctypes.byref(t))
    if st == 7:
        return None
    if st not in (0, 4, 5, 8):
        _check(st)
    return {"status": STATUS[st], "answer": bool(ans.value), "bits": int(bits.value),
            "t_done_ns": int(t.value)}


def abcore_serve_counters(g: Graph) -> dict:
    """The serving engine's counters."""
    c = (ctypes.c_int64 * 8)()
    _check(load().abcore_serve_counters(g.handle, c, 8))
    return {"windows": int(c[0]), "answered": int(c[1]), "rejected": int(c[2]),
            "decided_without_peel": int(c[3]), "core_snapshots": int(c[4]),
            "snapshot_ms": c[5] / 1e3, "timed_out": int(c[6]), "device_slots": int(c[7])}


def abcore_serve_stop(g: Graph) -> dict:
    """Drains and stops the engine; returns its counters."""
    c = (ctypes.c_int64 * 3)()
    _check(load().abcore_serve_stop(g.handle, c))
    info_u, info_l, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(load().abcore_graph_info(g.handle, ctypes.byref(info_u), ctypes.byref(info_l),
                                    ctypes.byref(m)))
    g.m = int(m.value)
    return {"windows": int(c[0]), "answered": int(c[1]), "rejected": int(c[2])}


def abcore_core_numbers(g: Graph, stream=None):
    """(core int32 CUDA tensor[n], max core number)."""
    import torch
    core = torch.empty(max(1, g.n), dtype=torch.int32, device="cuda")
    mx = ctypes.c_int32()
    _check(load().abcore_core_numbers(g.handle, _ptr(core), ctypes.byref(mx), _stream(stream)))
    return core[: g.n], int(mx.value)


def abcore_components(g: Graph, stream=None):
    import torch
    comp = torch.empty(max(1, g.n), dtype=torch.int32, device="cuda")
    _check(load().abcore_components(g.handle, _ptr(comp), _stream(stream)))
    return comp[: g.n]


def abcore_query(g: Graph, u: int, v: int, op: int, alpha: int, beta: int, stream=None):
    """Apply one edge update and return (answer, endpoint_bits)."""
    ans = ctypes.c_int32()
    bits = ctypes.c_uint32()
    upd = abcore_edge_update(int(u), int(v), int(op))
    _check(load().abcore_query(g.handle, upd, int(alpha), int(beta), ctypes.byref(ans),
                               ctypes.byref(bits), _stream(stream)))
    g.m += int(op)
    return bool(ans.value), int(bits.value)


def abcore_query_set(g: Graph, u: int, v: int, op: int, alpha: int, beta: int,
                     connected: bool = False, out=None, stream=None):
    """Apply one edge update; return (answer, endpoint_bits, bitmask tensor,
    set size): the core members the scoped peel leaves in the component(s)
    of u and v, or with connected=True those connected to u or v."""
    import torch
    if out is None:
        out = torch.empty(max(1, g.nwords), dtype=torch.int32, device="cuda")
    ans = ctypes.c_int32()
    bits = ctypes.c_uint32()
    cnt = ctypes.c_int64()
    upd = abcore_edge_update(int(u), int(v), int(op))
    _check(load().abcore_query_set(g.handle, upd, int(alpha), int(beta), int(bool(connected)),
                                   ctypes.byref(ans), ctypes.byref(bits), _ptr(out),
                                   ctypes.byref(cnt), _stream(stream)))
    g.m += int(op)
    return bool(ans.value), int(bits.value), out, int(cnt.value)


def abcore_community(g: Graph, q: int, alpha: int, beta: int, connected: bool = False,
                     out=None, stream=None):
    """(bitmask tensor, size) of the (alpha,beta)-core members around vertex
    q (unified id): its component's members, or with connected=True the
    connected part of the core containing q."""
    import torch
    if out is None:
        out = torch.empty(max(1, g.nwords), dtype=torch.int32, device="cuda")
    cnt = ctypes.c_int64()
    _check(load().abcore_community(g.handle, int(q), int(alpha), int(beta), int(bool(connected)),
                                   _ptr(out), ctypes.byref(cnt), _stream(stream)))
    return out, int(cnt.value)


def abcore_alpha_offsets(g: Graph, alphas, stream=None):
    """(alpha_offset of each alpha, delta) -- the query parameters of Sec. VI-B."""
    a, q = _u32_array(alphas)
    off = (ctypes.c_uint32 * max(1, q))()
    d = ctypes.c_int32()
    _check(load().abcore_alpha_offsets(g.handle, a, q, off, ctypes.byref(d), _stream(stream)))
    return [int(x) for x in list(off)[:q]], int(d.value)


def abcore_default_query(g: Graph, stream=None):
    """The default (alpha, beta) of Sec. VI-B."""
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().abcore_default_query(g.handle, ctypes.byref(a), ctypes.byref(b),
                                       _stream(stream)))
    return int(a.value), int(b.value)


def abcore_tuned(g: Graph, kind: int = 1):
    """(grid, claim, ms) cached for the handle's architecture and shape
    (kind 0 single queries, 1 batches), or None."""
    gr, cl, ms, found = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    _check(load().abcore_tuned(g.handle, int(kind), ctypes.byref(gr), ctypes.byref(cl),
                               ctypes.byref(ms), ctypes.byref(found)))
    return (int(gr.value), int(cl.value), float(ms.value)) if found.value else None


def abcore_tune_cache(path, mode: int):
    """Tuning cache file: mode 0 load, 1 save, 2 clear."""
    _check(load().abcore_tune_cache(None if path is None else str(path).encode(), int(mode)))
