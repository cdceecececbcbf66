"""Seeded synthetic inputs for the (alpha,beta)-core workloads.

This package generates edge lists, query parameters and edge-update streams.
It holds none of the core computation; both the oracle and the device library
consume its outputs.  The arithmetic lives in ``gen.cpp`` (SplitMix64 counter
streams, Lemire bounded integers, Vose alias tables); this module only
marshals arrays.

Workloads (the paper's datasets are not available, so these stand in for the
scale and degree skew of its Table I graphs):

* ``uniform``  -- pairs drawn uniformly, first m distinct pairs kept.
* ``chung_lu`` -- endpoints drawn with probability proportional to power-law
  expected degrees (degree-distribution exponent gamma per layer, capped),
  first m distinct pairs kept.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbigraph_gen.so")
_lib = None

# The five workload shapes.  Seeds: graph seed k, query/update seed k + 1000.
CONFIGS = {
    1: dict(kind="uniform", n_upper=2_000, n_lower=1_500, m=20_000, seed=1),
    2: dict(kind="chung_lu", n_upper=1_000_000, n_lower=500_000, m=20_000_000,
            gamma_upper=2.1, gamma_lower=2.1, cap=50_000, seed=2),
    3: dict(kind="chung_lu", n_upper=50_000_000, n_lower=20_000_000, m=1_000_000_000,
            gamma_upper=2.0, gamma_lower=2.3, cap=50_000, seed=3),
    4: dict(kind="chung_lu", n_upper=10_000_000, n_lower=5_000_000, m=200_000_000,
            gamma_upper=2.1, gamma_lower=2.1, cap=50_000, seed=4),
    5: dict(kind="chung_lu", n_upper=20_000_000, n_lower=10_000_000, m=500_000_000,
            gamma_upper=2.1, gamma_lower=2.1, cap=50_000, seed=5),
}


def build() -> str:
    """Compile ``gen.cpp`` into ``libbigraph_gen.so`` (always recompiles)."""
    global _lib
    src = os.path.join(_HERE, "gen.cpp")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ABC_BIGRAPH_GEN_LIB: another build of the same source (the sanitizer test loads
    # one compiled with AddressSanitizer and UndefinedBehaviorSanitizer)
    path = os.environ.get("ABC_BIGRAPH_GEN_LIB", _LIB_PATH)
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(path)
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.bg_uniform.restype = ctypes.c_int64
    lib.bg_uniform.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                               i32p, i32p]
    lib.bg_chung_lu.restype = ctypes.c_int64
    lib.bg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.bg_loguniform_pairs.restype = None
    lib.bg_loguniform_pairs.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_uint64, i32p, i32p]
    lib.bg_update_stream.restype = ctypes.c_int64
    lib.bg_update_stream.argtypes = [
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_double,
        ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i32p, i32p, i32p, i32p, i32p, f64p]
    lib.bg_splitmix_draw.restype = ctypes.c_uint64
    lib.bg_splitmix_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.bg_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def splitmix_draw(seed: int, tag: int, i: int) -> int:
    return int(_load().bg_splitmix_draw(seed, tag, i))


def uniform(n_upper: int, n_lower: int, m: int, seed: int):
    """First m distinct uniformly drawn (u, v) pairs, sorted by (u, v)."""
    eu = np.empty(m, np.int32)
    ev = np.empty(m, np.int32)
    r = _load().bg_uniform(n_upper, n_lower, m, seed, _p32(eu), _p32(ev))
    if r != m:
        raise ValueError(f"uniform generator failed ({r})")
    return eu, ev


def chung_lu(n_upper: int, n_lower: int, m: int, gamma_upper: float, gamma_lower: float,
             cap: float, seed: int):
    """First m distinct Chung-Lu pairs, sorted by (u, v)."""
    eu = np.empty(m, np.int32)
    ev = np.empty(m, np.int32)
    r = _load().bg_chung_lu(n_upper, n_lower, m, gamma_upper, gamma_lower, cap, seed,
                            _p32(eu), _p32(ev))
    if r != m:
        raise ValueError(f"Chung-Lu generator failed ({r})")
    return eu, ev


def scaled(cfg: int, factor: float) -> dict:
    """A config with vertex and edge counts multiplied by ``factor`` (cap kept
    below a twentieth of the scaled edge count so the skew stays feasible)."""
    c = dict(CONFIGS[cfg])
    c["n_upper"] = max(8, int(c["n_upper"] * factor))
    c["n_lower"] = max(8, int(c["n_lower"] * factor))
    c["m"] = max(16, int(c["m"] * factor))
    if "cap" in c:
        c["cap"] = float(min(c["cap"], max(16, c["m"] // 20)))
    return c


def make_graph(spec: dict):
    """Edge arrays for a config dict (see ``CONFIGS``)."""
    if spec["kind"] == "uniform":
        return uniform(spec["n_upper"], spec["n_lower"], spec["m"], spec["seed"])
    return chung_lu(spec["n_upper"], spec["n_lower"], spec["m"], spec["gamma_upper"],
                    spec["gamma_lower"], spec["cap"], spec["seed"])


def edge_hash(eu: np.ndarray, ev: np.ndarray) -> str:
    """SHA-256 of the canonical (sorted, int32 little-endian interleaved) list."""
    order = np.lexsort((ev, eu))
    pairs = np.stack([eu[order], ev[order]], axis=1).astype("<i4")
    return hashlib.sha256(pairs.tobytes()).hexdigest()


def loguniform_pairs(q: int, lo: int, hi: int, seed: int):
    a = np.empty(q, np.int32)
    b = np.empty(q, np.int32)
    _load().bg_loguniform_pairs(q, lo, hi, seed, _p32(a), _p32(b))
    return a, b


def update_stream(spec: dict, eu: np.ndarray, ev: np.ndarray, count: int, seed: int,
                  ins_permille: int = 700, qlo: int = 2, qhi: int = 64):
    """Edge-update stream (70% insertions by default) with per-update (alpha,
    beta) and unit-mean exponential inter-arrival gaps."""
    eu = np.ascontiguousarray(eu, np.int32)
    ev = np.ascontiguousarray(ev, np.int32)
    out = {k: np.empty(count, np.int32) for k in ("u", "v", "op", "alpha", "beta")}
    gap = np.empty(count, np.float64)
    gu = spec.get("gamma_upper", 2.1)
    gl = spec.get("gamma_lower", 2.1)
    cap = spec.get("cap", 50_000)
    r = _load().bg_update_stream(
        spec["n_upper"], spec["n_lower"], len(eu), _p32(eu), _p32(ev), gu, gl, cap,
        spec["seed"], seed, count, ins_permille, qlo, qhi, _p32(out["u"]), _p32(out["v"]),
        _p32(out["op"]), _p32(out["alpha"]), _p32(out["beta"]),
        gap.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if r != count:
        raise ValueError(f"update stream generator failed ({r})")
    out["gap"] = gap
    return out
