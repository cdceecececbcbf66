"""Multithreaded CPU peel of the (alpha,beta)-core (OpenMP, ``cpu_peel.c``):
the host-side comparison point of the benchmark, the frontier peeling of
Sec. III-A run on all host threads.  Independent of the device library and
of the oracle; its results are checked against the oracle in the tests."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcpu_peel.so")
_lib = None


def build() -> str:
    """Compile ``cpu_peel.c`` (always recompiles)."""
    global _lib
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O3", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                    os.path.join(_HERE, "cpu_peel.c"), "-o", tmp], check=True)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ABC_CPU_PEEL_LIB: another build of the same source (the sanitizer test loads
    # one compiled with AddressSanitizer and UndefinedBehaviorSanitizer)
    path = os.environ.get("ABC_CPU_PEEL_LIB", _LIB_PATH)
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.cp_peel.restype = ctypes.c_int
    lib.cp_peel.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64,
                            ctypes.c_int64, vp, ctypes.c_int, vp]
    lib.cp_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().cp_max_threads())


def peel(n_upper: int, n_lower: int, off: np.ndarray, cols: np.ndarray, alpha: int, beta: int,
         threads: int = 0):
    """(member bool array, rounds) of the (alpha,beta)-core of the unified
    CSR (off int64[n+1], cols int32[2m])."""
    off = np.ascontiguousarray(off, np.int64)
    cols = np.ascontiguousarray(cols, np.int32)
    n = int(n_upper) + int(n_lower)
    member = np.zeros(max(1, n), np.uint8)
    rounds = ctypes.c_int64()
    rc = _load().cp_peel(int(n_upper), int(n_lower), ctypes.c_void_p(off.ctypes.data),
                         ctypes.c_void_p(cols.ctypes.data), int(alpha), int(beta),
                         ctypes.c_void_p(member.ctypes.data), int(threads),
                         ctypes.byref(rounds))
    if rc != 0:
        raise MemoryError("cpu peel failed")
    return member[:n].astype(bool), int(rounds.value)
