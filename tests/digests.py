"""SHA-256 digests of little-endian arrays, shared by the golden-writing
script (oracle outputs) and the GPU tests (device outputs).  No part of the
method's arithmetic lives here."""
from __future__ import annotations

import hashlib

import numpy as np

CHUNK = 1 << 26


def sha_array(a, dtype: str) -> str:
    """SHA-256 of ``a`` as a contiguous little-endian array of ``dtype``."""
    h = hashlib.sha256()
    a = np.asarray(a)
    for s in range(0, len(a), CHUNK):
        h.update(np.ascontiguousarray(a[s:s + CHUNK], dtype).tobytes())
    return h.hexdigest()


def sha_edges(eu, ev) -> str:
    """SHA-256 of the interleaved int32 (u, v) pairs, which must be strictly
    sorted by (u, v) (checked chunk by chunk)."""
    h = hashlib.sha256()
    prev = None
    for s in range(0, len(eu), CHUNK):
        u = np.asarray(eu[s:s + CHUNK], np.int64)
        v = np.asarray(ev[s:s + CHUNK], np.int64)
        k = u * (1 << 32) + v
        if len(k) > 1 and not bool(np.all(k[1:] > k[:-1])):
            raise ValueError("edge list not strictly sorted")
        if prev is not None and len(k) and not k[0] > prev:
            raise ValueError("edge list not strictly sorted across chunks")
        if len(k):
            prev = int(k[-1])
        h.update(np.stack([eu[s:s + CHUNK], ev[s:s + CHUNK]], axis=1).astype("<i4").tobytes())
    return h.hexdigest()
