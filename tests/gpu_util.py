"""Helpers shared by the GPU parity tests."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    import paper_2606_07148_amd as pkg
    if not (os.path.exists(pkg.LIB_PATH) and os.path.exists(pkg.DEBUG_LIB_PATH)):
        sys.path.insert(0, ROOT)
        import __graft_entry__
        __graft_entry__.build()
    return pkg.load()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def bits_np(t):
    return t.cpu().numpy().view(np.uint32)


def say(*args):
    print(*args, flush=True)


def serve_all(g, ups, max_inflight):
    """Submits the stream in order, polling while admission is full; returns
    the results in ticket order."""
    import paper_2606_07148_amd as pkg
    n = len(ups["u"])
    tickets, results = [], {}
    waiting = []
    i = 0
    while i < n or waiting:
        if i < n:
            t = pkg.abcore_try_submit(g, ups["u"][i], ups["v"][i], ups["op"][i],
                                      ups["alpha"][i], ups["beta"][i])
            if t is not None:
                tickets.append(t)
                waiting.append(t)
                i += 1
                continue
        still = []
        for t in waiting:
            r = pkg.abcore_poll(g, t)
            if r is None:
                still.append(t)
            else:
                results[t] = r
        waiting = still
    assert tickets == list(range(tickets[0], tickets[0] + n))
    return [results[t] for t in tickets]
