"""Helpers shared by the GPU parity tests."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    import paper_2606_07148_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
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
