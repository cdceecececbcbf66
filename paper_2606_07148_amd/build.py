"""Builds libabcore.so for gfx950 from csrc/*.hip with hipcc (always
recompiles; objects go to _build/, which is not committed), and
libabcore_debug.so from the same sources with per-vertex enqueue counters
(ABC_DEBUG_ENQUEUE), which tests load to check the crossing rule."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libabcore.so")
DEBUG_LIB_PATH = os.path.join(HERE, "libabcore_debug.so")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Wno-unused-function", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def _compile(src: str, obj: str, defines: tuple) -> None:
    cmd = ["hipcc", "-c", *HIP_FLAGS, *[f"-D{d}" for d in defines], src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")


def _link(objs: list, path: str) -> None:
    tmp = path + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, path)


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    variants = [(LIB_PATH, "abcore", ()), (DEBUG_LIB_PATH, "abcore_debug", ("ABC_DEBUG_ENQUEUE",))]
    jobs = []
    for path, sub, defines in variants:
        out_dir = os.path.join(ROOT, "_build", sub)
        os.makedirs(out_dir, exist_ok=True)
        objs = [os.path.join(out_dir, os.path.basename(s) + ".o") for s in srcs]
        jobs.append((path, objs, [(s, o, defines) for s, o in zip(srcs, objs)]))
    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(lambda t: _compile(*t), [c for _, _, cs in jobs for c in cs]))
    for path, objs, _ in jobs:
        _link(objs, path)
        if verbose:
            print("built", path)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
