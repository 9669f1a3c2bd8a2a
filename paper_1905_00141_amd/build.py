"""Builds libmra.so (HIP kernels for gfx950 + host code) in-tree.

    python -m paper_1905_00141_amd.build [--changed]

--changed recompiles only the sources newer than their objects.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libmra.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + INCLUDE, "-I" + CSRC]
HIP_SOURCES = ["mra_chain.hip", "mra_finish.hip", "mra_gram.hip", "mra_pred.hip", "mra_api.hip", "mra_mlp.hip", "mra_bench.hip", "mra_tree_gpu.hip"]
HOST_SOURCES = ["mra_tree.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {os.path.basename(cmd[-1])}")
    return r


def _stale(obj: str, src: str) -> bool:
    """An object is rebuilt when it is older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + \
        [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force) or only those changed since their object."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD_DIR, s + ".o")
        objs.append(o)
        if force or _stale(o, os.path.join(CSRC, s)):
            jobs.append([HIPCC] + HIP_FLAGS + ["-c", "-o", o, os.path.join(CSRC, s)])
    for s in HOST_SOURCES:
        o = os.path.join(BUILD_DIR, s + ".o")
        objs.append(o)
        # host-only tree builder: plain IEEE expression evaluation (no FMA contraction)
        if force or _stale(o, os.path.join(CSRC, s)):
            jobs.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=off",
                         "-I" + INCLUDE, "-I" + CSRC, "-c", "-o", o, os.path.join(CSRC, s)])
    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(_run, jobs))
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, force="--changed" not in sys.argv)
