"""Build libpfe.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1612_06496_amd.build

Each source compiles to its own object (in parallel), then one link.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpfe.so")
OBJ = os.path.join(ROOT, "_build")

SOURCES = ["alloc.hip", "graph.hip", "solver.hip", "learned.hip", "kmeans.hip", "eigen.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {cmd[-1]}")
    return res


def build(verbose: bool = False, extra_flags=None, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = list(SOURCES)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in srcs]
    cc = hipcc()
    cmds = [[cc, *HIPCC_FLAGS, *(extra_flags or []), "-I", INCLUDE, "-I", CSRC, "-c",
             os.path.join(CSRC, s), "-o", o] for s, o in zip(srcs, objs)]
    # the largest translation unit first
    order = sorted(range(len(cmds)), key=lambda i: -os.path.getsize(os.path.join(CSRC, srcs[i])))
    with ThreadPoolExecutor(max(1, min(jobs, len(cmds)))) as ex:
        list(ex.map(lambda i: _run(cmds[i], verbose), order))
    tmp = LIB + ".tmp"
    _run([cc, "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
