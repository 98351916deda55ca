"""Build libjag.so in-tree: host C++ with g++, device code with hipcc for gfx950.

    python -m paper_2602_10258_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libjag.so")
BUILD = os.path.join(ROOT, "_build")

HOST_SRC = ["api.cpp", "builder.cpp"]
DEV_SRC = ["search.hip", "serve_kernels.hip", "predictor.hip", "serve.hip", "build.hip", "probe.hip", "batch.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3", "-fopenmp-simd", "-Wall",
              "-Wno-unused-function", f"-I{INC}", f"-I{CSRC}"]
DEV_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", f"-I{INC}", f"-I{CSRC}"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HOST_SRC:
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, s),
                     "-o", os.path.join(BUILD, s + ".o")])
    for s in DEV_SRC:
        jobs.append([HIPCC, *DEV_FLAGS, "-c", os.path.join(CSRC, s),
                     "-o", os.path.join(BUILD, s + ".o")])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and r.stderr.strip():
                print(r.stderr, file=sys.stderr)
    objs = [os.path.join(BUILD, s + ".o") for s in HOST_SRC + DEV_SRC]
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        sys.exit("hipcc not found")
    build()
