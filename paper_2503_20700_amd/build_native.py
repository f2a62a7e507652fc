"""Build the native library libdmrg_mi355x.so in-tree for gfx950.

Host C++ sources are compiled with g++, the HIP executor with hipcc
(--offload-arch=gfx950, packed-FP32 instructions disabled), and everything is
linked by hipcc into paper_2503_20700_amd/_lib/.  Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT, "libdmrg_mi355x.so")
HOST_SRC = ["su2.cpp", "spin.cpp", "planner.cpp", "hpsi.cpp", "api.cpp", "driver.cpp", "batch.cpp", "orbital.cpp"]
HIP_SRC = ["exec_hip.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-std=c++17", "-O3", "-fPIC", "-Wall", "-Wno-unused-variable", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    objdir = os.path.join(OUT, "obj")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for s in HOST_SRC:
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", os.path.join(objdir, s + ".o")])
    for s in HIP_SRC:
        jobs.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", os.path.join(objdir, s + ".o")])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr)
    objs = [os.path.join(objdir, s + ".o") for s in HOST_SRC + HIP_SRC]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
