"""Build the HIP library ``libcans_poisson.so`` in-tree for gfx950.

    python -m paper_2001_05234_amd.build

Compiles every source under ``csrc/`` with hipcc (one process per
translation unit, in parallel) and links them into one shared object next to
this file.  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcans_poisson.so")
SOURCES = ["k_x64.hip", "k_y64.hip", "k_x32f.hip", "k_x32i.hip", "k_y32.hip", "k_zsolve.hip", "k_resid.hip",
           "k_project.hip", "plan.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
OBJDIR = os.path.join(HERE, "_build")


def flags() -> list:
    return ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    objs, cmds = [], []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, s.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC] + flags() + ["-c", os.path.join(CSRC, s), "-o", obj])
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 8)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(run, cmds))
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    run(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
