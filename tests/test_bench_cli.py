"""bench.py's command-line contract, on the CPU: one GPU only, side workloads
only with a solve mode, and the workload text of a face-located z."""
import dataclasses
import os
import subprocess
import sys

import bench
from paper_2001_05234_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_side_workloads_need_a_solve_mode():
    for flags in (["--shift=-1.0"], ["--face-z"]):
        r = run(*flags)
        assert r.returncode == 2
        assert "--solve-only" in r.stderr


def test_workload_text_and_digest():
    pr = inputs.config("c3")
    assert "1024x512x384, bc PP/PP/NN" in bench.workload_text("c3", pr, "auto")
    face = dataclasses.replace(pr, nz=pr.nz - 1, bc=tuple(pr.bc[:4]) + (3, 3), rhs_kind="uniform")
    assert "1024x512x383, bc PP/PP/FdFd" in bench.workload_text("c3", face, "auto")
    d = bench.source_digest()
    assert len(d) == 16 and int(d, 16) >= 0
