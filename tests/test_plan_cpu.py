"""The host's tile planners, checked without a GPU: tests/plan_check.cpp is compiled against
the library's own planner source and run over the single-stream workload, equal frames,
empty and tiny segments, and 3000 random chunk mixes (sizes, grid limits, tile limits).  It
also runs a model of two launches of a stream whose chunks wait for decisions, on the
planner's own tiles: with each grid at most half the device's workgroup slots they always
finish, whatever order the dispatcher places workgroups in; with full grids the model
shows the deadlock that rule avoids."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1011_0235_amd", "csrc")


def test_planners_cover_and_balance(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "plan_check")
    cmd = [cxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "plan_check.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all plans valid" in out.stdout
    head = float(out.stdout.split("headline balance")[1].split()[0])
    assert 1.0 <= head <= 1.03
    assert "300 of 300 runs finished at half capacity" in out.stdout
