"""Compile-time resource checks of the counting kernels (host only: hipcc cross-compiles for
gfx950 without a GPU).

No kernel may touch per-lane scratch memory.  The main kernel takes its parameter block by
value; if any helper that receives it by reference is left out of line, the compiler copies
the whole block (over 1 KiB) into each lane's private memory on entry, which costs more than
the histogram itself.  The generated code must hold no scratch load or store at all, and the
reserved private segment must stay small (the register allocator may reserve an emergency
spill slot of a few bytes that no instruction uses).  Occupancy must stay at >= 3 wavefronts
per SIMD (three workgroups of four wavefronts per CU)."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_kernels_use_no_scratch(tmp_path):
    from paper_1011_0235_amd import build
    src = os.path.join(ROOT, "paper_1011_0235_amd", "csrc", "kernels.hip")
    cmd = (["hipcc"] + build.hip_flags() + ["-Rpass-analysis=kernel-resource-usage", "-c", src,
                                           "-o", str(tmp_path / "k.o")])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z /\[\]]+?):\s+(\d+)", line)
        if m and name:
            kernels[name][m.group(1).strip()] = int(m.group(2))
    assert any("hist_main" in k for k in kernels), list(kernels)
    for k, res in kernels.items():
        assert res.get("ScratchSize [bytes/lane]", 0) <= 64, (k, res)
        assert res.get("VGPRs Spill", 0) == 0, (k, res)
        if "hist_main" in k:
            assert res.get("Occupancy [waves/SIMD]", 0) >= 3, (k, res)
    asm = tmp_path / "k.s"
    r = subprocess.run(["hipcc"] + build.hip_flags() + ["--cuda-device-only", "-S", src, "-o", str(asm)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    text = asm.read_text()
    assert not re.search(r"^\s*(scratch_(load|store)|buffer_(load|store)_\w+\s.*s\[0:3\])", text, re.M)
