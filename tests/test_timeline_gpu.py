"""The diagnostic timeline build (libhistmi_timeline.so): one launch per workload broken down
into the steps of the paper's Table 1 (Sec. III.A).  It runs in its own process, since it
loads the diagnostic library in place of libhistmi.so."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_timeline_breakdown():
    r = subprocess.run([sys.executable, "-m", "paper_1011_0235_amd.timeline", "--json"], cwd=ROOT,
                       capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert set(out) == {"hist_u8_64MiB_random", "hist_u8_1MiB", "stream_push_66x4MiB"}
    for name, row in out.items():
        ends = [s["ends_us"] for s in row["steps"]]
        assert [s["step"] for s in row["steps"]] == ["start", "count", "flush", "merge"], name
        assert all(e > 0 for e in ends) and ends == sorted(ends), (name, ends)
        assert 0 < row["span_us"] < 10000, name
        assert row["workgroups"] >= 1
    big = out["hist_u8_64MiB_random"]
    assert big["counts_sum_to_n"]
    assert big["read_probe"]["GBps"] > 0
    assert big["workgroups"] > 256 and out["stream_push_66x4MiB"]["workgroups"] >= 256
