"""Host-side logic of bench.py (no GPU): the one-GPU guard and the build-tagged
counter table that the bench line's `traffic` comes from."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2408_13782_amd import build  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_table_names_the_current_sources():
    """The committed counter table was taken on the library built from these
    sources: the bench reports its traffic for every step kernel of the three
    workloads, and nothing for any other build."""
    tag = build.source_tag()
    for wl, kinds in (("paper", {"rows_forward", "cols", "rows_backward", "update"}),
                      ("large", {"rows_forward", "cols", "rows_backward", "update"}),
                      ("small", {"chain_fused", "update"})):
        t = bench.load_traffic(wl, tag)
        assert t is not None and set(t) == kinds, wl
        assert all(v > 0 for v in t.values())
    assert bench.load_traffic("paper", "0" * 16) is None
    assert bench.load_traffic("no-such-workload", tag) is None


def test_traffic_is_calibrated_by_the_copy_probe():
    """HBM bytes per launch = FETCH_SIZE and WRITE_SIZE scaled by what the
    counters read for a copy of known size: the paper-shaped chain moves 34.56
    MB per batch, the update 24.82 MB."""
    t = bench.load_traffic("paper", build.source_tag())
    chain = t["rows_forward"] + t["cols"] + t["rows_backward"]
    assert abs(chain / 1e6 - 34.56) < 0.01
    assert abs(t["update"] / 1e6 - 24.82) < 0.01
    text = open(os.path.join(ROOT, "profiles", "hbm_traffic.md")).read()
    data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    cal = data["calibration"]
    assert cal["copy_read_kib"] == cal["copy_written_kib"] == 262144
    assert 1.9 < cal["copy_read_kib"] / cal["fetch_kib"] < 2.1
    assert cal["write_kib"] == pytest.approx(cal["copy_written_kib"])
