"""The benchmark's command-line contract and its traffic bookkeeping (no GPU)."""

import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_measured_traffic_table_is_well_formed():
    assert set(bench.MEASURED_TRAFFIC) >= {"jvp_ad", "dcgs_update"}
    for name, m in bench.MEASURED_TRAFFIC.items():
        assert re.fullmatch(r"[0-9a-f]{16}", m["sources"]), name
        assert m["orth"] in ("cgs2", "dcgs2"), name
        assert 0.5 < m["ratio"] <= 1.5, name


def test_traffic_reported_only_for_the_measured_sources():
    h = bench.kernel_sources_hash()
    assert re.fullmatch(r"[0-9a-f]{16}", h) and h == bench.kernel_sources_hash()
    m = bench.MEASURED_TRAFFIC["dcgs_update"]
    assert bench.measured_traffic("dcgs_update", 1e8, m["orth"], sources=m["sources"]) == round(m["ratio"] * 1e8)
    assert bench.measured_traffic("dcgs_update", 1e8, m["orth"], sources="0" * 16) is None
    assert bench.measured_traffic("dcgs_update", 1e8, "cgs2" if m["orth"] == "dcgs2" else "dcgs2",
                                  sources=m["sources"]) is None
    assert bench.measured_traffic("vy", 1e8, m["orth"], sources=m["sources"]) is None
