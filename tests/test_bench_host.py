"""Host-side pieces of bench.py: the algorithmic byte count of a search, the
committed HBM-traffic figure and its source check, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes():
    # 12 R + s X + (s + 4) X with s = 20 (three objectives) or 16 (two)
    assert bench.alg_bytes(6640816, 251779422, 3) == 3313548968
    assert bench.alg_bytes(10, 100, 2) == 12 * 100 + 16 * 10 + 20 * 10
    assert bench.alg_bytes(0, 0, 3) == 0


def test_traffic_follows_the_profiled_sources(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "k_search_halves_o3_plain3d_n20000.md")) as f:
        line = next(l for l in f if l.startswith("traffic:"))
    kv = dict(t.split("=", 1) for t in line.split()[1:])
    expect = int(1024 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                         float(kv["write_kib"]) * float(kv["write_scale"])))
    monkeypatch.setattr(bench, "search_source_hash", lambda: kv["source_sha256_16"])
    assert bench.measured_traffic() == expect
    # sources that no longer hash to the profiled ones: no traffic figure
    monkeypatch.setattr(bench, "search_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None


def test_source_hash_is_stable():
    h = bench.search_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.search_source_hash() == h


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout
