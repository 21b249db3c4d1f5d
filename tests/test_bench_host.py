"""CPU: the bench's host-side bookkeeping (no GPU): how a timed region is cut into graph spans and
fusion depths, how launch times are averaged from the HIP-event totals, the refusal of more
than one GPU, and the lookup of the stored counter traffic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_region_depth_splits_short_regions_into_whole_graph_spans():
    # the default depth unless a short region would leave single steps over
    assert bench.region_depth(10000, 6) == 6          # long: 1,666 launches, 4 single steps
    assert bench.region_depth(20, 6) == 5             # 20 = 2 x (2 x 5)
    assert bench.region_depth(24, 6) == 6             # already whole
    assert bench.region_depth(30, 6) == 5
    assert bench.region_depth(7, 6) == 6              # no depth splits 7 into an even count
    for steps in range(2, 400):
        k = bench.region_depth(steps, 6)
        assert 2 <= k <= 6
        if k != 6:
            assert steps % (2 * k) == 0


def test_graph_size_fits_the_region():
    assert bench.graph_size(10000, 6, 8) == 8
    assert bench.graph_size(20, 5, 8) == 4            # one graph covers the 20 steps
    assert bench.graph_size(20, 4, 8) == 4            # 16 of 20 steps, an even count
    assert bench.graph_size(7, 6, 8) == 0             # not even two launches fit
    for steps in range(1, 300):
        for K in (2, 4, 5, 6, 8):
            g = bench.graph_size(steps, K, 8)
            assert g == 0 or (g % 2 == 0 and 2 <= g <= 8 and g * K <= steps)


def test_launch_stats_average_graph_and_eager_launches():
    prof = {"graph": {"count": 2, "total_ms": 0.8}, "fused": {"count": 4, "total_ms": 0.2}}
    kind, n, avg = bench.launch_stats(prof, 8)
    assert kind == "fused" and n == 2 * 8 + 4 and abs(avg - 1.0 / 20) < 1e-15
    kind, n, avg = bench.launch_stats({"fused": {"count": 5, "total_ms": 0.25}}, 4)
    assert (kind, n) == ("fused", 5) and abs(avg - 0.05) < 1e-15
    # one launch per half-step: a step is an edge and a triangle launch
    prof = {"edge": {"count": 10, "total_ms": 0.2}, "tri": {"count": 10, "total_ms": 0.1}}
    kind, n, avg = bench.launch_stats(prof, 0)
    assert (kind, n) == ("edge+tri", 10) and abs(avg - 0.03) < 1e-15
    assert bench.launch_stats({}, 8) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_stored_traffic_applies_only_to_its_configuration(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    cfg = {"triangles": 4004450, "steps_per_launch": 6, "tile_tris": 1536, "prec": "f32", "order": "morton"}
    rec = {"kernel": "k_fused", "source_hash": "abc", "config": cfg, "bytes_per_launch": 123}
    with open(bench.traffic_file("torus1415", 6), "w") as f:
        json.dump(rec, f)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.measured_traffic("k_fused", cfg) == 123
    assert bench.measured_traffic("k_fused", dict(cfg, tile_tris=2048)) is None
    assert bench.measured_traffic("k_fused", dict(cfg, steps_per_launch=5)) is None   # no file
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "other")              # sources changed
    assert bench.measured_traffic("k_fused", cfg) is None
