"""GPU: the reported bench line, run in-process on the short timed region the full test run uses.

A timed region shorter than one graph span (20 steps against graphs of 8 fused launches of
6 steps) must still be timed, from whole graph spans (the depth drops to 5 steps per launch,
one graph of 4 launches), and the line must carry the value, the roofline of the fused kernel
as a fraction of the HBM peak, the single-step figure and the CPU oracle baseline.
"""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_on_a_short_timed_region():
    print("case: bench torus1415 --steps 20 --warmup 5 --cpu-steps 2 in-process", flush=True)
    sys.path.insert(0, ROOT)
    import bench
    args = bench.parse(["--steps", "20", "--warmup", "5", "--cpu-steps", "2"])
    out = bench.bench_torus(args)
    json.dumps(out)
    assert out["value"] > 0 and out["ms_per_step"] > 0 and out["steps"] == 20
    assert out["config"]["triangles"] == 4004450 and out["config"]["edges"] == 6006675
    assert out["dtype"] == "f32"
    r = out["roofline"]
    assert r["kernel"] == "k_fused" and r["launches_timed"] == 20 // r["steps_per_launch"]
    assert out["config"]["graph_launches"] * r["steps_per_launch"] == 20
    assert 0 < r["frac"] <= 1 and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert r["algorithmic_bytes_per_launch"] == 64 * 4004450
    s = r["single_step"]
    assert 0 < s["frac"] <= 1 and s["ms_per_step"] > 0
    c = out["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["nproc"] >= 1
    assert c["value_1_thread"] > 0
