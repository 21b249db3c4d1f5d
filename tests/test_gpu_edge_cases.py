"""GPU: degenerate and boundary cases of the stepping path, each against the oracle or the
single-step launches.

* the smallest meshes: an 8-triangle closed box (one interior node) and a 4 x 4 torus
  (32 triangles), where one tile holds the whole mesh and its halo rings wrap around the
  torus, at every fusion depth;
* a torus split into two tiles whose halos cover each other completely (K = 8);
* zero-step calls, all-zero media, empty sources and a current set on non-plasma edges;
* argument errors of the launch configuration;
* HIP-graph replay (fused or one step per launch) equal to eager launches, with tails.
"""
import sys

import numpy as np
import pytest

import oracle
from meshgen import lattice_mesh
from common import rel_l2, cavity_state, packet_state

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def _run(ty, xy, tri, periodic, dt, E0, B0, steps, prec, fusion, tile=0, media=None, src=None,
         order="morton"):
    m = ty.Mesh(xy, tri, periodic)
    m.reorder(order, 1)
    sim = ty.Sim(m, dt, prec)
    if media is not None:
        sim.set_media(*media)
    if src is not None:
        sim.set_source(*src)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_fusion(fusion, tile)
    sim.step(steps)
    return {f: sim.get_state(f) for f in ("E", "B", "J", "Q")}, sim


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_eight_triangle_box(ty, prec):
    _note(f"case: box3 (8 triangles) {prec} fusion 1/2/4/8 vs oracle")
    xy, tri = lattice_mesh(3, 0.2, 0, periodic=False)
    om = oracle.OracleMesh(xy, tri, False)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    E0, B0 = cavity_state(om)
    ref = om.step(E0, B0, dt, 77)
    base = None
    for k in range(1, 9):
        got, _ = _run(ty, xy, tri, False, dt, E0, B0, 77, prec, k, order="none")
        tol = 1e-12 if prec == "f64" else 1e-5
        assert rel_l2(got["E"], ref["E"]) < tol and rel_l2(got["B"], ref["B"]) < tol, k
        if base is None:
            base = got
        else:
            assert np.array_equal(got["E"], base["E"]) and np.array_equal(got["B"], base["B"]), k


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_smallest_torus_one_tile_all_depths(ty, prec):
    n = 4
    _note(f"case: torus{n} (32 triangles, one tile) {prec} fusion 1..8, plasma everywhere")
    xy, tri = lattice_mesh(n, 0.25, 0, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    E0, B0 = packet_state(om, dt, n, cells=4.0, sigma=0.5)
    wp2 = np.full(om.nt, (0.3 / dt) ** 2 * 1e-2)
    media = (wp2, 0.1 / dt * 1e-2)
    ref = om.step(E0, B0, dt, 61, wp2=om.edge_wp2(wp2), nu=media[1])
    base = None
    for k in range(1, 9):
        got, sim = _run(ty, xy, tri, True, dt, E0, B0, 61, prec, k, tile=256, media=media)
        if k > 1:
            info = sim.fusion_info()
            assert info["tiles"] == 1 and info["special_tiles"] == 1
        tol = 1e-12 if prec == "f64" else 1e-5
        for f in ("E", "B", "J", "Q"):
            assert rel_l2(got[f], ref[f]) < tol, (k, f)
        if base is None:
            base = got
        else:
            for f in ("E", "B", "J", "Q"):
                assert np.array_equal(got[f], base[f]), (k, f)


def test_two_tiles_whose_halos_wrap(ty):
    n = 16
    _note(f"case: torus{n} (512 triangles) K=8 with 256-triangle tiles, fp64")
    xy, tri = lattice_mesh(n, 0.25, 5, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    E0, B0 = packet_state(om, dt, n, cells=6.0, sigma=0.3)
    ref = om.step(E0, B0, dt, 64)
    got, sim = _run(ty, xy, tri, True, dt, E0, B0, 64, "f64", 8, tile=256)
    assert sim.fusion_info()["tiles"] == 2
    assert rel_l2(got["E"], ref["E"]) < 1e-12 and rel_l2(got["B"], ref["B"]) < 1e-12


def test_zero_steps_empty_media_and_sources(ty):
    n = 24
    _note(f"case: torus{n} zero steps, all-zero media, empty source")
    xy, tri = lattice_mesh(n, 0.25, 9, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    E0, B0 = packet_state(om, dt, n, cells=8.0)
    m = ty.Mesh(xy, tri, True)
    sim = ty.Sim(m, dt, "f64")
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.step(0)
    assert np.array_equal(sim.get_state("B"), B0) and sim.steps == 0
    # all-zero plasma frequency and an empty source leave no special edge: plain stepping
    sim.set_media(np.zeros(om.nt), 0.0)
    sim.set_source(np.zeros((0, 2), np.int32), np.zeros(0), 1.0, 1.0)
    sim.set_fusion(4, 0)
    sim.step(50)
    assert np.count_nonzero(sim.get_state("J")) == 0 and np.count_nonzero(sim.get_state("Q")) == 0
    assert sim.fusion_info()["special_tiles"] == 0
    ref = om.step(E0, B0, dt, 50)
    assert rel_l2(sim.get_state("E"), ref["E"]) < 1e-12
    # a current on an edge without plasma is rejected
    J = np.zeros(om.ne)
    J[3] = 1.0
    with pytest.raises(ty.TyeeError):
        sim.set_state("J", J)


def test_launch_configuration_errors(ty):
    _note("case: launch configuration argument errors")
    xy, tri = lattice_mesh(8, 0.25, 2, periodic=True)
    m = ty.Mesh(xy, tri, True)
    sim = ty.Sim(m, 1e-3, "f32")
    for bad in ((9, 0), (-1, 0), (16, 0), (4, 100), (4, 10000)):
        with pytest.raises(ty.TyeeError):
            sim.set_fusion(*bad)
    with pytest.raises(ty.TyeeError):
        sim.set_graph(3)
    with pytest.raises(ty.TyeeError):
        sim.step(-1)
    with pytest.raises(ty.TyeeError):
        sim.set_source(np.array([[0, 0]], np.int32), np.ones(1), 1.0, 1.0)
    with pytest.raises(ty.TyeeError):
        ty.Sim(m, -1.0, "f32")


@pytest.mark.parametrize("fusion", [1, 4])
def test_graph_replay_equals_eager_launches(ty, fusion):
    n = 40
    _note(f"case: torus{n} fp32 graph replay (8 launches) vs eager, fusion {fusion}, 203 steps")
    xy, tri = lattice_mesh(n, 0.25, 21, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, _ = m.cfl()
    dt = 0.5 * 2 / np.sqrt(lam)
    v = m.view()
    E0, B0 = packet_state(v, dt, n, cells=8.0)
    out = []
    for graph in (0, 8):
        sim = ty.Sim(m, dt, "f32")
        sim.set_state("E", E0)
        sim.set_state("B", B0)
        sim.set_fusion(fusion, 0)
        sim.set_graph(graph)
        for chunk in (50, 100, 53):      # replays, then eager tails
            sim.step(chunk)
        out.append((sim.get_state("E"), sim.get_state("B")))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_copy_probe_rate_is_plausible(ty):
    _note("case: device copy-rate probe, 256 MiB x 5")
    gbs = ty.copy_bandwidth(256 << 20, 5)
    _note(f"  {gbs:.0f} GB/s")
    assert 1000.0 < gbs < 8000.0 * 1.05        # below the published 8 TB/s peak


def test_launch_timing_counts(ty):
    # per-kind HIP-event timing counts every launch of the kinds asked for; graph replays are
    # timed whole; the last step call's time covers its launches
    n = 48
    _note(f"case: torus{n} launch timing counts (single, fused, graph) and a batch's borrowed sim")
    xy, tri = lattice_mesh(n, 0.25, 23, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, _ = m.cfl()
    dt = 0.5 * 2 / np.sqrt(lam)
    sim = ty.Sim(m, dt, "f32")
    sim.set_fusion(1, 0)
    sim.set_profiling(True, kinds=["edge", "tri"])
    sim.step(10)
    t = sim.kernel_times()
    assert t["edge"]["count"] == 10 and t["tri"]["count"] == 10 and t["edge"]["total_ms"] > 0
    assert sim.last_step_ms() >= 0.5 * (t["edge"]["total_ms"] + t["tri"]["total_ms"])
    sim.set_fusion(4, 0)
    sim.set_profiling(True, kinds=["fused"])
    sim.step(40)
    t = sim.kernel_times()
    assert set(t) == {"fused"} and t["fused"]["count"] == 10
    sim.set_graph(4)
    sim.set_profiling(True, kinds=["graph"])
    sim.step(48)                                  # 3 replays of 4 launches of 4 steps
    t = sim.kernel_times()
    assert set(t) == {"graph"} and t["graph"]["count"] == 3
    # timing replays and fused launches together keeps the replays: a remainder shorter than
    # a graph span (4 + 4 steps) runs as two fused launches outside a graph
    sim.set_profiling(True, kinds=["graph", "fused"])
    sim.step(40)
    t = sim.kernel_times()
    assert t["graph"]["count"] == 2 and t["fused"]["count"] == 2
    sim.set_profiling(False)
    sim.step(8)
    assert sim.kernel_times() == {} and sim.steps == 10 + 40 + 48 + 40 + 8
    # a batch hands out its union's simulation for the same queries
    b = ty.Batch([m, m], [dt, dt], "f32")
    b.set_fusion(4, 0)
    b.step(8)
    u = b.sim()
    assert u.fusion_info()["steps_per_launch"] == 4 and u.steps == 8
    assert u.diagnostics()["nonfinite"] == 0
