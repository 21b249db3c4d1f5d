"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Both sides receive the same seeded (xy, tri) and dt; each samples the closed-form initial
fields on its own geometry. Tolerances: FP64 fields within 1e-12 relative L2; FP32 fields
(geometry and coefficients from FP64) within 1e-5 after 100 steps; reorderings and fusion
depths bit-identical after the inverse permutation.
"""
import sys

import numpy as np
import pytest

import oracle
from meshgen import (lattice_mesh, make_workload, triangle_particle_mask, line_source_pairs,
                     scramble, plasma_workload)
from common import rel_l2, cavity_state, packet_state

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def _pair(xy, tri, periodic):
    return oracle.OracleMesh(xy, tri, periodic), None


def run_gpu(ty, xy, tri, periodic, dt, E0_fn, steps, prec, order="none", seed=0, fusion=1,
            media=None, source=None, gamma=None, chunks=1, tile=0, want_info=False):
    m = ty.Mesh(xy, tri, periodic)
    m.reorder(order, seed)
    view = m.view()
    E0, B0 = E0_fn(view)
    sim = ty.Sim(m, dt, prec)
    if gamma is not None:
        sim.set_edge_scale(gamma)
    if media is not None:
        sim.set_media(*media)
    if source is not None:
        sim.set_source(*source)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_fusion(fusion, tile)
    for c in range(chunks):
        sim.step(steps // chunks + (steps % chunks if c == chunks - 1 else 0))
    out = {f: sim.get_state(f) for f in ("E", "B", "J", "Q")}
    if want_info:
        return out, view, sim.fusion_info()
    return out, view


def test_c1_cavity_fp64_full_2000_steps(ty):
    _note("case: cavity45 fp64 2000 steps")
    w = make_workload("cavity45")
    om = oracle.OracleMesh(w["xy"], w["tri"], False)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    E0, B0 = cavity_state(om)
    ref = om.step(E0, B0, dt, 2000)
    got, _ = run_gpu(ty, w["xy"], w["tri"], False, dt, cavity_state, 2000, "f64")
    assert rel_l2(got["E"], ref["E"]) < 1e-12
    assert rel_l2(got["B"], ref["B"]) < 1e-12


@pytest.mark.parametrize("order", ["none", "random", "morton", "rcm"])
def test_periodic_fp32_100_steps(ty, order):
    n = 96
    _note(f"case: torus{n} fp32 100 steps order={order}")
    xy, tri = lattice_mesh(n, 0.25, 1, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    fn = lambda side: packet_state(side, dt, n)
    E0, B0 = fn(om)
    ref = om.step(E0, B0, dt, 100)
    got, _ = run_gpu(ty, xy, tri, True, dt, fn, 100, "f32", order=order, seed=3)
    assert rel_l2(got["E"], ref["E"]) < 1e-5
    assert rel_l2(got["B"], ref["B"]) < 1e-5


def test_reorderings_bit_identical_fp64(ty):
    n = 40
    _note(f"case: torus{n} fp64 reorder bit-exactness")
    xy, tri = lattice_mesh(n, 0.25, 2, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    fn = lambda side: packet_state(side, dt, n, cells=8.0, sigma=0.2)
    base, _ = run_gpu(ty, xy, tri, True, dt, fn, 300, "f64", order="none")
    ref = om.step(*fn(om), dt, 300)
    assert rel_l2(base["E"], ref["E"]) < 1e-12 and rel_l2(base["B"], ref["B"]) < 1e-12
    for order in ("random", "morton", "rcm"):
        got, _ = run_gpu(ty, xy, tri, True, dt, fn, 300, "f64", order=order, seed=9)
        assert np.array_equal(got["E"], base["E"]), order
        assert np.array_equal(got["B"], base["B"]), order


def test_scrambled_input_and_chunked_steps(ty):
    n = 20
    _note("case: cavity20 scrambled winding, chunked stepping fp64")
    xy, tri = lattice_mesh(n, 0.2, 4, periodic=False)
    st, _ = scramble(tri, 1)
    om = oracle.OracleMesh(xy, st, False)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    ref = om.step(*cavity_state(om), dt, 500)
    got, _ = run_gpu(ty, xy, st, False, dt, cavity_state, 500, "f64", order="rcm", chunks=5)
    assert rel_l2(got["E"], ref["E"]) < 1e-12 and rel_l2(got["B"], ref["B"]) < 1e-12


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_plasma_and_source(ty, prec, tol):
    n = 48
    _note(f"case: torus{n} plasma+source {prec}")
    xy, tri = lattice_mesh(n, 0.25, 5, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    chi = triangle_particle_mask(xy, tri, True, side=0.5, center=(0.6, 0.5))
    wp2_tri = (0.02 / dt) ** 2 * chi.astype(float)     # omega_p dt = 0.02
    pairs, w = line_source_pairs(xy, tri, True, 1.0, 1.0 / n)
    w = w * (0.01 / dt)
    omega = 2 * np.pi / (200 * dt)       # a source period of 200 steps
    fn = lambda side: packet_state(side, dt, n, cells=10.0)
    E0, B0 = fn(om)
    ref = om.step(E0, B0, dt, 300, wp2=om.edge_wp2(wp2_tri), nu=0.05 / dt / 100,
                  src=(pairs, w, omega, 1.0))
    got, _ = run_gpu(ty, xy, tri, True, dt, fn, 300, prec,
                     media=(wp2_tri, 0.05 / dt / 100), source=(pairs, w, omega, 1.0),
                     order="morton")
    for f in ("E", "B", "J", "Q"):
        assert rel_l2(got[f], ref[f]) < tol, f
    assert np.max(np.abs(ref["Q"])) > 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("fusion,tile,chunks", [(2, 0, 1), (4, 0, 3), (8, 1024, 1), (4, 256, 2),
                                               (3, 0, 1), (5, 0, 2), (6, 0, 1), (7, 512, 1)])
def test_plasma_fused_bit_identical(ty, prec, fusion, tile, chunks):
    # conforming particle and line source: the fused launch splits tiles into a plain class
    # and a class holding special edges; every field, the current and the charge must equal
    # the single-step launches bit for bit (203 steps: fused launches plus single-step tails)
    w = plasma_workload(64)
    n, xy, tri = w["n"], w["xy"], w["tri"]
    _note(f"case: plasma{n} {prec} fusion={fusion} tile={tile} chunks={chunks} bit-exactness")
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    fn = lambda side: packet_state(side, dt, n, cells=8.0)
    media = (w["wp2_tri"], w["nu"])
    src = (w["src_pairs"], w["src_weights"], w["src_omega"], w["src_cycles"])
    base, _ = run_gpu(ty, xy, tri, True, dt, fn, 203, prec, order="morton", fusion=1,
                      media=media, source=src)
    got, _, info = run_gpu(ty, xy, tri, True, dt, fn, 203, prec, order="morton", fusion=fusion,
                           media=media, source=src, tile=tile, chunks=chunks, want_info=True)
    assert info["steps_per_launch"] == fusion
    assert 0 < info["special_tiles"] < info["tiles"] or info["tiles"] == 1
    for f in ("E", "B", "J", "Q"):
        assert np.array_equal(got[f], base[f]), f
    ref = om.step(*fn(om), dt, 203, wp2=om.edge_wp2(w["wp2_tri"]), nu=w["nu"], src=src)
    tol = 1e-12 if prec == "f64" else 1e-5
    for f in ("E", "B", "J", "Q"):
        assert rel_l2(got[f], ref[f]) < tol, f
    assert np.max(np.abs(ref["J"])) > 0 and np.max(np.abs(ref["Q"])) > 0


def test_edge_scale_fp64(ty):
    n = 30
    _note("case: torus30 learned-scale coefficients fp64")
    xy, tri = lattice_mesh(n, 0.25, 6, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    gamma = 1.0 + 0.1 * np.sin(np.arange(om.ne) * 0.37)
    dt = 0.5 * 2 / np.sqrt(om.power(gamma=gamma)[0])
    fn = lambda side: packet_state(side, dt, n, cells=8.0)
    ref = om.step(*fn(om), dt, 400, gamma=gamma)
    got, _ = run_gpu(ty, xy, tri, True, dt, fn, 400, "f64", gamma=gamma, order="rcm")
    assert rel_l2(got["E"], ref["E"]) < 1e-12 and rel_l2(got["B"], ref["B"]) < 1e-12


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("fusion,tile", [(2, 0), (4, 0), (8, 0), (4, 512), (8, 1024), (2, 256),
                                         (3, 0), (5, 0), (6, 0), (7, 0), (6, 1536), (5, 768)])
def test_fusion_depth_bit_identical(ty, fusion, tile, prec):
    n = 64
    _note(f"case: torus{n} {prec} fusion={fusion} tile={tile} bit-exactness")
    xy, tri = lattice_mesh(n, 0.25, 7, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    fn = lambda side: packet_state(side, dt, n)
    base, _ = run_gpu(ty, xy, tri, True, dt, fn, 37, prec, order="morton", fusion=1)
    got, _ = run_gpu(ty, xy, tri, True, dt, fn, 37, prec, order="morton", fusion=fusion,
                     tile=tile)
    assert np.array_equal(got["E"], base["E"]) and np.array_equal(got["B"], base["B"])


@pytest.mark.parametrize("order", ["none", "random", "rcm"])
def test_fusion_any_numbering_and_closed_box(ty, order):
    n = 40
    _note(f"case: cavity{n} fp64 fusion=4 order={order}")
    xy, tri = lattice_mesh(n, 0.2, 3, periodic=False)
    om = oracle.OracleMesh(xy, tri, False)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    ref = om.step(*cavity_state(om), dt, 203)
    base, _ = run_gpu(ty, xy, tri, False, dt, cavity_state, 203, "f64", order=order, fusion=1)
    got, _ = run_gpu(ty, xy, tri, False, dt, cavity_state, 203, "f64", order=order, fusion=4,
                     tile=512, chunks=7)
    assert np.array_equal(got["E"], base["E"]) and np.array_equal(got["B"], base["B"])
    assert rel_l2(got["E"], ref["E"]) < 1e-12 and rel_l2(got["B"], ref["B"]) < 1e-12
