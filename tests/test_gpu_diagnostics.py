"""GPU: probes against the oracle, leap-frog energy and discrete Gauss law through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
from meshgen import lattice_mesh, triangle_particle_mask, line_source_pairs
from common import rel_l2, packet_state, cavity_state

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def test_probes_match_oracle_trajectory(ty):
    n = 48
    _note("case: torus48 fp64 probes E/B every 8 steps with fusion 4")
    xy, tri = lattice_mesh(n, 0.25, 11, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    v = m.view()
    sim = ty.Sim(m, dt, "f64")
    E0, B0 = packet_state(v, dt, n, cells=8.0)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_fusion(4, 512)
    rng = np.random.default_rng(0)
    eids = rng.choice(om.ne, 50, replace=False).astype(np.int32)
    tids = rng.choice(om.nt, 40, replace=False).astype(np.int32)
    pe = sim.add_probe("E", eids, every=8, max_samples=10)
    pb = sim.add_probe("B", tids, every=8, max_samples=10)
    sim.step(30)
    sim.step(70)           # 100 steps: samples at 8, 16, ..., 80 (capacity 10 -> 8..80)
    se, sb = sim.read_probe(pe), sim.read_probe(pb)
    assert se.shape == (10, 50) and sb.shape == (10, 40)
    E, B = packet_state(om, dt, n, cells=8.0)
    for t in range(10):
        r = om.step(E, B, dt, 8, n0=8 * t)
        E, B = r["E"], r["B"]
        assert rel_l2(se[t], E[eids]) < 1e-12
        assert rel_l2(sb[t], B[tids]) < 1e-12


def test_leapfrog_energy_conserved_on_gpu(ty):
    _note("case: cavity30 fp64 W_h conservation, fusion 8")
    xy, tri = lattice_mesh(30, 0.25, 12, periodic=False)
    m = ty.Mesh(xy, tri, False)
    m.reorder("morton")
    lam, _, _ = m.cfl()
    dt = 0.5 * 2 / np.sqrt(lam)
    v = m.view()
    sim = ty.Sim(m, dt, "f64")
    rng = np.random.default_rng(3)
    sim.set_state("E", rng.standard_normal(m.ne))
    sim.set_state("B", rng.standard_normal(m.nt))
    sim.set_fusion(8, 256)
    w0 = sim.diagnostics()["energy_h"]
    sim.step(1600)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0 and d["step"] == 1600
    assert abs(d["energy_h"] / w0 - 1) < 1e-11
    # eq. 8 form differs from W_h by O((omega dt)^2) but stays bounded
    assert 0.1 < d["energy"] / w0 < 10


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 2e-4)])
def test_gauss_law_and_plasma_probes(ty, prec, tol):
    n = 40
    _note(f"case: torus40 {prec} plasma+source Gauss law and J/Q probes")
    xy, tri = lattice_mesh(n, 0.25, 13, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    chi = triangle_particle_mask(xy, tri, True, side=0.5, center=(0.6, 0.5)).astype(float)
    wp2_tri = (0.03 / dt) ** 2 * chi
    pairs, w = line_source_pairs(xy, tri, True, 1.0, 1.0 / n)
    w = w * (0.01 / dt)
    omega = 2 * np.pi / (150 * dt)
    m = ty.Mesh(xy, tri, True)
    m.reorder("rcm")
    v = m.view()
    sim = ty.Sim(m, dt, prec)
    E0, B0 = packet_state(v, dt, n, cells=8.0)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_media(wp2_tri, 1e-3 / dt)
    sim.set_source(pairs, w, omega, 2.0)
    g0 = sim.gauss()
    plasma_edges = np.nonzero(om.edge_wp2(wp2_tri))[0][:20].astype(np.int32)
    pj = sim.add_probe("J", plasma_edges, every=25, max_samples=8)
    pq = sim.add_probe("Q", np.arange(0, om.nv, 7, dtype=np.int32), every=25, max_samples=8)
    sim.step(200)
    g1 = sim.gauss()
    assert np.max(np.abs(g1 - g0)) < tol * np.max(np.abs(g0))
    ref_E, ref_B = packet_state(om, dt, n, cells=8.0)
    # the Gauss residual at the start and after 200 steps equals the oracle's (D E) - Q
    assert np.max(np.abs(g0 - om.div(ref_E))) < tol * np.max(np.abs(g0))
    J = Q = None
    sj, sq = sim.read_probe(pj), sim.read_probe(pq)
    assert len(sj) == 8
    for t in range(8):
        r = om.step(ref_E, ref_B, dt, 25, n0=25 * t, J=J, Q=Q, wp2=om.edge_wp2(wp2_tri),
                    nu=1e-3 / dt, src=(pairs, w, omega, 2.0))
        ref_E, ref_B, J, Q = r["E"], r["B"], r["J"], r["Q"]
        t_tol = 1e-11 if prec == "f64" else 1e-4
        assert rel_l2(sj[t], J[plasma_edges]) < t_tol
        assert rel_l2(sq[t], Q[::7]) < t_tol
    g_ref = om.div(ref_E) - Q
    assert np.max(np.abs(g1 - g_ref)) < tol * np.max(np.abs(g_ref))


@pytest.mark.parametrize("prec,periodic,tol", [("f64", True, 1e-12), ("f32", True, 1e-6),
                                               ("f64", False, 1e-12)])
def test_device_diagnostics_match_host_sums(ty, prec, periodic, tol):
    n = 36
    _note(f"case: diagnostics reduction vs host sums, {prec} periodic={periodic}, learned scale")
    xy, tri = lattice_mesh(n, 0.25, 13, periodic=periodic)
    m = ty.Mesh(xy, tri, periodic)
    m.reorder("rcm")
    v = m.view()
    gamma = 1.0 + 0.05 * np.sin(np.arange(m.ne) * 0.7)
    lam, _, _ = m.cfl(gamma=gamma)
    dt = 0.5 * 2 / np.sqrt(lam)
    sim = ty.Sim(m, dt, prec)
    sim.set_edge_scale(gamma)
    rng = np.random.default_rng(4)
    sim.set_fusion(4, 0)
    E0, B0 = rng.standard_normal(m.ne), rng.standard_normal(m.nt)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.step(37)
    d = sim.diagnostics()
    E, B = sim.get_state("E"), sim.get_state("B")
    # the oracle, canonical numbering, same start (outer edges hold no field), same scale
    om = oracle.OracleMesh(xy, tri, periodic)
    E0 = np.where(om.interior, E0, 0.0)
    r = om.step(E0, B0, dt, 37, gamma=gamma, want_prev=True)
    # eq. 8 W and the leap-frog invariant W_h against the oracle's (FP64 serial sums); FP32
    # fields from a rough (random) start drift from FP64 by ~1e-6 in 37 steps
    otol = 1e-12 if prec == "f64" else 2e-5
    assert abs(d["energy"] / om.energy(r["E"], r["B"]) - 1) < otol
    assert abs(d["energy_h"] / om.energy(r["E"], r["B_prev"], r["B"]) - 1) < otol
    # the device reduction against the oracle's sum over the device's own fields
    assert abs(d["energy"] / om.energy(E, B) - 1) < tol
    assert abs(d["max_abs_E"] / np.max(np.abs(E)) - 1) < 1e-6
    assert d["max_abs_B"] == np.max(np.abs(B))
    assert d["nonfinite"] == 0 and d["step"] == 37
    assert sim.diagnostics() == d                      # deterministic
