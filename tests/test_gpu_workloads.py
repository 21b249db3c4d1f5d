"""GPU parity at the workloads' full sizes, in the launch configuration the bench times.

* torus1415 (4,004,450 triangles) FP32, Morton order, default fusion: 100 steps against the
  FP64 oracle element by element (relative L2 <= 1e-5), then replayed from graphs of 8 fused
  launches (the bench's configuration) to 10^4 steps, against the oracle element by element
  (relative L2 <= 1e-3), with the leap-frog energy and the nodal divergence conserved.
* 10^4-step FP32 parity (<= 1e-3) on a reduced torus.
* plasma2830 (16,017,830 triangles, conforming plasma particle, soft line source) FP32: 100
  steps against the oracle (E, B, J, Q), then to 5,000 steps, again element by element (E, B,
  J, Q), with the discrete Gauss law.

The oracle's per-cell loops run on all the host threads OpenMP is given.
"""
import sys

import numpy as np
import pytest

import oracle
from meshgen import lattice_mesh, make_workload, plasma_workload
from common import rel_l2, packet_state

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def test_torus1415_full_size_fp32(ty):
    _note("case: torus1415 full size fp32 fused (bench configuration)")
    w = make_workload("torus1415")
    xy, tri, n = w["xy"], w["tri"], w["n"]
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, ok = m.cfl()
    assert ok
    dt = 0.5 * 2 / np.sqrt(lam)
    v = m.view()
    sim = ty.Sim(m, dt, "f32")
    sim.set_fusion(0, 0)
    E0, B0 = packet_state(v, dt, n)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.step(100)
    E_gpu, B_gpu = sim.get_state("E"), sim.get_state("B")
    om = oracle.OracleMesh(xy, tri, True)
    ref = om.step(*packet_state(om, dt, n), dt, 100)
    _note(f"  rel L2 E {rel_l2(E_gpu, ref['E']):.2e} B {rel_l2(B_gpu, ref['B']):.2e}")
    assert rel_l2(E_gpu, ref["E"]) < 1e-5 and rel_l2(B_gpu, ref["B"]) < 1e-5
    # to 10^4 steps from graphs of 8 fused launches (the bench's replay), element by element
    w0 = sim.diagnostics()["energy_h"]
    div0 = om.div(E_gpu)
    sim.set_graph(8)
    sim.step(9900)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0 and d["step"] == 10000
    E_gpu, B_gpu = sim.get_state("E"), sim.get_state("B")
    _note("  oracle: 9,900 further steps")
    ref = om.step(ref["E"], ref["B"], dt, 9900, n0=100)
    eE, eB = rel_l2(E_gpu, ref["E"]), rel_l2(B_gpu, ref["B"])
    _note(f"  10^4 steps: rel L2 E {eE:.2e} B {eB:.2e}; W_h drift {d['energy_h'] / w0 - 1:.2e}")
    assert eE < 1e-3 and eB < 1e-3
    assert abs(d["energy_h"] / w0 - 1) < 1e-4
    div1 = om.div(E_gpu)
    assert np.max(np.abs(div1 - div0)) < 1e-4 * np.max(np.abs(div0)) + 1e-6


def test_fp32_ten_thousand_steps_reduced_torus(ty):
    n = 128
    _note(f"case: torus{n} fp32 10^4 steps fused vs oracle")
    xy, tri = lattice_mesh(n, 0.25, 1, periodic=True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    v = m.view()
    sim = ty.Sim(m, dt, "f32")
    sim.set_fusion(4, 0)
    E0, B0 = packet_state(v, dt, n)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.step(10000)
    ref = om.step(*packet_state(om, dt, n), dt, 10000)
    eE, eB = rel_l2(sim.get_state("E"), ref["E"]), rel_l2(sim.get_state("B"), ref["B"])
    _note(f"  rel L2 E {eE:.2e} B {eB:.2e}")
    assert eE < 1e-3 and eB < 1e-3


def test_plasma2830_full_size_fp32(ty):
    _note("case: plasma2830 full size fp32 (particle + source, bench configuration)")
    w = plasma_workload()
    xy, tri, n = w["xy"], w["tri"], w["n"]
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, ok = m.cfl()
    assert ok
    dt = 0.5 * 2 / np.sqrt(lam)
    v = m.view()
    src = (w["src_pairs"], w["src_weights"], w["src_omega"], w["src_cycles"])
    sim = ty.Sim(m, dt, "f32")
    sim.set_fusion(0, 0)
    sim.set_media(w["wp2_tri"], w["nu"])
    sim.set_source(*src)
    # a packet centred on the particle, so the plasma current is driven from the first step
    fn = lambda side: packet_state(side, dt, n, cells=20.0)
    E0, B0 = fn(v)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    g0 = sim.gauss()
    sim.step(100)
    got = {f: sim.get_state(f) for f in ("E", "B", "J", "Q")}
    _note("  oracle: mesh + 100 steps")
    om = oracle.OracleMesh(xy, tri, True)
    ref = om.step(*fn(om), dt, 100, wp2=om.edge_wp2(w["wp2_tri"]), nu=w["nu"], src=src)
    errs = {f: rel_l2(got[f], ref[f]) for f in got}
    _note("  rel L2 " + " ".join(f"{f} {e:.2e}" for f, e in errs.items()))
    assert np.max(np.abs(ref["J"])) > 0 and np.max(np.abs(ref["Q"])) > 0
    for f, e in errs.items():
        assert e < 1e-5, f
    # to 5,000 steps: element by element again, and (D E - Q) stays at its initial value
    sim.step(4900)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0 and d["step"] == 5000
    got = {f: sim.get_state(f) for f in ("E", "B", "J", "Q")}
    _note("  oracle: 4,900 further steps")
    ref = om.step(ref["E"], ref["B"], dt, 4900, n0=100, J=ref["J"], Q=ref["Q"],
                  wp2=om.edge_wp2(w["wp2_tri"]), nu=w["nu"], src=src)
    errs = {f: rel_l2(got[f], ref[f]) for f in got}
    _note("  5,000 steps: rel L2 " + " ".join(f"{f} {e:.2e}" for f, e in errs.items()))
    for f, e in errs.items():
        assert e < 1e-3, f
    del om, ref
    g1 = sim.gauss()
    # scale: the largest nodal sum of |d E| (the terms FP32 rounds), and the charge itself
    E1 = got["E"]
    mag = np.zeros(len(g1))
    np.add.at(mag, v["edge_nodes"][:, 0], np.abs(v["d"] * E1))
    np.add.at(mag, v["edge_nodes"][:, 1], np.abs(v["d"] * E1))
    Q1 = got["Q"]
    res = np.max(np.abs(g1 - g0))
    _note(f"  Gauss-law residual after 5,000 steps {res:.3e} (max nodal |d E| sum "
          f"{np.max(mag):.3e}, max |Q| {np.max(np.abs(Q1)):.3e})")
    assert np.max(np.abs(Q1)) > 1e-2 * np.max(mag)      # the charge is not negligible
    assert res < 1e-3 * np.max(mag)
