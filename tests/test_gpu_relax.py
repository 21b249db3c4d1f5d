"""GPU: jello relaxation of the mesh nodes (Section 3, Fig. 5b) through the C ABI.

* the Euler iterate of the spring forces equals the oracle's, node by node, on a closed box
  (outline anchored) and on a torus, with extra anchors honoured;
* the remeshed output is a Delaunay triangulation of the moved nodes (independent check);
* the best iterate is returned with its omega_max (checked by the oracle's power iteration),
  never above the input's;
* the leap-frog run on a relaxed mesh matches the oracle (FP64, C1 family);
* at the bench's size (the 4M-triangle torus), patches of the mesh against the oracle's Euler
  steps, every node the patch's cut cannot reach.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import relax as OR
from meshgen import lattice_mesh, cavity_mode
from common import rel_l2

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


@pytest.mark.parametrize("periodic", [False, True])
def test_euler_iterate_matches_oracle(ty, periodic):
    n = 12
    _note(f"case: relax {n}x{n} periodic={periodic}: 1 round of 20 Euler steps vs oracle")
    xy, tri = lattice_mesh(n, 0.3, 41, periodic=periodic)
    m = ty.Mesh(xy, tri, periodic)
    om = oracle.OracleMesh(xy, tri, periodic)
    anchors = np.array([5, 17, 40], np.int32)
    x1, t1, omegas, st = m.relax(rounds=1, iters=20, step=0.05, keep_best=False, anchors=anchors)
    fixed = om.node_bnd.astype(bool)
    fixed[anchors] = True
    a0, _ = OR.rest_lengths(om.nt, 1.0)
    ref = OR.euler(xy, om.tri, periodic, 1.0, 1.0, a0, 20, 0.05, fixed)
    d = x1 - ref
    if periodic:
        d -= np.round(d)
    _note(f"  max |x - x_ref| {np.max(np.abs(d)):.2e}; flips {st['flips']}; omega "
          f"{omegas[0]:.4e} -> {omegas[1]:.4e}")
    assert np.max(np.abs(d)) < 1e-13
    assert np.array_equal(x1[fixed], xy[fixed])
    assert st["step_used"] == 0.05 and st["best_round"] == 1
    # the output triangulation is Delaunay for the moved nodes (the oracle accepts only
    # positive dual lengths), same counts
    r = oracle.OracleMesh(x1, t1, periodic)
    assert np.min(r.d[r.interior] / r.elen[r.interior]) > 0
    assert (r.nv, r.nt, r.ne) == (om.nv, om.nt, om.ne)
    assert abs(r.S.sum() - 1.0) < 1e-12
    lam, _, _ = r.power()
    assert abs(np.sqrt(lam) / omegas[1] - 1) < 1e-9
    assert st["energy_final"] < st["energy_initial"]


def test_best_iterate_and_a_relaxed_cavity_run(ty):
    n = 45
    _note(f"case: relax the {n}x{n} cavity (jitter 0.2), 8 rounds x 100 steps, then 2,000 FP64 "
          "steps on the relaxed mesh vs oracle")
    xy, tri = lattice_mesh(n, 0.2, 0, periodic=False)
    m = ty.Mesh(xy, tri, False)
    x1, t1, omegas, st = m.relax(rounds=8, iters=100, step=0.05)
    _note(f"  omega per round {np.array2string(omegas, precision=4)}; best round "
          f"{st['best_round']}, flips {st['flips']}")
    assert st["omega_best"] == np.min(omegas) and st["omega_best"] <= st["omega_initial"]
    assert st["omega_best"] == omegas[st["best_round"]]
    om = oracle.OracleMesh(x1, t1, False)
    lam, _, ok = om.power()
    assert ok and abs(np.sqrt(lam) / st["omega_best"] - 1) < 1e-9
    # outline nodes stay where they were
    out = (xy[:, 0] == 0) | (xy[:, 0] == 1) | (xy[:, 1] == 0) | (xy[:, 1] == 1)
    assert np.array_equal(x1[out], xy[out])
    # leap-frog on the relaxed mesh, its own eq. 20 step: FP64 GPU against the oracle
    dt = 0.5 * 2 / np.sqrt(lam)
    mr = ty.Mesh(x1, t1, False)
    mr.reorder("morton")
    v = mr.view()
    sim = ty.Sim(mr, dt, "f64")
    sim.set_state("B", cavity_mode(v["O"], 1, 1))
    sim.set_fusion(4, 0)
    sim.step(2000)
    ref = om.step(np.zeros(om.ne), cavity_mode(om.O, 1, 1), dt, 2000)
    eE, eB = rel_l2(sim.get_state("E"), ref["E"]), rel_l2(sim.get_state("B"), ref["B"])
    _note(f"  relaxed mesh, 2,000 steps at dt {dt:.4e}: rel L2 E {eE:.2e} B {eB:.2e}")
    assert eE < 1e-12 and eB < 1e-12


def _patch_check(xy, tri, x_new, centre, radius, steps, step, a0):
    """Advance the patch of `tri` around `centre` (triangles whose centroid, taken with minimum
    images on the unit torus, lies within `radius`) by the oracle's Euler steps, with the nodes
    whose star the patch cuts held fixed, and compare every node the cut cannot reach in
    `steps` steps (a step moves a node by the forces of the triangles it belongs to) with
    `x_new`. Returns (compared nodes, largest difference)."""
    mi = lambda d: d - np.round(d)
    v0 = xy[tri[:, 0]]
    cen = v0 + (mi(xy[tri[:, 1]] - v0) + mi(xy[tri[:, 2]] - v0)) / 3.0
    sel = np.sum(mi(cen - np.asarray(centre)) ** 2, axis=1) < radius ** 2
    sub = tri[sel]
    full_count = np.bincount(tri.reshape(-1), minlength=len(xy))
    sub_count = np.bincount(sub.reshape(-1), minlength=len(xy))
    cut = (sub_count > 0) & (sub_count < full_count)
    fixed = (sub_count == 0) | cut
    ref = OR.euler(xy, sub, False, 1.0, 1.0, a0, steps, step, fixed)
    reached = cut.copy()
    for _ in range(steps):
        reached[sub[np.any(reached[sub], axis=1)].reshape(-1)] = True
    cmp = (sub_count > 0) & ~reached
    return int(cmp.sum()), float(np.max(np.abs(mi(x_new[cmp] - ref[cmp]))))


def test_torus1415_relaxation_sampled_against_oracle(ty):
    """The bench's relaxation input at its size (1415 x 1415 torus, jitter 0.25, seed 1: 4.0M
    triangles): one round of 20 Euler steps (step 0.05) on the GPU. The oracle's Euler steps
    loop over edges and triangles in Python, so it takes three patches of the mesh (triangles
    within 35 lattice spacings of a centre), the nodes whose star the patch cuts held fixed,
    and every node the cut cannot reach in 20 steps must agree (the bar of the small cases,
    1e-13 in the unit torus)."""
    n = 1415
    _note(f"case: relax torus{n} (4.0M triangles): 1 round of 20 Euler steps, three patches vs oracle")
    xy, tri = lattice_mesh(n, 0.25, 1, periodic=True)
    m = ty.Mesh(xy, tri, True)
    x1, t1, omegas, st = m.relax(rounds=1, iters=20, step=0.05, keep_best=False)
    assert st["step_used"] == 0.05
    a0, _ = OR.rest_lengths(len(tri), 1.0)
    for c in ((0.31, 0.47), (0.66, 0.28), (0.52, 0.73)):
        k, worst = _patch_check(xy, np.asarray(tri, np.int64), x1, c, 35.0 / n, 20, 0.05, a0)
        _note(f"  patch at {c}: {k} nodes compared, max |x - x_ref| {worst:.2e}")
        assert k > 200 and worst < 1e-13
