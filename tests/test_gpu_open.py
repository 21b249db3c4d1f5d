"""GPU: the triangle mesh tied to a PML frame (tyee_open_*) against the open-boundary oracle.

Element by element on the same seeded states: FP64 within 1e-12 (relative L2 per field, the
arithmetic differs only in the order of a few additions), FP32 within 1e-5 after 200 steps
(the FP32 leap-frog's rounding grows about linearly with steps from 6e-8 per operation; the
triangle-mesh solver's FP32 bar). The frame cells' split parts are compared separately. The
largest eigenvalue of the mixed operator against the oracle's power iteration. At a larger size
the properties the frame is for: a pulse leaves the box through the PML, stays with a reflecting
frame, and the leap-frog energy is conserved without damping. At the bench's size (4.6M
triangles, graphs of 8 steps) every cell the box's sides cannot reach in 200 steps against the
closed-box oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.open import OpenMesh
from meshgen import box_mesh, box_tri_mesh

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(kind):
    if kind == "tri":
        return box_tri_mesh(12, 9, 1.0, 0.1, 4)
    return box_mesh(10, 8, 0.15, 5, h=1.0)


def _random_state(ref, seed):
    rng = np.random.default_rng(seed)
    E = np.where(ref.inner, rng.standard_normal(ref.ne), 0.0)
    Bx = rng.standard_normal(ref.ncell)
    By = np.where(ref.split, rng.standard_normal(ref.ncell), 0.0)
    return E, Bx, By


@pytest.mark.parametrize("kind,prec,steps,tol", [("tri", "f64", 200, 1e-12), ("square", "f64", 200, 1e-12),
                                                 ("tri", "f32", 200, 1e-5), ("square", "f32", 200, 1e-5)])
def test_stepping_matches_oracle(ty, kind, prec, steps, tol):
    _note(f"case: open {kind} box with a 4-layer PML frame, {prec}, {steps} steps")
    xy, tri, Lx, Ly = _case(kind)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, 4, 0.7, 2.0)
    dt = 0.6 * 2 / ref.omega_max()
    E, Bx, By = _random_state(ref, 3)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    sim = ty.Open(m, ty.pml(4, 0.7, 2.0), dt, prec)
    assert (sim.ne, sim.ncell, sim.nf) == (ref.ne, ref.ncell, ref.nf)
    sim.set_state("E", E)
    sim.set_state("BX", Bx)
    sim.set_state("BY", By)
    sim.step(steps)
    Er, Bxr, Byr = ref.step(E, Bx, By, dt, steps)
    e, bx, by = sim.get_state("E"), sim.get_state("BX"), sim.get_state("BY")
    errs = (_rel(e, Er), _rel(bx, Bxr), _rel(by[ref.nt:], Byr[ref.nt:]))
    _note(f"  rel L2 E {errs[0]:.2e} Bx {errs[1]:.2e} By {errs[2]:.2e}")
    assert max(errs) <= tol
    assert np.all(e[~ref.inner] == 0.0) and np.all(by[:ref.nt] == 0.0)
    # the damping acts: the state decays in the frame against the undamped run's energy
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(bx))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replay_matches_eager_launches(ty, prec):
    """Whole graphs of 8 steps and a remainder of eager steps give the same bits as eager
    launches alone (the same kernels in the same order), and a state set and read back is
    unchanged up to the |e| scaling of E."""
    _note(f"case: open tri box, graph replay against eager launches, {prec}, 203 steps")
    xy, tri, Lx, Ly = _case("tri")
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, 4, 0.7, 2.0)
    dt = 0.6 * 2 / ref.omega_max()
    E, Bx, By = _random_state(ref, 5)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    out = []
    for graph in (8, 0):
        sim = ty.Open(m, ty.pml(4, 0.7, 2.0), dt, prec)
        sim.set_graph(graph)
        sim.set_state("E", E)
        sim.set_state("BX", Bx)
        sim.set_state("BY", By)
        e0 = sim.get_state("E")
        rt = 1e-15 if prec == "f64" else 1e-7
        assert np.all(np.abs(e0 - E) <= rt * np.abs(E) + 1e-300)
        sim.step(203)
        out.append([sim.get_state(f) for f in ("E", "BX", "BY")])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_cfl_matches_oracle(ty):
    xy, tri, Lx, Ly = _case("tri")
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, 3, 0.5, 1.0)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    sim = ty.Open(m, ty.pml(3, 0.5, 1.0), 0.01, "f64")
    lam, iters, ok = sim.cfl(rtol=1e-13)
    assert ok and abs(np.sqrt(lam) - ref.omega_max(rtol=1e-14)) <= 1e-8 * np.sqrt(lam)


def test_pulse_leaves_through_the_pml_at_size(ty):
    _note("case: 96 x 96 triangular-lattice box (21k triangles), 16-layer frame, FP32, a centred pulse")
    xy, tri, Lx, Ly = box_tri_mesh(96, 96, 1.0, 0.1, 7)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    g = ty.open_frame(m, ty.pml(16, 1.0, 0.0))
    nt = g["n_cells"] - g["n_frame_cells"]
    O, S = g["O"], g["S"]
    r2 = np.sum((O - [Lx / 2, Ly / 2]) ** 2, axis=1)
    B0 = np.where(np.arange(len(S)) < nt, np.exp(-r2 / 8.0), 0.0)
    e0 = np.sum(S[:nt] * B0[:nt] ** 2)
    left = {}
    for smax in (0.0, 1.5):
        sim = ty.Open(m, ty.pml(16, 1.0, smax), 1.0, "f32")
        lam, _, ok = sim.cfl(rtol=1e-10)
        assert ok
        dt = 0.5 * 2 / np.sqrt(lam)
        sim = ty.Open(m, ty.pml(16, 1.0, smax), dt, "f32")
        sim.set_state("BX", B0)
        n = int(2.0 * (Lx + Ly) / dt)
        sim.step(n)
        B = sim.get_state("BX") + sim.get_state("BY")
        left[smax] = float(np.sum(S[:nt] * B[:nt] ** 2) / e0)
        _note(f"  sigma_max {smax}: {n} steps, energy left in the box {left[smax]:.2e}")
    assert left[0.0] > 0.05 and left[1.5] < 3e-3


def test_energy_conserved_without_damping(ty):
    xy, tri, Lx, Ly = _case("tri")
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, 4, 0.7, 0.0)
    dt = 0.9 * 2 / ref.omega_max()
    E, Bx, By = _random_state(ref, 9)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    sim = ty.Open(m, ty.pml(4, 0.7, 0.0), dt, "f64")
    sim.set_state("E", E)
    sim.set_state("BX", Bx)
    sim.set_state("BY", By)
    W = []
    b_old = Bx + By
    for _ in range(50):
        sim.step(1)
        e = sim.get_state("E")
        b_new = sim.get_state("BX") + sim.get_state("BY")
        W.append(ref.energy(e, b_old, b_new))
        b_old = b_new
    assert (max(W) - min(W)) / W[0] < 1e-12


def test_timing_and_errors(ty):
    xy, tri, Lx, Ly = _case("square")
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    sim = ty.Open(m, ty.pml(2, 1.0, 1.0), 0.05, "f32")
    sim.set_timing(True)
    sim.step(5)
    t = sim.kernel_ms()
    assert t["steps"] == 5 and t["edge_ms"] > 0 and t["cell_ms"] > 0
    with pytest.raises(ty.TyeeError):
        ty.Open(m, ty.pml(2, 1.0, 1.0), -1.0, "f32")
    with pytest.raises(ty.TyeeError):
        ty.Open(m, ty.pml(0, 1.0, 1.0), 0.05, "f32")
    with pytest.raises(ty.TyeeError):
        sim.set_graph(-1)
    with pytest.raises(ty.TyeeError):
        sim.set_graph(2000)


def _reached_from_sides(om, inner, steps):
    """Edges and triangles that the box's side edges reach in `steps` leap-frog steps: an E
    update reaches every edge of a reached triangle, a B update every triangle of a reached
    edge. Advanced by fronts (only the cells reached in the last update can reach new ones)."""
    te, tt = ~inner, np.zeros(om.nt, bool)
    fresh_e, fresh_t = np.nonzero(te)[0], np.zeros(0, np.int64)
    for _ in range(steps):
        new_e = np.unique(om.A[fresh_t].reshape(-1))
        new_e = new_e[~te[new_e]]
        te[new_e] = True
        cand = np.concatenate([om.R[fresh_e], om.L[fresh_e], om.R[new_e], om.L[new_e]])
        cand = np.unique(cand[cand >= 0])
        fresh_t = cand[~tt[cand]]
        tt[fresh_t] = True
        fresh_e = np.zeros(0, np.int64)
    return te, tt


@pytest.mark.parametrize("fusion", [1, 0])
def test_open1415_bench_configuration_interior_against_oracle(ty, fusion):
    """The bench's open1415 case at its size (1415 x 1415 triangular-lattice box, jitter 0.1,
    seed 11: 4.6M triangles, tied to a 16-layer frame, sigma_max 1, cubic grading), FP32, in the
    bench's launch configuration (graphs of 8 steps): 200 steps from a seeded random state in
    the box, the frame at rest. The frame is too large for the open-boundary oracle at this size,
    but away from the box's sides the scheme is the closed box's: the FP64 oracle advances the
    box with conducting sides, and every edge and triangle the sides cannot reach in 200 steps
    is compared element by element (the sides' influence is followed exactly through the mesh:
    a step's E update reaches the edges of a reached triangle, its B update the triangles of a
    reached edge). FP32 bar 1e-5 (relative L2 per field over the compared cells), as for the
    frame at small sizes. Both launch configurations of the bench: graphs of single steps, and
    the fused box with the frame's band."""
    _note(f"case: open1415 (4.6M triangles + 16-layer frame) FP32, {'graphs of 8 steps' if fusion == 1 else 'fused box'}, "
          "200 steps, interior against the closed-box oracle")
    xy, tri, Lx, Ly = box_tri_mesh(1415.0, 1415.0, 1.0, 0.1, 11)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    rng = np.random.default_rng(5)
    inner = (om.R >= 0) & (om.L >= 0)
    E0 = np.where(inner, rng.standard_normal(om.ne), 0.0)
    B0 = rng.standard_normal(om.nt)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    sim = ty.Open(m, ty.pml(16, 1.0, 1.0, 3.0), dt, "f32")
    if fusion != 1:
        sim.set_fusion(m, fusion)
    assert sim.nt == om.nt and sim.ne > om.ne
    E = np.zeros(sim.ne)
    E[:om.ne] = E0
    Bx = np.zeros(sim.ncell)
    Bx[:om.nt] = B0
    sim.set_state("E", E)
    sim.set_state("BX", Bx)
    sim.set_state("BY", np.zeros(sim.ncell))
    sim.step(200)
    e_gpu, b_gpu = sim.get_state("E")[:om.ne], sim.get_state("BX")[:om.nt]
    del sim
    ref = om.step(E0, B0, dt, 200)
    te, tt = _reached_from_sides(om, inner, 200)
    ce, ct = ~te, ~tt
    errs = (_rel(e_gpu[ce], ref["E"][ce]), _rel(b_gpu[ct], ref["B"][ct]))
    _note(f"  {ce.sum()} edges and {ct.sum()} triangles compared: rel L2 E {errs[0]:.2e} B {errs[1]:.2e}")
    assert ct.sum() > om.nt // 4
    assert max(errs) <= 1e-5


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-12)])
@pytest.mark.parametrize("K,tile", [(6, 256), (3, 512), (0, 0)])
def test_fused_box_matches_oracle(ty, prec, tol, K, tile):
    """Fused stepping of the box (tyee_open_set_fusion): a 60 x 50 triangular-lattice box with
    an 8-layer frame, 203 steps (whole groups of K plus a remainder of single steps) from a
    random state in the box and the frame, against the open-boundary oracle element by element
    at the single-step bars, against the single-step launches, and bit for bit between the
    fused groups replayed from graphs and launched one by one."""
    _note(f"case: open tri box 60 x 50, 8-layer frame, fused K={K} tile={tile}, {prec}, 203 steps")
    xy, tri, Lx, Ly = box_tri_mesh(60.0, 50.0, 1.0, 0.1, 3)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, 8, 1.0, 1.0)
    dt = 0.6 * 2 / ref.omega_max()
    E, Bx, By = _random_state(ref, 7)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    out = {}
    for fused, graph in ((False, 8), (True, 8), (True, 0)):
        sim = ty.Open(m, ty.pml(8, 1.0, 1.0), dt, prec)
        sim.set_graph(graph)
        if fused:
            sim.set_fusion(m, K, tile)
        sim.set_state("E", E)
        sim.set_state("BX", Bx)
        sim.set_state("BY", By)
        sim.step(203)
        out[(fused, graph)] = (sim.get_state("E"), sim.get_state("BX"), sim.get_state("BY"))
    for a, b in zip(out[(True, 8)], out[(True, 0)]):     # graphs of 8 groups replay the eager groups
        assert np.array_equal(a, b)
    out = {False: out[(False, 8)], True: out[(True, 8)]}
    Er, Bxr, Byr = ref.step(E, Bx, By, dt, 203)
    e, bx, by = out[True]
    errs = (_rel(e, Er), _rel(bx, Bxr), _rel(by[ref.nt:], Byr[ref.nt:]))
    _note(f"  fused vs oracle: rel L2 E {errs[0]:.2e} Bx {errs[1]:.2e} By {errs[2]:.2e}")
    assert max(errs) <= tol
    e1, bx1, by1 = out[False]
    d = (_rel(e, e1), _rel(bx, bx1), _rel(by[ref.nt:], by1[ref.nt:]))
    _note(f"  fused vs single-step: {d[0]:.2e} {d[1]:.2e} {d[2]:.2e}")
    assert max(d) <= tol
    assert np.all(e[~ref.inner] == 0.0)


def test_fused_box_arguments_and_switching_off(ty):
    """tyee_open_set_fusion refuses another mesh and bad depths or tiles; depth 1 switches it
    off (single steps again, bit for bit); the state carries over either way."""
    _note("case: open fused box: argument errors, switching on and off mid-run")
    xy, tri, Lx, Ly = box_tri_mesh(30.0, 24.0, 1.0, 0.1, 2)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    xy2, tri2, Lx2, Ly2 = box_tri_mesh(30.0, 26.0, 1.0, 0.1, 2)
    other = ty.Mesh(xy2, tri2, False, L=Lx2, Ly=Ly2)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, 4, 0.7, 2.0)
    dt = 0.6 * 2 / ref.omega_max()
    E, Bx, By = _random_state(ref, 9)
    runs = {}
    for mode in ("single", "switch"):
        sim = ty.Open(m, ty.pml(4, 0.7, 2.0), dt, "f64")
        for bad in ((other, 6, 0), (m, 9, 0), (m, -1, 0), (m, 6, 100)):
            with pytest.raises(ty.TyeeError):
                sim.set_fusion(*bad)
        sim.set_state("E", E)
        sim.set_state("BX", Bx)
        sim.set_state("BY", By)
        if mode == "switch":
            sim.set_fusion(m, 4, 256)
        sim.step(40)
        if mode == "switch":
            sim.set_fusion(m, 1)
        sim.step(37)
        runs[mode] = (sim.get_state("E"), sim.get_state("BX"), sim.get_state("BY"))
    Er, Bxr, Byr = ref.step(E, Bx, By, dt, 77)
    for got, want in zip(runs["switch"], (Er, Bxr, Byr)):
        assert _rel(got, want) <= 1e-12
    for a, b in zip(runs["switch"], runs["single"]):
        assert _rel(a, b) <= 1e-12
