"""GPU: the three-dimensional scheme on tetrahedra (tyee_tet_sim_*) against the tetrahedral
oracle.

Element by element on the same seeded states after 200 steps: FP64 within max(1e-12, 2 N delta)
(relative L2 per field), delta the largest relative difference between the two sides' dual
coefficients A*_e and d_f, which they compute by different formulas (the Voronoi polygon's
shoelace sum against the sum of face kites): a coefficient off by delta moves a mode's phase by
at most N theta delta after N steps, theta = omega dt <= 2 (delta is about 2e-15 on the BCC
meshes, so the bar is 1e-12 there; 1.1e-12 on the irregular mesh). FP32 within 1e-5 (the FP32 leap-frog's
rounding, about 6e-8 per operation, grows about linearly with the steps; the triangle solver's
FP32 bar). Meshes: the direct BCC construction, an irregular Qhull Delaunay mesh (jitter 0.15 h:
edges in 3 to 7 faces, so rows of every length; at 0.25 h a near-degenerate Voronoi polygon,
A* = 2e-7, makes the two sides' independent dual-area formulas differ by 3e-10 and the FP64
comparison a test of conditioning) and a 49k-tetrahedron box (many work-groups and a ragged
last one). Graph replay against eager launches bit for bit; the leap-frog phase of an
eigenvector start; the energy without damping. At 1.3M tetrahedra, properties that hold at any
size: the discrete divergence of B in every tetrahedron stays where it started, and the FP32
energy stays within its rounding. At the bench's size (12M tetrahedra, one graph of 8 steps),
three balls of the mesh against the oracle on their sub-meshes, every cell the cut cannot reach.
"""
import sys

import numpy as np
import pytest

from meshgen.tet import bcc_box
from oracle.tet import TetMesh

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


CASES = {"bcc": ((6, 5, 4), 1.0, 0.05, 3, "direct"), "qhull": ((5, 4, 4), 1.0, 0.15, 5, "qhull"),
         "bigger": ((16, 16, 16), 0.5, 0.05, 5, "direct")}
_cache = {}


def _mesh(kind):
    if kind not in _cache:
        dims, h, jit, seed, method = CASES[kind]
        xyz, tets, L = bcc_box(*dims, h, jit, seed, method=method)
        _cache[kind] = (xyz, tets, TetMesh(xyz, tets, L))
    return _cache[kind]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _state(m, seed):
    rng = np.random.default_rng(seed)
    E = np.where(m.inner_edge, rng.standard_normal(m.ne), 0.0)
    B = rng.standard_normal(m.nf)            # wall faces too: their B never changes
    return E, B


@pytest.mark.parametrize("kind,prec,tol", [("bcc", "f64", 1e-12), ("qhull", "f64", 1e-12), ("bigger", "f64", 1e-12),
                                           ("bcc", "f32", 1e-5), ("qhull", "f32", 1e-5), ("bigger", "f32", 1e-5)])
def test_stepping_matches_oracle(ty, kind, prec, tol):
    _note(f"case: tetrahedra {kind} {CASES[kind][0]}, {prec}, 200 steps")
    xyz, tets, m = _mesh(kind)
    dt = 0.6 * 2 / m.omega_max()
    E, B = _state(m, 1)
    T = ty.Tet(xyz, tets)
    v = T.view()
    ie, fi = m.inner_edge, m.inner_face
    delta = max(np.max(np.abs(v["dual_area"][ie] / m.dual_area[ie] - 1.0)), np.max(np.abs(v["d"][fi] / m.d[fi] - 1.0)))
    if prec == "f64":
        tol = max(tol, 2 * 200 * delta)
    sim = ty.TetSim(T, dt, prec)
    sim.set_state("E", E)
    sim.set_state("B", B)
    sim.step(200)
    Er, Br = m.step(E, B, dt, 200)
    e, b = sim.get_state("E"), sim.get_state("B")
    errs = (_rel(e, Er), _rel(b, Br))
    _note(f"  rel L2 E {errs[0]:.2e} B {errs[1]:.2e} (coefficient difference {delta:.1e}, bar {tol:.1e})")
    assert max(errs) <= tol
    assert np.all(e[~m.inner_edge] == 0.0)
    assert np.all(np.abs(b[~m.inner_face] - B[~m.inner_face]) <= (1e-15 if prec == "f64" else 1e-7) *
                  np.abs(B[~m.inner_face]))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replay_matches_eager_launches(ty, prec):
    _note(f"case: tetrahedra qhull, graph replay against eager launches, {prec}, 203 steps")
    xyz, tets, m = _mesh("qhull")
    dt = 0.6 * 2 / m.omega_max()
    E, B = _state(m, 2)
    T = ty.Tet(xyz, tets)
    out = []
    for graph in (8, 0):
        sim = ty.TetSim(T, dt, prec)
        sim.set_graph(graph)
        sim.set_state("E", E)
        sim.set_state("B", B)
        rt = 1e-15 if prec == "f64" else 1e-7
        assert np.all(np.abs(sim.get_state("E") - E) <= rt * np.abs(E))
        assert np.all(np.abs(sim.get_state("B") - B) <= rt * np.abs(B))
        sim.step(203)
        out.append((sim.get_state("E"), sim.get_state("B")))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_leap_frog_phase_of_an_eigenvector(ty):
    xyz, tets, m = _mesh("bcc")
    K, Me = m.operator()
    s = np.sqrt(Me)
    w, V = np.linalg.eigh(0.5 * ((K.toarray() * s[:, None]) / s[None, :] + ((K.toarray() * s[:, None]) / s[None, :]).T))
    k = np.argmax(w > 1e-6 * w.max()) + 3
    v = np.zeros(m.ne)
    v[m.inner_edge] = V[:, k] / s
    dt = 0.9 * 2 / np.sqrt(w.max())
    theta = np.arccos(1.0 - 0.5 * dt * dt * w[k])
    sim = ty.TetSim(ty.Tet(xyz, tets), dt, "f64")
    sim.set_state("E", v)
    sim.set_state("B", 0.5 * dt * m.curl_e(v))
    sim.step(300)
    assert np.max(np.abs(sim.get_state("E") - np.cos(300 * theta) * v)) < 1e-9 * np.max(np.abs(v))


def test_energy_conserved_without_damping(ty):
    xyz, tets, m = _mesh("qhull")
    E, B = _state(m, 3)
    B = np.where(m.inner_face, B, 0.0)
    dt = 0.9 * 2 / m.omega_max()
    sim = ty.TetSim(ty.Tet(xyz, tets), dt, "f64")
    sim.set_state("E", E)
    sim.set_state("B", B)
    W, b_old = [], B
    for _ in range(50):
        sim.step(1)
        b_new = sim.get_state("B")
        W.append(m.energy(sim.get_state("E"), b_old, b_new))
        b_old = b_new
    assert (max(W) - min(W)) / W[0] < 1e-12


def _tet_faces(tets, face):
    """For every tetrahedron its four faces' ids in the canonical face list."""
    nv = int(max(tets.max(), face.max())) + 1
    tri = np.sort(tets[:, [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]].reshape(-1, 3).astype(np.int64), axis=1)
    key = (tri[:, 0] * nv + tri[:, 1]) * nv + tri[:, 2]
    fk = (face[:, 0].astype(np.int64) * nv + face[:, 1]) * nv + face[:, 2]
    return np.searchsorted(fk, key).reshape(-1, 4)


def test_divergence_and_energy_at_size(ty):
    _note("case: 48^3 BCC box (1.33M tetrahedra), FP32, 2,000 steps from a Gaussian B")
    xyz, tets, L = bcc_box(48, 48, 48, 1.0, 0.05, 9)
    T = ty.Tet(xyz, tets)
    v = T.view()
    lam, _, ok = T.cfl(max_iter=5000, rtol=1e-8)
    assert ok
    dt = 0.5 * 2 / np.sqrt(lam)
    face = v["face"]
    cen = xyz[face].mean(axis=1)
    fa = xyz[face[:, 0]]
    nrm = np.cross(xyz[face[:, 1]] - fa, xyz[face[:, 2]] - fa)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r2 = np.sum((cen - 24.0) ** 2, axis=1)
    inner = v["d"] > 0
    B0 = np.where(inner, np.exp(-r2 / 18.0) * nrm[:, 2], 0.0)
    sim = ty.TetSim(T, dt, "f32")
    sim.set_state("B", B0)
    # signed face fluxes per tetrahedron: +1 where the face normal points out of it
    tf = _tet_faces(np.asarray(tets, np.int64), face)
    opp = xyz[np.asarray(tets)[:, [0, 1, 2, 3]]]
    out_sign = np.sign(np.einsum("tqk,tqk->tq", nrm[tf], xyz[face[tf, 0]] - opp))

    def div(B):
        return np.sum(out_sign * (v["farea"] * B)[tf], axis=1)

    def energy(E, b_old, b_new):
        return float(np.sum(v["dual_area"] * v["elen"] * E ** 2) + np.sum(v["farea"] * v["d"] * b_old * b_new))

    d0 = div(sim.get_state("B"))
    sim.step(1)
    b1 = sim.get_state("B")
    W0 = energy(sim.get_state("E"), B0, b1)
    sim.step(1998)
    b_old = sim.get_state("B")
    sim.step(1)
    b_new = sim.get_state("B")
    W1 = energy(sim.get_state("E"), b_old, b_new)
    drift = abs(W1 - W0) / W0
    ddiv = np.max(np.abs(div(b_new) - d0)) / np.max(np.abs(v["farea"] * B0))
    _note(f"  energy drift {drift:.2e}, divergence change {ddiv:.2e} of the largest face flux")
    assert drift < 1e-4
    assert ddiv < 1e-4


def test_timing_and_errors(ty):
    xyz, tets, m = _mesh("bcc")
    T = ty.Tet(xyz, tets)
    sim = ty.TetSim(T, 0.05, "f32")
    sim.set_timing(True)
    sim.step(5)
    t = sim.kernel_ms()
    assert t["steps"] == 5 and t["edge_ms"] > 0 and t["face_ms"] > 0
    with pytest.raises(ty.TyeeError):
        ty.TetSim(T, -1.0, "f32")
    with pytest.raises(ty.TyeeError):
        sim.set_graph(-1)


def test_tet100_bench_configuration_sampled_against_oracle(ty):
    """The bench's tet100 mesh at its size (100^3 BCC box, jitter 0.05 h, seed 0: 12M
    tetrahedra), FP32, in the bench's launch configuration (graphs of 8 steps): one graph of 8
    steps from a seeded random state. The oracle cannot build the whole mesh, so it takes three
    balls of it: the tetrahedra whose centroids lie within 14 h of a centre, with the global node
    ids (so edges and faces keep their orientation), advanced 8 steps. The ball's cut faces act
    as walls there, so only the edges and faces the cut cannot reach in 8 steps are compared:
    the cut's influence is followed exactly through the sub-mesh's incidences (a step's E update
    reaches every edge of a reached face, its B update every face with a reached edge). FP32
    bar 1e-5 (relative L2 per field over the compared cells)."""
    _note("case: tet100 (12M tetrahedra) FP32, one graph of 8 steps, three balls against the oracle")
    xyz, tets, L = bcc_box(100, 100, 100, 1.0, 0.05, 0)
    T = ty.Tet(xyz, tets)
    v = T.view()
    nv = np.int64(T.nv)
    ekey = v["edge"][:, 0].astype(np.int64) * nv + v["edge"][:, 1]
    f64 = v["face"].astype(np.int64)
    fkey = (f64[:, 0] * nv + f64[:, 1]) * nv + f64[:, 2]
    assert np.all(np.diff(ekey) > 0) and np.all(np.diff(fkey) > 0)       # canonical order
    dt = 0.5 * 2 / np.sqrt(65.64)        # CFL 0.5 of this mesh's omega_max^2 (the bench's power iteration)
    rng = np.random.default_rng(11)
    E0 = np.where(v["dual_area"] > 0, rng.standard_normal(T.ne), 0.0)
    B0 = rng.standard_normal(T.nf)
    sim = ty.TetSim(T, dt, "f32")
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.step(8)
    e_gpu, b_gpu = sim.get_state("E"), sim.get_state("B")
    del sim, v
    cen = xyz[tets].mean(axis=1)
    for p in ([31.3, 48.6, 57.2], [66.1, 35.4, 40.8], [50.5, 70.2, 28.9]):
        sub = tets[np.sum((cen - np.array(p)) ** 2, axis=1) < 14.0 ** 2]
        m = TetMesh(xyz, sub)
        ie = np.searchsorted(ekey, m.edge[:, 0] * nv + m.edge[:, 1])
        fk = (m.face[:, 0] * nv + m.face[:, 1]) * nv + m.face[:, 2]       # rows sorted
        jf = np.searchsorted(fkey, fk)
        assert np.array_equal(ekey[ie], m.edge[:, 0] * nv + m.edge[:, 1]) and np.array_equal(fkey[jf], fk)
        Er, Br = m.step(E0[ie], B0[jf], dt, 8)
        # cells the cut reaches within 8 steps
        te, tf = ~m.inner_edge, ~m.inner_face
        for _ in range(8):
            te[m.face_edge[tf].reshape(-1)] = True
            tf = tf | np.any(te[m.face_edge], axis=1)
        ce, cf = ~te, ~tf
        errs = (_rel(e_gpu[ie][ce], Er[ce]), _rel(b_gpu[jf][cf], Br[cf]))
        _note(f"  ball at {p}: {len(sub)} tetrahedra, {ce.sum()} edges and {cf.sum()} faces compared, "
              f"rel L2 E {errs[0]:.2e} B {errs[1]:.2e}")
        assert ce.sum() > 1000 and cf.sum() > 2000
        assert max(errs) <= 1e-5
