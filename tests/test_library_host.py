"""Host side of the library (no GPU): exports, connectivity, geometry and orderings against
the oracle, error paths and the omega_max iteration."""
import ctypes
import re
import os

import numpy as np
import pytest

import oracle
from meshgen import lattice_mesh, scramble, equilateral_torus

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def test_every_declared_symbol_is_exported(ty):
    header = open(os.path.join(ROOT, "include", "tyee.h")).read()
    declared = set(re.findall(r"\b(tyee_[a-z_0-9]+)\s*\(", header))
    assert len(declared) >= 20
    lib = ctypes.CDLL(ty.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(ty.EXPORTS)


@pytest.mark.parametrize("periodic,n,jitter,seed", [(False, 45, 0.2, 0), (True, 64, 0.25, 1),
                                                    (True, 50, 0.3, 100)])
def test_connectivity_and_geometry_match_oracle(ty, periodic, n, jitter, seed):
    xy, tri = lattice_mesh(n, jitter, seed, periodic=periodic)
    tri, _ = scramble(tri, seed + 1)
    m = ty.Mesh(xy, tri, periodic)
    o = oracle.OracleMesh(xy, tri, periodic)
    v = m.view()
    for a, b in (("tri", "tri"), ("edge_nodes", "edge"), ("R", "R"), ("L", "L"), ("A", "A"),
                 ("sgn", "s")):
        assert np.array_equal(v[a], getattr(o, b)), a
    for a in ("elen", "hR", "hL", "d", "S", "O", "C"):
        ref = getattr(o, a)
        err = np.max(np.abs(v[a] - ref) / np.maximum(np.abs(ref), 1e-300 + np.max(np.abs(ref))))
        assert err < 1e-12, a
    np.testing.assert_array_equal(v["evec"], o.evec)
    info = m.info()
    assert info["n_edges"] == o.ne and info["n_boundary_edges"] == o.nb
    assert abs(info["sum_area"] - 1) < 1e-12 and abs(info["sum_dual_area"] - 1) < 1e-12


@pytest.mark.parametrize("kind", ["none", "random", "morton", "rcm"])
@pytest.mark.parametrize("periodic", [False, True])
def test_orderings_bit_exact_against_oracle(ty, kind, periodic):
    xy, tri = lattice_mesh(70, 0.25, 3, periodic=periodic)
    m = ty.Mesh(xy, tri, periodic)
    o = oracle.OracleMesh(xy, tri, periodic)
    for seed in (0, 12345):
        m.reorder(kind, seed)
        v = m.view()
        pt, pe = o.order(kind, seed)
        assert np.array_equal(v["perm_t"], pt)
        assert np.array_equal(v["perm_e"], pe)


def test_rcm_with_several_components(ty):
    # two disjoint boxes in one mesh: RCM must restart per component
    xy1, t1 = lattice_mesh(8, 0.2, 1, periodic=False)
    xy2, t2 = lattice_mesh(6, 0.2, 2, periodic=False)
    xy = np.vstack([xy1, xy2 + [2.0, 0.0]])
    tri = np.vstack([t1, t2 + len(xy1)]).astype(np.int32)
    m = ty.Mesh(xy, tri, False, L=3.0)
    o = oracle.OracleMesh(xy, tri, False, L=3.0)
    m.reorder("rcm")
    assert np.array_equal(m.view()["perm_t"], o.order("rcm")[0])


def test_error_codes(ty):
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 0.8], [1.5, 0.8]])
    with pytest.raises(ty.TyeeError) as e:
        ty.Mesh(xy, np.array([[0, 1, 2], [0, 1, 2]]), False, L=2.0)
    assert e.value.code == -4
    with pytest.raises(ty.TyeeError) as e:
        ty.Mesh(np.array([[0, 0], [1, 0], [2, 0.0]]), np.array([[0, 1, 2]]), False, L=2.0)
    assert e.value.code == -3
    with pytest.raises(ty.TyeeError) as e:
        ty.Mesh(xy, np.array([[0, 1, 3], [0, 3, 2]]), False, L=2.0)
    assert e.value.code == -2
    xy3, tri3 = lattice_mesh(6, 0.2, 1, periodic=True)
    with pytest.raises(ty.TyeeError) as e:
        ty.Mesh(xy3, tri3[:-1], True)
    assert e.value.code == -5
    with pytest.raises(ty.TyeeError) as e:
        ty.Mesh(xy3, np.array([[0, 1, 99]]), True)
    assert e.value.code == -1
    m = ty.Mesh(xy3, tri3, True)
    with pytest.raises(ty.TyeeError):
        m.reorder(7)


def test_cfl_matches_oracle_and_closed_form(ty):
    xy, tri, Lx, Ly = equilateral_torus(12, 8)
    m = ty.Mesh(xy, tri, True, Lx, Ly)
    lam, it, ok = m.cfl(rtol=1e-14)
    assert ok and abs(np.sqrt(lam) - 2 * np.sqrt(6)) < 1e-9        # omega_max = 2 sqrt(6)/a
    xy, tri = lattice_mesh(40, 0.25, 8, periodic=True)
    m = ty.Mesh(xy, tri, True)
    o = oracle.OracleMesh(xy, tri, True)
    gamma = 1 + 0.05 * np.cos(np.arange(m.ne))
    for g in (None, gamma):
        lam, _, ok = m.cfl(gamma=g)
        lam_o, _, ok_o = o.power(gamma=g)
        assert ok and ok_o and abs(lam / lam_o - 1) < 1e-10


def test_phase_error_needs_a_periodic_mesh(ty):
    # argument checks happen on the host before any device work
    xy, tri = lattice_mesh(10, 0.2, 0, periodic=False)
    m = ty.Mesh(xy, tri, False)
    with pytest.raises(ty.TyeeError):
        m.phase_error_timestepped(1e-3, np.array([2 * np.pi, 0.0]))


def test_copy_probe_rejects_bad_sizes(ty):
    for nbytes, reps in ((100, 1), (1 << 20, 0), (1 << 40, 1)):
        with pytest.raises(ty.TyeeError):
            ty.copy_bandwidth(nbytes, reps)


def test_mode_solver_rejects_bad_arguments(ty):
    # all checked on the host before any device call
    xy, tri = lattice_mesh(6, 0.2, 1, periodic=False)        # 50 triangles
    m = ty.Mesh(xy, tri, False)
    bad = [dict(n_modes=0), dict(n_modes=51), dict(n_modes=300),
           dict(n_modes=10, block=9), dict(n_modes=10, block=51), dict(n_modes=1, block=1),
           dict(n_modes=10, degree=-1), dict(n_modes=10, degree=100001),
           dict(n_modes=10, tol=0.0), dict(n_modes=10, max_iter=0)]
    for kw in bad:
        with pytest.raises(ty.TyeeError) as e:
            m.modes(**kw)
        assert e.value.code == -1, kw                          # TYEE_EINVAL
    with pytest.raises(ValueError):
        m.modes(10, which="middle")
    out = np.zeros(10)
    from paper_1812_01448_amd import tyee as raw
    assert raw.lib.tyee_mesh_modes(m._h, None, 7, 10, 0, 0, 1e-10, 10, 0, None,
                                   out.ctypes.data, None, None, None) == -1


def test_rayleigh_quotient_diagnostic_matches_oracle(ty):
    # host FP64 diagnostic: equals the oracle's Rayleigh-quotient phase error with and without
    # a per-edge scale, and the honeycomb closed form on the equilateral torus
    from oracle import learned as OL
    xy, tri = lattice_mesh(24, 0.3, 3, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    waves = 2 * np.pi * np.array([[1.0, 0.0], [2.0, 3.0], [-1.0, 4.0]])
    gamma = 1.0 + 0.05 * np.sin(np.arange(om.ne) * 0.3)
    for g in (None, gamma):
        got = m.phase_error_rq(dt, waves, gamma=g)
        ref = [OL.rq_phase_error(om, g, dt, k) for k in waves]
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-14)
    xy, tri, Lx, Ly = equilateral_torus(12, 8, a=1.0)
    m = ty.Mesh(xy, tri, True, L=Lx, Ly=Ly)
    delta = np.array([[0.0, -1 / np.sqrt(3)], [0.5, 1 / (2 * np.sqrt(3))], [-0.5, 1 / (2 * np.sqrt(3))]])
    k = 2 * np.pi * np.array([2 / Lx, 1 / Ly])
    w2 = 4.0 * (3.0 - np.sum(np.cos(delta @ k)))
    expect = 2 / 0.1 * np.arcsin(np.sqrt(w2) * 0.1 / 2) / np.hypot(*k) - 1
    assert abs(m.phase_error_rq(0.1, k)[0] - expect) < 1e-12


def _scramble_diagonals(xy, tri, periodic, seed, frac=0.3):
    """Flip a random set of interior edges (triangle-disjoint, convex quads only): a
    non-Delaunay triangulation of the same nodes."""
    from meshgen.lattice import _interior_pairs
    tri = np.array(tri, np.int32, copy=True)
    h1, h2 = _interior_pairs(tri, len(xy))
    rng = np.random.default_rng(seed)
    used = set()

    def rel(a, b):
        d = xy[b] - xy[a]
        return d - np.round(d) if periodic else d

    n = 0
    for k in rng.permutation(len(h1))[: int(frac * len(h1))]:
        t1, q1, t2, q2 = h1[k] // 3, h1[k] % 3, h2[k] // 3, h2[k] % 3
        if t1 in used or t2 in used:
            continue
        u, v, o1 = tri[t1, q1], tri[t1, (q1 + 1) % 3], tri[t1, (q1 + 2) % 3]
        o2 = tri[t2, (q2 + 2) % 3]
        # convex quad u, o2, v, o1: both new triangles counter-clockwise
        cross = lambda a, b: a[0] * b[1] - a[1] * b[0]
        c1 = cross(rel(o1, u), rel(o1, o2))
        c2 = cross(rel(o2, v), rel(o2, o1))
        if c1 <= 0 or c2 <= 0:
            continue
        tri[t1] = (o1, u, o2)
        tri[t2] = (o2, v, o1)
        used.update((t1, t2))
        n += 1
    return tri, n


@pytest.mark.parametrize("periodic", [False, True])
def test_lawson_flips_restore_the_delaunay_triangulation(ty, periodic):
    # the Delaunay triangulation of points in general position is unique: flipping a random
    # set of diagonals and handing the result to the library's flips must give it back
    from meshgen import count_non_delaunay
    xy, tri = lattice_mesh(20, 0.25, 9, periodic=periodic)
    bad, n = _scramble_diagonals(xy, tri, periodic, 3)
    assert n > 50 and count_non_delaunay(xy, bad, periodic) > 0
    fixed, flips = ty.flip(xy, bad, periodic)
    assert flips >= n and count_non_delaunay(xy, fixed, periodic) == 0
    key = lambda t: sorted(tuple(sorted(r)) for r in np.asarray(t).tolist())
    assert key(fixed) == key(tri)
    # counter-clockwise output (the oracle keeps counter-clockwise rows as given), accepted by
    # the oracle's strict Delaunay check
    om = oracle.OracleMesh(xy, fixed, periodic)
    assert np.array_equal(om.tri, fixed) and om.nt == len(tri)
    again, none = ty.flip(xy, fixed, periodic)
    assert none == 0 and np.array_equal(again, fixed)


def test_lawson_flip_errors(ty):
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0], [0.0, 1.0]])
    with pytest.raises(ty.TyeeError) as e:
        ty.flip(xy, np.array([[0, 1, 2]]), False, L=2.0)
    assert e.value.code == -3                      # degenerate
    with pytest.raises(ty.TyeeError) as e:
        ty.flip(xy, np.array([[0, 1, 7]]), False, L=2.0)
    assert e.value.code == -1                      # node id out of range


@pytest.mark.parametrize("kind,layers,width,smax,grading",
                         [("tri", 3, 0.5, 0.0, 3.0), ("tri", 4, 0.7, 2.0, 3.0), ("square", 2, 1.25, 1.5, 2.0)])
def test_open_frame_matches_oracle(ty, kind, layers, width, smax, grading):
    """The library's PML frame (built on the host) against the oracle's own builder: the same
    canonical numbering, coordinates, edges, cell-edge sets, lengths, centre distances, areas,
    centres and damping profiles."""
    from meshgen import box_mesh, box_tri_mesh
    from oracle.open import OpenMesh
    if kind == "tri":
        xy, tri, Lx, Ly = box_tri_mesh(8, 6, 1.0, 0.1, 1)
    else:
        xy, tri, Lx, Ly = box_mesh(6, 5, 0.15, 2, h=1.0)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    ref = OpenMesh(om, layers, width, smax, grading)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    g = ty.open_frame(m, ty.pml(layers, width, smax, grading))
    assert (g["n_nodes"], g["n_edges"], g["n_cells"], g["n_frame_cells"]) == (ref.nv, ref.ne, ref.ncell, ref.nf)
    assert g["n_inner_edges"] == int(ref.inner.sum())
    assert np.array_equal(g["xy"], ref.xy) and np.array_equal(g["edge"], ref.edge)
    for j in range(ref.ncell):
        got = g["cell_edge"][j]
        assert sorted(got[got >= 0].tolist()) == sorted(ref.cell_edges[j]), j
    # a rectangle lists its sides parallel to y first
    vert = np.abs(np.diff(g["xy"][g["edge"]], axis=1)[:, 0, 0]) == 0.0
    assert np.all(vert[g["cell_edge"][ref.nt:, :2]]) and not np.any(vert[g["cell_edge"][ref.nt:, 2:]])
    for k, v in (("elen", ref.elen), ("d", ref.d), ("S", ref.S), ("O", ref.O), ("sigma_e", ref.sigma_e),
                 ("sigma_x", ref.sigma_x), ("sigma_y", ref.sigma_y)):
        assert np.max(np.abs(g[k] - v)) <= 1e-14 * max(1.0, np.max(np.abs(v))), k


def test_open_frame_errors(ty):
    from meshgen import box_tri_mesh
    xy, tri, Lx, Ly = box_tri_mesh(8, 6, 1.0, 0.1, 1)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    for bad in (ty.pml(0, 1.0, 1.0), ty.pml(2, 0.0, 1.0), ty.pml(2, 1.0, -1.0), ty.pml(2, 1.0, 1.0, -1.0)):
        with pytest.raises(ty.TyeeError) as e:
            ty.open_frame(m, bad)
        assert e.value.code == -1
    # the mesh must fill the box it is declared on
    wide = ty.Mesh(xy, tri, False, L=Lx + 1.0, Ly=Ly)
    with pytest.raises(ty.TyeeError) as e:
        ty.open_frame(wide, ty.pml(2, 1.0, 1.0))
    assert e.value.code == -1
    xt, tt = lattice_mesh(8, 0.2, 3, periodic=True)
    torus = ty.Mesh(xt, tt, True)
    with pytest.raises(ty.TyeeError) as e:
        ty.open_frame(torus, ty.pml(2, 0.1, 1.0))
    assert e.value.code == -1


@pytest.mark.parametrize("dims,jitter,method", [((3, 4, 2), 0.05, "direct"), ((4, 3, 3), 0.25, "qhull")])
def test_tet_mesh_matches_oracle(ty, dims, jitter, method):
    """The tetrahedral builder against the oracle's: canonical edges, faces and face edges bit
    for bit, geometry and the Voronoi dual to 1e-12, omega_max to 1e-10. The Qhull mesh at
    jitter 0.25 is an irregular Delaunay mesh (edges in 3 to 9 faces)."""
    from meshgen.tet import bcc_box
    from oracle.tet import TetMesh
    xyz, tets, L = bcc_box(*dims, 1.0, jitter, 2, method=method)
    # hand the library the tetrahedra in scrambled vertex order: it reorients them
    rng = np.random.default_rng(0)
    scr = np.array([t[rng.permutation(4)] for t in tets], np.int32)
    T = ty.Tet(xyz, scr)
    m = TetMesh(xyz, tets, L)
    v = T.view()
    assert (T.ne, T.nf, T.nt, T.n_inner_edge, T.n_inner_face) == (m.ne, m.nf, m.nt, m.inner_edge.sum(),
                                                                    m.inner_face.sum())
    assert np.array_equal(v["edge"], m.edge) and np.array_equal(v["face"], m.face)
    assert np.array_equal(v["face_edge"], m.face_edge)
    for k, ref in (("elen", m.elen), ("dual_area", m.dual_area), ("farea", m.farea), ("d", m.d)):
        assert np.max(np.abs(v[k] - ref)) <= 1e-12 * np.max(np.abs(ref)), k
    lam, it, ok = T.cfl(rtol=1e-14)
    assert ok and abs(np.sqrt(lam) - m.omega_max()) <= 1e-10 * np.sqrt(lam)


def test_tet_mesh_errors(ty):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.3, 0.3, 1.0], [0.3, 0.3, -0.05], [0.2, 0.2, 0.5]])
    cases = [
        (np.array([[0, 1, 2, 7]]), -1),                        # index out of range
        (np.array([[0, 1, 2, 2]]), -3),                        # no volume
        (np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]]), -4),   # face in three tetrahedra
        (np.array([[0, 1, 2, 3], [0, 1, 2, 5]]), -4),          # both on one side of (a, b, c)
        (np.array([[0, 1, 2, 3], [0, 1, 2, 4]]), -2),          # q inside the sphere of (a, b, c, p)
    ]
    for tets, code in cases:
        with pytest.raises(ty.TyeeError) as e:
            ty.Tet(xyz, tets)
        assert e.value.code == code, tets
    with pytest.raises(ValueError):
        ty.Tet(xyz[:, :2], [[0, 1, 2, 3]])
