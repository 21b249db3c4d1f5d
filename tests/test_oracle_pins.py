"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Hand-derived tiny meshes, mesh identities (Euler characteristic, area sums, circumcentre
equidistance), the skew-adjointness of M in metric (7) (eqs. 7-10), the exact spectrum of the
equilateral mesh (the honeycomb dual), PEC cavity eigenfrequencies, the exact leap-frog time
phase and the stability threshold of eq. 20, conservation of div E (Section 1) and of the discrete
energy, and closed-form Drude oscillation/decay.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from meshgen import (lattice_mesh, equilateral_torus, count_non_delaunay, scramble,
                     cavity_mode)

SQ3 = np.sqrt(3.0)


def rhombus():
    # two equilateral triangles of side 1 sharing the edge 1-2
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, SQ3 / 2], [1.5, SQ3 / 2]])
    tri = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    return xy, tri


def test_hand_checked_rhombus_topology_and_geometry():
    xy, tri = rhombus()
    m = oracle.OracleMesh(xy, tri, periodic=False, L=2.0)
    # edges in lexicographic (lo, hi) order
    assert m.edge.tolist() == [[0, 1], [0, 2], [1, 2], [1, 3], [2, 3]]
    # edge 1-2 runs 1->2 along the counter-clockwise boundary of triangle 0, 2->1 of triangle 1
    assert (m.R[2], m.L[2]) == (0, 1)
    assert m.nb == 4 and m.ne == 5
    assert m.A.tolist() == [[0, 2, 1], [3, 4, 2]]
    assert m.s.tolist() == [[1, 1, -1], [1, -1, -1]]
    # equilateral: circumcentre = centroid, d = a/sqrt(3) split equally
    np.testing.assert_allclose(m.O, [[0.5, SQ3 / 6], [1.0, SQ3 / 3]], atol=1e-15)
    np.testing.assert_allclose([m.hR[2], m.hL[2], m.d[2]],
                               [1 / (2 * SQ3), 1 / (2 * SQ3), 1 / SQ3], rtol=1e-14)
    np.testing.assert_allclose(m.S, [SQ3 / 4, SQ3 / 4], rtol=1e-14)
    np.testing.assert_allclose(m.elen, 1.0, rtol=1e-15)


def test_winding_and_row_order_do_not_matter():
    xy, tri = lattice_mesh(9, 0.2, 7, periodic=False)
    a = oracle.OracleMesh(xy, tri, periodic=False)
    st, perm = scramble(tri, 3)
    b = oracle.OracleMesh(xy, st, periodic=False)
    assert np.array_equal(a.edge, b.edge)
    # every edge sees the same triangles (modulo the row shuffle)
    def mapped(x):
        return np.where(x >= 0, perm[np.maximum(x, 0)], -1)
    np.testing.assert_array_equal(mapped(b.R), a.R)
    np.testing.assert_array_equal(mapped(b.L), a.L)
    np.testing.assert_allclose(b.d, a.d, rtol=1e-12)
    np.testing.assert_allclose(b.S, a.S[perm], rtol=1e-13)


@pytest.mark.parametrize("periodic", [False, True])
def test_mesh_identities(periodic):
    xy, tri = lattice_mesh(24, 0.25, 11, periodic=periodic)
    m = oracle.OracleMesh(xy, tri, periodic=periodic)
    # Euler characteristic: disc 1, torus 0
    assert m.nv - m.ne + m.nt == (0 if periodic else 1)
    # sum of areas = domain area; sum |e| d / 2 = domain area (dual cells tile it too)
    assert abs(m.S.sum() - 1.0) < 1e-13
    assert abs((m.elen * m.d).sum() / 2 - 1.0) < 1e-13
    assert np.all(m.S > 0)
    # circumcentre equidistant from the three vertices (minimum image)
    P = xy[m.tri]
    D = P - m.O[:, None, :]
    if periodic:
        D -= np.round(D)
    r = np.hypot(D[..., 0], D[..., 1])
    assert np.max(np.abs(r - r[:, :1]) / r[:, :1]) < 1e-11
    # each edge: its two triangles lie on the side the sign says (R left of e, L right)
    i = m.interior
    assert np.all(m.d[i] > 0) and count_non_delaunay(xy, tri, periodic) == 0


def test_error_paths():
    xy, tri = rhombus()
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(xy, np.array([[0, 1, 2], [0, 1, 2]], np.int32), False, 2.0)
    assert e.value.code == oracle.ENONMANIFOLD
    xy2 = np.array([[0, 0], [1, 0], [2, 0]], float)
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(xy2, np.array([[0, 1, 2]], np.int32), False, 2.0)
    assert e.value.code == oracle.EDEGENERATE
    # flipping the shared edge of a Delaunay rhombus makes it non-Delaunay
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(xy, np.array([[0, 1, 3], [0, 3, 2]], np.int32), False, 2.0)
    assert e.value.code == oracle.ENOTDELAUNAY
    xy3, tri3 = lattice_mesh(6, 0.2, 1, periodic=True)
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(xy3, tri3[:-1], True)
    assert e.value.code == oracle.EPERIODIC


def dense_ops(m, gamma=None):
    LB = np.stack([m.apply_LB(np.eye(m.nt)[j], gamma) for j in range(m.nt)], axis=1)
    LE = np.stack([m.apply_LE(np.eye(m.ne)[i], gamma) for i in range(m.ne)], axis=1)
    return LB, LE


@pytest.mark.parametrize("periodic", [False, True])
def test_operator_skew_adjoint_in_metric_7(periodic):
    xy, tri = lattice_mesh(8, 0.25, 5, periodic=periodic)
    m = oracle.OracleMesh(xy, tri, periodic=periodic)
    gamma = 1.0 + 0.1 * np.sin(np.arange(m.ne))
    for g in (None, gamma):
        LB, LE = dense_ops(m, g)
        w = np.where(m.interior, m.d * m.elen, 0.0)
        lhs = m.S[:, None] * LE[:, m.interior]
        rhs = -(w[:, None] * LB)[m.interior].T
        assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))
    # spectrum of M: imaginary, +- pairs, static kernel of the expected dimension
    LB, LE = dense_ops(m)
    keep = m.interior
    nt, ni = m.nt, int(keep.sum())
    M = np.zeros((nt + ni, nt + ni))
    M[:nt, nt:] = LE[:, keep]
    M[nt:, :nt] = LB[keep]
    ev = np.linalg.eigvals(M)
    scale = np.max(np.abs(ev))
    assert np.max(np.abs(ev.real)) < 1e-9 * scale
    im = np.sort(ev.imag)
    np.testing.assert_allclose(im, -im[::-1], atol=1e-9 * scale)
    n_zero = int(np.sum(np.abs(ev) < 1e-8 * scale))
    expected = (m.nv + 2) if periodic else (int((m.node_bnd == 0).sum()) + 1)
    assert n_zero == expected


def test_equilateral_spectrum_is_the_honeycomb_closed_form():
    nx, ny, a = 6, 4, 1.0
    xy, tri, Lx, Ly = equilateral_torus(nx, ny, a)
    m = oracle.OracleMesh(xy, tri, True, Lx, Ly)
    LB, LE = dense_ops(m)
    K = -LE @ LB
    lam = np.sort(np.linalg.eigvals(K).real)
    # honeycomb of circumcentres, bonds of length a/sqrt(3)
    delta = np.array([[0.0, -a / SQ3], [a / 2, a / (2 * SQ3)], [-a / 2, a / (2 * SQ3)]])
    ex = []
    for m1 in range(nx):
        for m2 in range(ny):
            k = 2 * np.pi * np.array([m1 / Lx, m2 / Ly])
            f = np.abs(np.exp(1j * delta @ k).sum())
            ex += [4 / a ** 2 * (3 - f), 4 / a ** 2 * (3 + f)]
    np.testing.assert_allclose(lam, np.sort(ex), atol=1e-12)
    # power iteration gives the top of the same closed-form spectrum
    lam_max, _, ok = m.power(rtol=1e-14, max_iter=20000)
    assert ok and abs(lam_max - max(ex)) < 1e-9 * max(ex)


def cavity_eigs(n, jitter, seed, count):
    xy, tri = lattice_mesh(n, jitter, seed, periodic=False)
    m = oracle.OracleMesh(xy, tri, periodic=False)
    LB, LE = dense_ops(m)
    SK = (m.S[:, None] * (-LE @ LB))
    SK = 0.5 * (SK + SK.T)
    lam = scipy.linalg.eigh(SK, np.diag(m.S), eigvals_only=True)
    return np.sqrt(np.clip(lam[1:count + 1], 0, None)), m


def test_pec_cavity_eigenfrequencies_converge_to_analytic():
    # closed resonator: omega = pi sqrt(m^2 + n^2) (the "exact analytic solution" of Fig. 4)
    exact = np.pi * np.sqrt(np.array([1, 1, 2, 4, 4, 5, 5]))
    errs = []
    for n in (13, 25):
        w, _ = cavity_eigs(n, 0.2, 0, len(exact))
        errs.append(np.max(np.abs(w / exact - 1)))
    assert errs[1] < 5e-3
    assert errs[1] < errs[0] / 2.5          # second-order convergence (about 4x)


def test_cavity_te11_frequency_from_time_stepping():
    # 45 x 45 closed cavity, B = cos(pi x) cos(pi z), E = 0, dt = 0.5 * 2/omega_max
    from scipy.optimize import curve_fit
    xy, tri = lattice_mesh(45, 0.2, 0, periodic=False)
    m = oracle.OracleMesh(xy, tri, periodic=False)
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    B0 = cavity_mode(m.O, 1, 1)
    E, B = np.zeros(m.ne), B0.copy()
    nrm = np.sum(m.S * B0 * B0)
    ts, zs = [], []
    for k in range(40):
        r = m.step(E, B, dt, 50, n0=50 * k)
        E, B = r["E"], r["B"]
        ts.append((50 * (k + 1) + 0.5) * dt)
        zs.append(np.sum(m.S * B * B0) / nrm)
    (amp, w), _ = curve_fit(lambda t, a, w: a * np.cos(w * t), np.array(ts), np.array(zs),
                            p0=(1.0, 4.4))
    assert abs(w / (np.pi * np.sqrt(2)) - 1) < 1e-3
    assert abs(amp - 1) < 1e-3


def test_leapfrog_exact_time_phase_and_eq20_threshold():
    xy, tri = lattice_mesh(10, 0.2, 2, periodic=False)
    m = oracle.OracleMesh(xy, tri, periodic=False)
    LB, LE = dense_ops(m)
    SK = m.S[:, None] * (-LE @ LB)
    lam, V = scipy.linalg.eigh(0.5 * (SK + SK.T), np.diag(m.S))
    for idx in (1, 7, len(lam) - 1):
        w = np.sqrt(lam[idx])
        dt = 0.9 * 2 / lam[-1] ** 0.5
        v = V[:, idx] / np.max(np.abs(V[:, idx]))
        N = 137
        r = m.step(np.zeros(m.ne), v, dt, N)
        theta = 2 * np.arcsin(w * dt / 2)       # sin(theta/2) = omega dt / 2
        c = np.cos(theta * (N + 0.5)) / np.cos(theta / 2)
        np.testing.assert_allclose(r["B"], c * v, atol=1e-10)
    # eq. 20: omega_max dt just below 2 stays bounded, just above grows
    wmax = np.sqrt(m.power()[0])
    rng = np.random.default_rng(0)
    B0 = rng.standard_normal(m.nt)
    for f, grows in ((0.99, False), (1.01, True)):
        dt = f * 2 / wmax
        r = m.step(np.zeros(m.ne), B0, dt, 300)
        ratio = np.linalg.norm(r["B"]) / np.linalg.norm(B0)
        assert (ratio > 1e3) == grows


def test_power_iteration_matches_dense_top_eigenvalue():
    _, m = cavity_eigs(12, 0.25, 4, 1)
    LB, LE = dense_ops(m)
    lam_dense = np.max(np.linalg.eigvals(-LE @ LB).real)
    lam, it, ok = m.power(rtol=1e-13)
    assert ok and abs(lam - lam_dense) < 1e-9 * lam_dense


@pytest.mark.parametrize("periodic", [False, True])
def test_energy_and_divergence_conserved(periodic):
    xy, tri = lattice_mesh(16, 0.25, 9, periodic=periodic)
    m = oracle.OracleMesh(xy, tri, periodic=periodic)
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    rng = np.random.default_rng(1)
    E0 = np.where(m.interior, rng.standard_normal(m.ne), 0.0)
    B0 = rng.standard_normal(m.nt)
    # W_h^0 needs B^{-1/2} = B^{1/2} - dt L_E E^0
    Bm = B0 - dt * m.apply_LE(E0)
    W0 = m.energy(E0, Bm, B0)
    r = m.step(E0, B0, dt, 1000, want_prev=True)
    W1 = m.energy(r["E"], r["B_prev"], r["B"])
    assert abs(W1 / W0 - 1) < 1e-12
    inner = m.node_bnd == 0
    div0, div1 = m.div(E0)[inner], m.div(r["E"])[inner]
    assert np.max(np.abs(div1 - div0)) < 1e-12 * np.max(np.abs(div0))


def gradient_field(m, seed):
    phi = np.random.default_rng(seed).standard_normal(m.nv)
    return (phi[m.edge[:, 1]] - phi[m.edge[:, 0]]) / m.elen


def test_drude_plasma_oscillation_and_collision_decay():
    # equilateral torus: omega_max = 2 sqrt(6)/a, so dt = 0.2 is inside eq. 20
    xy, tri, Lx, Ly = equilateral_torus(8, 6)
    m = oracle.OracleMesh(xy, tri, True, Lx, Ly)
    E0 = gradient_field(m, 0)           # curl-free: L_E E0 = 0, so B stays 0
    assert np.max(np.abs(m.apply_LE(E0))) < 1e-12 * np.max(np.abs(E0))
    wp, dt, N = 0.8, 0.2, 400
    wp2 = np.full(m.ne, wp * wp)
    r = m.step(E0, np.zeros(m.nt), dt, N, wp2=wp2, nu=0.0)
    theta = np.arccos(1 - wp * wp * dt * dt / 2)
    np.testing.assert_allclose(r["E"], E0 * np.cos(theta * (N + 0.5)) / np.cos(theta / 2),
                               atol=1e-11)
    assert np.max(np.abs(r["B"])) < 1e-9
    # with collisions and no field: j decays by (1 - nu dt/2)/(1 + nu dt/2) per step
    nu = 0.05
    J0 = gradient_field(m, 1)
    r = m.step(np.zeros(m.ne), np.zeros(m.nt), dt, 1, J=J0, wp2=np.full(m.ne, 1e-300), nu=nu)
    np.testing.assert_allclose(r["J"], J0 * (1 - nu * dt / 2) / (1 + nu * dt / 2), rtol=1e-14)
    # damped oscillation: energy-like amplitude shrinks monotonically over periods
    r = m.step(E0, np.zeros(m.nt), dt, 2000, wp2=wp2, nu=nu)
    amp = np.max(np.abs(r["E"])) / np.max(np.abs(E0))
    assert amp < np.exp(-nu / 2 * 2000 * dt) * 1.2


def test_gauss_law_with_plasma_and_source():
    from meshgen import triangle_particle_mask, line_source_pairs
    xy, tri = lattice_mesh(20, 0.25, 4, periodic=True)
    m = oracle.OracleMesh(xy, tri, periodic=True)
    chi = triangle_particle_mask(xy, tri, True, side=0.5, center=(0.6, 0.5))
    wp2 = m.edge_wp2(0.64 * chi)
    pairs, w = line_source_pairs(xy, tri, True, 1.0, 1 / 20, x0=0.2, z0=0.25, z1=0.75)
    assert len(pairs) > 5 and np.count_nonzero(wp2) > 10
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    rng = np.random.default_rng(2)
    E0, B0 = rng.standard_normal(m.ne), rng.standard_normal(m.nt)
    src = (pairs, w, 1.0, 10)
    r = m.step(E0, B0, dt, 500, wp2=wp2, nu=0.05, src=src)
    g0 = m.div(E0) - 0.0
    g1 = m.div(r["E"]) - r["Q"]
    assert np.max(np.abs(g1 - g0)) < 1e-11 * np.max(np.abs(g0))
    assert np.max(np.abs(r["Q"])) > 1e-8           # charge really moved
    # linearity in the source amplitude
    z = m.step(np.zeros(m.ne), np.zeros(m.nt), dt, 300, src=(pairs, w, 1.0, 10))
    z2 = m.step(np.zeros(m.ne), np.zeros(m.nt), dt, 300, src=(pairs, 2 * w, 1.0, 10))
    np.testing.assert_allclose(z2["E"], 2 * z["E"], rtol=1e-12, atol=1e-300)


def test_splitmix64_and_morton_reference_values():
    # published splitmix64 outputs for state 0 (first three draws)
    assert oracle.splitmix64(0) == 0xE220A8397B1DCDAF
    g = 0x9E3779B97F4A7C15
    assert oracle.splitmix64(g) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(2 * g) == 0x06C45D188009454F
    # Z-order of a 4x4 grid, x in the even bits
    z = np.zeros((4, 4), int)
    for x in range(4):
        for y in range(4):
            z[y, x] = oracle.morton(x, y)
    assert z.tolist() == [[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]]
    assert oracle.morton(65535, 65535) == 2 ** 32 - 1


def bandwidth(m, perm_t):
    inv = np.empty_like(perm_t)
    inv[perm_t] = np.arange(len(perm_t))
    i = m.interior
    return int(np.max(np.abs(inv[m.R[i]] - inv[m.L[i]])))


@pytest.mark.parametrize("periodic", [False, True])
def test_orderings_are_bijections_with_expected_locality(periodic):
    xy, tri = lattice_mesh(30, 0.25, 6, periodic=periodic)
    m = oracle.OracleMesh(xy, tri, periodic=periodic)
    bw = {}
    for kind in ("none", "random", "morton", "rcm"):
        pt, pe = m.order(kind, seed=5)
        assert np.array_equal(np.sort(pt), np.arange(m.nt))
        assert np.array_equal(np.sort(pe), np.arange(m.ne))
        bw[kind] = bandwidth(m, pt)
        if kind in ("morton", "rcm"):
            # edges appear in order of first use by the reordered triangles
            inv = np.empty_like(pe)
            inv[pe] = np.arange(m.ne)
            seq = inv[m.A[pt]].reshape(-1)
            _, first_pos = np.unique(seq, return_index=True)
            assert np.all(np.diff(first_pos) > 0)
    assert bw["rcm"] < bw["random"] / 5
    assert bw["morton"] < bw["random"]
    # RCM on a strip of triangles (path-shaped dual graph) reaches bandwidth 1, and starts
    # from a pseudo-peripheral triangle at one end of the strip
    from meshgen import lawson_flip
    rng = np.random.default_rng(0)
    strip_xy = np.array([[i, j] for j in range(2) for i in range(12)], float)
    strip_xy[:, 1] += rng.uniform(-0.1, 0.1, 24)
    strip_tri = []
    for i in range(11):
        a, b, c, d = i, i + 1, 12 + i + 1, 12 + i
        strip_tri += [[a, b, c], [a, c, d]]
    strip_tri, _ = lawson_flip(strip_xy, np.array(strip_tri, np.int32), False)
    sm = oracle.OracleMesh(strip_xy, strip_tri, False, 12.0, 2.0)
    pt, _ = sm.order("rcm")
    assert bandwidth(sm, pt) == 1
    deg = (sm.interior[sm.A]).sum(1)
    assert deg[pt[0]] == 1 and deg[pt[-1]] == 1


def kite():
    # two isosceles triangles on the base P(0,-1) - Q(0,1): apex A(-2, 0) on the left, B(3, 0)
    # on the right.  Circumcentres lie on the x axis at (1 - a^2)/(2a) from the base for apex
    # distance a: O_A = (-3/4, 0), O_B = (4/3, 0); the base runs P -> Q counter-clockwise
    # around PQA, so R(PQ) = PQA with hR = 3/4, L(PQ) = PBQ with hL = 4/3, d = 25/12
    xy = np.array([[0.0, -1.0], [0.0, 1.0], [-2.0, 0.0], [3.0, 0.0]])
    tri = np.array([[0, 1, 2], [0, 3, 1]], np.int32)
    return xy, tri


def test_edge_plasma_frequency_rule_hand_derived():
    """The per-edge plasma frequency squared (eq. 5 on edges): every interior edge of a
    homogeneous medium carries the medium's value; the base of the kite, with plasma on one
    side only, carries wp2 times that side's half dual length over d."""
    xy, tri = kite()
    m = oracle.OracleMesh(xy, tri, periodic=False, L=5.0)
    assert m.edge[0].tolist() == [0, 1] and (m.R[0], m.L[0]) == (0, 1)
    np.testing.assert_allclose([m.hR[0], m.hL[0], m.d[0]], [0.75, 4 / 3, 25 / 12], rtol=1e-14)
    np.testing.assert_allclose(m.edge_wp2([0.64, 0.0]), [0.64 * 9 / 25, 0, 0, 0, 0], rtol=1e-14)
    np.testing.assert_allclose(m.edge_wp2([0.0, 0.64]), [0.64 * 16 / 25, 0, 0, 0, 0], rtol=1e-14)
    np.testing.assert_allclose(m.edge_wp2([0.64, 0.64]), [0.64, 0, 0, 0, 0], rtol=1e-14)
    for periodic in (True, False):
        xy, tri = lattice_mesh(16, 0.25, 8, periodic=periodic)
        m = oracle.OracleMesh(xy, tri, periodic=periodic)
        w = m.edge_wp2(np.full(m.nt, 0.64))
        i = m.interior
        # (hR c + hL c) / d rounds with an error of a few ulps of c (|hR| + |hL|) / d, large
        # where hR and hL nearly cancel (near-cocircular quads)
        bound = 4 * np.finfo(float).eps * 0.64 * (np.abs(m.hR[i]) + np.abs(m.hL[i])) / m.d[i]
        assert np.all(np.abs(w[i] - 0.64) <= bound)
        assert np.all(w[~m.interior] == 0.0)


def test_source_waveform_values_hand_evaluated():
    """The soft source J = w g(t) with g(t) = sin(omega t) sin^2(pi t / T), T = cycles 2 pi /
    omega, and g = 0 outside [0, T): with B = 0 and E = 0 one step gives E^1 = -dt w g(dt/2) on
    the source edge (eq. 6 with the source term), so the first step reads g at t = dt / 2."""
    xy, tri = rhombus()
    m = oracle.OracleMesh(xy, tri, periodic=False, L=2.0)
    z_e, z_b = np.zeros(m.ne), np.zeros(m.nt)

    def first_step(dt, pair, w, n0=0):
        return m.step(z_e, z_b, dt, 1, n0=n0, src=(np.array([pair]), np.array([w]), 1.0, 10))["E"]

    # t = pi/2 (omega = 1, T = 20 pi): g = sin^2(pi / 40)
    e = first_step(np.pi, [1, 2], 1.0)
    assert e[2] == pytest.approx(-np.pi * np.sin(np.pi / 40) ** 2, rel=1e-14)
    assert np.all(np.delete(e, 2) == 0.0)
    # the weight follows the direction the pair is given in: 2 -> 1 is against e (1 -> 2)
    e = first_step(np.pi, [2, 1], 2.0)
    assert e[2] == pytest.approx(2 * np.pi * np.sin(np.pi / 40) ** 2, rel=1e-14)
    # t = 19 pi / 2: sin(omega t) = -1, g = -sin^2(19 pi / 40)
    e = first_step(19 * np.pi, [1, 2], 1.0)
    assert e[2] == pytest.approx(19 * np.pi * np.sin(19 * np.pi / 40) ** 2, rel=1e-13)
    # t = T (the pulse has ended) and t < 0 (not started): no source
    assert np.all(first_step(40 * np.pi, [1, 2], 1.0) == 0.0)
    assert np.all(first_step(1.0, [1, 2], 1.0, n0=-1) == 0.0)
    # n0 shifts the time: step n0 reads g at (n0 + 1/2) dt
    e = first_step(np.pi / 3, [1, 2], 1.0, n0=1)
    assert e[2] == pytest.approx(-np.pi / 3 * np.sin(np.pi / 40) ** 2, rel=1e-14)


def test_threaded_oracle_is_bit_identical_to_one_thread():
    """Every per-cell update keeps its arithmetic and order under OpenMP, and the nodal charge
    is a per-node gather in ascending edge order: the thread count changes no bit."""
    from meshgen import triangle_particle_mask, line_source_pairs
    xy, tri = lattice_mesh(40, 0.25, 21, periodic=True)
    m = oracle.OracleMesh(xy, tri, periodic=True)
    chi = triangle_particle_mask(xy, tri, True, side=0.5, center=(0.6, 0.5))
    wp2 = m.edge_wp2(0.64 * chi)
    pairs, w = line_source_pairs(xy, tri, True, 1.0, 1 / 40, x0=0.2, z0=0.25, z1=0.75)
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    rng = np.random.default_rng(5)
    E0, B0 = rng.standard_normal(m.ne), rng.standard_normal(m.nt)
    gamma = 1 + 0.05 * rng.standard_normal(m.ne)
    kw = dict(wp2=wp2, nu=0.05, src=(pairs, w, 1.0 / dt / 50, 2), gamma=gamma, want_prev=True)
    before = oracle.get_threads()
    try:
        oracle.set_threads(1)
        a = m.step(E0, B0, dt, 60, **kw)
        pa = m.power(gamma=gamma)
        oracle.set_threads(max(4, before))
        assert oracle.get_threads() >= 4
        b = m.step(E0, B0, dt, 60, **kw)
        pb = m.power(gamma=gamma)
    finally:
        oracle.set_threads(before)
    for k in ("E", "B", "J", "Q", "B_prev"):
        assert np.array_equal(a[k], b[k]), k
    assert pa == pb
    assert np.max(np.abs(a["Q"])) > 0
