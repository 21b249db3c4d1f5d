"""Pins of the three-dimensional oracle (``oracle/tet.py``) and its input generator against
facts from outside them.

* the direct BCC construction is the Delaunay tetrahedralisation (the same tetrahedra as
  Qhull's, no face fails the sphere test) and fills the box;
* a hand-derived corner tetrahedron: circumcentre, face areas, edge lengths;
* the pyramids from each tetrahedron's circumcentre to its faces add up to the box's volume
  (pins A_f, d_f and the circumcentres); the Voronoi polygon areas equal the sum over the
  faces around the edge of (1/2) h d, with h the in-plane distance from the edge to the face's
  circumcentre (a second construction of A*_e);
* curl of a gradient and divergence of a curl vanish exactly (the signs s(f, e) and the face
  normals); K has exactly one zero eigenvalue per interior node (the gradients) and no negative
  one;
* the PEC box's eigenvalues converge at second order to pi^2 ((l/Lx)^2 + (m/Ly)^2 + (n/Lz)^2);
* time stepping reproduces the leap-frog phase cos(N theta) of an eigenvector start
  (2 - 2 cos theta = dt^2 lambda) and conserves the leap-frog energy.
"""
import numpy as np
import pytest

from meshgen.tet import bcc_box, insphere_violations
from oracle.tet import TetMesh


def _set(t):
    return {tuple(sorted(r)) for r in np.asarray(t).tolist()}


@pytest.mark.parametrize("dims,jitter,seed", [((3, 3, 3), 0.05, 1), ((6, 4, 5), 0.08, 2), ((8, 8, 8), 0.05, 3)])
def test_direct_bcc_is_the_delaunay_tetrahedralisation(dims, jitter, seed):
    x1, t1, L = bcc_box(*dims, 0.5, jitter, seed)
    x2, t2, _ = bcc_box(*dims, 0.5, jitter, seed, method="qhull")
    assert np.array_equal(x1, x2)
    assert _set(t1) == _set(t2)
    assert len(t1) == 12 * dims[0] * dims[1] * dims[2]
    assert insphere_violations(x1, t1) == 0
    a, b, c, d = (x1[t1[:, q]] for q in range(4))
    vol = np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a) / 6.0
    assert np.all(vol > 0) and abs(vol.sum() - L[0] * L[1] * L[2]) < 1e-12 * L[0] * L[1] * L[2]
    with pytest.raises(ValueError):
        bcc_box(*dims, 0.5, 0.09, seed)


def test_corner_tetrahedron_by_hand():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    m = TetMesh(xyz, np.array([[0, 1, 2, 3]]))
    assert np.allclose(m.C[0], [0.5, 0.5, 0.5], atol=1e-15)
    assert np.allclose(np.sort(m.farea), [0.5, 0.5, 0.5, np.sqrt(3) / 2], atol=1e-15)
    assert np.allclose(np.sort(m.elen), [1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)], atol=1e-15)
    assert m.ne == 6 and m.nf == 4 and not m.inner_face.any() and not m.inner_edge.any()
    # face (0, 1, 2) lies in z = 0 with its normal along +z (right-hand rule of 0 -> 1 -> 2)
    f = [i for i, fc in enumerate(m.face.tolist()) if fc == [0, 1, 2]][0]
    assert np.allclose(m.fnormal[f], [0, 0, 1])


@pytest.fixture(scope="module")
def small():
    xyz, tets, L = bcc_box(3, 4, 2, 1.0, 0.05, 1)
    return TetMesh(xyz, tets, L), L


def test_circumcentre_pyramids_fill_the_box(small):
    m, L = small
    i = m.inner_face
    total = np.sum(m.farea[i] * m.d[i]) / 3.0
    b = ~i
    t = np.where(m.front[b] >= 0, m.front[b], m.back[b])
    toward = np.where(m.front[b] >= 0, 1.0, -1.0)        # the tetrahedron's side of the face
    h = toward * np.einsum("ij,ij->i", m.C[t] - m.xyz[m.face[b, 0]], m.fnormal[b])
    total += np.sum(m.farea[b] * h) / 3.0
    assert abs(total - L[0] * L[1] * L[2]) < 1e-12 * L[0] * L[1] * L[2]
    assert m.d[i].min() > 0 and m.dual_area[m.inner_edge].min() > 0


def test_voronoi_area_equals_the_sum_of_face_kites(small):
    m, _ = small
    alt = np.zeros(m.ne)
    for f in np.nonzero(m.inner_face)[0]:
        a, b, c = m.face[f]
        P = m.xyz
        # the face's circumcentre: where the dual edge meets the face plane
        cf = m.C[m.front[f]] - np.dot(m.C[m.front[f]] - P[a], m.fnormal[f]) * m.fnormal[f]
        for q, (p, r, w) in enumerate([(a, b, c), (b, c, a), (a, c, b)]):
            t = (P[r] - P[p]) / np.linalg.norm(P[r] - P[p])
            u = (P[w] - P[p]) - np.dot(P[w] - P[p], t) * t
            u /= np.linalg.norm(u)
            alt[m.face_edge[f, q]] += 0.5 * np.dot(cf - 0.5 * (P[p] + P[r]), u) * m.d[f]
    i = m.inner_edge
    assert np.max(np.abs(alt[i] - m.dual_area[i]) / m.dual_area[i]) < 1e-12


def test_curl_grad_and_div_curl_vanish(small):
    m, _ = small
    G = np.zeros((m.ne, m.nv))
    G[np.arange(m.ne), m.edge[:, 0]] = -1.0
    G[np.arange(m.ne), m.edge[:, 1]] = 1.0
    C = np.zeros((m.nf, m.ne))
    for q in range(3):
        C[np.arange(m.nf), m.face_edge[:, q]] = m.face_sign[:, q]
    D = np.zeros((m.nt, m.nf))
    for f in range(m.nf):
        if m.front[f] >= 0:
            D[m.front[f], f] -= 1.0          # the normal points into the front tetrahedron
        if m.back[f] >= 0:
            D[m.back[f], f] += 1.0
    assert np.abs(C @ G).max() == 0.0
    assert np.abs(D @ C).max() == 0.0
    # the curl of the oracle's stepping: a gradient field leaves B unchanged
    phi = np.random.default_rng(0).standard_normal(m.nv)
    E = (phi[m.edge[:, 1]] - phi[m.edge[:, 0]]) / m.elen
    assert np.abs(m.curl_e(E)).max() < 1e-12


def test_null_space_is_the_gradients(small):
    m, _ = small
    lam = m.spectrum()
    zero = np.abs(lam) < 1e-9 * lam.max()
    assert zero.sum() == m.inner_node.sum()
    assert lam.min() > -1e-12 * lam.max()


def _box_modes(Lx, Ly, Lz, count):
    vals = []
    for l in range(5):
        for mm in range(5):
            for n in range(5):
                if (l > 0) + (mm > 0) + (n > 0) >= 2:
                    vals += [np.pi ** 2 * ((l / Lx) ** 2 + (mm / Ly) ** 2 + (n / Lz) ** 2)] * (2 if l and mm and n else 1)
    return np.sort(vals)[:count]


def test_box_modes_converge_at_second_order():
    exact = _box_modes(1.0, 1.25, 0.75, 6)
    errs = []
    for k in (4, 8):
        xyz, tets, L = bcc_box(k, 5 * k // 4, 3 * k // 4, 1.0 / k, 0.05, 7)
        lam = TetMesh(xyz, tets, L).modes_near(exact[2], 6)
        errs.append(np.abs(lam - exact) / exact)
    assert np.all(errs[1] < 0.012)
    assert np.all(errs[0] / errs[1] > 3.5)          # measured 4.1 - 4.5


def test_leap_frog_phase_of_an_eigenvector(small):
    m, _ = small
    K, Me = m.operator()
    s = np.sqrt(Me)
    Ks = (K.toarray() * s[:, None]) / s[None, :]
    w, V = np.linalg.eigh(0.5 * (Ks + Ks.T))
    k = np.argmax(w > 1e-6 * w.max()) + 5                # a mode above the gradients
    lam = w[k]
    v = np.zeros(m.ne)
    v[m.inner_edge] = V[:, k] / s
    dt = 0.9 * 2 / np.sqrt(w.max())
    theta = np.arccos(1.0 - 0.5 * dt * dt * lam)
    B = 0.5 * dt * m.curl_e(v)                            # B^{1/2} for E^0 = v at rest
    N = 300
    E, _ = m.step(v, B, dt, N)
    assert np.max(np.abs(E - np.cos(N * theta) * v)) < 1e-10 * np.max(np.abs(v))


def test_energy_is_conserved(small):
    m, _ = small
    rng = np.random.default_rng(4)
    E = np.where(m.inner_edge, rng.standard_normal(m.ne), 0.0)
    B = np.where(m.inner_face, rng.standard_normal(m.nf), 0.0)
    dt = 0.9 * 2 / m.omega_max()
    W = []
    for _ in range(100):
        E2, B2 = m.step(E, B, dt, 1)
        W.append(m.energy(E2, B, B2))
        E, B = E2, B2
    assert (max(W) - min(W)) / W[0] < 1e-12
