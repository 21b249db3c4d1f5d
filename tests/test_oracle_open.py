"""Pins of the open-boundary oracle (``oracle/open.py``) against facts from outside it.

* the mixed mesh is a disc (Euler characteristic 1), its cells tile the enlarged box, and the
  edge areas |e| d / 2 plus the outer wall's half cells add up to the same area;
* every centre distance across an edge is positive and every rectangle's centre lies on its
  sides' perpendicular bisectors;
* without damping the leap-frog energy (metric (7)) is conserved to rounding, with a frame;
* with no layers the scheme is the pinned triangle oracle's, step for step;
* with the PML a centred pulse leaves the box: after two crossing times less than 3e-3 of its
  energy is left in the box, while a reflecting frame (sigma = 0) keeps a large part and a
  damping of the wrong sign blows up.
"""
import numpy as np
import pytest

import oracle
from oracle.open import OpenMesh
from meshgen import box_mesh, box_tri_mesh


def _mesh(kind="tri"):
    if kind == "tri":
        xy, tri, Lx, Ly = box_tri_mesh(8, 6, 1.0, 0.1, 1)
    else:
        xy, tri, Lx, Ly = box_mesh(6, 5, 0.15, 2, h=1.0)
    return oracle.OracleMesh(xy, tri, False, Lx, Ly)


@pytest.mark.parametrize("kind,layers,width", [("tri", 3, 0.5), ("square", 2, 1.25), ("tri", 1, 0.3)])
def test_frame_geometry(kind, layers, width):
    om = _mesh(kind)
    m = OpenMesh(om, layers, width, 1.0)
    depth = layers * width
    area = (om.Lx + 2 * depth) * (om.Ly + 2 * depth)
    assert m.nv - m.ne + m.ncell == 1
    assert abs(m.S.sum() - area) < 1e-12 * area
    # the outer wall's cells are rectangles: a half of their depth on the wall side
    wall = ~m.inner
    cell = np.where(m.left >= 0, m.left, m.right)
    half = np.where(wall, 0.5 * m.S[cell] / m.elen, 0.0)
    assert np.all(cell[wall] >= m.nt)
    total = 0.5 * np.sum(m.elen[m.inner] * m.d[m.inner]) + 0.5 * np.sum(m.elen[wall] * half[wall])
    assert abs(total - area) < 1e-12 * area
    assert np.all(m.d[m.inner] > 0)
    # rectangles: the centre is equidistant from the corners
    for j in range(m.nt, m.ncell):
        nodes = np.unique(m.edge[m.cell_edges[j]].ravel())
        r = np.hypot(*(m.xy[nodes] - m.O[j]).T)
        assert len(nodes) == 4 and np.ptp(r) < 1e-12 * r.max()
    # every frame cell is split and damped; triangles are not
    assert np.all(m.split[m.nt:]) and not np.any(m.split[:m.nt])
    assert np.all(m.sigma_x[:m.nt] == 0) and np.all(m.sigma_y[:m.nt] == 0)
    assert np.all((m.sigma_x[m.nt:] > 0) | (m.sigma_y[m.nt:] > 0))
    assert np.all(m.sigma_e[:om.ne] == 0)


def test_energy_is_conserved_without_damping():
    om = _mesh()
    m = OpenMesh(om, 3, 0.5, 0.0)
    rng = np.random.default_rng(0)
    E = np.where(m.inner, rng.standard_normal(m.ne), 0.0)
    Bx, By = rng.standard_normal(m.ncell), np.where(m.split, rng.standard_normal(m.ncell), 0.0)
    dt = 0.9 * 2 / m.omega_max()
    W = []
    for _ in range(300):
        E2, Bx2, By2 = m.step(E, Bx, By, dt, 1)
        W.append(m.energy(E2, Bx + By, Bx2 + By2))
        E, Bx, By = E2, Bx2, By2
    assert (max(W) - min(W)) / W[0] < 1e-13


@pytest.mark.parametrize("kind", ["tri", "square"])
def test_no_layers_is_the_triangle_oracle(kind):
    om = _mesh(kind)
    m = OpenMesh(om, 0, 1.0, 0.0)
    assert m.ne == om.ne and m.ncell == om.nt
    rng = np.random.default_rng(1)
    E = np.where(m.inner, rng.standard_normal(m.ne), 0.0)
    B = rng.standard_normal(m.ncell)
    ref = om.step(E, B, 0.05, 25)
    Eo, Bo, _ = m.step(E, B, np.zeros(m.ncell), 0.05, 25)
    assert np.max(np.abs(ref["E"] - Eo)) < 1e-12 and np.max(np.abs(ref["B"] - Bo)) < 1e-12


def test_the_pml_absorbs_a_pulse():
    xy, tri, Lx, Ly = box_tri_mesh(16, 16, 1.0, 0.1, 2)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    left = {}
    for smax in (0.0, 2.0, -0.5):
        m = OpenMesh(om, 8, 1.0, smax)
        dt = 0.5 * 2 / OpenMesh(om, 8, 1.0, 0.0).omega_max()
        r2 = np.sum((m.O - [Lx / 2, Ly / 2]) ** 2, axis=1)
        B0 = np.where(m.split, 0.0, np.exp(-r2 / 2.0))
        tri_c = ~m.split
        n = int(2.0 * (Lx + Ly) / dt)
        E, Bx, By = m.step(np.zeros(m.ne), B0, np.zeros(m.ncell), dt, n)
        B = Bx + By
        e_in = np.sum(m.S[tri_c] * B[tri_c] ** 2)
        left[smax] = e_in / np.sum(m.S[tri_c] * B0[tri_c] ** 2)
    # (measured: 0.109, 8.9e-4, 1.3e3)
    assert left[0.0] > 0.05                         # a reflecting frame keeps a part of the pulse
    assert left[2.0] < 3e-3                         # the PML lets it go
    assert not np.isfinite(left[-0.5]) or left[-0.5] > 100 * left[0.0]   # the wrong sign grows
