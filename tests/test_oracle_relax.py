"""Pins of the jello-relaxation oracle (Section 3, Fig. 5b) against facts that do not come
from the oracle itself: the forces are minus the gradient of the spring energy (central
differences), they sum to zero and carry no torque (translation and rotation invariance), a
perfect equilateral torus at its own rest length feels no force, hand-derived forces on a
right triangle, and the energy falls along small Euler steps (a damped gradient flow)."""
import numpy as np
import pytest

from oracle import relax as OR
from meshgen import lattice_mesh, equilateral_torus


def _fd_grad(xy, tri, periodic, Lx, Ly, a0, k_e, k_h, eps=1e-7):
    g = np.zeros_like(xy)
    for v in range(len(xy)):
        for c in range(2):
            p, m = xy.copy(), xy.copy()
            p[v, c] += eps
            m[v, c] -= eps
            g[v, c] = (OR.energy(p, tri, periodic, Lx, Ly, a0, k_e, k_h) -
                       OR.energy(m, tri, periodic, Lx, Ly, a0, k_e, k_h)) / (2 * eps)
    return g


@pytest.mark.parametrize("periodic", [False, True])
def test_forces_are_minus_the_energy_gradient(periodic):
    xy, tri = lattice_mesh(5, 0.3, 4, periodic=periodic)
    a0, _ = OR.rest_lengths(len(tri), 1.0)
    for k_e, k_h in ((1.0, 0.0), (0.0, 1.0), (1.0, 0.7)):
        F = OR.forces(xy, tri, periodic, 1.0, 1.0, a0, k_e, k_h)
        g = _fd_grad(xy, tri, periodic, 1.0, 1.0, a0, k_e, k_h)
        assert np.max(np.abs(F + g)) < 1e-6 * np.max(np.abs(F))
        # translation invariance: the forces balance
        assert np.max(np.abs(F.sum(0))) < 1e-12 * np.max(np.abs(F))
        if not periodic:
            # rotation invariance: no net torque about the origin
            torque = np.sum(xy[:, 0] * F[:, 1] - xy[:, 1] * F[:, 0])
            assert abs(torque) < 1e-12 * np.max(np.abs(F))


def test_equilateral_torus_at_its_rest_length_is_at_rest():
    xy, tri, Lx, Ly = equilateral_torus(6, 4, a=0.25)
    a0, h0 = OR.rest_lengths(len(tri), Lx * Ly)
    assert a0 == pytest.approx(0.25, rel=1e-14) and h0 == pytest.approx(0.25 * np.sqrt(3) / 2, rel=1e-14)
    F = OR.forces(xy, tri, True, Lx, Ly, a0)
    assert np.max(np.abs(F)) < 1e-13
    assert OR.energy(xy, tri, True, Lx, Ly, a0) < 1e-28


def test_right_triangle_forces_by_hand():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2]])
    s2 = np.sqrt(2.0)
    # edge springs at rest length 1: only the hypotenuse (length sqrt 2) is stretched; it pulls
    # nodes 1 and 2 toward each other with force (sqrt 2 - 1) along it
    F = OR.forces(xy, tri, False, 2.0, 2.0, 1.0, k_e=1.0, k_h=0.0)
    f = (s2 - 1) * np.array([-1.0, 1.0]) / s2
    np.testing.assert_allclose(F, [[0, 0], f, -f], atol=1e-15)
    # height springs at rest height h0 = sqrt(3)/2.  Apex 0 stands 1/sqrt 2 off the hypotenuse:
    # the spring pushes it away along (-1,-1)/sqrt 2 and each base end along (1,1)/(2 sqrt 2),
    # both with s0 = h0 - 1/sqrt 2.  Apex 1 stands 1 off leg 0-2: it is pulled toward it along
    # (1,0) and node 0 along (-1,0) with s1 = h0 - 1 (node 2 slides along the leg: no force);
    # likewise apex 2 over leg 0-1 with s2 = h0 - 1 along (0,1) and (0,-1) on node 0.
    F = OR.forces(xy, tri, False, 2.0, 2.0, 1.0, k_e=0.0, k_h=1.0)
    h0 = np.sqrt(3) / 2
    s0, s1 = h0 - 1 / s2, h0 - 1.0
    q = np.array([1.0, 1.0]) / (2 * s2)
    expect = np.array([s0 * np.array([-1.0, -1.0]) / s2 + s1 * np.array([-1.0, 0.0])
                       + s1 * np.array([0.0, -1.0]),
                       s0 * q + s1 * np.array([1.0, 0.0]),
                       s0 * q + s1 * np.array([0.0, 1.0])])
    np.testing.assert_allclose(F, expect, atol=1e-15)
    e = OR.energy(xy, tri, False, 2.0, 2.0, 1.0, k_e=0.0, k_h=1.0)
    assert e == pytest.approx(0.5 * ((1 / s2 - h0) ** 2 + 2 * (1 - h0) ** 2), rel=1e-14)


@pytest.mark.parametrize("periodic", [False, True])
def test_energy_falls_along_small_euler_steps(periodic):
    xy, tri = lattice_mesh(8, 0.3, 5, periodic=periodic)
    a0, _ = OR.rest_lengths(len(tri), 1.0)
    anchored = None
    if not periodic:
        anchored = (xy[:, 0] == 0) | (xy[:, 0] == 1) | (xy[:, 1] == 0) | (xy[:, 1] == 1)
    e = [OR.energy(xy, tri, periodic, 1.0, 1.0, a0)]
    x = xy
    for _ in range(5):
        x = OR.euler(x, tri, periodic, 1.0, 1.0, a0, 2, 0.05, anchored)
        e.append(OR.energy(x, tri, periodic, 1.0, 1.0, a0))
    assert all(b < a for a, b in zip(e, e[1:]))
    if anchored is not None:
        assert np.array_equal(x[anchored], xy[anchored])
