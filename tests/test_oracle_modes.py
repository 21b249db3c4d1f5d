"""Pins of the oracle's mode solver (``OracleMesh.modes``) against facts from outside it.

* its sparse operators equal the C core's operators applied to unit vectors;
* the equilateral torus gives the honeycomb closed form, all modes;
* a closed box gives the resonator frequencies pi sqrt((m/Lx)^2 + (n/Ly)^2) with second-order
  convergence, through the dense and the sparse solver;
* the top mode (of the whole spectrum, and as the first of the highest modes, dense and sparse)
  equals the C core's power iteration; a uniform scale gamma multiplies every eigenvalue by
  gamma^2;
* every pair is an eigenpair of the C core's matrix-free operator, S-orthonormal, with one
  static (zero) mode on a connected mesh.

Pins of the whole spectrum (``OracleMesh.spectrum``): the honeycomb closed form on the
equilateral torus; the sums of the eigenvalues and of their squares equal the traces of K and
K^2 written out from the weights gamma^2 |e|/d and the areas S (K's definition from eqs. 3-4);
on a tiny mesh, the eigenvalues of the non-symmetric K built column by column from the C core
(a general eigenvalue routine); S-orthonormal eigenpairs of the matrix-free operator.
"""
import numpy as np
import pytest

import oracle
from meshgen import lattice_mesh, box_mesh, equilateral_torus

SQ3 = np.sqrt(3.0)


def test_sparse_operators_equal_unit_vector_application():
    for periodic in (False, True):
        xy, tri = lattice_mesh(9, 0.25, 4, periodic=periodic)
        m = oracle.OracleMesh(xy, tri, periodic)
        gamma = 1.0 + 0.1 * np.cos(np.arange(m.ne))
        for g in (None, gamma):
            LB, LE = m.sparse_ops(g)
            LBd = np.stack([m.apply_LB(np.eye(m.nt)[j], g) for j in range(m.nt)], axis=1)
            LEd = np.stack([m.apply_LE(np.eye(m.ne)[i], g) for i in range(m.ne)], axis=1)
            assert np.array_equal(LB.toarray(), LBd) and np.array_equal(LE.toarray(), LEd)


def test_all_modes_of_the_equilateral_torus_are_the_honeycomb_closed_form():
    nx, ny, a = 6, 4, 1.0
    xy, tri, Lx, Ly = equilateral_torus(nx, ny, a)
    m = oracle.OracleMesh(xy, tri, True, Lx, Ly)
    lam, V = m.modes(m.nt)
    delta = np.array([[0.0, -a / SQ3], [a / 2, a / (2 * SQ3)], [-a / 2, a / (2 * SQ3)]])
    ex = []
    for m1 in range(nx):
        for m2 in range(ny):
            k = 2 * np.pi * np.array([m1 / Lx, m2 / Ly])
            f = np.abs(np.exp(1j * delta @ k).sum())
            ex += [4 / a ** 2 * (3 - f), 4 / a ** 2 * (3 + f)]
    np.testing.assert_allclose(lam, np.sort(ex), atol=1e-12)


@pytest.mark.parametrize("sparse", [False, True])
def test_box_modes_converge_to_the_resonator_frequencies(sparse):
    # box 1 x 1.5: exact omega^2 = pi^2 ((m/1)^2 + (n/1.5)^2), m, n >= 0 not both zero
    Lx, Ly = 1.0, 1.5
    exact = np.sort([np.pi ** 2 * ((p / Lx) ** 2 + (q / Ly) ** 2)
                     for p in range(6) for q in range(6)])[1:9]
    errs = []
    for n in ((12, 24) if not sparse else (30, 60)):
        xy, tri, _, _ = box_mesh(n, int(1.5 * n), 0.2, 3, h=1.0 / n)
        m = oracle.OracleMesh(xy, tri, False, Lx, Ly)
        assert (m.nt > 4000) == (sparse and n == 60) or not sparse
        lam, _ = m.modes(9)
        assert abs(lam[0]) < 1e-9 * lam[1]
        errs.append(np.max(np.abs(np.sqrt(lam[1:]) / np.sqrt(exact) - 1)))
    assert errs[1] < errs[0] / 2.5                 # second order: about 4x per halving of h
    assert errs[1] < (2e-3 if sparse else 1e-2)


def test_top_mode_is_the_power_iteration_and_gamma_scales_the_spectrum():
    xy, tri = lattice_mesh(10, 0.25, 6, periodic=True)
    m = oracle.OracleMesh(xy, tri, True)
    lam, _ = m.modes(m.nt)
    top, _, ok = m.power(rtol=1e-14, max_iter=200000)
    assert ok and abs(lam[-1] - top) < 1e-9 * top
    # the highest modes are the top of the same spectrum, descending
    hi, Vh = m.modes(5, which="highest")
    np.testing.assert_allclose(hi, lam[::-1][:5], rtol=1e-12)
    assert np.max(np.abs(Vh.T @ (m.S[:, None] * Vh) - np.eye(5))) < 1e-12
    lam2, _ = m.modes(20, gamma=np.full(m.ne, 1.1))
    np.testing.assert_allclose(lam2[1:], 1.21 * lam[1:20], rtol=1e-10)
    # sparse path (more than 4,000 triangles)
    xy, tri, Lx, Ly = box_mesh(50, 50, 0.2, 7, h=0.02)
    mb = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    assert mb.nt > 4000
    hi, _ = mb.modes(3, which="highest")
    top, _, ok = mb.power(rtol=1e-14, max_iter=400000)
    assert ok and abs(hi[0] - top) < 1e-9 * top and hi[0] >= hi[1] >= hi[2]


@pytest.mark.parametrize("periodic", [False, True])
def test_modes_are_s_orthonormal_eigenpairs_of_the_matrix_free_operator(periodic):
    xy, tri = lattice_mesh(14, 0.25, 8, periodic=periodic)
    m = oracle.OracleMesh(xy, tri, periodic)
    gamma = 1.0 + 0.05 * np.sin(np.arange(m.ne) * 0.7)
    lam, V = m.modes(40, gamma)
    top = m.power(gamma)[0]
    for c in range(40):
        kv = -m.apply_LE(m.apply_LB(V[:, c], gamma), gamma)
        assert np.sqrt(np.sum(m.S * (kv - lam[c] * V[:, c]) ** 2)) < 1e-10 * top
    G = V.T @ (m.S[:, None] * V)
    assert np.max(np.abs(G - np.eye(40))) < 1e-12
    assert np.all(lam[1:] > 1e-6 * top) and abs(lam[0]) < 1e-10 * top
    # the static mode is the constant field
    v0 = V[:, 0] / V[np.argmax(np.abs(V[:, 0])), 0]
    assert np.max(np.abs(v0 - 1.0)) < 1e-9


def test_whole_spectrum_of_the_equilateral_torus_is_the_honeycomb_closed_form():
    nx, ny, a = 8, 6, 1.0
    xy, tri, Lx, Ly = equilateral_torus(nx, ny, a)
    m = oracle.OracleMesh(xy, tri, True, Lx, Ly)
    lam, V = m.spectrum()
    delta = np.array([[0.0, -a / SQ3], [a / 2, a / (2 * SQ3)], [-a / 2, a / (2 * SQ3)]])
    ex = []
    for m1 in range(nx):
        for m2 in range(ny):
            k = 2 * np.pi * np.array([m1 / Lx, m2 / Ly])
            f = np.abs(np.exp(1j * delta @ k).sum())
            ex += [4 / a ** 2 * (3 - f), 4 / a ** 2 * (3 + f)]
    assert len(lam) == m.nt == len(ex)
    np.testing.assert_allclose(lam, np.sort(ex), atol=1e-12)
    assert np.max(np.abs(V.T @ (m.S[:, None] * V) - np.eye(m.nt))) < 1e-12
    lam_only, none = m.spectrum(vectors=False)
    assert none is None and np.max(np.abs(lam_only - lam)) < 1e-12


def _traces(m, gamma):
    """trace K and trace K^2 from K's entries: (K B)_j = (1/S_j) sum over interior edges i of j
    of w_i (B_j - B_other), w_i = gamma_i^2 |e_i| / d_i."""
    w = np.where(m.interior, gamma ** 2 * m.elen / np.where(m.d != 0, m.d, 1.0), 0.0)
    diag = np.zeros(m.nt)
    i = np.nonzero(m.interior)[0]
    np.add.at(diag, m.R[i], w[i] / m.S[m.R[i]])
    np.add.at(diag, m.L[i], w[i] / m.S[m.L[i]])
    # K_RL K_LR = w^2 / (S_R S_L); a pair of triangles sharing two edges (periodic strips) is
    # not made here
    off2 = 2.0 * np.sum(w[i] ** 2 / (m.S[m.R[i]] * m.S[m.L[i]]))
    return diag.sum(), np.sum(diag ** 2) + off2


@pytest.mark.parametrize("periodic", [False, True])
def test_whole_spectrum_sums_are_the_traces_of_k_and_k_squared(periodic):
    xy, tri = lattice_mesh(12, 0.25, 11, periodic=periodic)
    m = oracle.OracleMesh(xy, tri, periodic)
    gamma = 1.0 + 0.1 * np.cos(np.arange(m.ne) * 1.3)
    lam, V = m.spectrum(gamma)
    t1, t2 = _traces(m, gamma)
    assert abs(lam.sum() - t1) < 1e-11 * t1
    assert abs(np.sum(lam ** 2) - t2) < 1e-11 * t2
    top = lam[-1]
    for c in range(0, m.nt, 7):
        kv = -m.apply_LE(m.apply_LB(V[:, c], gamma), gamma)
        assert np.sqrt(np.sum(m.S * (kv - lam[c] * V[:, c]) ** 2)) < 1e-11 * top
    assert np.max(np.abs(V.T @ (m.S[:, None] * V) - np.eye(m.nt))) < 1e-11


def test_whole_spectrum_of_a_tiny_mesh_is_the_general_eigenvalues_of_k():
    xy, tri, Lx, Ly = box_mesh(3, 3, 0.15, 2, h=0.5)
    m = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    K = np.stack([-m.apply_LE(m.apply_LB(np.eye(m.nt)[j])) for j in range(m.nt)], axis=1)
    ev = np.linalg.eigvals(K)                      # K itself is not symmetric (S differs)
    assert np.max(np.abs(ev.imag)) < 1e-10 * np.max(np.abs(ev.real))
    lam, _ = m.spectrum()
    np.testing.assert_allclose(lam, np.sort(ev.real), atol=1e-11 * lam[-1])


def test_nearest_modes_are_the_middle_of_the_whole_spectrum():
    xy, tri, Lx, Ly = box_mesh(16, 24, 0.15, 4, h=0.25)
    m = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam, V = m.spectrum()
    k = m.nt // 2
    sigma = 0.5 * (lam[k] + lam[k + 1])
    near, W = m.modes(10, which="nearest", sigma=sigma)
    idx = np.argsort(np.abs(lam - sigma))[:10]
    np.testing.assert_allclose(near, np.sort(lam[idx]), atol=1e-11 * lam[-1])
    # the same eigenvectors (simple eigenvalues here), up to sign
    for c, j in enumerate(np.sort(idx)):
        assert abs(abs(np.sum(m.S * W[:, c] * V[:, j])) - 1.0) < 1e-8
