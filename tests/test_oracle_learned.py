"""Pins of the learned-correction oracle: closed forms on the equilateral mesh, geometric
identities of the features, finite-difference checks of both analytic gradients, and the
exact leap-frog phase of an eigenmode measured by the time-stepped phase error."""
import numpy as np
import pytest

import oracle
from oracle import learned as L
from meshgen import lattice_mesh, equilateral_torus, scramble

SQ3 = np.sqrt(3.0)


@pytest.fixture(scope="module")
def eq_mesh():
    xy, tri, Lx, Ly = equilateral_torus(12, 8, a=1.0)
    return oracle.OracleMesh(xy, tri, True, Lx, Ly)


@pytest.fixture(scope="module")
def jit_mesh():
    xy, tri = lattice_mesh(24, 0.3, 3, periodic=True)
    return oracle.OracleMesh(xy, tri, True)


def test_features_closed_form_on_equilateral_mesh(eq_mesh):
    f = L.features(eq_mesh)
    expect = [1 / SQ3, np.pi / 3, np.pi / 3, 1 / SQ3, 1 / SQ3, 0.0, 1 / np.sqrt(SQ3 / 4), 0.0]
    np.testing.assert_allclose(f, np.tile(expect, (eq_mesh.ne, 1)), atol=1e-12)


def test_features_geometry_and_symmetry(jit_mesh):
    f = L.features(jit_mesh)
    # d/|e| = (cot a_R + cot a_L)/2: the half dual length is (|e|/2) cot(opposite angle)
    np.testing.assert_allclose(f[:, 0], (1 / np.tan(f[:, 1]) + 1 / np.tan(f[:, 2])) / 2,
                               rtol=1e-9)
    m = jit_mesh
    assert np.all(f[:, 1] <= f[:, 2]) and np.all(f[:, 3] <= f[:, 4])
    assert np.all((f[:, 3] >= 1 / SQ3 - 1e-12))           # circumradius >= side / sqrt(3)
    # winding and row order of the input do not change any edge's features
    st, _ = scramble(m.tri, 4)
    m2 = oracle.OracleMesh(m.xy, st, True)
    np.testing.assert_allclose(L.features(m2), f, rtol=1e-10, atol=1e-12)


def _theta(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, L.N_PARAMS)


def test_mlp_identity_init_and_fd_gradient(jit_mesh):
    f = L.features(jit_mesh)[:200]
    mu, sd = f.mean(0), f.std(0) + 1e-3
    th = _theta(1)
    p0 = th.copy()
    p0[-(L.H2 + 1):] = 0.0                                 # w3 = b3 = 0
    assert np.all(L.mlp_forward(p0, f, mu, sd) == 1.0)
    rng = np.random.default_rng(2)
    up = rng.standard_normal(len(f))
    grad = L.mlp_param_grad(th, f, mu, sd, up)
    h = 1e-6
    for idx in list(range(0, L.N_PARAMS, 97)) + [L.N_PARAMS - 1]:
        tp, tm = th.copy(), th.copy()
        tp[idx] += h
        tm[idx] -= h
        fd = (np.dot(up, L.mlp_forward(tp, f, mu, sd)) - np.dot(up, L.mlp_forward(tm, f, mu, sd))) / (2 * h)
        assert abs(fd - grad[idx]) < 1e-7 * max(1.0, abs(fd)), idx
    g = L.mlp_forward(th, f, mu, sd)
    assert np.all((g > 0.9) & (g < 1.1))


def test_rq_closed_form_on_equilateral_mesh(eq_mesh):
    m = eq_mesh
    delta = np.array([[0.0, -1 / SQ3], [0.5, 1 / (2 * SQ3)], [-0.5, 1 / (2 * SQ3)]])
    dt = 0.1
    for m1, m2 in ((1, 0), (2, 1), (3, 2), (0, 1)):
        k = 2 * np.pi * np.array([m1 / m.Lx, m2 / m.Ly])
        w2 = 4.0 * (3.0 - np.sum(np.cos(delta @ k)))
        expect = 2 / dt * np.arcsin(np.sqrt(w2) * dt / 2) / np.hypot(*k) - 1
        assert abs(L.rq_phase_error(m, None, dt, k) - expect) < 1e-12


def test_rq_loss_gradient_fd(jit_mesh):
    m = jit_mesh
    rng = np.random.default_rng(3)
    gamma = 1 + 0.05 * rng.standard_normal(m.ne)
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    waves = [2 * np.pi * np.array(v, float) for v in ((1, 0), (2, 3), (-1, 4))]
    loss, grad = L.rq_loss_grad(m, gamma, dt, waves)
    assert loss > 0
    h = 1e-6
    for i in rng.choice(m.ne, 12, replace=False):
        gp, gm = gamma.copy(), gamma.copy()
        gp[i] += h
        gm[i] -= h
        fd = (L.rq_loss_grad(m, gp, dt, waves)[0] - L.rq_loss_grad(m, gm, dt, waves)[0]) / (2 * h)
        assert abs(fd - grad[i]) < 1e-6 * max(abs(fd), 1e-12) + 1e-14
    # scaling every coefficient by c scales omega_RQ by c (before the leap-frog asin)
    k = waves[0]
    kn = np.hypot(*k)
    e1 = L.rq_phase_error(m, None, dt, k)
    e2 = L.rq_phase_error(m, np.full(m.ne, 1.01), dt, k)
    s1 = np.sin((1 + e1) * kn * dt / 2)             # omega_RQ dt / 2 of the plain operator
    assert abs((1 + e2) - 2 / dt * np.arcsin(1.01 * s1) / kn) < 1e-12


def test_timestepped_phase_error_of_an_eigenmode(eq_mesh):
    # k along x on the equilateral torus: exp(i k.O) is an exact eigenvector of K with
    # omega = (4/a) sin(k a / 4); leap-frog then advances its phase by theta per step with
    # sin(theta/2) = omega dt / 2.
    m = eq_mesh
    dt = 0.5 * 2 / (2 * np.sqrt(6))
    for m1 in (1, 2):
        k = np.array([2 * np.pi * m1 / m.Lx, 0.0])
        om_ex = 4 * np.sin(k[0] / 4)
        expect = 2 / dt * np.arcsin(om_ex * dt / 2) / k[0] - 1
        got = L.timestepped_phase_error(m, None, dt, k, 400, samples=200)
        assert abs(got - expect) < 2e-3 * abs(expect) + 1e-5
        assert abs(L.rq_phase_error(m, None, dt, k) - expect) < 1e-12


def test_ts_phase_error_gradient_fd(jit_mesh):
    m = jit_mesh
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    rng = np.random.default_rng(5)
    gamma = 1 + 0.04 * rng.standard_normal(m.ne)
    k = 2 * np.pi * np.array([3.0, 1.0])
    n = L.ts_steps(k, dt)
    e, de = L.ts_phase_error_grad(m, gamma, dt, k, n)
    h = 1e-5         # the long recurrence carries ~1e-13 of rounding in the error itself
    for i in rng.choice(m.ne, 8, replace=False):
        gp, gm = gamma.copy(), gamma.copy()
        gp[i] += h
        gm[i] -= h
        fd = (L.ts_phase_error_grad(m, gp, dt, k, n)[0] - L.ts_phase_error_grad(m, gm, dt, k, n)[0]) / (2 * h)
        assert abs(fd - de[i]) < 1e-5 * abs(fd) + 1e-10, (i, fd, de[i])
    waves = [k, 2 * np.pi * np.array([1.0, -2.0])]
    loss, grad = L.ts_loss_grad(m, gamma, dt, waves)
    i = int(rng.integers(m.ne))
    gp, gm = gamma.copy(), gamma.copy()
    gp[i] += h
    gm[i] -= h
    fd = (L.ts_loss_grad(m, gp, dt, waves)[0] - L.ts_loss_grad(m, gm, dt, waves)[0]) / (2 * h)
    assert abs(fd - grad[i]) < 1e-5 * abs(fd) + 1e-10


def test_ts_phase_error_of_an_eigenmode_and_against_full_stepping(eq_mesh, jit_mesh):
    # equilateral torus, k along x: exact eigenvector, so the phase advances theta per step
    # with sin(theta/2) = omega dt / 2, omega = 4 sin(k/4)
    m = eq_mesh
    dt = 0.5 * 2 / (2 * np.sqrt(6))
    k = np.array([2 * np.pi * 2 / m.Lx, 0.0])
    theta = 2 * np.arcsin(4 * np.sin(k[0] / 4) * dt / 2)
    n = L.ts_steps(k, dt, 2.0)            # the measured phase must stay below pi
    e, _ = L.ts_phase_error_grad(m, None, dt, k, n)
    # exact solution of the recurrence for an eigenvector: x_n = c1 e^{-i theta n} + c2 e^{i theta n}
    # with x_0 = e^{-i a}, x_{-1} = e^{i a}, a = |k| dt / 2
    a = k[0] * dt / 2
    c1 = (np.exp(1j * a) - np.exp(-1j * a) * np.exp(-1j * theta)) / (2j * np.sin(theta))
    c2 = np.exp(-1j * a) - c1
    xn = c1 * np.exp(-1j * theta * n) + c2 * np.exp(1j * theta * n)
    expect = -np.angle(xn / np.exp(-1j * a)) / (k[0] * n * dt) - 1
    assert abs(e - expect) < 1e-10
    assert abs(e - (theta / (k[0] * dt) - 1)) < 5e-3      # close to the pure eigen phase
    # on a jittered mesh the B-only recurrence and the full E/B stepping agree on the phase
    m = jit_mesh
    dt = 0.5 * 2 / np.sqrt(m.power()[0])
    k = 2 * np.pi * np.array([2.0, 1.0])
    n = L.ts_steps(k, dt, 3.0)
    e_b, _ = L.ts_phase_error_grad(m, None, dt, k, n)
    e_full = L.timestepped_phase_error(m, None, dt, k, n, samples=30)
    assert abs(e_b - e_full) < 0.05 * abs(e_full)


def test_stiff_edge_term_value_and_gradient():
    # beta * mean over edges with d/|e| < tau of (gamma - target)^2: a hand-computed case
    feat = np.zeros((5, L.N_FEAT))
    feat[:, 0] = [0.001, 0.5, 0.01, 0.3, 0.019]        # edges 0, 2, 4 are below tau = 0.02
    gamma = np.array([1.0, 1.05, 0.95, 1.1, 0.9])
    loss, grad = L.stiff_reg_loss_grad(feat, gamma, tau=0.02, beta=2.0, target=0.9)
    expect = 2.0 * ((1.0 - 0.9) ** 2 + (0.95 - 0.9) ** 2 + 0.0) / 3
    assert abs(loss - expect) < 1e-15
    assert np.all(grad[[1, 3]] == 0.0) and grad[4] == 0.0
    h = 1e-7
    for i in range(5):
        gp, gm = gamma.copy(), gamma.copy()
        gp[i] += h
        gm[i] -= h
        fd = (L.stiff_reg_loss_grad(feat, gp, 0.02, 2.0, 0.9)[0]
              - L.stiff_reg_loss_grad(feat, gm, 0.02, 2.0, 0.9)[0]) / (2 * h)
        assert abs(fd - grad[i]) < 1e-8
    # no stiff edge: no term
    feat[:, 0] = 0.5
    assert L.stiff_reg_loss_grad(feat, gamma, 0.02, 2.0, 0.9)[0] == 0.0
