"""GPU: lowest resonator modes (tyee_mesh_modes) against the oracle's eigenpairs.

Eigenvalues are unique and compared directly: |lambda_gpu - lambda_oracle| <= 1e-9 x the
Gershgorin bound the solver reports (the residual tolerance asked for is 1e-12 of it, and an
eigenvalue error is at most the residual). Eigenvectors are unique only up to sign, and up to
a rotation inside a cluster of equal eigenvalues: each GPU mode must lie in the oracle's
eigenspace of its cluster, S-distance <= 1e-6 (residual / gap bound with gaps >= 1e-4 of the
bound), and every GPU pair must be an S-orthonormal eigenpair of the oracle's matrix-free
operator.
"""
import sys

import numpy as np
import pytest

import oracle
from meshgen import box_mesh, box_tri_mesh, equilateral_torus, lattice_mesh

pytestmark = pytest.mark.gpu

SQ3 = np.sqrt(3.0)


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def _check(om, got, lam_ref, V_ref, gamma=None, ev_tol=1e-9, vec_tol=1e-6, cluster=1e-7):
    bound = got["lambda_bound"]
    lam, V = got["omega2"], got["modes"].T
    n = len(lam)
    assert got["converged"]
    assert np.max(np.abs(lam - lam_ref[:n])) <= ev_tol * bound
    G = V.T @ (om.S[:, None] * V)
    assert np.max(np.abs(G - np.eye(n))) < 1e-11
    for c in range(n):
        kv = -om.apply_LE(om.apply_LB(V[:, c], gamma), gamma)
        assert np.sqrt(np.sum(om.S * (kv - lam[c] * V[:, c]) ** 2)) <= 1e-10 * bound
        near = np.nonzero(np.abs(lam_ref - lam[c]) <= cluster * bound)[0]
        P = V_ref[:, near]
        proj = P @ (P.T @ (om.S * V[:, c]))
        assert np.sqrt(np.sum(om.S * (V[:, c] - proj) ** 2)) <= vec_tol, c


@pytest.mark.parametrize("order", ["none", "morton"])
def test_box_modes_match_oracle(ty, order):
    _note(f"case: box 24 x 36 triangular lattice (+-0.1h), 40 lowest modes, order {order}")
    xy, tri, Lx, Ly = box_tri_mesh(24, 36, 1.0, 0.1, 5)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(60)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    m.reorder(order)
    got = m.modes(40, tol=1e-12, max_iter=400)
    _note(f"  iters {got['iters']} applies {got['applies']} filter {got['filter_ms']:.1f} ms")
    _check(om, got, lam_ref, V_ref)
    assert abs(got["omega2"][0]) <= 1e-9 * got["lambda_bound"]          # static mode


def test_highest_modes_match_oracle_and_the_power_iteration(ty):
    _note("case: box 24 x 36 triangular lattice, 16 highest modes (the paper's order)")
    xy, tri, Lx, Ly = box_tri_mesh(24, 36, 1.0, 0.1, 5)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(40, which="highest")
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    m.reorder("morton")
    got = m.modes(16, which="highest", tol=1e-12, max_iter=400)
    _note(f"  iters {got['iters']} applies {got['applies']}")
    assert np.all(np.diff(got["omega2"]) <= 0)                       # descending
    _check(om, got, lam_ref, V_ref)
    lam_cfl, _, ok = m.cfl(rtol=1e-14, max_iter=400000)
    assert ok and abs(got["omega2"][0] - lam_cfl) <= 1e-9 * lam_cfl


def test_square_lattice_box_and_gamma(ty):
    _note("case: jittered square-lattice box 14 x 14, per-edge gamma, 24 modes")
    xy, tri, Lx, Ly = box_mesh(14, 14, 0.2, 2, h=1.0 / 14)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    gamma = 1.0 + 0.05 * np.sin(np.arange(om.ne) * 0.37)
    lam_ref, V_ref = om.modes(40, gamma)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    m.reorder("morton")
    got = m.modes(24, gamma=gamma, block=48, degree=200, tol=1e-12, max_iter=2000)
    _note(f"  iters {got['iters']} applies {got['applies']}")
    _check(om, got, lam_ref, V_ref, gamma=gamma)


def test_equilateral_torus_closed_form_and_degenerate_clusters(ty):
    nx, ny, a = 12, 8, 1.0
    _note(f"case: equilateral torus {nx} x {ny}: honeycomb closed form, degenerate clusters")
    xy, tri, Lx, Ly = equilateral_torus(nx, ny, a)
    om = oracle.OracleMesh(xy, tri, True, Lx, Ly)
    lam_ref, V_ref = om.modes(80)
    m = ty.Mesh(xy, tri, True, L=Lx, Ly=Ly)
    got = m.modes(48, block=80, tol=1e-12, max_iter=400)
    delta = np.array([[0.0, -a / SQ3], [a / 2, a / (2 * SQ3)], [-a / 2, a / (2 * SQ3)]])
    ex = []
    for m1 in range(nx):
        for m2 in range(ny):
            k = 2 * np.pi * np.array([m1 / Lx, m2 / Ly])
            f = np.abs(np.exp(1j * delta @ k).sum())
            ex += [4 / a ** 2 * (3 - f), 4 / a ** 2 * (3 + f)]
    ex = np.sort(ex)
    # sorted eigenvalues are unique even where the wanted count ends inside a cluster
    assert np.max(np.abs(got["omega2"] - ex[:48])) <= 1e-9 * got["lambda_bound"]
    _check(om, got, lam_ref, V_ref)


def test_largest_block_uses_the_global_memory_small_kernels(ty):
    # a block of 256 does not fit a packed triangle in LDS: Cholesky and Jacobi then run on
    # global memory
    _note("case: box 30 x 40 triangular lattice, 200 modes, block 256 (global-memory small kernels)")
    xy, tri, Lx, Ly = box_tri_mesh(30, 40, 1.0, 0.1, 11)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(256)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    m.reorder("morton")
    got = m.modes(200, block=256, tol=1e-11, max_iter=100)
    _note(f"  iters {got['iters']} applies {got['applies']} total {got['total_ms']:.0f} ms")
    _check(om, got, lam_ref, V_ref)


@pytest.mark.parametrize("n_modes,block", [(21, 37), (150, 191), (150, 192), (150, 201)])
def test_odd_and_largest_lds_block_widths(ty, n_modes, block):
    # an odd block gives the round-robin Jacobi a ghost row and column: 37 and 191 in LDS, 201
    # (too large for LDS) in global memory; 191 and 192 fill the LDS Jacobi's table and work split
    _note(f"case: box 16 x 24 triangular lattice, {n_modes} modes, block {block}")
    xy, tri, Lx, Ly = box_tri_mesh(16, 24, 1.0, 0.1, 3)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(min(om.nt, block + 40))
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    m.reorder("morton")
    got = m.modes(n_modes, block=block, tol=1e-11, max_iter=300)
    _note(f"  iters {got['iters']} applies {got['applies']}")
    _check(om, got, lam_ref, V_ref)


@pytest.mark.parametrize("block", [2, 3, 4, 5, 6])
def test_small_blocks(ty, block):
    # blocks of up to 4 vectors (at most two Jacobi pairs) compute every round's rotations in
    # a phase of their own; from 5 on the pair-slot waves compute the next round's
    _note(f"case: 4 x 3 box (24 triangles), {min(block, 2)} lowest modes, block {block}")
    xy, tri, Lx, Ly = box_mesh(4, 3, 0.1, 1, h=0.5)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(om.nt)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    got = m.modes(min(block, 2), block=block, tol=1e-12, max_iter=2000)
    _note(f"  iters {got['iters']} applies {got['applies']}")
    _check(om, got, lam_ref, V_ref)


def test_every_block_width_up_to_48(ty):
    # every block width from 2 to 48 (the Jacobi's work split and pair schedule depend on it),
    # eigenvalues against the oracle's dense spectrum
    _note("case: 6 x 4 box (48 triangles), blocks 2 .. 48, half as many modes")
    xy, tri, Lx, Ly = box_mesh(6, 4, 0.1, 1, h=0.5)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, _ = om.modes(om.nt)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    for block in range(2, om.nt + 1):
        k = max(1, block // 2)
        got = m.modes(k, block=block, tol=1e-11, max_iter=3000)
        assert got["converged"], block
        assert np.max(np.abs(got["omega2"] - lam_ref[:k])) <= 1e-9 * got["lambda_bound"], block


def test_whole_spectrum_of_a_tiny_mesh(ty):
    _note("case: 2 x 2 box (8 triangles), every mode, block = n_t")
    xy, tri, Lx, Ly = box_mesh(2, 2, 0.1, 1, h=0.5)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(om.nt)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    got = m.modes(om.nt, block=om.nt, tol=1e-13, max_iter=50)
    _check(om, got, lam_ref, V_ref)


def test_fig4_resonator_full_size(ty):
    _note("case: Fig. 4 resonator 70 x 101, h = 1 (16,497 triangles), 128 lowest modes")
    xy, tri, Lx, Ly = box_tri_mesh(70, 101, 1.0, 0.1, 0)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam_ref, V_ref = om.modes(160)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    m.reorder("morton")
    got = m.modes(128, block=160, tol=1e-11, max_iter=200)
    _note(f"  iters {got['iters']} applies {got['applies']} filter {got['filter_ms']:.1f} ms "
          f"total {got['total_ms']:.1f} ms")
    # sampled eigenvector checks: every 8th mode
    bound = got["lambda_bound"]
    assert got["converged"]
    assert np.max(np.abs(got["omega2"] - lam_ref[:128])) <= 1e-9 * bound
    V = got["modes"].T
    for c in range(0, 128, 8):
        near = np.nonzero(np.abs(lam_ref - got["omega2"][c]) <= 1e-7 * bound)[0]
        P = V_ref[:, near]
        r = V[:, c] - P @ (P.T @ (om.S * V[:, c]))
        assert np.sqrt(np.sum(om.S * r * r)) <= 1e-5, c


def test_repeatable_and_reports_non_convergence(ty):
    _note("case: box 16 x 24: bit-identical repeat; max_iter = 1 reports non-convergence")
    xy, tri, Lx, Ly = box_tri_mesh(16, 24, 1.0, 0.1, 9)
    m = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    a = m.modes(20, tol=1e-10)
    b = m.modes(20, tol=1e-10)
    assert np.array_equal(a["omega2"], b["omega2"]) and np.array_equal(a["modes"], b["modes"])
    c = m.modes(20, degree=2, tol=1e-14, max_iter=1)
    assert not c["converged"] and c["iters"] == 1 and np.max(c["residual"]) > 1e-14


def test_device_omega_max_at_the_bench_size(ty):
    """eq. 20's omega_max on the device (FP64) at the bench's size: the highest mode of the
    4M-triangle torus from the block solver against the host power iteration, and (a relaxed
    mesh has no isolated top mode) of the jello-relaxed 45 x 45 cavity."""
    n = 1415
    _note(f"case: torus{n} (4.0M triangles): omega_max^2 from the device's highest mode vs the host power iteration")
    xy, tri = lattice_mesh(n, 0.25, 1, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam_cfl, it, ok = m.cfl(rtol=1e-14, max_iter=20000)
    got = m.modes(4, which="highest", tol=1e-11, max_iter=400, want_vectors=False)
    _note(f"  host {lam_cfl:.15e} ({it} iterations), device {got['omega2'][0]:.15e} "
          f"(iters {got['iters']}, applies {got['applies']}, {got['total_ms']:.1f} ms)")
    assert ok and got["converged"]
    assert abs(got["omega2"][0] - lam_cfl) <= 1e-10 * lam_cfl
    # a relaxed mesh: no near-cocircular outlier, so the top of the spectrum is a cluster
    xy, tri = lattice_mesh(45, 0.2, 0, periodic=False)
    x1, t1, _, _ = ty.Mesh(xy, tri, False).relax(rounds=8, iters=100, step=0.05)
    mr = ty.Mesh(x1, t1, False)
    lam_cfl, it, ok = mr.cfl(rtol=1e-14, max_iter=400000)
    got = mr.modes(8, which="highest", tol=1e-11, max_iter=400, want_vectors=False)
    _note(f"  relaxed cavity45: host {lam_cfl:.15e} ({it} iterations), device {got['omega2'][0]:.15e}")
    assert ok and got["converged"]
    assert abs(got["omega2"][0] - lam_cfl) <= 1e-10 * lam_cfl
