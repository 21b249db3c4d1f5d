"""GPU: the learned edge scale (features, MLP forward/backward, Adam, gate) against the oracle.

* loss, per-wave phase errors, dL/dtheta and gamma from the HIP kernels vs the FP64 oracle;
* the initial model (gamma = 1) reproduces the plain method bit-exactly;
* training on the GPU lowers the loss;
* the time-stepped phase error of the library equals the oracle's;
* end to end at reduced size: train, gate and evaluate on held-out meshes, showing what the
  trained network gains over the plain coefficients.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import learned as OL
from meshgen import lattice_mesh, periodic_wavevector
from common import rel_l2, packet_state

pytestmark = pytest.mark.gpu

ANGLES = np.arange(12) * np.pi / 12


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def waves_for(n, cells=(8, 10, 16, 32), angles=ANGLES):
    return np.array([periodic_wavevector(a, r, 1.0 / n)[0] for a in angles for r in cells])


def training_set(ty, sizes, seed0, jitter=0.3):
    out = []
    for k, n in enumerate(sizes):
        xy, tri = lattice_mesh(n, jitter, seed0 + k, periodic=True)
        m = ty.Mesh(xy, tri, True)
        om = oracle.OracleMesh(xy, tri, True)
        lam, _, _ = m.cfl()
        out.append(dict(n=n, xy=xy, tri=tri, mesh=m, om=om, dt=0.5 * 2 / np.sqrt(lam),
                        waves=waves_for(n)))
    return out


def test_learner_matches_oracle(ty):
    _note("case: learner loss/grad/gamma vs oracle on 3 meshes x 12 waves")
    ts = training_set(ty, [16, 20, 24], 300)
    for t in ts:
        t["waves"] = waves_for(t["n"], cells=(8, 16), angles=np.arange(6) * np.pi / 6)
    W = np.stack([t["waves"] for t in ts])
    lr = ty.Learner([t["mesh"] for t in ts], [t["dt"] for t in ts], W, phase=2.0)
    lr.regulariser(tau=0.05, beta=1e-3, target=0.9)
    feats = [OL.features(t["om"]) for t in ts]
    F = np.concatenate(feats)
    mu, sd = F.mean(0), F.std(0) + 1e-6
    lr.normaliser(mu, sd)
    theta = np.random.default_rng(7).uniform(-0.4, 0.4, OL.N_PARAMS)
    lr.set_params(theta)
    theta32 = lr.params()                      # the values the GPU holds (FP32)
    loss, grad, errs = lr.loss_grad(want_errors=True)
    ref_loss, ref_grad = 0.0, np.zeros(OL.N_PARAMS)
    for t, f, e_row in zip(ts, feats, errs):
        gam = OL.mlp_forward(theta32, f, mu, sd)
        assert np.max(np.abs(lr.gamma(t["mesh"]) - gam)) < 2e-6
        l, dg = OL.ts_loss_grad(t["om"], gam, t["dt"], t["waves"], phase=2.0)
        ref_loss += l / len(ts)
        ref_grad += OL.mlp_param_grad(theta32, f, mu, sd, dg / len(ts))
    # the stiff-edge term is a mean over all training meshes' stiff edges
    gall = np.concatenate([OL.mlp_forward(theta32, f, mu, sd) for f in feats])
    rl, rg = OL.stiff_reg_loss_grad(F, gall, tau=0.05, beta=1e-3, target=0.9)
    assert np.count_nonzero(F[:, 0] < 0.05) > 0
    ref_loss += rl
    ref_grad += OL.mlp_param_grad(theta32, F, mu, sd, rg)
    for t, f, e_row in zip(ts, feats, errs):
        gam = OL.mlp_forward(theta32, f, mu, sd)
        ref_e = [OL.ts_phase_error_grad(t["om"], gam, t["dt"], k, OL.ts_steps(k, t["dt"]))[0]
                 for k in t["waves"]]
        assert np.max(np.abs(e_row - ref_e)) < 2e-6, np.max(np.abs(e_row - ref_e))
    # per parameter: the FP32 recurrences (N <= 2,500 steps, worst-case linear growth of the
    # rounding, N 2^-24 < 1.5e-4) bound every component by 3e-4 of the largest one
    err = np.abs(grad - ref_grad)
    bound = 3e-4 * np.max(np.abs(ref_grad))
    _note(f"  loss {loss:.6e} ref {ref_loss:.6e}; grad rel L2 {rel_l2(grad, ref_grad):.2e}, "
          f"worst parameter {np.max(err) / bound:.3f} of the bound")
    assert abs(loss / ref_loss - 1) < 1e-3
    assert np.all(err <= bound)


def test_identity_model_is_plain_and_training_lowers_loss(ty):
    _note("case: gamma = 1 bit-exact, 150 Adam steps on the GPU")
    ts = training_set(ty, [32, 40], 400)
    lr = ty.Learner([t["mesh"] for t in ts], [t["dt"] for t in ts],
                    np.stack([t["waves"] for t in ts]), phase=2.0)
    lr.init(seed=3)
    t = ts[0]
    g = lr.gamma(t["mesh"])
    assert np.all(g == 1.0)
    v = t["mesh"].view()
    out = []
    for gamma in (None, g):
        sim = ty.Sim(t["mesh"], t["dt"], "f32")
        if gamma is not None:
            sim.set_edge_scale(gamma)
        E, B = packet_state(v, t["dt"], t["n"], cells=8.0)
        sim.set_state("E", E)
        sim.set_state("B", B)
        sim.step(40)
        out.append(sim.get_state("E"))
    assert np.array_equal(out[0], out[1])
    hist = lr.train(150, 3e-3)
    final, _, _ = lr.loss_grad(want_grad=False)
    _note(f"  loss {hist[0]:.4e} -> {final:.4e}")
    assert final < 0.5 * hist[0]
    g2 = lr.gamma(t["mesh"])
    assert np.all((g2 > 0.9) & (g2 < 1.1)) and np.std(g2) > 0


def test_timestepped_phase_error_matches_oracle(ty):
    _note("case: time-stepped phase error library vs oracle")
    xy, tri = lattice_mesh(24, 0.25, 11, periodic=True)
    m = ty.Mesh(xy, tri, True)
    om = oracle.OracleMesh(xy, tri, True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    k, _, _ = periodic_wavevector(0.3, 8.0, 1 / 24)
    g = 1 + 0.03 * np.cos(np.arange(om.ne))
    n = 4000
    phase = n * np.hypot(*k) * dt          # N = round(phase/(|k| dt)) = 4000
    for gamma in (None, g):
        a = m.phase_error_timestepped(dt, k, phase=phase, samples=20, gamma=gamma, prec="f64")
        b = OL.timestepped_phase_error(om, gamma, dt, k, n, samples=20)
        assert abs(a - b) < 1e-9, (a, b)
    # several waves in one call equal one call per wave
    ks = np.array([k, periodic_wavevector(1.1, 10.0, 1 / 24)[0]])
    many = m.phase_error_timestepped(dt, ks, phase=2.0, samples=10, prec="f64")
    one = [m.phase_error_timestepped(dt, kk, phase=2.0, samples=10, prec="f64") for kk in ks]
    np.testing.assert_array_equal(many, one)


def test_trained_network_gains_over_plain_on_held_out_meshes(ty):
    _note("case: train 8 meshes (n=32), gate + evaluate on 3 held-out meshes (n=48)")
    angles = np.arange(6) * np.pi / 6
    train = training_set(ty, [32] * 8, 500)
    lr = ty.Learner([t["mesh"] for t in train], [t["dt"] for t in train],
                    np.stack([waves_for(32, cells=(8, 10, 16), angles=angles)] * len(train)))
    lr.init(seed=1)
    hist = lr.train(200, 3e-3)
    _note(f"  training loss {hist[0]:.4e} -> {hist[-1]:.4e}")
    held = training_set(ty, [48] * 3, 900)
    gains = []
    for t in held:
        gam = lr.gamma(t["mesh"])
        w10 = waves_for(t["n"], cells=(10,), angles=angles)
        gate = t["mesh"].gate(gam, w10)
        _note(f"  held-out (time-stepped, 10 cells/lambda): plain {gate['err_plain']:.4e} "
              f"learned {gate['err_learned']:.4e} dt ratio "
              f"{gate['dt_learned'] / gate['dt_plain']:.4f} accepted {gate['accepted']}")
        assert gate["converged"] and gate["accepted"]
        gains.append(gate["err_plain"] / gate["err_learned"])
        # the oracle's own time stepping agrees on one wave
        k = w10[1]
        om = t["om"]
        ep = OL.timestepped_phase_error(om, None, gate["dt_plain"], k,
                                        OL.ts_steps(k, gate["dt_plain"]), samples=20)
        el = OL.timestepped_phase_error(om, gam, gate["dt_learned"], k,
                                        OL.ts_steps(k, gate["dt_learned"]), samples=20)
        _note(f"    oracle at {np.degrees(np.arctan2(k[1], k[0])):.0f} deg: plain {ep:.4e} "
              f"learned {el:.4e}")
        assert abs(el) < abs(ep)
    assert np.mean(gains) > 2.0


def test_gate_rejects_a_scale_that_slows_the_waves(ty):
    # a uniform scale c multiplies every coupling by c^2, so omega_max scales by c exactly;
    # c = 0.95 slows waves that already lag (plain errors are negative here): rejected
    _note("case: gate with gamma = 0.95 everywhere on a held-out mesh (n=48)")
    xy, tri = lattice_mesh(48, 0.3, 910, periodic=True)
    m = ty.Mesh(xy, tri, True)
    w10 = waves_for(48, cells=(10,), angles=np.arange(4) * np.pi / 4)
    gate = m.gate(np.full(m.ne, 0.95), w10)
    _note(f"  plain {gate['err_plain']:.4e} scaled {gate['err_learned']:.4e} "
          f"omega ratio {gate['omega_learned'] / gate['omega_plain']:.12f}")
    assert gate["converged"] and not gate["accepted"]
    assert abs(gate["omega_learned"] / gate["omega_plain"] - 0.95) < 1e-9
    assert abs(gate["dt_learned"] * 0.95 - gate["dt_plain"]) < 1e-9 * gate["dt_plain"]
    assert gate["err_learned"] > gate["err_plain"]


def test_learned_pieces_at_the_held_out_size(ty):
    # a held-out evaluation mesh at full size (707 x 707, 999,698 triangles): the scale at
    # every edge, the power iteration of the gate, and one time-stepped phase error (a short
    # sampled wave, so the oracle's two FP64 runs finish in seconds) against the oracle
    n = 707
    _note(f"case: learned pieces on a {n}x{n} held-out mesh vs oracle")
    xy, tri = lattice_mesh(n, 0.3, 200, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    om = oracle.OracleMesh(xy, tri, True)
    small = training_set(ty, [24], 77)
    lr = ty.Learner([small[0]["mesh"]], [small[0]["dt"]], np.stack([small[0]["waves"]]))
    F = OL.features(om)
    mu, sd = F.mean(0), F.std(0) + 1e-6
    lr.normaliser(mu, sd)
    lr.set_params(np.random.default_rng(11).uniform(-0.4, 0.4, OL.N_PARAMS))
    theta32 = lr.params()
    g = lr.gamma(m)
    g_ref = OL.mlp_forward(theta32, F, mu, sd)
    _note(f"  gamma max |diff| {np.max(np.abs(g - g_ref)):.2e} over {m.ne} edges")
    assert np.max(np.abs(g - g_ref)) < 2e-6
    # the gate's stability part: omega_max with and without the scale
    w = waves_for(n, cells=(10,), angles=np.array([0.3]))
    gate = m.gate(g, w, prec="f32")
    lam_p, _, ok_p = om.power()
    lam_l, _, ok_l = om.power(gamma=g)
    _note(f"  omega_max plain {gate['omega_plain']:.9e} (oracle {np.sqrt(lam_p):.9e}), "
          f"scaled {gate['omega_learned']:.9e} (oracle {np.sqrt(lam_l):.9e})")
    assert gate["converged"] and ok_p and ok_l
    assert abs(gate["omega_plain"] / np.sqrt(lam_p) - 1) < 1e-8
    assert abs(gate["omega_learned"] / np.sqrt(lam_l) - 1) < 1e-8
    # one time-stepped phase error (5 cells per wavelength, 0.5 rad of travel), FP32 stepping
    dt = gate["dt_learned"]
    k = periodic_wavevector(0.9, 5.0, 1.0 / n)[0]
    nsteps = max(10, int(round(0.5 / (np.hypot(*k) * dt))))
    got = m.phase_error_timestepped(dt, k, phase=0.5, samples=10, gamma=g, prec="f32")
    ref = OL.timestepped_phase_error(om, g, dt, k, nsteps, samples=10)
    _note(f"  phase error {got:.9e} oracle {ref:.9e} ({nsteps} steps)")
    assert abs(got - ref) < 1e-6
    # the folded scale in the stepping path the simulations use: default fused launches (6 steps
    # on 1536-triangle tiles) replayed from graphs of 8, 240 FP32 steps of a packet, element by
    # element against the oracle's FP64 run with the same scale
    sim = ty.Sim(m, dt, "f32")
    sim.set_edge_scale(g)
    sim.set_fusion(0, 0)
    sim.set_graph(8)
    v = m.view()
    E0, B0 = packet_state(v, dt, n)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.step(240)
    ref = om.step(*packet_state(om, dt, n), dt, 240, gamma=g)
    eE, eB = rel_l2(sim.get_state("E"), ref["E"]), rel_l2(sim.get_state("B"), ref["B"])
    _note(f"  scaled stepping, {sim.fusion_info()['steps_per_launch']} steps per launch, 240 steps: "
          f"rel L2 E {eE:.2e} B {eB:.2e}")
    assert sim.fusion_info()["steps_per_launch"] == 6
    assert eE < 1e-5 and eB < 1e-5
