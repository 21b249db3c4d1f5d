"""GPU: batched stepping of uneven meshes, hipGraph replay and the autotuner.

Every batch member must be bit-identical to its standalone simulation (same dt, numbering,
precision); graph replays bit-identical to eager launches; the autotuner must restore the
fields it advanced while timing trials.
"""
import sys

import numpy as np
import pytest

import oracle
from meshgen import lattice_mesh, periodic_wavevector, plane_wave_packet
from meshgen.workloads import batch_lattice_sizes
from common import rel_l2, packet_state

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def _members(ty, sizes, seed0, periodic=True):
    out = []
    for k, n in enumerate(sizes):
        per = periodic if isinstance(periodic, bool) else periodic[k]
        xy, tri = lattice_mesh(int(n), 0.25, seed0 + k, periodic=per)
        m = ty.Mesh(xy, tri, per)
        lam, _, _ = m.cfl()
        dt = 0.5 * 2 / np.sqrt(lam)
        out.append(dict(xy=xy, tri=tri, n=int(n), periodic=per, mesh=m, dt=dt))
    return out


def _initial(mem, view, k):
    if mem["periodic"]:
        kv, _, _ = periodic_wavevector(0.3 + 0.7 * k, 8.0 + 3 * k, 1.0 / mem["n"])
        B, E = plane_wave_packet(view["O"], view["C"], view["evec"] / view["elen"][:, None], kv,
                                 mem["dt"], sigma=0.15)
        return E, B
    from meshgen import cavity_mode
    return np.zeros(len(view["elen"])), cavity_mode(view["O"], 1, 2)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_members_bit_identical_to_standalone(ty, prec):
    sizes = [20, 9, 33, 14, 27, 6]
    periodic = [True, True, False, True, False, True]
    _note(f"case: batch of {len(sizes)} uneven meshes {prec}, fusion 4 tile 512 + graph")
    mem = _members(ty, sizes, 40, periodic)
    for m in mem:
        m["mesh"].reorder("morton")
    batch = ty.Batch([m["mesh"] for m in mem], [m["dt"] for m in mem], prec)
    views = [m["mesh"].view() for m in mem]
    for k, (m, v) in enumerate(zip(mem, views)):
        E, B = _initial(m, v, k)
        batch.set_state(k, "E", E)
        batch.set_state(k, "B", B)
    batch.set_fusion(4, 512)
    batch.set_graph(2)
    batch.step(41)
    batch.step(40)
    for k, (m, v) in enumerate(zip(mem, views)):
        sim = ty.Sim(m["mesh"], m["dt"], prec)
        E, B = _initial(m, v, k)
        sim.set_state("E", E)
        sim.set_state("B", B)
        sim.step(81)
        assert np.array_equal(batch.get_state(k, "E"), sim.get_state("E")), k
        assert np.array_equal(batch.get_state(k, "B"), sim.get_state("B")), k
    # one member against the oracle
    om = oracle.OracleMesh(mem[1]["xy"], mem[1]["tri"], True)
    E, B = _initial(mem[1], dict(O=om.O, C=om.C, evec=om.evec, elen=om.elen), 1)
    ref = om.step(E, B, mem[1]["dt"], 81)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel_l2(batch.get_state(1, "E"), ref["E"]) < tol
    assert rel_l2(batch.get_state(1, "B"), ref["B"]) < tol


def test_graph_replay_bit_identical(ty):
    n = 60
    _note("case: torus60 fp32 fusion 4 with graphs of 8 launches vs eager")
    xy, tri = lattice_mesh(n, 0.25, 9, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, _ = m.cfl()
    dt = 0.5 * 2 / np.sqrt(lam)
    v = m.view()
    out = []
    for graph in (0, 8):
        sim = ty.Sim(m, dt, "f32")
        E, B = packet_state(v, dt, n)
        sim.set_state("E", E)
        sim.set_state("B", B)
        sim.set_fusion(4, 1024)
        sim.set_graph(graph)
        sim.step(100)       # 3 graphs of 32 steps + 4 single steps
        sim.set_state("B", sim.get_state("B"))     # state upload between replays
        sim.step(70)
        out.append((sim.get_state("E"), sim.get_state("B")))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_autotuner_restores_state_and_picks_a_setting(ty):
    sizes = [30, 12, 45, 20]
    _note("case: batch of 4, autotune 16 steps per trial")
    mem = _members(ty, sizes, 70)
    batch = ty.Batch([m["mesh"] for m in mem], [m["dt"] for m in mem], "f32")
    views = [m["mesh"].view() for m in mem]
    for k, (m, v) in enumerate(zip(mem, views)):
        E, B = _initial(m, v, k)
        batch.set_state(k, "E", E)
        batch.set_state(k, "B", B)
    before = [batch.get_state(k, "E") for k in range(4)]
    seen = []
    res = batch.tune(16, progress=seen.append)
    assert len(res) == 2 * (1 + 4 * 4)
    assert seen == res            # one report per trial, as it ends, with the same record
    assert all(r["ms_per_step"] > 0 for r in res)
    after = [batch.get_state(k, "E") for k in range(4)]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    batch.step(24)
    ref = ty.Sim(mem[2]["mesh"], mem[2]["dt"], "f32")
    E, B = _initial(mem[2], views[2], 2)
    ref.set_state("E", E)
    ref.set_state("B", B)
    ref.step(24)
    # the tuner may have renumbered the members: compare in canonical order, to FP32 rounding
    assert rel_l2(batch.get_state(2, "E"), ref.get_state("E")) < 1e-6


@pytest.mark.slow
def test_batch256_full_size_members(ty):
    """The batched workload at its stated length: 256 members, 2,000 steps from graphs of 8
    fused launches; four members bit-identical to their standalone runs and sixteen, spread
    over the sizes, against the oracle element by element."""
    sizes = batch_lattice_sizes(256, seed=4)
    _note(f"case: batch256 full size ({int(np.sum(2 * sizes ** 2))} triangles), 2,000 steps")
    mem = _members(ty, sizes, 1000)
    for m in mem:
        m["mesh"].reorder("morton")
    batch = ty.Batch([m["mesh"] for m in mem], [m["dt"] for m in mem], "f32")
    info = batch.info()
    assert info["members"] == 256 and info["triangles"] == int(np.sum(2 * sizes ** 2))
    views = [m["mesh"].view() for m in mem]
    for k, (m, v) in enumerate(zip(mem, views)):
        E, B = _initial(m, v, k % 7)
        batch.set_state(k, "E", E)
        batch.set_state(k, "B", B)
    batch.set_fusion(4, 0)
    batch.set_graph(8)
    batch.step(2000)
    assert batch.sim().diagnostics()["nonfinite"] == 0
    for k in (0, int(np.argmin(sizes)), int(np.argmax(sizes)), 255):
        m = mem[k]
        sim = ty.Sim(m["mesh"], m["dt"], "f32")
        E, B = _initial(m, views[k], k % 7)
        sim.set_state("E", E)
        sim.set_state("B", B)
        sim.step(2000)
        assert np.array_equal(batch.get_state(k, "E"), sim.get_state("E")), k
        assert np.array_equal(batch.get_state(k, "B"), sim.get_state("B")), k
    order = np.argsort(sizes)
    worst = 0.0
    for k in order[np.linspace(0, 255, 16).astype(int)]:
        om = oracle.OracleMesh(mem[k]["xy"], mem[k]["tri"], True)
        E, B = _initial(mem[k], dict(O=om.O, C=om.C, evec=om.evec, elen=om.elen), k % 7)
        ref = om.step(E, B, mem[k]["dt"], 2000)
        eE = rel_l2(batch.get_state(k, "E"), ref["E"])
        eB = rel_l2(batch.get_state(k, "B"), ref["B"])
        worst = max(worst, eE, eB)
        assert eE < 1e-3 and eB < 1e-3, k
    _note(f"  16 members vs oracle after 2,000 steps: worst rel L2 {worst:.2e}")
