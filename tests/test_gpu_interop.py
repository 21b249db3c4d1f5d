"""GPU: caller-owned field buffers (torch tensors) bound to a simulation.

Stepping with bound buffers equals stepping with library memory bit for bit (fused launches
alternate between the two buffers, single steps update the current one); the tensors hold the
scaled edge field and B in device numbering; a change made through torch is what the next
steps advance; unbinding keeps the state.
"""
import sys

import numpy as np
import pytest

from meshgen import lattice_mesh
from common import packet_state

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ty():
    import paper_1812_01448_amd as ty
    return ty


def test_bound_torch_buffers(ty):
    import torch
    n = 40
    _note(f"case: torus{n} fp32 with E and B bound to torch tensors, fused and single steps")
    xy, tri = lattice_mesh(n, 0.25, 31, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, _ = m.cfl()
    dt = 0.5 * 2 / np.sqrt(lam)
    v = m.view()
    E0, B0 = packet_state(v, dt, n, cells=8.0)
    stream = torch.cuda.current_stream().cuda_stream

    def make():
        s = ty.Sim(m, dt, "f32", stream=stream)
        s.set_state("E", E0)
        s.set_state("B", B0)
        s.set_fusion(4, 0)
        return s

    ref = make()
    sim = make()
    tE = [torch.empty(m.ne, dtype=torch.float32, device="cuda") for _ in range(2)]
    tB = [torch.empty(m.nt, dtype=torch.float32, device="cuda") for _ in range(2)]
    sim.bind_external("E", tE[0], tE[1])
    sim.bind_external("B", tB[0], tB[1])
    for s in (ref, sim):
        for chunk in (12, 7, 20):          # fused launches and single-step tails
            s.step(chunk)
    assert np.array_equal(sim.get_state("E"), ref.get_state("E"))
    assert np.array_equal(sim.get_state("B"), ref.get_state("B"))
    cur = sim.current_buffer()
    assert cur == ref.current_buffer()
    torch.cuda.synchronize()
    E = sim.get_state("E")
    Et = E[v["perm_e"]] * v["elen"][v["perm_e"]]
    np.testing.assert_allclose(tE[cur].cpu().numpy(), Et, rtol=1e-6, atol=1e-30)
    np.testing.assert_array_equal(tB[cur].cpu().numpy().astype(np.float64),
                                  sim.get_state("B")[v["perm_t"]])
    # double the state through torch on the shared stream: the linear scheme then advances
    # exactly twice the reference state (scaling by 2 commutes with every rounding)
    tE[cur].mul_(2.0)
    tB[cur].mul_(2.0)
    for s in (ref, sim):
        s.step(9)
    assert np.array_equal(sim.get_state("E"), 2.0 * ref.get_state("E"))
    assert np.array_equal(sim.get_state("B"), 2.0 * ref.get_state("B"))
    before = sim.get_state("B")
    sim.bind_external("E", None, None)
    sim.bind_external("B", None, None)
    assert np.array_equal(sim.get_state("B"), before)
    sim.step(4)
    ref.step(4)
    assert np.array_equal(sim.get_state("B"), 2.0 * ref.get_state("B"))
    with pytest.raises(ty.TyeeError):
        sim.bind_external("J", tE[0], tE[1])
    with pytest.raises(ty.TyeeError):
        sim.bind_external("E", tE[0], tE[0])
