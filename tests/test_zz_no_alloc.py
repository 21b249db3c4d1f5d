"""GPU: the allocation-free diagnostics entry point against the allocating one.

Two calls in a row on the shared fixed scratch, the second on a smaller mesh (fewer partial
sums than the first left behind), then the first mesh again: each must return exactly what
tyee_sim_diagnostics returns for the same state (the totals are added in the same order).
"""
import numpy as np
import pytest

from meshgen import lattice_mesh
from common import packet_state

pytestmark = pytest.mark.gpu


def _sim(ty, n, prec, seed):
    xy, tri = lattice_mesh(n, 0.25, seed, periodic=True)
    m = ty.Mesh(xy, tri, True)
    m.reorder("morton")
    lam, _, _ = m.cfl()
    dt = 0.5 * 2 / np.sqrt(lam)
    sim = ty.Sim(m, dt, prec)
    E0, B0 = packet_state(m.view(), dt, n, cells=10.0)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_fusion(4, 0)
    return sim


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_diagnostics_match_the_allocating_entry_point(prec):
    import paper_1812_01448_amd as ty
    print(f"case: diagnostics_noalloc vs diagnostics, {prec}, torus 300 then torus 40",
          flush=True)
    big, small = _sim(ty, 300, prec, 31), _sim(ty, 40, prec, 32)
    # the fixed scratch needs the weight tables, which only the allocating call builds
    with pytest.raises(ty.TyeeError, match="tables are not built"):
        big.diagnostics_noalloc()
    for sim, steps in ((big, 37), (small, 21), (big, 8)):
        sim.step(steps)
        ref = sim.diagnostics()
        got = sim.diagnostics_noalloc()
        assert got == ref, (got, ref)
        assert got["nonfinite"] == 0 and got["energy_h"] > 0
        assert sim.diagnostics_noalloc() == ref          # a repeat reads the same bits
    # a new edge scale invalidates the tables until the allocating call rebuilds them
    small.set_edge_scale(np.full(small.ne, 1.01))
    with pytest.raises(ty.TyeeError, match="tables are not built"):
        small.diagnostics_noalloc()
    ref = small.diagnostics()
    assert small.diagnostics_noalloc() == ref
