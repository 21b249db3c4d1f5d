"""CPU checks of the seeded inputs that are more than a lattice: the conforming plasma
particle mesh (Delaunay, Euler count, sides present as edges, exact particle area) and the
plasma workload's parameters."""
import numpy as np
import pytest

import oracle
from meshgen import (conforming_particle_mesh, count_non_delaunay, lattice_mesh, particle_corners,
                     plasma_workload)


@pytest.mark.parametrize("n,seed", [(64, 3), (150, 8)])
def test_conforming_particle_mesh(n, seed):
    xy, tri, inside, seg = conforming_particle_mesh(n, 0.25, seed)
    assert len(tri) == 2 * len(xy)                       # torus: V - E + F = 0 with E = 3F/2
    assert count_non_delaunay(xy, tri, True) == 0
    u, v = tri.reshape(-1), tri[:, [1, 2, 0]].reshape(-1)
    keys = set(zip(np.minimum(u, v).tolist(), np.maximum(u, v).tolist()))
    assert all((min(a, b), max(a, b)) in keys for a, b in seg.tolist())
    om = oracle.OracleMesh(xy, tri, True)                # every dual length positive
    area = np.sqrt(3.0) / 4 * 0.25 ** 2
    assert abs(om.S[inside > 0].sum() - area) < 1e-12
    # far from the sides the lattice triangulation is untouched
    xy0, tri0 = lattice_mesh(n, 0.25, seed, True)
    c = particle_corners()
    far0 = np.all(np.abs(xy0[tri0].mean(1) - c.mean(0)) > 0.3, axis=1)
    key0 = {tuple(sorted(map(tuple, np.round(xy0[t], 15).tolist()))) for t in tri0[far0]}
    key1 = {tuple(sorted(map(tuple, np.round(xy[t], 15).tolist()))) for t in tri}
    assert key0 <= key1


def test_plasma_workload_small():
    w = plasma_workload(96)
    assert w["wp2_tri"].max() == pytest.approx((0.8 * 96) ** 2)
    assert np.all(w["wp2_tri"][w["inside"] == 0] == 0)
    assert w["nu"] == pytest.approx(0.05 * 96) and w["src_omega"] == pytest.approx(96)
    assert len(w["src_pairs"]) > 0 and np.all(w["src_pairs"][:, 0] < w["src_pairs"][:, 1])
