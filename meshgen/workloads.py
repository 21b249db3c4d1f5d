"""Named synthetic workloads (shapes, sizes and value distributions of the paper's setting).

* cavity45      closed unit-square resonator, 45 x 45 lattice, interior jitter +-0.2 h
* torus1415     periodic unit square, 1415 x 1415 lattice, jitter +-0.25 h (about 4.0M triangles)
* plasma2830    periodic unit square, 2830 x 2830 lattice, jitter +-0.25 h (about 16M triangles),
                with an equilateral plasma particle whose sides are mesh edges and a soft line
                source (plasma_workload)
* batch256      256 periodic meshes with triangle counts log-uniform in [5k, 500k]
* learn_train / learn_eval   periodic meshes with jitter +-0.3 h for the learned correction

Any of them can be requested at a smaller lattice size n for tests.
"""
import numpy as np

from .lattice import lattice_mesh
from .media import conforming_particle_mesh, line_source_pairs

WORKLOADS = {
    "cavity45": dict(n=45, jitter=0.2, seed=0, periodic=False),
    "torus1415": dict(n=1415, jitter=0.25, seed=1, periodic=True),
    "plasma2830": dict(n=2830, jitter=0.25, seed=3, periodic=True),
    "learn_train": dict(n=316, jitter=0.3, seed=100, periodic=True),
    "learn_eval": dict(n=707, jitter=0.3, seed=200, periodic=True),
}


def make_workload(name, n=None, seed=None, jitter=None):
    """Mesh of a named workload: dict(xy, tri, periodic, L, h, n, jitter, seed)."""
    w = dict(WORKLOADS[name])
    if n is not None:
        w["n"] = int(n)
    if seed is not None:
        w["seed"] = int(seed)
    if jitter is not None:
        w["jitter"] = float(jitter)
    xy, tri = lattice_mesh(w["n"], w["jitter"], w["seed"], w["periodic"])
    h = 1.0 / w["n"] if w["periodic"] else 1.0 / (w["n"] - 1)
    return dict(xy=xy, tri=tri, periodic=w["periodic"], L=1.0, h=h, n=w["n"],
                jitter=w["jitter"], seed=w["seed"], name=name)


def batch_lattice_sizes(count=256, tmin=5e3, tmax=5e5, seed=4):
    """Lattice sizes N_k = round(sqrt(T_k / 2)) for T_k ~ log-uniform[tmin, tmax]."""
    rng = np.random.default_rng(seed)
    T = np.exp(rng.uniform(np.log(tmin), np.log(tmax), size=count))
    return np.maximum(4, np.round(np.sqrt(T / 2.0))).astype(int)


def plasma_workload(n=2830, seed=3, jitter=0.25):
    """The plasma-particle workload in mesh units (length unit h = 1/n, c = 1).

    Particle: equilateral, side 0.25, centroid (0.6, 0.5), sides conforming to mesh edges;
    plasma frequency 0.8 and collision rate 0.05 per mesh-unit time inside it. Source: soft
    current on the mesh lines along x = 0.2, 0.25 <= z <= 0.75, polarised along z, unit
    amplitude, angular frequency 1 per mesh-unit time, 10 cycles. All rates are returned
    in the unit square's time (rate / h).
    """
    xy, tri, inside, segments = conforming_particle_mesh(n, jitter, seed)
    h = 1.0 / n
    pairs, w = line_source_pairs(xy, tri, True, 1.0, h)
    return dict(xy=xy, tri=tri, inside=inside, segments=segments, periodic=True, L=1.0, h=h,
                n=n, seed=seed, jitter=jitter, wp2_tri=(0.8 / h) ** 2 * inside.astype(np.float64),
                nu=0.05 / h, src_pairs=pairs, src_weights=w, src_omega=1.0 / h, src_cycles=10.0,
                name="plasma%d" % n)
