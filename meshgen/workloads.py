"""Named synthetic workloads (shapes, sizes and value distributions of the paper's setting).

* cavity45      closed unit-square resonator, 45 x 45 lattice, interior jitter +-0.2 h
* torus1415     periodic unit square, 1415 x 1415 lattice, jitter +-0.25 h (about 4.0M triangles)
* plasma2830    periodic unit square, 2830 x 2830 lattice, jitter +-0.25 h (about 16M triangles),
                with a triangular plasma particle and a soft line source
* batch256      256 periodic meshes with triangle counts log-uniform in [5k, 500k]
* learn_train / learn_eval   periodic meshes with jitter +-0.3 h for the learned correction

Any of them can be requested at a smaller lattice size n for tests.
"""
import numpy as np

from .lattice import lattice_mesh

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
