"""Write fig4_spectrum.npy: every eigenvalue of K on the Fig. 4 resonator mesh, from the oracle.

The mesh is the seeded 70 x 101 box of the test-suite (triangular lattice, h = 1, jitter 0.1 h,
seed 0: 16,497 triangles); the eigenvalues come from OracleMesh.spectrum (the dense library
eigensolver, about two minutes on eight cores).  Run from the repository root:
    python tests/golden/make_fig4_spectrum.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from meshgen import box_tri_mesh  # noqa: E402

OUT = os.path.join(HERE, "fig4_spectrum.npy")
MESH = (70, 101, 1.0, 0.1, 0)


def main():
    xy, tri, Lx, Ly = box_tri_mesh(*MESH)
    m = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    lam, _ = m.spectrum(vectors=False)
    np.save(OUT, lam)
    print(f"{OUT}: {len(lam)} eigenvalues, {lam[0]:.3e} .. {lam[-1]:.6f}")


if __name__ == "__main__":
    main()
