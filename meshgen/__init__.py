"""Seeded synthetic inputs for the triangular Yee-like solver.

This package is the one input source that both the GPU library and the CPU oracle consume.
It holds none of the solver's arithmetic: no connectivity, no dual lengths, no coefficients,
no stepping. It produces

* node clouds and triangles (the mesh-creation stage of Section 3: seeding, then a Delaunay
  triangulation, then flip refinement until every edge passes the empty-circumcircle test),
* per-triangle media masks and source node pairs, which are defined on the input itself,
* closed-form fields (cavity modes, plane-wave packets) evaluated at points that the caller
  takes from one side's own geometry,
* tetrahedra of a box (the Delaunay tetrahedralisation of a jittered BCC lattice) for the
  three-dimensional form of the scheme.

Every random draw comes from ``numpy.random.default_rng(seed)``.
"""
from .lattice import (lattice_mesh, box_mesh, box_tri_mesh, incircle, lawson_flip, count_non_delaunay, equilateral_torus,
                      triangle_centroids, scramble)
from .fields import (cavity_mode, plane_wave_packet, periodic_wavevector,
                     random_angle, source_waveform)
from .media import (triangle_particle_mask, line_source_pairs, conforming_particle_mesh,
                    particle_corners)
from .workloads import WORKLOADS, make_workload, plasma_workload
from .tet import bcc_box, insphere_violations

__all__ = [
    "lattice_mesh", "box_mesh", "box_tri_mesh", "incircle", "lawson_flip", "count_non_delaunay", "triangle_centroids",
    "scramble", "equilateral_torus", "cavity_mode", "plane_wave_packet", "periodic_wavevector", "random_angle",
    "source_waveform", "triangle_particle_mask", "line_source_pairs", "conforming_particle_mesh",
    "particle_corners", "WORKLOADS", "make_workload", "plasma_workload", "bcc_box", "insphere_violations",
]
