"""Media and source placement defined on the input node cloud and triangles.

Both are plain inputs: a 0/1 flag per input triangle (inside a triangular particle, the
plasma-like object of Fig. 3) and a list of node pairs with weights for a soft line
current source.
"""
import numpy as np

from .lattice import triangle_centroids, _unwrap


def triangle_particle_mask(xy, tri, periodic, L=1.0, side=0.25, center=(0.6, 0.5),
                           angle=np.pi / 2):
    """1 for input triangles whose vertex-average lies inside an equilateral triangle.

    The particle has the given side length, centroid and orientation (angle of the
    direction from the centroid to its first corner).
    """
    c = triangle_centroids(xy, tri, periodic, L)
    R = side / np.sqrt(3.0)
    corners = np.array([[center[0] + R * np.cos(angle + 2 * np.pi * q / 3),
                         center[1] + R * np.sin(angle + 2 * np.pi * q / 3)]
                        for q in range(3)])
    inside = np.ones(len(c), dtype=bool)
    for q in range(3):
        a, b = corners[q], corners[(q + 1) % 3]
        cross = (b[0] - a[0]) * (c[:, 1] - a[1]) - (b[1] - a[1]) * (c[:, 0] - a[0])
        inside &= cross > 0.0
    return inside.astype(np.uint8)


def line_source_pairs(xy, tri, periodic, L, h, x0=0.2, z0=0.25, z1=0.75, amp=1.0,
                      pol=(0.0, 1.0)):
    """Node pairs of the mesh lines lying along the segment x = x0, z in [z0, z1].

    A line is selected when its midpoint is within h/2 of x = x0 and z0 <= z <= z1. Its
    weight is amp * (t . pol) with t the unit vector from the lower to the higher node
    index. Returns (pairs int32[n, 2] with pairs[:,0] < pairs[:,1], weights float64[n]).
    """
    tri = np.asarray(tri)
    u = tri.reshape(-1)
    v = tri[:, [1, 2, 0]].reshape(-1)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    key = np.unique(lo.astype(np.int64) * len(xy) + hi)
    lo, hi = (key // len(xy)).astype(np.int64), (key % len(xy)).astype(np.int64)
    d = _unwrap(xy[hi] - xy[lo], L, periodic)
    mid = xy[lo] + 0.5 * d
    if periodic:
        mid = np.mod(mid, L)
    sel = (np.abs(mid[:, 0] - x0) < 0.5 * h) & (mid[:, 1] >= z0) & (mid[:, 1] <= z1)
    t = d[sel] / np.hypot(d[sel, 0], d[sel, 1])[:, None]
    w = amp * (t @ np.asarray(pol, dtype=np.float64))
    pairs = np.stack([lo[sel], hi[sel]], axis=1).astype(np.int32)
    keep = w != 0.0
    return np.ascontiguousarray(pairs[keep]), np.ascontiguousarray(w[keep])
