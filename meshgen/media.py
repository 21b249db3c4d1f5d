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


def particle_corners(side=0.25, center=(0.6, 0.5), angle=np.pi / 2):
    """Corners (counter-clockwise) of the equilateral particle."""
    R = side / np.sqrt(3.0)
    return np.array([[center[0] + R * np.cos(angle + 2 * np.pi * q / 3),
                      center[1] + R * np.sin(angle + 2 * np.pi * q / 3)] for q in range(3)])


def _distance_to_sides(p, corners):
    out = np.full(len(p), np.inf)
    for q in range(3):
        a, b = corners[q], corners[(q + 1) % 3]
        ab = b - a
        t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
        out = np.minimum(out, np.hypot(*(p - a - t[:, None] * ab).T))
    return out


def conforming_particle_mesh(n, jitter, seed, L=1.0, side=0.25, center=(0.6, 0.5),
                             angle=np.pi / 2, clear=0.5):
    """Periodic jittered-lattice Delaunay mesh whose edges follow the particle's sides.

    Each side is split into round(side/h) equal pieces whose end points join the cloud;
    lattice points closer than clear*h to a side are dropped. With clear >= 1/2 the circle
    on each piece as diameter holds no other point, so every piece is a Delaunay edge and
    the particle is a union of triangles. Only a band around the sides changes: lattice
    triangles with no vertex within 4h of a side are kept, the rest comes from a Delaunay
    triangulation (scipy's Qhull) of the points within 10h of a side. Both margins exceed
    twice the largest empty circle of the cloud, so the union is the Delaunay
    triangulation of the whole modified cloud.

    Returns (xy, tri, inside uint8[n_t], segments int32[m, 2] of node pairs on the sides).
    """
    from scipy.spatial import Delaunay
    from .lattice import lattice_mesh

    h = L / n
    xy0, tri0 = lattice_mesh(n, jitter, seed, periodic=True, L=L)
    corners = particle_corners(side, center, angle)
    if np.any(corners - 10 * h < 0) or np.any(corners + 10 * h > L):
        raise ValueError("particle too close to the domain edge for this n")
    m = max(1, int(round(side / h)))
    seg_pts = np.concatenate([corners[q] + np.outer(np.arange(m) / m, corners[(q + 1) % 3] - corners[q])
                              for q in range(3)])
    dist = _distance_to_sides(xy0, corners)
    keep = dist >= clear * h
    near = dist < 4 * h                 # band whose triangles are rebuilt
    band = (dist < 10 * h) & keep       # lattice points handed to Qhull
    # node numbering: kept lattice points in lattice order, then the side points
    new_id = np.full(len(xy0), -1, np.int64)
    new_id[keep] = np.arange(int(keep.sum()))
    n_keep = int(keep.sum())
    xy = np.concatenate([xy0[keep], seg_pts])
    outer = ~near[tri0].any(axis=1)
    tri_a = new_id[tri0[outer]]
    loc = np.concatenate([np.nonzero(band)[0], -1 - np.arange(len(seg_pts))])
    pts = np.concatenate([xy0[band], seg_pts])
    dt = Delaunay(pts)
    simp = dt.simplices
    glob = np.where(loc >= 0, new_id[np.maximum(loc, 0)], n_keep + (-1 - loc))
    in_near = np.concatenate([near[band], np.ones(len(seg_pts), bool)])
    tri_b = glob[simp[in_near[simp].any(axis=1)]]
    tri = np.concatenate([tri_a, tri_b]).astype(np.int32)
    # counter-clockwise
    p0 = xy[tri[:, 0]]
    d1 = xy[tri[:, 1]] - p0
    d1 -= L * np.round(d1 / L)
    d2 = xy[tri[:, 2]] - p0
    d2 -= L * np.round(d2 / L)
    cw = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0] < 0
    tri[cw] = tri[cw][:, ::-1]
    inside = triangle_particle_mask(xy, tri, True, L, side, center, angle)
    seg_ids = n_keep + np.arange(len(seg_pts))
    segments = np.stack([seg_ids, np.roll(seg_ids, -1)], 1).astype(np.int32)
    return xy, np.ascontiguousarray(tri), inside, segments
