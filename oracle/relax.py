"""FP64 oracle of the jello mesh relaxation (TEST INFRASTRUCTURE ONLY).

Section 3 (mesh generation, Fig. 5b) relaxes a seeded node cloud by treating it as nodes joined
by springs along the triangle edges and along the triangle heights, whose rest lengths are those
of a perfect mesh of equilateral triangles covering the domain.  The motion is strongly damped
and the second time derivative is dropped, so each node moves along its net spring force
(the "jello" model), integrated with Euler steps; seeding nodes of the geometry stay anchored,
and the node cloud is remeshed (flips) between rounds.

Written here from those definitions, in plain Python loops over edges and triangles (small
meshes only):
- `rest_lengths`: side a of the equilateral triangle that tiles the domain with n_t triangles,
  and its height a sqrt(3)/2;
- `energy`: sum over edges of k_e/2 (l - a)^2 plus, over every triangle and each of its three
  vertices, k_h/2 (h - a sqrt(3)/2)^2 with h the distance of the vertex from the opposite side;
- `forces`: minus the gradient of that energy, per node, from the analytic derivatives of
  lengths and heights;
- `euler`: x <- x + tau F(x) for the nodes not anchored (wrapped into the torus).
"""
import numpy as np


def _mi(d, L, periodic):
    """Minimum image of a coordinate difference."""
    return d - L * np.round(d / L) if periodic else d


def rest_lengths(n_tris, area):
    """(a, h): equilateral side and height for n_tris triangles covering `area`."""
    a = np.sqrt(4.0 * area / (np.sqrt(3.0) * n_tris))
    return a, a * np.sqrt(3.0) / 2.0


def edges_of(tri):
    """Undirected edges (lo, hi) of a triangle list, each once, sorted."""
    s = set()
    for t in tri:
        for q in range(3):
            a, b = int(t[q]), int(t[(q + 1) % 3])
            s.add((min(a, b), max(a, b)))
    return sorted(s)


def _vec(xy, i, j, Lx, Ly, periodic):
    """x_j - x_i (minimum image)."""
    return np.array([_mi(xy[j, 0] - xy[i, 0], Lx, periodic), _mi(xy[j, 1] - xy[i, 1], Ly, periodic)])


def _cross(u, w):
    return u[0] * w[1] - u[1] * w[0]


def _perp(u):
    """u rotated by +90 degrees."""
    return np.array([-u[1], u[0]])


def energy(xy, tri, periodic, Lx, Ly, a0, k_e=1.0, k_h=1.0):
    h0 = a0 * np.sqrt(3.0) / 2.0
    e = 0.0
    for lo, hi in edges_of(tri):
        ln = np.linalg.norm(_vec(xy, lo, hi, Lx, Ly, periodic))
        e += 0.5 * k_e * (ln - a0) ** 2
    for t in tri:
        for q in range(3):
            c, a, b = int(t[q]), int(t[(q + 1) % 3]), int(t[(q + 2) % 3])
            u = _vec(xy, a, b, Lx, Ly, periodic)          # the side opposite vertex c
            w = _vec(xy, a, c, Lx, Ly, periodic)
            h = _cross(u, w) / np.linalg.norm(u)           # > 0 for a counter-clockwise triangle
            e += 0.5 * k_h * (h - h0) ** 2
    return e


def forces(xy, tri, periodic, Lx, Ly, a0, k_e=1.0, k_h=1.0):
    """F = -grad E per node [n_v, 2] (triangles counter-clockwise)."""
    h0 = a0 * np.sqrt(3.0) / 2.0
    F = np.zeros_like(xy, dtype=np.float64)
    for lo, hi in edges_of(tri):
        d = _vec(xy, lo, hi, Lx, Ly, periodic)             # from lo to hi
        ln = np.linalg.norm(d)
        f = k_e * (ln - a0) * d / ln                       # pulls the ends together when stretched
        F[lo] += f
        F[hi] -= f
    for t in tri:
        for q in range(3):
            c, a, b = int(t[q]), int(t[(q + 1) % 3]), int(t[(q + 2) % 3])
            u = _vec(xy, a, b, Lx, Ly, periodic)
            w = _vec(xy, a, c, Lx, Ly, periodic)
            lu = np.linalg.norm(u)
            h = _cross(u, w) / lu
            # h = (u x w)/|u|, u = b - a, w = c - a:
            #   dh/dc = perp(u)/|u|,  dh/db = -perp(w)/|u| - h u/|u|^2,  dh/da = -(dh/db + dh/dc)
            dc = _perp(u) / lu
            db = -_perp(w) / lu - h * u / lu ** 2
            da = -(db + dc)
            s = -k_h * (h - h0)
            F[c] += s * dc
            F[b] += s * db
            F[a] += s * da
    return F


def euler(xy, tri, periodic, Lx, Ly, a0, steps, tau, anchored=None, k_e=1.0, k_h=1.0):
    """`steps` Euler steps of the overdamped (jello) motion; anchored nodes do not move."""
    x = np.array(xy, np.float64, copy=True)
    free = np.ones(len(x), bool) if anchored is None else ~np.asarray(anchored, bool)
    for _ in range(steps):
        F = forces(x, tri, periodic, Lx, Ly, a0, k_e, k_h)
        x[free] = x[free] + tau * F[free]
        if periodic:
            x[:, 0] = np.mod(x[:, 0], Lx)
            x[:, 1] = np.mod(x[:, 1], Ly)
    return x
