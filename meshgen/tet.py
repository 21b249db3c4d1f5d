"""Seeded tetrahedral meshes of a box for the three-dimensional form of the scheme.

The Conclusion of the paper carries the method to three dimensions with tetrahedra: E (and j)
on edges, B on faces, n on nodes. The mesh here is the Delaunay tetrahedralisation of a
jittered body-centred cubic lattice (cube corners plus cube centres), whose Delaunay cells are
congruent, well-shaped tetrahedra with no five cospherical points; scipy's Qhull builds it.
Only the triangulation is produced here: no edges, faces, circumcentres or coefficients.
"""
import numpy as np


def _bcc_points(nx, ny, nz, h, jitter, seed):
    """Jittered BCC points numbered by (z, y, x) of their lattice positions, and the maps from
    lattice indices to point ids (corner[i, j, k], centre[i, j, k])."""
    rng = np.random.default_rng(seed)
    gi, gj, gk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    corners = np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1).astype(np.float64)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    centres = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1).astype(np.float64) + 0.5
    lat = np.concatenate([corners, centres])
    order = np.lexsort((lat[:, 0], lat[:, 1], lat[:, 2]))
    rank = np.empty(len(lat), np.int64)
    rank[order] = np.arange(len(lat))
    nc = len(corners)
    corner_id = rank[:nc].reshape(nx + 1, ny + 1, nz + 1)
    centre_id = rank[nc:].reshape(nx, ny, nz)
    lat = lat[order]
    jit = rng.uniform(-jitter, jitter, size=lat.shape)
    on_side = (lat <= 0.0) | (lat >= np.array([nx, ny, nz], np.float64))
    jit[on_side] = 0.0      # on a side it moves within the side, on a box edge along it, a corner stays
    return (lat + jit) * h, corner_id, centre_id


def _finish(xyz, tets, L, h):
    """Orient every tetrahedron positively, check that they fill the box, sort by centroid."""
    a, b, c, d = (xyz[tets[:, q]] for q in range(4))
    vol6 = np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)
    keep = np.abs(vol6) > 1e-9 * h ** 3
    tets, vol6 = tets[keep], vol6[keep]
    neg = vol6 < 0
    tets[neg] = tets[neg][:, [0, 2, 1, 3]]
    total, box = np.sum(np.abs(vol6)) / 6.0, L[0] * L[1] * L[2]
    if abs(total - box) > 1e-9 * box:
        raise RuntimeError(f"the tetrahedra fill {total} of the box's {box}")
    cen = xyz[tets].mean(axis=1)
    tets = tets[np.lexsort((cen[:, 0], cen[:, 1], cen[:, 2]))]
    return tets.astype(np.int32)


def bcc_box(nx, ny, nz, h, jitter, seed, method="direct"):
    """Delaunay tetrahedralisation of a jittered BCC lattice filling [0, nx h] x [0, ny h] x [0, nz h].

    Points: the cube corners (i, j, k) h for 0 <= i <= nx, ... and the cube centres
    (i + 1/2, j + 1/2, k + 1/2) h. Interior points move by U(-jitter h, +jitter h) per axis;
    points on a side of the box move only within that side (corners and points on the box's
    edges stay), so the box is filled exactly. Points are numbered by (z, y, x) of their lattice
    positions, tetrahedra by the (z, y, x) of their centroids, each with positive volume
    (det[b - a, c - a, d - a] > 0).

    method "direct" writes the BCC Delaunay cells down: the octahedron between two neighbouring
    cube centres and their shared square splits into four tetrahedra about the centre-to-centre
    axis (the octahedron's shortest diagonal, h against sqrt(2) h, so small jitter keeps it
    Delaunay: none of 370k tetrahedra over 8 seeds failed the sphere test at 0.08 h, three did at
    0.09 h), and the pyramid between a cube centre and a square on the box's side into two,
    along the square's diagonal that passes the in-plane circle test (on that side the sphere
    test reduces to it). It takes jitter <= 0.08. "qhull" asks scipy's Qhull instead (slow above ~10^5 points; the tests
    check the two agree).
    Returns (xyz float64[n_v, 3], tets int32[n_t, 4], (Lx, Ly, Lz)).
    """
    xyz, corner, centre = _bcc_points(nx, ny, nz, h, jitter, seed)
    L = (float(nx * h), float(ny * h), float(nz * h))
    if method == "qhull":
        from scipy.spatial import Delaunay
        tets = Delaunay(xyz, qhull_options="Qbb Qc Qz Q12").simplices.astype(np.int64)
        return xyz, _finish(xyz, tets, L, h), L
    if method != "direct":
        raise ValueError("method must be 'direct' or 'qhull'")
    if jitter > 0.08:
        raise ValueError("the direct construction is Delaunay for jitter up to 0.08 h")
    out = []
    dims = (nx, ny, nz)
    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3
        n_a, n_u, n_v = dims[ax], dims[u], dims[v]
        # squares normal to ax at plane index p, spanning cells (iu, iv) of the other two axes
        P, IU, IV = np.meshgrid(np.arange(n_a + 1), np.arange(n_u), np.arange(n_v), indexing="ij")
        P, IU, IV = P.ravel(), IU.ravel(), IV.ravel()

        def corner_at(pp, a_u, a_v):
            idx = [None, None, None]
            idx[ax], idx[u], idx[v] = pp, a_u, a_v
            return corner[idx[0], idx[1], idx[2]]

        def centre_at(pp, a_u, a_v):
            idx = [None, None, None]
            idx[ax], idx[u], idx[v] = pp, a_u, a_v
            return centre[idx[0], idx[1], idx[2]]

        sq = np.stack([corner_at(P, IU, IV), corner_at(P, IU + 1, IV), corner_at(P, IU + 1, IV + 1),
                       corner_at(P, IU, IV + 1)], axis=1)          # cyclic around the square
        inner = (P > 0) & (P < n_a)
        pi = P[inner]
        c1 = centre_at(pi - 1, IU[inner], IV[inner])
        c2 = centre_at(pi, IU[inner], IV[inner])
        s_in = sq[inner]
        for q in range(4):
            out.append(np.stack([c1, c2, s_in[:, q], s_in[:, (q + 1) % 4]], axis=1))
        side = ~inner
        ps = P[side]
        c = centre_at(np.where(ps == 0, 0, ps - 1), IU[side], IV[side])
        s_sd = sq[side]
        # in-plane circle test: is the square's 4th corner inside the circle of corners 1, 2, 3?
        q2 = xyz[s_sd][:, :, [u, v]]
        rel = q2[:, :3] - q2[:, 3:4]
        m = np.concatenate([rel, np.sum(rel ** 2, axis=2, keepdims=True)], axis=2)
        e1, e2 = q2[:, 1] - q2[:, 0], q2[:, 2] - q2[:, 0]
        orient = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
        flip = np.linalg.det(m) * np.sign(orient) > 1e-12 * h ** 4      # inside: use diagonal 2-4
        d13 = np.stack([np.stack([c, s_sd[:, 0], s_sd[:, 1], s_sd[:, 2]], axis=1),
                        np.stack([c, s_sd[:, 0], s_sd[:, 2], s_sd[:, 3]], axis=1)])
        d24 = np.stack([np.stack([c, s_sd[:, 1], s_sd[:, 2], s_sd[:, 3]], axis=1),
                        np.stack([c, s_sd[:, 1], s_sd[:, 3], s_sd[:, 0]], axis=1)])
        out.append(np.where(flip[None, :, None], d24, d13).reshape(-1, 4))
    tets = np.concatenate(out).astype(np.int64)
    return xyz, _finish(xyz, tets, L, h), L


def insphere_violations(xyz, tets):
    """Number of interior faces whose opposite vertex of one tetrahedron lies strictly inside the
    circumsphere of the other (the local Delaunay test): the 4 x 4 determinant of the four
    vertices lifted to the paraboloid about the point, negative for a point inside the sphere of
    a positively oriented tetrahedron."""
    nt, nv = len(tets), len(xyz)
    tets = np.asarray(tets, np.int64)
    faces = np.sort(np.stack([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]],
                              tets[:, [0, 1, 2]]], axis=1).reshape(-1, 3), axis=1)
    owner = np.repeat(np.arange(nt), 4)
    opp = tets.reshape(-1)
    key = (faces[:, 0] * nv + faces[:, 1]) * nv + faces[:, 2]
    srt = np.argsort(key, kind="stable")
    ks = key[srt]
    pair = np.nonzero(ks[1:] == ks[:-1])[0]
    t, p = owner[srt[pair]], opp[srt[pair + 1]]
    rel = xyz[tets[t]] - xyz[p][:, None, :]
    m = np.concatenate([rel, np.sum(rel ** 2, axis=2, keepdims=True)], axis=2)
    a, b, c, d = (xyz[tets[t, k]] for k in range(4))
    orient = np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)
    scale = np.max(np.abs(rel).reshape(len(t), -1), axis=1) ** 5
    return int(np.sum(np.linalg.det(m) * np.sign(orient) < -1e-12 * scale))
