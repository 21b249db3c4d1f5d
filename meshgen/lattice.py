"""Jittered-lattice Delaunay triangulations (Section 3: seeding, Delaunay, flips).

A lattice of points is jittered, each lattice square is split along the diagonal that the
empty-circumcircle test selects, and Lawson flips then repair any edge whose neighbouring
triangles still violate the test (the flip operation of Fig. 5a). The result is a Delaunay
triangulation of the seeded cloud, either of a closed box (boundary points on the box sides)
or of a periodic square (a torus, node indices wrapping).
"""
import numpy as np


def _unwrap(delta, L, periodic):
    """Minimum-image difference vectors on a periodic square of side L."""
    if not periodic:
        return delta
    return delta - L * np.round(delta / L)


def incircle(a, b, c, d):
    """Classical in-circle determinant for arrays of 2-D points (shape [..., 2]).

    Positive when d lies strictly inside the circumcircle of the counter-clockwise
    triangle (a, b, c), zero when the four points are cocircular.
    """
    adx, ady = a[..., 0] - d[..., 0], a[..., 1] - d[..., 1]
    bdx, bdy = b[..., 0] - d[..., 0], b[..., 1] - d[..., 1]
    cdx, cdy = c[..., 0] - d[..., 0], c[..., 1] - d[..., 1]
    ad2 = adx * adx + ady * ady
    bd2 = bdx * bdx + bdy * bdy
    cd2 = cdx * cdx + cdy * cdy
    return (ad2 * (bdx * cdy - cdx * bdy)
            + bd2 * (cdx * ady - adx * cdy)
            + cd2 * (adx * bdy - bdx * ady))


def lattice_mesh(n, jitter, seed, periodic, L=1.0):
    """Delaunay triangulation of a jittered n x n point lattice.

    periodic=False: closed box [0, L]^2, spacing h = L/(n-1); interior points move by
    U(-jitter*h, +jitter*h) per axis, points on the box sides stay fixed.
    periodic=True: torus [0, L)^2, spacing h = L/n; every point moves by U(+-jitter*h) per
    axis and is wrapped into [0, L).

    Node (i, j) (i along the first axis x, j along the second axis z) has index j*n + i.
    Returns (xy float64[n_v, 2], tri int32[n_t, 3]); triangles are counter-clockwise.
    """
    n = int(n)
    if periodic and n < 4:
        raise ValueError("periodic lattice needs n >= 4")
    if not periodic and n < 2:
        raise ValueError("box lattice needs n >= 2")
    rng = np.random.default_rng(seed)
    h = L / n if periodic else L / (n - 1)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([i.ravel(), j.ravel()], axis=1).astype(np.float64)
    jit = rng.uniform(-jitter, jitter, size=base.shape)
    if not periodic:
        on_side = ((i == 0) | (i == n - 1) | (j == 0) | (j == n - 1)).ravel()
        jit[on_side] = 0.0
    xy = (base + jit) * h
    if periodic:
        xy = np.mod(xy, L)
    else:
        # keep the box sides exact
        xy[i.ravel() == n - 1, 0] = L
        xy[j.ravel() == n - 1, 1] = L

    m = n if periodic else n - 1
    qj, qi = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()

    def idx(ii, jj):
        if periodic:
            return (jj % n) * n + (ii % n)
        return jj * n + ii

    a, b, c, d = idx(qi, qj), idx(qi + 1, qj), idx(qi + 1, qj + 1), idx(qi, qj + 1)
    pa = xy[a]
    pb = pa + _unwrap(xy[b] - pa, L, periodic)
    pc = pa + _unwrap(xy[c] - pa, L, periodic)
    pd = pa + _unwrap(xy[d] - pa, L, periodic)
    # diagonal a-c unless d is strictly inside circle(a, b, c); ties keep a-c
    use_bd = incircle(pa, pb, pc, pd) > 0.0
    t1 = np.where(use_bd[:, None], np.stack([a, b, d], 1), np.stack([a, b, c], 1))
    t2 = np.where(use_bd[:, None], np.stack([b, c, d], 1), np.stack([a, c, d], 1))
    tri = np.concatenate([t1, t2], axis=0).astype(np.int32)
    tri, _ = lawson_flip(xy, tri, periodic, L)
    return xy, tri


def box_mesh(nx, ny, jitter, seed, h=1.0):
    """Delaunay triangulation of a jittered lattice filling the closed box [0, nx h] x [0, ny h].

    (nx + 1) x (ny + 1) points with spacing h; points on the box sides stay fixed, interior
    points move by U(-jitter*h, +jitter*h) per axis. Node (i, j) has index j*(nx+1) + i.
    Returns (xy float64[n_v, 2], tri int32[2 nx ny, 3], Lx, Ly); triangles counter-clockwise.
    """
    nx, ny = int(nx), int(ny)
    if nx < 1 or ny < 1:
        raise ValueError("box needs nx, ny >= 1")
    rng = np.random.default_rng(seed)
    j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    i, j = i.ravel(), j.ravel()
    jit = rng.uniform(-jitter, jitter, size=(len(i), 2))
    jit[(i == 0) | (i == nx) | (j == 0) | (j == ny)] = 0.0
    xy = (np.stack([i, j], axis=1).astype(np.float64) + jit) * h
    xy[i == nx, 0] = nx * h
    xy[j == ny, 1] = ny * h
    qj, qi = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    idx = lambda ii, jj: jj * (nx + 1) + ii
    a, b, c, d = idx(qi, qj), idx(qi + 1, qj), idx(qi + 1, qj + 1), idx(qi, qj + 1)
    use_bd = incircle(xy[a], xy[b], xy[c], xy[d]) > 0.0
    t1 = np.where(use_bd[:, None], np.stack([a, b, d], 1), np.stack([a, b, c], 1))
    t2 = np.where(use_bd[:, None], np.stack([b, c, d], 1), np.stack([a, c, d], 1))
    tri = np.concatenate([t1, t2], axis=0).astype(np.int32)
    tri, _ = lawson_flip(xy, tri, False, max(nx, ny) * h)
    return xy, tri, nx * h, ny * h


def box_tri_mesh(Lx, Ly, h, jitter, seed):
    """Delaunay triangulation of a jittered triangular lattice filling the box [0, Lx] x [0, Ly].

    Rows are hy = Ly / round(Ly / (h sqrt(3)/2)) apart; even rows hold nx + 1 points at
    x = k hx (hx = Lx / round(Lx / h)), odd rows are shifted by hx/2 and close with a point on
    each side, so nearly every triangle is close to equilateral. Points on the box sides stay
    fixed; the others move by U(-jitter*hx, +jitter*hx) per axis. Neighbouring rows are joined
    by merging them in x order, and Lawson flips make the result Delaunay.
    Returns (xy float64[n_v, 2], tri int32[n_t, 3], Lx, Ly); triangles counter-clockwise.
    """
    nx = max(1, int(round(Lx / h)))
    ny = max(1, int(round(Ly / (h * np.sqrt(3.0) / 2.0))))
    hx, hy = Lx / nx, Ly / ny
    rng = np.random.default_rng(seed)
    rows, pts = [], []
    for r in range(ny + 1):
        xs = np.arange(nx + 1) * hx if r % 2 == 0 else \
            np.concatenate([[0.0], (np.arange(nx) + 0.5) * hx, [Lx]])
        ids = np.arange(len(xs)) + sum(len(p) for p in pts)
        p = np.stack([xs, np.full(len(xs), r * hy)], axis=1)
        pts.append(p)
        rows.append(ids)
    xy = np.concatenate(pts)
    jit = rng.uniform(-jitter, jitter, size=xy.shape) * hx
    side = (xy[:, 0] <= 0.0) | (xy[:, 0] >= Lx) | (xy[:, 1] <= 0.0) | (xy[:, 1] >= Ly)
    jit[side] = 0.0
    xy = xy + jit
    tri = []
    for r in range(ny):
        lo, hi = rows[r], rows[r + 1]
        i = k = 0
        while i < len(lo) - 1 or k < len(hi) - 1:
            # advance along the row whose next point lies further left
            step_lo = k == len(hi) - 1 or (i < len(lo) - 1 and xy[lo[i + 1], 0] <= xy[hi[k + 1], 0])
            if step_lo:
                tri.append((lo[i], lo[i + 1], hi[k]))
                i += 1
            else:
                tri.append((lo[i], hi[k + 1], hi[k]))
                k += 1
    tri = np.array(tri, dtype=np.int32)
    tri, _ = lawson_flip(xy, tri, False, max(Lx, Ly))
    return xy, tri, float(Lx), float(Ly)


def _interior_pairs(tri, nv):
    """Half-edge index pairs (t*3+q) that share an undirected edge."""
    u = tri.reshape(-1).astype(np.int64)
    v = tri[:, [1, 2, 0]].reshape(-1).astype(np.int64)
    key = np.minimum(u, v) * nv + np.maximum(u, v)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    return order[:-1][same], order[1:][same]


def _violations(xy, tri, periodic, L):
    h1, h2 = _interior_pairs(tri, len(xy))
    t1, q1 = h1 // 3, h1 % 3
    t2, q2 = h2 // 3, h2 % 3
    o2 = tri[t2, (q2 + 2) % 3]
    p0 = xy[tri[t1, 0]]
    pa = p0
    pb = p0 + _unwrap(xy[tri[t1, 1]] - p0, L, periodic)
    pc = p0 + _unwrap(xy[tri[t1, 2]] - p0, L, periodic)
    pd = p0 + _unwrap(xy[o2] - p0, L, periodic)
    bad = incircle(pa, pb, pc, pd) > 0.0
    return t1[bad], q1[bad], t2[bad], q2[bad]


def count_non_delaunay(xy, tri, periodic, L=1.0):
    """Number of interior edges whose neighbour apex lies inside the circumcircle."""
    return int(len(_violations(xy, np.asarray(tri), periodic, L)[0]))


def lawson_flip(xy, tri, periodic, L=1.0, max_rounds=200):
    """Flip edges that fail the empty-circumcircle test until none is left (Fig. 5a).

    Each round flips a set of violating edges that share no triangle, then re-tests.
    Triangles must be counter-clockwise. Returns (tri, number of flips).
    """
    tri = np.array(tri, dtype=np.int32, copy=True)
    flips = 0
    for _ in range(max_rounds):
        t1, q1, t2, q2 = _violations(xy, tri, periodic, L)
        if len(t1) == 0:
            return tri, flips
        used = set()
        for a, qa, b, qb in zip(t1.tolist(), q1.tolist(), t2.tolist(), q2.tolist()):
            if a in used or b in used:
                continue
            used.add(a)
            used.add(b)
            u, v, o1 = tri[a, qa], tri[a, (qa + 1) % 3], tri[a, (qa + 2) % 3]
            o2 = tri[b, (qb + 2) % 3]
            tri[a] = (o1, u, o2)
            tri[b] = (o2, v, o1)
            flips += 1
    raise RuntimeError("Lawson flips did not converge")


def triangle_centroids(xy, tri, periodic, L=1.0):
    """Vertex-average of each input triangle (minimum image on a torus), wrapped into [0, L)."""
    tri = np.asarray(tri)
    p0 = xy[tri[:, 0]]
    d1 = _unwrap(xy[tri[:, 1]] - p0, L, periodic)
    d2 = _unwrap(xy[tri[:, 2]] - p0, L, periodic)
    c = p0 + (d1 + d2) / 3.0
    return np.mod(c, L) if periodic else c


def scramble(tri, seed):
    """Randomly rotate/reverse each triangle's vertex order and shuffle the rows.

    The solver must not depend on the winding or the row order it is handed.
    Returns (scrambled tri, row permutation such that scrambled[k] ~ tri[perm[k]]).
    """
    rng = np.random.default_rng(seed)
    tri = np.asarray(tri, dtype=np.int32)
    nt = len(tri)
    roll = rng.integers(0, 3, size=nt)
    rev = rng.integers(0, 2, size=nt).astype(bool)
    cols = (np.arange(3)[None, :] + roll[:, None]) % 3
    out = np.take_along_axis(tri, cols, axis=1)
    out[rev] = out[rev][:, ::-1]
    perm = rng.permutation(nt)
    return np.ascontiguousarray(out[perm]), perm


def equilateral_torus(nx, ny, a=1.0):
    """Periodic mesh of equilateral triangles of side a (ny even).

    Domain [0, nx*a) x [0, ny*a*sqrt(3)/2); row r is shifted by a/2 * (r mod 2).
    Returns (xy, tri, Lx, Ly).
    """
    if ny % 2 or nx < 3 or ny < 4:
        raise ValueError("need nx >= 3 and even ny >= 4")
    hy = a * np.sqrt(3.0) / 2.0
    r, c = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    xy = np.stack([(c + 0.5 * (r % 2)) * a, r * hy], axis=-1).reshape(-1, 2)
    idx = lambda rr, cc: (rr % ny) * nx + (cc % nx)
    r, c = r.ravel(), c.ravel()
    even = (r % 2) == 0
    # even rows: up (c, c+1, row above c), down (c+1, above c+1, above c)
    # odd rows:  up (c, c+1, above c+1),    down (c, above c+1, above c)
    up = np.where(even[:, None],
                  np.stack([idx(r, c), idx(r, c + 1), idx(r + 1, c)], 1),
                  np.stack([idx(r, c), idx(r, c + 1), idx(r + 1, c + 1)], 1))
    dn = np.where(even[:, None],
                  np.stack([idx(r, c + 1), idx(r + 1, c + 1), idx(r + 1, c)], 1),
                  np.stack([idx(r, c), idx(r + 1, c + 1), idx(r + 1, c)], 1))
    tri = np.concatenate([up, dn]).astype(np.int32)
    return xy, tri, nx * a, ny * hy
