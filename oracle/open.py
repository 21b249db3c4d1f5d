"""FP64 oracle of the open boundary (TEST INFRASTRUCTURE ONLY).

The Conclusion of the paper ties a triangle mesh with rectangular outer boundaries to a
structured rectangular frame that carries PML layers, since the scheme works on mixed meshes
(triangles plus quads). Written here from that description and the scheme of Section 1, in
plain numpy, with its own frame builder:

- the frame: the triangle mesh fills the box [0, Lx] x [0, Ly]; each side is continued outwards
  by `layers` rows of rectangles `width` deep whose columns are bounded by that side's boundary
  nodes, and each corner by a block of layers x layers squares; the frame's outer boundary is a
  perfect conductor (E = 0);
- every cell keeps B at its circumcentre (a rectangle's is its centre, which lies on the
  perpendicular bisector of every side, as a triangle's circumcentre does), every edge E along
  its tangent (lower node id to higher): eq. 3 dE/dt = (B_left - B_right)/d with d the distance
  between the two centres across the edge, eq. 4 dB/dt = -(1/S) sum over the cell's edges of
  s |e| E, s = +1 where the edge runs counter-clockwise around the cell;
- the PML (split field, graded polynomially): sigma(rho) = sigma_max (rho / (layers width))^grading
  with rho the distance beyond the box in x (sigma_x) or in y (sigma_y); a frame cell's B is the
  sum of Bx, driven by its two vertical edges and damped by sigma_x, and By, driven by its two
  horizontal edges and damped by sigma_y; an edge parallel to x is damped by sigma_y at its
  midpoint, one parallel to y by sigma_x; triangles and the edges inside the box are undamped;
- leap-frog, E then B, with each damping term taken at the half step:
  X <- (1 - sigma dt/2)/(1 + sigma dt/2) X + dt/(1 + sigma dt/2) (drive).

Canonical numbering: mesh nodes, edges and triangles keep the triangle oracle's ids; frame nodes
follow, ordered by (y, x); frame edges follow the mesh edges, ordered by their (lower, higher)
node ids; frame cells follow the triangles, ordered by the (y, x) of their centres.
"""
import numpy as np


def _sigma(rho, sigma_max, depth, grading):
    return sigma_max * np.clip(rho / depth, 0.0, None) ** grading


class OpenMesh:
    """The triangle mesh of `om` (an OracleMesh of a closed box) with a PML frame."""

    def __init__(self, om, layers, width, sigma_max, grading=3.0):
        if om.periodic:
            raise ValueError("the frame needs a closed box")
        layers, width = int(layers), float(width)
        if layers < 0 or (layers > 0 and not width > 0.0):
            raise ValueError("layers >= 0 and width > 0")
        Lx, Ly = om.Lx, om.Ly
        self.Lx, self.Ly, self.layers, self.width = Lx, Ly, layers, width
        self.sigma_max, self.grading = float(sigma_max), float(grading)
        self.nv0, self.ne0, self.nt = om.nv, om.ne, om.nt
        xy0 = om.xy
        tol = 1e-9 * max(Lx, Ly)
        bnd = np.nonzero(om.node_bnd)[0]

        def side(mask, key):
            ids = bnd[mask(xy0[bnd])]
            return ids[np.argsort(xy0[ids, key], kind="stable")]

        bottom = side(lambda p: np.abs(p[:, 1]) <= tol, 0)
        top = side(lambda p: np.abs(p[:, 1] - Ly) <= tol, 0)
        left = side(lambda p: np.abs(p[:, 0]) <= tol, 1)
        right = side(lambda p: np.abs(p[:, 0] - Lx) <= tol, 1)
        # rectangles as corner points (x0, x1, y0, y1) and the mesh node ids on their inner side
        rects = []
        h = width
        for k in range(layers):
            for a in range(len(bottom) - 1):
                x0, x1 = xy0[bottom[a], 0], xy0[bottom[a + 1], 0]
                rects.append((x0, x1, -(k + 1) * h, -k * h if k else 0.0))
            for a in range(len(top) - 1):
                x0, x1 = xy0[top[a], 0], xy0[top[a + 1], 0]
                rects.append((x0, x1, Ly + k * h if k else Ly, Ly + (k + 1) * h))
            for b in range(len(left) - 1):
                y0, y1 = xy0[left[b], 1], xy0[left[b + 1], 1]
                rects.append((-(k + 1) * h, -k * h if k else 0.0, y0, y1))
            for b in range(len(right) - 1):
                y0, y1 = xy0[right[b], 1], xy0[right[b + 1], 1]
                rects.append((Lx + k * h if k else Lx, Lx + (k + 1) * h, y0, y1))
            for r in range(layers):
                xl = (-(k + 1) * h, -k * h if k else 0.0)
                xr = (Lx + k * h if k else Lx, Lx + (k + 1) * h)
                yb = (-(r + 1) * h, -r * h if r else 0.0)
                yt = (Ly + r * h if r else Ly, Ly + (r + 1) * h)
                for xs in (xl, xr):
                    for ys in (yb, yt):
                        rects.append((xs[0], xs[1], ys[0], ys[1]))
        # nodes: the mesh's, then the frame's new points ordered by (y, x)
        known = {(float(xy0[i, 0]), float(xy0[i, 1])): int(i) for i in bnd}
        new = set()
        for (x0, x1, y0, y1) in rects:
            for p in ((x0, y0), (x1, y0), (x1, y1), (x0, y1)):
                if p not in known:
                    new.add(p)
        new = sorted(new, key=lambda p: (p[1], p[0]))
        for q, p in enumerate(new):
            known[p] = self.nv0 + q
        self.nv = self.nv0 + len(new)
        self.xy = np.concatenate([xy0, np.array(new, np.float64).reshape(-1, 2)])
        # frame cells ordered by the (y, x) of their centres
        rects.sort(key=lambda r: (0.5 * (r[2] + r[3]), 0.5 * (r[0] + r[1])))
        self.nf = len(rects)
        corners = np.array([[known[(x0, y0)], known[(x1, y0)], known[(x1, y1)], known[(x0, y1)]]
                            for (x0, x1, y0, y1) in rects], np.int64).reshape(-1, 4)
        # edges: the mesh's, then the frame's by (lower, higher) node id
        mesh_edge = {(int(a), int(b)): i for i, (a, b) in enumerate(om.edge)}
        frame_pairs = set()
        for c in corners:
            for q in range(4):
                a, b = int(c[q]), int(c[(q + 1) % 4])
                key = (min(a, b), max(a, b))
                if key not in mesh_edge:
                    frame_pairs.add(key)
        frame_pairs = sorted(frame_pairs)
        self.ne = self.ne0 + len(frame_pairs)
        self.edge = np.concatenate([np.asarray(om.edge, np.int64),
                                    np.array(frame_pairs, np.int64).reshape(-1, 2)])
        eid = dict(mesh_edge)
        for q, key in enumerate(frame_pairs):
            eid[key] = self.ne0 + q
        # cells: triangles then rectangles; their edges, centres and areas
        self.ncell = self.nt + self.nf
        cell_edges = [list(map(int, om.A[j])) for j in range(self.nt)]
        for c in corners:
            cell_edges.append([eid[(min(int(c[q]), int(c[(q + 1) % 4])), max(int(c[q]), int(c[(q + 1) % 4])))]
                               for q in range(4)])
        self.cell_edges = cell_edges
        R = np.array(rects, np.float64).reshape(-1, 4)
        self.O = np.concatenate([om.O, np.stack([0.5 * (R[:, 0] + R[:, 1]), 0.5 * (R[:, 2] + R[:, 3])], 1)])
        self.S = np.concatenate([om.S, (R[:, 1] - R[:, 0]) * (R[:, 3] - R[:, 2])])
        centroid = np.concatenate([xy0[om.tri].mean(axis=1), self.O[self.nt:]])
        # edge geometry and its two cells (left and right of the tangent lower -> higher id)
        p0, p1 = self.xy[self.edge[:, 0]], self.xy[self.edge[:, 1]]
        t = p1 - p0
        self.elen = np.hypot(t[:, 0], t[:, 1])
        self.left = np.full(self.ne, -1, np.int64)
        self.right = np.full(self.ne, -1, np.int64)
        for j, es in enumerate(cell_edges):
            for i in es:
                rel = centroid[j] - p0[i]
                if t[i, 0] * rel[1] - t[i, 1] * rel[0] > 0.0:
                    self.left[i] = j
                else:
                    self.right[i] = j
        self.inner = (self.left >= 0) & (self.right >= 0)
        nrm = np.stack([-t[:, 1], t[:, 0]], 1) / self.elen[:, None]   # towards the left cell
        L_, R_ = np.maximum(self.left, 0), np.maximum(self.right, 0)
        self.d = np.where(self.inner, np.sum((self.O[L_] - self.O[R_]) * nrm, axis=1), 0.0)
        self.vertical = np.abs(t[:, 0]) <= 1e-12 * self.elen
        # damping
        depth = max(layers * width, 1e-300)
        rho = lambda v, L: np.maximum(0.0, np.maximum(-v, v - L))
        mid = 0.5 * (p0 + p1)
        sx = lambda p: _sigma(rho(p[:, 0], Lx), self.sigma_max, depth, self.grading)
        sy = lambda p: _sigma(rho(p[:, 1], Ly), self.sigma_max, depth, self.grading)
        self.sigma_e = np.where(self.vertical, sx(mid), sy(mid))
        self.split = np.arange(self.ncell) >= self.nt
        self.sigma_x = np.where(self.split, sx(self.O), 0.0)
        self.sigma_y = np.where(self.split, sy(self.O), 0.0)
        # incidence as flat arrays: cell, edge, sign (+1 where the cell is the edge's left cell)
        ci, ei = [], []
        for j, es in enumerate(cell_edges):
            ci += [j] * len(es)
            ei += es
        self.inc_cell, self.inc_edge = np.array(ci, np.int64), np.array(ei, np.int64)
        self.inc_sign = np.where(self.left[self.inc_edge] == self.inc_cell, 1.0, -1.0)

    # -- the scheme ---------------------------------------------------------------------
    def step(self, E, Bx, By, dt, nsteps):
        """nsteps leap-frog steps of E [ne], Bx [ncell], By [ncell] (By is zero on triangles);
        returns copies. The frame's outer edges stay at zero (perfect conductor)."""
        E = np.array(E, np.float64, copy=True)
        Bx = np.array(Bx, np.float64, copy=True)
        By = np.array(By, np.float64, copy=True)
        half = 0.5 * dt
        caE = (1 - self.sigma_e * half) / (1 + self.sigma_e * half)
        cbE = dt / (1 + self.sigma_e * half)
        cax = (1 - self.sigma_x * half) / (1 + self.sigma_x * half)
        cbx = dt / (1 + self.sigma_x * half)
        cay = (1 - self.sigma_y * half) / (1 + self.sigma_y * half)
        cby = dt / (1 + self.sigma_y * half)
        inner = self.inner
        L_, R_ = self.left[inner], self.right[inner]
        vert_inc = self.vertical[self.inc_edge]
        for _ in range(nsteps):
            B = Bx + By
            E[inner] = caE[inner] * E[inner] + cbE[inner] * (B[L_] - B[R_]) / self.d[inner]
            c = self.inc_sign * self.elen[self.inc_edge] * E[self.inc_edge]
            cv = np.zeros(self.ncell)
            ch = np.zeros(self.ncell)
            np.add.at(cv, self.inc_cell[vert_inc], c[vert_inc])
            np.add.at(ch, self.inc_cell[~vert_inc], c[~vert_inc])
            tri = ~self.split
            Bx[tri] = Bx[tri] - dt * (cv[tri] + ch[tri]) / self.S[tri]
            sp = self.split
            Bx[sp] = cax[sp] * Bx[sp] - cbx[sp] * cv[sp] / self.S[sp]
            By[sp] = cay[sp] * By[sp] - cby[sp] * ch[sp] / self.S[sp]
        return E, Bx, By

    def energy(self, E, Bold, Bnew):
        """Leap-frog energy sum |e| d E^2 + sum S B_old B_new (metric (7)); conserved without
        damping."""
        i = self.inner
        return float(np.sum(self.elen[i] * self.d[i] * E[i] ** 2) + np.sum(self.S * Bold * Bnew))

    def omega_max(self, iters=20000, rtol=1e-12, seed=0):
        """sqrt of the largest eigenvalue of K = -L_E L_B (undamped), by power iteration on the
        symmetric S^(1/2) K S^(-1/2)."""
        import scipy.sparse as sp
        i = np.nonzero(self.inner)[0]
        rows = np.concatenate([i, i])
        cols = np.concatenate([self.left[i], self.right[i]])
        vals = np.concatenate([1.0 / self.d[i], -1.0 / self.d[i]])
        LB = sp.csr_matrix((vals, (rows, cols)), shape=(self.ne, self.ncell))
        LE = sp.csr_matrix((-self.inc_sign * self.elen[self.inc_edge] / self.S[self.inc_cell],
                            (self.inc_cell, self.inc_edge)), shape=(self.ncell, self.ne))
        K = -(LE @ LB)
        rs = np.sqrt(self.S)
        A = sp.diags(rs) @ K @ sp.diags(1.0 / rs)
        x = np.random.default_rng(seed).uniform(-1.0, 1.0, self.ncell)
        lam = 0.0
        for _ in range(iters):
            y = A @ x
            new = float(np.dot(x, y) / np.dot(x, x))
            x = y / np.linalg.norm(y)
            if abs(new - lam) <= rtol * abs(new):
                lam = new
                break
            lam = new
        return float(np.sqrt(lam))
