"""FP64 oracle of the three-dimensional scheme on tetrahedra (TEST INFRASTRUCTURE ONLY).

The Conclusion of the paper carries the method to three dimensions: tetrahedra in place of
triangles, E (and j) on edges, B on faces, the charge on nodes. Written here from that sentence
and the two-dimensional scheme of Section 1 (eqs. 3-4), in plain numpy, with its own mesh
builder. The dual is the Voronoi diagram of the nodes, as the triangles' circumcentres are in
two dimensions:

- E_e is the component of E along edge e, tangent from the lower node id to the higher;
- B_f is the component of B along the unit normal of face f = (a, b, c), a < b < c, taken by the
  right-hand rule of a -> b -> c; s(f, e) = +1 where that circuit runs along e's tangent;
- Faraday on the face: A_f dB_f/dt = -sum over f's edges of s(f, e) |e| E_e;
- Ampere on the edge's Voronoi polygon (the circumcentres of the tetrahedra around e, in the
  plane that bisects e): A*_e dE_e/dt = sum over the faces around e of s(f, e) d_f B_f, where
  d_f = (C_front - C_back) . n_f is the signed distance between the circumcentres of the two
  tetrahedra on either side of f (the dual edge crosses f at right angles);
- the box's walls are perfect conductors: E = 0 on the edges of boundary faces, whose B then
  never changes;
- leap-frog, E then B (as in two dimensions), dt below 2/omega_max (eq. 20).

A*_e is the area of the Voronoi polygon itself: the tetrahedra around e sorted by the angle of
their centroids about e, their circumcentres joined in that order, the shoelace sum taken with
the right-hand rule about e's tangent.

Canonical numbering: nodes as given; edges by (lower, higher) node id; faces by their sorted
node triples; tetrahedra as given.
"""
import numpy as np


def _unique_rows(keys):
    """Unique rows of an int64 array in lexicographic order and the inverse map."""
    u, inv = np.unique(keys, axis=0, return_inverse=True)
    return u, inv.reshape(-1)


class TetMesh:
    """A tetrahedral mesh of the box [0, Lx] x [0, Ly] x [0, Lz] with conducting walls."""

    def __init__(self, xyz, tets, L=None):
        self.xyz = np.asarray(xyz, np.float64)
        tets = np.asarray(tets, np.int64).copy()
        self.L = L
        x = self.xyz
        a, b, c, d = (x[tets[:, q]] for q in range(4))
        vol6 = np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)
        if np.any(vol6 == 0.0):
            raise ValueError("a tetrahedron has no volume")
        neg = vol6 < 0
        tets[neg] = tets[neg][:, [0, 2, 1, 3]]
        self.tets = tets
        self.vol = np.abs(vol6) / 6.0
        self.nv, self.nt = len(x), len(tets)

        # edges
        pairs = np.sort(tets[:, [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]].reshape(-1, 2), axis=1)
        self.edge, inv = _unique_rows(pairs)
        self.ne = len(self.edge)
        self.tet_edge = inv.reshape(-1, 6)
        # faces, each with the tetrahedra on either side
        tri = np.sort(tets[:, [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]].reshape(-1, 3), axis=1)
        self.face, finv = _unique_rows(tri)
        self.nf = len(self.face)
        self.tet_face = finv.reshape(-1, 4)
        owner = np.repeat(np.arange(self.nt), 4)
        opposite = tets[:, [0, 1, 2, 3]].reshape(-1)    # the vertex of the tetrahedron not on the face
        fa, fb, fc = (x[self.face[:, q]] for q in range(3))
        nrm = np.cross(fb - fa, fc - fa)
        self.farea = 0.5 * np.linalg.norm(nrm, axis=1)
        self.fnormal = nrm / (2.0 * self.farea[:, None])
        side = np.einsum("ij,ij->i", x[opposite] - fa[finv], self.fnormal[finv])
        self.front = np.full(self.nf, -1)
        self.back = np.full(self.nf, -1)
        # the tetrahedron whose fourth vertex lies on the +n side is in front
        self.front[finv[side > 0]] = owner[side > 0]
        self.back[finv[side < 0]] = owner[side < 0]
        self.inner_face = (self.front >= 0) & (self.back >= 0)
        # face -> edges with s(f, e): (a, b) +1, (b, c) +1, (a, c) -1
        key = {tuple(e): i for i, e in enumerate(self.edge.tolist())}
        F = self.face
        self.face_edge = np.array([[key[(p, q)], key[(q, r)], key[(p, r)]] for p, q, r in F.tolist()],
                                  dtype=np.int64).reshape(-1, 3)
        self.face_sign = np.tile(np.array([1.0, 1.0, -1.0]), (self.nf, 1))
        # conducting walls: the edges of boundary faces
        bnd_edge = np.zeros(self.ne, bool)
        bnd_edge[self.face_edge[~self.inner_face].reshape(-1)] = True
        self.inner_edge = ~bnd_edge
        bnd_node = np.zeros(self.nv, bool)
        bnd_node[self.face[~self.inner_face].reshape(-1)] = True
        self.inner_node = ~bnd_node

        # geometry: circumcentres by solving 2 (p - a) . C' = |p - a|^2 for p = b, c, d
        a = x[tets[:, 0]]
        A = np.stack([x[tets[:, 1]] - a, x[tets[:, 2]] - a, x[tets[:, 3]] - a], axis=1)
        rhs = 0.5 * np.sum(A ** 2, axis=2)
        self.C = a + np.linalg.solve(A, rhs[..., None])[..., 0]
        self.elen = np.linalg.norm(x[self.edge[:, 1]] - x[self.edge[:, 0]], axis=1)
        self.d = np.zeros(self.nf)
        i = self.inner_face
        self.d[i] = np.einsum("ij,ij->i", self.C[self.front[i]] - self.C[self.back[i]], self.fnormal[i])
        self.dual_area = self._voronoi_areas()

    def _voronoi_areas(self):
        """A*_e of every inner edge: the shoelace area of its Voronoi polygon."""
        x = self.xyz
        around = [[] for _ in range(self.ne)]
        for t in range(self.nt):
            for e in self.tet_edge[t]:
                around[e].append(t)
        out = np.zeros(self.ne)
        cen = x[self.tets].mean(axis=1)
        for e in np.nonzero(self.inner_edge)[0]:
            p, q = x[self.edge[e, 0]], x[self.edge[e, 1]]
            t = (q - p) / np.linalg.norm(q - p)
            ref = np.cross(t, [1.0, 0.0, 0.0])
            if np.linalg.norm(ref) < 0.5:
                ref = np.cross(t, [0.0, 1.0, 0.0])
            u = ref / np.linalg.norm(ref)
            v = np.cross(t, u)
            ts = np.array(around[e])
            w = cen[ts] - p
            ang = np.arctan2(w @ v, w @ u)
            poly = self.C[ts[np.argsort(ang)]]
            pu, pv = poly @ u, poly @ v
            out[e] = 0.5 * np.sum(pu * np.roll(pv, -1) - np.roll(pu, -1) * pv)
        return out

    # operators on full-length vectors (boundary entries held at zero)
    def curl_e(self, E):
        """-(1/A_f) sum s(f, e) |e| E_e: dB/dt of every face."""
        return -np.sum(self.face_sign * self.elen[self.face_edge] * E[self.face_edge], axis=1) / self.farea

    def curl_b(self, B):
        """(1/A*_e) sum over faces around e of s(f, e) d_f B_f: dE/dt of every inner edge."""
        acc = np.zeros(self.ne)
        np.add.at(acc, self.face_edge.reshape(-1), (self.face_sign * (self.d * B)[:, None]).reshape(-1))
        out = np.zeros(self.ne)
        i = self.inner_edge
        out[i] = acc[i] / self.dual_area[i]
        return out

    def step(self, E, B, dt, nsteps):
        """nsteps leap-frog steps: E^{n+1} = E^n + dt curl_b(B^{n+1/2}), then
        B^{n+3/2} = B^{n+1/2} + dt curl_e(E^{n+1}); returns copies."""
        E = np.array(E, np.float64, copy=True)
        B = np.array(B, np.float64, copy=True)
        for _ in range(nsteps):
            E = E + dt * self.curl_b(B)
            B = B + dt * self.curl_e(E)
        return E, B

    def energy(self, E, Bold, Bnew):
        """sum A*_e |e| E^2 + sum A_f d_f B_old B_new: the leap-frog invariant (the 3-D form of
        metric (7))."""
        i = self.inner_edge
        return float(np.sum(self.dual_area[i] * self.elen[i] * E[i] ** 2) +
                     np.sum(self.farea * self.d * Bold * Bnew))

    def operator(self):
        """K = -curl_b curl_e on E of the inner edges as a scipy sparse matrix, and the metric
        weights A*_e |e| in which it is symmetric (the energy's)."""
        import scipy.sparse as sp
        i = np.nonzero(self.inner_edge)[0]
        pos = -np.ones(self.ne, np.int64)
        pos[i] = np.arange(len(i))
        rows, cols, vals = [], [], []
        for q in range(3):
            e = self.face_edge[:, q]
            keep = pos[e] >= 0
            rows.append(np.nonzero(keep)[0])
            cols.append(pos[e[keep]])
            vals.append(self.face_sign[keep, q])
        Cm = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(self.nf, len(i)))
        W = sp.diags(self.d / self.farea)
        K = sp.diags(1.0 / self.dual_area[i]) @ (Cm.T @ W @ Cm) @ sp.diags(self.elen[i])
        return K.tocsr(), self.dual_area[i] * self.elen[i]

    def spectrum(self):
        """Every eigenvalue of K (dense, from the symmetric M^(1/2) K M^(-1/2))."""
        K, Me = self.operator()
        s = np.sqrt(Me)
        Ks = (K.toarray() * s[:, None]) / s[None, :]
        return np.linalg.eigvalsh(0.5 * (Ks + Ks.T))

    def modes_near(self, sigma, k):
        """The k eigenvalues of K nearest sigma (sparse shift-invert)."""
        import scipy.sparse as sp
        from scipy.sparse.linalg import eigsh
        K, Me = self.operator()
        s = np.sqrt(Me)
        Ks = sp.diags(s) @ K @ sp.diags(1.0 / s)
        Ks = 0.5 * (Ks + Ks.T)
        return np.sort(eigsh(Ks.tocsc(), k=k, sigma=sigma, which="LM", return_eigenvectors=False))

    def omega_max(self):
        """sqrt of K's largest eigenvalue."""
        import scipy.sparse as sp
        from scipy.sparse.linalg import eigsh
        K, Me = self.operator()
        s = np.sqrt(Me)
        Ks = sp.diags(s) @ K @ sp.diags(1.0 / s)
        Ks = 0.5 * (Ks + Ks.T)
        lam = eigsh(Ks.tocsc(), k=1, which="LA", return_eigenvectors=False, tol=1e-14)
        return float(np.sqrt(lam[0]))
