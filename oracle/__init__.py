"""Plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

The C core in ``oracle.c`` is the reference that the GPU library is checked against. Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg import this package; the
library never does. ``build()`` compiles the core with gcc (-O2 -ffp-contract=off); the
loader builds it on first use when it is missing.

Python-side helpers here are the evaluation formulas that sit on top of the stepper:
plasma-frequency averaging onto edges, source lookup by node pairs, the plane-wave phase
overlap used for the dispersion metric, and the resonator modes (eigenpairs of K = -L_E L_B
from the core's own operators and a library symmetric eigensolver).

`OracleMesh.edge_wp2` (the half-dual weighted average of per-triangle plasma frequencies onto
an edge of the particle boundary) and the source waveform of the C core are readings (the paper
gives no rule for either); both are pinned by hand-derived values (a homogeneous medium, a kite
with plasma on one side, the waveform at hand-evaluated times).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

OK, EINVAL, ENOTDELAUNAY, EDEGENERATE, ENONMANIFOLD, EPERIODIC, ENOTCONVERGED = \
    0, -1, -2, -3, -4, -5, -9
ORDER = {"none": 0, "random": 1, "morton": 2, "rcm": 3}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build():
    """Compile the C oracle into oracle/liborc.so."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("gamma", ctypes.c_void_p), ("wp2", ctypes.c_void_p),
                ("nu", ctypes.c_double), ("n_src", ctypes.c_int64),
                ("src_edge", ctypes.c_void_p), ("src_w", ctypes.c_void_p),
                ("src_omega", ctypes.c_double), ("src_cycles", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i64, f64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.orc_mesh_build.restype = vp
    lib.orc_mesh_build.argtypes = [vp, i64, vp, i64, ci, f64, f64, f64, ctypes.POINTER(ci)]
    lib.orc_mesh_free.argtypes = [vp]
    lib.orc_mesh_sizes.argtypes = [vp, vp]
    lib.orc_mesh_topology.argtypes = [vp] * 7
    lib.orc_mesh_geometry.argtypes = [vp] * 9
    lib.orc_node_boundary.argtypes = [vp, vp]
    lib.orc_apply_LB.argtypes = [vp, vp, vp, vp]
    lib.orc_apply_LE.argtypes = [vp, vp, vp, vp]
    lib.orc_step.restype = ci
    lib.orc_step.argtypes = [vp, ctypes.POINTER(_Params), i64, i64, vp, vp, vp, vp, vp]
    lib.orc_energy.restype = f64
    lib.orc_energy.argtypes = [vp, vp, vp, vp]
    lib.orc_div.argtypes = [vp, vp, vp]
    lib.orc_power.restype = ci
    lib.orc_power.argtypes = [vp, vp, i64, f64, ctypes.c_uint64, ctypes.POINTER(f64),
                              ctypes.POINTER(i64)]
    lib.orc_order.restype = ci
    lib.orc_order.argtypes = [vp, ci, ctypes.c_uint64, vp, vp]
    lib.orc_splitmix64.restype = ctypes.c_uint64
    lib.orc_splitmix64.argtypes = [ctypes.c_uint64]
    lib.orc_set_threads.argtypes = [ci]
    lib.orc_get_threads.restype = ci
    lib.orc_morton.restype = ctypes.c_uint64
    lib.orc_morton.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def set_threads(n):
    """Threads of the C core's per-cell loops (its results do not depend on the count)."""
    _load().orc_set_threads(int(n))


def get_threads():
    return int(_load().orc_get_threads())


def splitmix64(x):
    return int(_load().orc_splitmix64(ctypes.c_uint64(int(x) & (2 ** 64 - 1))))


def morton(qx, qz):
    return int(_load().orc_morton(int(qx), int(qz)))


class OracleMesh:
    """Topology, geometry and FP64 operators of one mesh (canonical numbering)."""

    def __init__(self, xy, tri, periodic, L=1.0, Ly=None, dual_tol=0.0):
        lib = _load()
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.periodic = bool(periodic)
        self.Lx, self.Ly = float(L), float(L if Ly is None else Ly)
        st = ctypes.c_int(0)
        h = lib.orc_mesh_build(_p(self.xy), len(self.xy), _p(tri), len(tri), int(periodic),
                               self.Lx, self.Ly, float(dual_tol), ctypes.byref(st))
        if not h:
            raise OracleError(st.value, "mesh build")
        self._h = ctypes.c_void_p(h)
        sz = np.zeros(4, np.int64)
        lib.orc_mesh_sizes(self._h, _p(sz))
        self.nv, self.ne, self.nt, self.nb = (int(v) for v in sz)
        ne, nt = self.ne, self.nt
        self.tri = np.zeros((nt, 3), np.int32)
        self.edge = np.zeros((ne, 2), np.int32)
        self.R = np.zeros(ne, np.int32)
        self.L = np.zeros(ne, np.int32)
        self.A = np.zeros((nt, 3), np.int32)
        self.s = np.zeros((nt, 3), np.int8)
        lib.orc_mesh_topology(self._h, _p(self.tri), _p(self.edge), _p(self.R), _p(self.L),
                              _p(self.A), _p(self.s))
        self.elen = np.zeros(ne)
        self.hR = np.zeros(ne)
        self.hL = np.zeros(ne)
        self.d = np.zeros(ne)
        self.S = np.zeros(nt)
        self.O = np.zeros((nt, 2))
        self.C = np.zeros((ne, 2))
        self.evec = np.zeros((ne, 2))
        lib.orc_mesh_geometry(self._h, _p(self.elen), _p(self.hR), _p(self.hL), _p(self.d),
                              _p(self.S), _p(self.O), _p(self.C), _p(self.evec))
        self.node_bnd = np.zeros(self.nv, np.uint8)
        lib.orc_node_boundary(self._h, _p(self.node_bnd))
        self.interior = (self.R >= 0) & (self.L >= 0)
        self.tangent = self.evec / self.elen[:, None]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_mesh_free(h)
            self._h = None

    # -- operators ---------------------------------------------------------------------
    def apply_LB(self, B, gamma=None):
        out = np.zeros(self.ne)
        B = np.ascontiguousarray(B, np.float64)
        g = None if gamma is None else np.ascontiguousarray(gamma, np.float64)
        _load().orc_apply_LB(self._h, _p(g), _p(B), _p(out))
        return out

    def apply_LE(self, E, gamma=None):
        out = np.zeros(self.nt)
        E = np.ascontiguousarray(E, np.float64)
        g = None if gamma is None else np.ascontiguousarray(gamma, np.float64)
        _load().orc_apply_LE(self._h, _p(g), _p(E), _p(out))
        return out

    def sparse_ops(self, gamma=None):
        """L_B (n_e x n_t) and L_E (n_t x n_e) as sparse matrices, read off this core's own
        operators: a row of L_B touches the two triangles of its edge, a row of L_E the three
        edges of its triangle, so applying each operator to the indicator of one colour class
        of a greedy colouring (no two columns of one row share a colour) yields every
        coefficient of that class at once."""
        import scipy.sparse as sp

        def colour(rows):
            # rows: [n_rows, k] column ids (-1 = none); colour columns so that each row's
            # columns differ
            ncol = int(rows.max()) + 1
            col = np.full(ncol, -1, np.int64)
            users = [[] for _ in range(ncol)]
            for r, cs in enumerate(rows.tolist()):
                for c in cs:
                    if c >= 0:
                        users[c].append(r)
            for c in range(ncol):
                taken = {int(col[o]) for r in users[c] for o in rows[r] if o >= 0 and o != c}
                k = 0
                while k in taken:
                    k += 1
                col[c] = k
            return col

        tri_of_edge = np.stack([self.R, self.L], 1)
        ct = colour(tri_of_edge)
        r_idx, c_idx, val = [], [], []
        for k in range(int(ct.max()) + 1):
            y = self.apply_LB((ct == k).astype(np.float64), gamma)
            for side in (self.R, self.L):
                hit = (side >= 0) & (ct[np.maximum(side, 0)] == k) & (y != 0.0)
                r_idx.append(np.nonzero(hit)[0])
                c_idx.append(side[hit])
                val.append(y[hit])
        LB = sp.csr_matrix((np.concatenate(val), (np.concatenate(r_idx), np.concatenate(c_idx))),
                           shape=(self.ne, self.nt))
        ce = colour(self.A)
        r_idx, c_idx, val = [], [], []
        rows = np.arange(self.nt)
        for k in range(int(ce.max()) + 1):
            y = self.apply_LE((ce == k).astype(np.float64), gamma)
            for q in range(3):
                e = self.A[:, q]
                hit = (ce[e] == k) & (y != 0.0)
                r_idx.append(rows[hit])
                c_idx.append(e[hit])
                val.append(y[hit])
        LE = sp.csr_matrix((np.concatenate(val), (np.concatenate(r_idx), np.concatenate(c_idx))),
                           shape=(self.nt, self.ne))
        return LB, LE

    def modes(self, count, gamma=None, which="lowest", sigma=0.0):
        """Lowest (or highest, or with which="nearest" nearest to sigma) `count` eigenpairs of
        K = -L_E L_B, the operator that eqs. 3-4 give for B once E is eliminated (Section 2,
        eigenvectors and the "complex time" method).

        K is self-adjoint and non-negative in the B part of metric (7) (weights S_j), so
        S^(1/2) K S^(-1/2) is symmetric; its eigenpairs come from a library symmetric solver
        (dense for up to 4,000 triangles, else sparse: shift-invert about a point just below
        zero for the lowest, the largest algebraic ones directly for the highest; "nearest" is
        always sparse shift-invert about sigma). Returns (lam [count], V [n_t, count]) with
        sum_j S_j V_jc V_jd = delta_cd, lam ascending for "lowest" and "nearest" and descending
        for "highest"; omega = sqrt(lam). The constant B is the static mode (lam = 0).
        """
        import scipy.linalg
        import scipy.sparse.linalg as sla
        count = int(count)
        if not 1 <= count <= self.nt or which not in ("lowest", "highest", "nearest"):
            raise OracleError(EINVAL, "modes count or which")
        A, irs = self._symmetric_k(gamma)
        if which == "nearest":
            lam, U = sla.eigsh(A.tocsc(), k=count, sigma=float(sigma), which="LM", tol=1e-14)
            order = np.argsort(lam)
            return lam[order], irs[:, None] * U[:, order]
        if self.nt <= 4000:
            lo = 0 if which == "lowest" else self.nt - count
            lam, U = scipy.linalg.eigh(A.toarray(), subset_by_index=[lo, lo + count - 1])
        elif which == "lowest":
            top = float(abs(A).sum(axis=1).max())
            lam, U = sla.eigsh(A.tocsc(), k=count, sigma=-1e-6 * top, which="LM")
        else:
            lam, U = sla.eigsh(A.tocsc(), k=count, which="LA", tol=1e-14)
        order = np.argsort(lam) if which == "lowest" else np.argsort(-lam)
        lam, U = lam[order], U[:, order]
        return lam, irs[:, None] * U

    def _symmetric_k(self, gamma=None):
        """S^(1/2) K S^(-1/2) (sparse, symmetrised) and S^(-1/2)."""
        import scipy.sparse as sp
        LB, LE = self.sparse_ops(gamma)
        K = -(LE @ LB)
        rs, irs = np.sqrt(self.S), 1.0 / np.sqrt(self.S)
        A = sp.diags(rs) @ K @ sp.diags(irs)
        return 0.5 * (A + A.T), irs

    def spectrum(self, gamma=None, vectors=True):
        """Every eigenpair of K = -L_E L_B (Section 2, Fig. 4: as many eigenvalues as B
        components, counted with the static constant field).

        The symmetric S^(1/2) K S^(-1/2) is formed densely and handed to a library dense
        symmetric eigensolver (divide and conquer): n_t^2 doubles of memory and O(n_t^3) work,
        about two minutes at 16,500 triangles without vectors.  Returns (lam [n_t] ascending,
        V [n_t, n_t] with S-orthonormal columns, or None).
        """
        import scipy.linalg
        A, irs = self._symmetric_k(gamma)
        if not vectors:
            return scipy.linalg.eigh(A.toarray(), eigvals_only=True, driver="evd"), None
        lam, U = scipy.linalg.eigh(A.toarray(), driver="evd")
        return lam, irs[:, None] * U

    # -- media and sources defined on the input ----------------------------------------
    def edge_wp2(self, wp2_tri):
        """Per-edge plasma frequency squared from per-triangle values.

        Each interior edge takes the half-dual-length weighted mean of its two triangles,
        (hR wp2_R + hL wp2_L)/d; outer edges carry no field and get 0 (a reading of the
        particle boundary of Fig. 3).
        """
        wt = np.asarray(wp2_tri, np.float64)
        out = np.zeros(self.ne)
        i = self.interior
        out[i] = (self.hR[i] * wt[self.R[i]] + self.hL[i] * wt[self.L[i]]) / self.d[i]
        return out

    def edge_ids(self, pairs):
        """Canonical edge ids and orientation signs (+1 when pair runs lo -> hi)."""
        pairs = np.asarray(pairs, np.int64).reshape(-1, 2)
        lo, hi = pairs.min(1), pairs.max(1)
        keys = self.edge[:, 0].astype(np.int64) * self.nv + self.edge[:, 1]
        q = lo * self.nv + hi
        ids = np.searchsorted(keys, q)
        if np.any(ids >= self.ne) or np.any(keys[np.minimum(ids, self.ne - 1)] != q):
            raise OracleError(EINVAL, "edge lookup")
        sign = np.where(pairs[:, 0] < pairs[:, 1], 1.0, -1.0)
        return ids.astype(np.int32), sign

    # -- stepping ----------------------------------------------------------------------
    def step(self, E, B, dt, nsteps, n0=0, J=None, Q=None, wp2=None, nu=0.0, gamma=None,
             src=None, want_prev=False):
        """Advance copies of (E, B[, J, Q]) by nsteps leap-frog steps; returns a dict.

        src = (pairs, weights, omega, cycles) for a soft source; weights refer to the pair
        direction given.
        """
        E = np.array(E, np.float64, copy=True)
        B = np.array(B, np.float64, copy=True)
        media = wp2 is not None
        J = (np.zeros(self.ne) if J is None else np.array(J, np.float64, copy=True)) \
            if media else None
        need_q = media or src is not None
        Q = (np.zeros(self.nv) if Q is None else np.array(Q, np.float64, copy=True)) \
            if need_q else None
        prm = _Params()
        prm.dt = float(dt)
        g = None if gamma is None else np.ascontiguousarray(gamma, np.float64)
        w2 = None if wp2 is None else np.ascontiguousarray(wp2, np.float64)
        prm.gamma, prm.wp2, prm.nu = _p(g), _p(w2), float(nu)
        keep = []
        if src is not None:
            pairs, w, omega, cycles = src
            ids, sign = self.edge_ids(pairs)
            w = np.ascontiguousarray(np.asarray(w, np.float64) * sign)
            keep += [ids, w]
            prm.n_src, prm.src_edge, prm.src_w = len(ids), _p(ids), _p(w)
            prm.src_omega, prm.src_cycles = float(omega), float(cycles)
        Bp = np.zeros(self.nt) if want_prev else None
        rc = _load().orc_step(self._h, ctypes.byref(prm), int(n0), int(nsteps), _p(E), _p(B),
                              _p(J), _p(Q), _p(Bp))
        if rc != OK:
            raise OracleError(rc, "step")
        return dict(E=E, B=B, J=J, Q=Q, B_prev=Bp)

    # -- diagnostics -------------------------------------------------------------------
    def energy(self, E, Bold, Bnew=None):
        Bnew = Bold if Bnew is None else Bnew
        a = [np.ascontiguousarray(x, np.float64) for x in (E, Bold, Bnew)]
        return float(_load().orc_energy(self._h, _p(a[0]), _p(a[1]), _p(a[2])))

    def div(self, E):
        out = np.zeros(self.nv)
        E = np.ascontiguousarray(E, np.float64)
        _load().orc_div(self._h, _p(E), _p(out))
        return out

    def power(self, gamma=None, max_iter=20000, rtol=1e-12, seed=0):
        """Largest eigenvalue of K = -L_E L_B (omega_max^2) and the iteration count."""
        lam = ctypes.c_double(0.0)
        it = ctypes.c_int64(0)
        g = None if gamma is None else np.ascontiguousarray(gamma, np.float64)
        rc = _load().orc_power(self._h, _p(g), int(max_iter), float(rtol), int(seed),
                               ctypes.byref(lam), ctypes.byref(it))
        if rc not in (OK, ENOTCONVERGED):
            raise OracleError(rc, "power iteration")
        return lam.value, it.value, rc == OK

    def omega_max(self, **kw):
        lam, _, _ = self.power(**kw)
        return float(np.sqrt(lam))

    def order(self, kind, seed=0):
        perm_t = np.zeros(self.nt, np.int32)
        perm_e = np.zeros(self.ne, np.int32)
        rc = _load().orc_order(self._h, ORDER[kind], int(seed), _p(perm_t), _p(perm_e))
        if rc != OK:
            raise OracleError(rc, "order")
        return perm_t, perm_e
