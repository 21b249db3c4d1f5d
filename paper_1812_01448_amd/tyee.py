"""Thin ctypes binding of libtyee (the C ABI declared in include/tyee.h).

Argument marshalling only: every step of the solver runs in the native library. The
library must have been built (``python paper_1812_01448_amd/build.py``); importing this
module without it raises immediately.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtyee.so")

OK, EINVAL, ENOTDELAUNAY, EDEGENERATE, ENONMANIFOLD, EPERIODIC, ENOMEM, EDEVICE, \
    EUNSTABLE, ENOTCONVERGED = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
PEC_BOX, PERIODIC = 0, 1
ORDER = {"none": 0, "random": 1, "morton": 2, "rcm": 3}
PREC = {"f32": 0, "f64": 1}
FIELD = {"E": 0, "B": 1, "J": 2, "Q": 3}


class TyeeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tyee error {code}: {msg}")
        self.code = code


class _Domain(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("dual_tol", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_tris", ctypes.c_int64), ("n_boundary_edges", ctypes.c_int64),
                ("min_dual_ratio", ctypes.c_double), ("max_dual_ratio", ctypes.c_double),
                ("sum_area", ctypes.c_double), ("sum_dual_area", ctypes.c_double),
                ("n_obtuse", ctypes.c_int64)]


_VIEW_FIELDS = ["tri", "edge_nodes", "R", "L", "A", "sgn", "elen", "evec", "hR", "hL", "d",
                "S", "O", "C", "perm_t", "perm_e"]


class _View(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in _VIEW_FIELDS]


class _Tune(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32),
                ("tile_tris", ctypes.c_int32), ("ms_per_step", ctypes.c_double)]


_TUNE_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.POINTER(_Tune), ctypes.c_void_p)


class _Gate(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("omega_plain", ctypes.c_double), ("omega_learned", ctypes.c_double),
                ("dt_plain", ctypes.c_double), ("dt_learned", ctypes.c_double),
                ("err_plain", ctypes.c_double), ("err_learned", ctypes.c_double)]


class _ModesStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("applies", ctypes.c_int64),
                ("lambda_bound", ctypes.c_double), ("filter_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class _SpectrumStats(ctypes.Structure):
    _fields_ = [("windows", ctypes.c_int32), ("iters", ctypes.c_int32), ("found", ctypes.c_int64),
                ("applies", ctypes.c_int64), ("below", ctypes.c_int64), ("retries", ctypes.c_int64),
                ("lambda_bound", ctypes.c_double), ("filter_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("max_residual", ctypes.c_double),
                ("min_gap", ctypes.c_double), ("sq_launches", ctypes.c_int64),
                ("sq_ms", ctypes.c_double)]


class _PmlParams(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int32), ("width", ctypes.c_double), ("sigma_max", ctypes.c_double),
                ("grading", ctypes.c_double)]


class _RelaxParams(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("iters", ctypes.c_int32), ("step", ctypes.c_double),
                ("k_edge", ctypes.c_double), ("k_height", ctypes.c_double), ("rest", ctypes.c_double),
                ("keep_best", ctypes.c_int32)]


class _RelaxStats(ctypes.Structure):
    _fields_ = [("omega_initial", ctypes.c_double), ("omega_best", ctypes.c_double),
                ("best_round", ctypes.c_int32), ("flips", ctypes.c_int64),
                ("energy_initial", ctypes.c_double), ("energy_final", ctypes.c_double),
                ("step_used", ctypes.c_double)]


class _Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("time", ctypes.c_double), ("energy", ctypes.c_double),
                ("energy_h", ctypes.c_double), ("max_abs_E", ctypes.c_double),
                ("max_abs_B", ctypes.c_double), ("nonfinite", ctypes.c_int32)]


EXPORTS = [
    "tyee_mesh_create", "tyee_mesh_reorder", "tyee_mesh_query", "tyee_mesh_view",
    "tyee_mesh_cfl", "tyee_mesh_destroy", "tyee_sim_create", "tyee_sim_set_state",
    "tyee_sim_get_state", "tyee_sim_set_media", "tyee_sim_set_source",
    "tyee_sim_set_edge_scale", "tyee_sim_set_fusion", "tyee_sim_step", "tyee_sim_sync",
    "tyee_sim_diagnostics", "tyee_sim_diagnostics_noalloc", "tyee_sim_last_step_ms", "tyee_sim_set_profiling",
    "tyee_sim_kernel_times", "tyee_sim_get_fusion", "tyee_sim_steps", "tyee_sim_destroy",
    "tyee_sim_gauss", "tyee_sim_add_probe", "tyee_sim_read_probe", "tyee_sim_set_graph",
    "tyee_batch_create", "tyee_batch_set_state", "tyee_batch_get_state", "tyee_batch_reorder",
    "tyee_batch_set_fusion", "tyee_batch_set_graph", "tyee_batch_step", "tyee_batch_sync",
    "tyee_batch_info", "tyee_batch_sim", "tyee_batch_tune", "tyee_batch_destroy",
    "tyee_mesh_features", "tyee_mesh_phase_error_rq", "tyee_phase_error_timestepped",
    "tyee_learner_create", "tyee_learner_init", "tyee_learner_set_params",
    "tyee_learner_get_params", "tyee_learner_normaliser", "tyee_learner_loss_grad",
    "tyee_learner_train", "tyee_learner_gamma", "tyee_learner_set_batch", "tyee_learner_set_path",
    "tyee_learner_destroy", "tyee_gate",
    "tyee_learner_regulariser", "tyee_copy_bandwidth", "tyee_sim_bind_external",
    "tyee_sim_current_buffer", "tyee_mesh_modes", "tyee_mesh_spectrum", "tyee_mesh_relax",
    "tyee_mesh_flip", "tyee_open_create", "tyee_open_sizes", "tyee_open_frame", "tyee_open_cfl",
    "tyee_open_set_state", "tyee_open_get_state", "tyee_open_step", "tyee_open_set_graph",
    "tyee_open_sync", "tyee_open_set_fusion",
    "tyee_open_set_timing", "tyee_open_kernel_ms", "tyee_open_destroy",
    "tyee_tet_create", "tyee_tet_sizes", "tyee_tet_view", "tyee_tet_cfl", "tyee_tet_destroy",
    "tyee_tet_sim_create", "tyee_tet_sim_set_state", "tyee_tet_sim_get_state", "tyee_tet_sim_step",
    "tyee_tet_sim_set_graph", "tyee_tet_sim_sync", "tyee_tet_sim_set_timing", "tyee_tet_sim_kernel_ms",
    "tyee_tet_sim_destroy",
    "tyee_batch_tune_progress",
    "tyee_last_error",
]
N_PARAMS = 1377
KERNELS = {"edge": 0, "tri": 1, "fused": 2, "special": 3, "charge": 4, "graph": 5}
KERNEL_NAMES = {"edge": "k_edge", "tri": "k_tri", "fused": "k_fused", "special": "k_special",
                "charge": "k_charge", "graph": "graph of k_fused"}


def _preload_hip_runtime():
    """PyTorch-ROCm wheels bundle their own HIP runtime under the same soname as the system
    one, and a process holds only the first one loaded; torch finds no GPU when it gets a
    runtime other than its own.  When such a wheel is installed (and torch is not imported
    yet), load its runtime before this library, so that both share it whatever the import
    order.  torch itself is not imported."""
    import importlib.util
    import sys
    if "torch" in sys.modules:
        return
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    path = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(path):
        ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtyee.so is not built ({LIB_PATH}); run python paper_1812_01448_amd/build.py")
    _preload_hip_runtime()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "tyee_mesh_create": [vp, i64, vp, i64, ctypes.POINTER(_Domain), ctypes.POINTER(vp)],
        "tyee_mesh_reorder": [vp, i32, ctypes.c_uint64],
        "tyee_mesh_query": [vp, ctypes.POINTER(_Info)],
        "tyee_mesh_view": [vp, ctypes.POINTER(_View)],
        "tyee_mesh_cfl": [vp, vp, i64, f64, ctypes.c_uint64, ctypes.POINTER(f64),
                          ctypes.POINTER(i64)],
        "tyee_sim_create": [vp, i32, f64, vp, ctypes.POINTER(vp)],
        "tyee_sim_set_state": [vp, i32, vp],
        "tyee_sim_get_state": [vp, i32, vp],
        "tyee_sim_set_media": [vp, vp, f64],
        "tyee_sim_set_source": [vp, vp, vp, i64, f64, f64],
        "tyee_sim_set_edge_scale": [vp, vp],
        "tyee_sim_set_fusion": [vp, i32, i32],
        "tyee_sim_step": [vp, i64],
        "tyee_sim_sync": [vp],
        "tyee_sim_diagnostics": [vp, ctypes.POINTER(_Diag)],
        "tyee_sim_diagnostics_noalloc": [vp, ctypes.POINTER(_Diag)],
        "tyee_sim_last_step_ms": [vp, ctypes.POINTER(f64)],
        "tyee_sim_set_profiling": [vp, ctypes.c_uint32],
        "tyee_sim_kernel_times": [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64)],
        "tyee_sim_get_fusion": [vp, vp],
        "tyee_sim_gauss": [vp, vp],
        "tyee_sim_set_graph": [vp, i32],
        "tyee_batch_create": [vp, vp, i64, i32, vp, ctypes.POINTER(vp)],
        "tyee_batch_set_state": [vp, i64, i32, vp],
        "tyee_batch_get_state": [vp, i64, i32, vp],
        "tyee_batch_reorder": [vp, i32, ctypes.c_uint64],
        "tyee_batch_set_fusion": [vp, i32, i32],
        "tyee_batch_set_graph": [vp, i32],
        "tyee_batch_step": [vp, i64],
        "tyee_batch_sync": [vp],
        "tyee_batch_info": [vp, vp],
        "tyee_batch_sim": [vp, ctypes.POINTER(vp)],
        "tyee_batch_tune": [vp, i64, vp, i64, ctypes.POINTER(i64)],
        "tyee_mesh_features": [vp, vp],
        "tyee_mesh_phase_error_rq": [vp, vp, f64, vp, i64, vp],
        "tyee_phase_error_timestepped": [vp, vp, f64, i32, vp, i64, f64, i64, vp, vp],
        "tyee_learner_create": [vp, vp, i64, vp, i64, f64, vp, ctypes.POINTER(vp)],
        "tyee_learner_init": [vp, ctypes.c_uint64],
        "tyee_learner_regulariser": [vp, f64, f64, f64],
        "tyee_learner_set_params": [vp, vp],
        "tyee_learner_get_params": [vp, vp],
        "tyee_learner_normaliser": [vp, vp, vp, vp, vp],
        "tyee_learner_loss_grad": [vp, ctypes.POINTER(f64), vp, vp],
        "tyee_learner_train": [vp, i64, f64, vp],
        "tyee_learner_gamma": [vp, vp, vp],
        "tyee_learner_set_batch": [vp, vp, i64],
        "tyee_learner_set_path": [vp, i32],
        "tyee_gate": [vp, vp, vp, i64, f64, f64, i32, vp, ctypes.POINTER(_Gate)],
        "tyee_sim_add_probe": [vp, i32, vp, i64, i64, i64, ctypes.POINTER(i32)],
        "tyee_sim_read_probe": [vp, i32, vp, i64, ctypes.POINTER(i64)],
        "tyee_copy_bandwidth": [i64, i32, ctypes.POINTER(f64)],
        "tyee_sim_bind_external": [vp, i32, vp, vp],
        "tyee_sim_current_buffer": [vp, ctypes.POINTER(i32)],
        "tyee_mesh_flip": [vp, i64, vp, i64, ctypes.POINTER(_Domain), ctypes.POINTER(i64)],
        "tyee_mesh_relax": [vp, ctypes.POINTER(_RelaxParams), vp, i64, vp, vp, vp, vp,
                            ctypes.POINTER(_RelaxStats)],
        "tyee_mesh_modes": [vp, vp, i32, i64, i32, i32, f64, i32, ctypes.c_uint64, vp, vp, vp, vp,
                            ctypes.POINTER(_ModesStats)],
        "tyee_mesh_spectrum": [vp, vp, i32, i32, f64, i32, ctypes.c_uint64, vp, vp, vp, vp,
                               ctypes.POINTER(_SpectrumStats)],
        "tyee_batch_tune_progress": [vp, i64, vp, i64, ctypes.POINTER(i64), _TUNE_PROGRESS, vp],
        "tyee_open_create": [vp, ctypes.POINTER(_PmlParams), i32, f64, vp, ctypes.POINTER(vp)],
        "tyee_open_sizes": [vp, vp],
        "tyee_open_frame": [vp, ctypes.POINTER(_PmlParams), vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "tyee_open_cfl": [vp, i64, f64, ctypes.c_uint64, ctypes.POINTER(f64), ctypes.POINTER(i64)],
        "tyee_open_set_state": [vp, i32, vp],
        "tyee_open_get_state": [vp, i32, vp],
        "tyee_open_step": [vp, i64],
        "tyee_open_set_graph": [vp, i32],
        "tyee_open_sync": [vp],
        "tyee_open_set_fusion": [vp, vp, i32, i32],
        "tyee_open_set_timing": [vp, i32],
        "tyee_open_kernel_ms": [vp, vp, ctypes.POINTER(i64)],
        "tyee_open_destroy": [vp],
        "tyee_tet_create": [vp, i64, vp, i64, ctypes.POINTER(vp)],
        "tyee_tet_sizes": [vp, vp],
        "tyee_tet_view": [vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "tyee_tet_cfl": [vp, i64, f64, ctypes.c_uint64, ctypes.POINTER(f64), ctypes.POINTER(i64)],
        "tyee_tet_destroy": [vp],
        "tyee_tet_sim_create": [vp, i32, f64, vp, ctypes.POINTER(vp)],
        "tyee_tet_sim_set_state": [vp, i32, vp],
        "tyee_tet_sim_get_state": [vp, i32, vp],
        "tyee_tet_sim_step": [vp, i64],
        "tyee_tet_sim_set_graph": [vp, i32],
        "tyee_tet_sim_sync": [vp],
        "tyee_tet_sim_set_timing": [vp, i32],
        "tyee_tet_sim_kernel_ms": [vp, vp, ctypes.POINTER(i64)],
        "tyee_tet_sim_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.tyee_mesh_destroy.argtypes = [vp]
    lib.tyee_mesh_destroy.restype = None
    lib.tyee_sim_destroy.argtypes = [vp]
    lib.tyee_sim_destroy.restype = None
    lib.tyee_learner_destroy.argtypes = [vp]
    lib.tyee_learner_destroy.restype = None
    lib.tyee_batch_destroy.argtypes = [vp]
    lib.tyee_batch_destroy.restype = None
    lib.tyee_sim_steps.argtypes = [vp]
    lib.tyee_sim_steps.restype = i64
    lib.tyee_last_error.argtypes = []
    lib.tyee_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise TyeeError(rc, lib.tyee_last_error().decode())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def flip(xy, tri, periodic, L=1.0, Ly=None):
    """Lawson flips (tyee_mesh_flip): returns (counter-clockwise Delaunay tri, number of flips)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    t = np.array(tri, dtype=np.int32, copy=True, order="C")
    dom = _Domain(PERIODIC if periodic else PEC_BOX, float(L), float(L if Ly is None else Ly), 0.0)
    n = ctypes.c_int64()
    _check(lib.tyee_mesh_flip(_ptr(xy), len(xy), _ptr(t), len(t), ctypes.byref(dom), ctypes.byref(n)))
    return t, n.value


class Mesh:
    """Connectivity, FP64 geometry and locality numbering of a triangle mesh."""

    def __init__(self, xy, tri, periodic, L=1.0, Ly=None, dual_tol=0.0):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        dom = _Domain(PERIODIC if periodic else PEC_BOX, float(L), float(L if Ly is None else Ly),
                      float(dual_tol))
        h = ctypes.c_void_p()
        _check(lib.tyee_mesh_create(_ptr(xy), len(xy), _ptr(tri), len(tri), ctypes.byref(dom),
                                    ctypes.byref(h)))
        self._h = h
        self.periodic = bool(periodic)
        info = self.info()
        self.nv, self.ne, self.nt, self.nb = (info["n_nodes"], info["n_edges"], info["n_tris"],
                                              info["n_boundary_edges"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_mesh_destroy(h)
            self._h = None

    def relax(self, rounds=10, iters=100, step=0.05, k_edge=1.0, k_height=1.0, rest=0.0,
              keep_best=True, anchors=None, stream=None):
        """Jello relaxation (tyee_mesh_relax): returns (xy, tri, omega per round, stats); build
        the relaxed mesh with Mesh(xy, tri, ...) on the same domain."""
        prm = _RelaxParams(int(rounds), int(iters), float(step), float(k_edge), float(k_height),
                           float(rest), 1 if keep_best else 0)
        anc = None if anchors is None else np.ascontiguousarray(anchors, np.int32)
        xy = np.zeros((self.nv, 2))
        tri = np.zeros((self.nt, 3), np.int32)
        om = np.zeros(int(rounds) + 1)
        st = _RelaxStats()
        _check(lib.tyee_mesh_relax(self._h, ctypes.byref(prm), _ptr(anc), 0 if anc is None else len(anc),
                                   None if stream is None else int(stream), _ptr(xy), _ptr(tri),
                                   _ptr(om), ctypes.byref(st)))
        return xy, tri, om, {n: getattr(st, n) for n, _ in _RelaxStats._fields_}

    def reorder(self, kind, seed=0):
        _check(lib.tyee_mesh_reorder(self._h, ORDER[kind] if isinstance(kind, str) else int(kind),
                                     int(seed)))

    def info(self):
        out = _Info()
        _check(lib.tyee_mesh_query(self._h, ctypes.byref(out)))
        return {n: getattr(out, n) for n, _ in _Info._fields_}

    def view(self):
        """Copies of the mesh arrays (canonical numbering)."""
        v = _View()
        _check(lib.tyee_mesh_view(self._h, ctypes.byref(v)))
        ne, nt = self.ne, self.nt
        spec = {"tri": (np.int32, (nt, 3)), "edge_nodes": (np.int32, (ne, 2)),
                "R": (np.int32, (ne,)), "L": (np.int32, (ne,)), "A": (np.int32, (nt, 3)),
                "sgn": (np.int8, (nt, 3)), "elen": (np.float64, (ne,)),
                "evec": (np.float64, (ne, 2)), "hR": (np.float64, (ne,)),
                "hL": (np.float64, (ne,)), "d": (np.float64, (ne,)), "S": (np.float64, (nt,)),
                "O": (np.float64, (nt, 2)), "C": (np.float64, (ne, 2)),
                "perm_t": (np.int32, (nt,)), "perm_e": (np.int32, (ne,))}
        out = {}
        for name, (dt, shape) in spec.items():
            n = int(np.prod(shape))
            buf = (ctypes.c_byte * (n * np.dtype(dt).itemsize)).from_address(getattr(v, name))
            out[name] = np.frombuffer(buf, dtype=dt).reshape(shape).copy()
        return out

    def features(self):
        out = np.zeros((self.ne, 8))
        _check(lib.tyee_mesh_features(self._h, _ptr(out)))
        return out

    def phase_error_rq(self, dt, waves, gamma=None):
        w = np.ascontiguousarray(waves, np.float64).reshape(-1, 2)
        g = None if gamma is None else _f64(gamma, self.ne)
        out = np.zeros(len(w))
        _check(lib.tyee_mesh_phase_error_rq(self._h, _ptr(g), float(dt), _ptr(w), len(w), _ptr(out)))
        return out

    def phase_error_timestepped(self, dt, waves, phase=2.0, samples=10, gamma=None, prec="f64",
                                stream=None):
        """Time-stepped phase error of each wave in `waves` ([n, 2] or one [2] wavevector)."""
        w = np.ascontiguousarray(waves, np.float64)
        single = w.ndim == 1
        w = w.reshape(-1, 2)
        g = None if gamma is None else _f64(gamma, self.ne)
        out = np.zeros(len(w))
        _check(lib.tyee_phase_error_timestepped(self._h, _ptr(g), float(dt), PREC[prec], _ptr(w),
                                                len(w), float(phase), int(samples),
                                                None if stream is None else int(stream),
                                                _ptr(out)))
        return float(out[0]) if single else out

    def gate(self, gamma, waves, cfl=0.5, phase=2.0, prec="f64", stream=None):
        g = _f64(gamma, self.ne)
        w = np.ascontiguousarray(waves, np.float64).reshape(-1, 2)
        r = _Gate()
        _check(lib.tyee_gate(self._h, _ptr(g), _ptr(w), len(w), float(cfl), float(phase),
                             PREC[prec], None if stream is None else int(stream),
                             ctypes.byref(r)))
        return {n: getattr(r, n) for n, _ in _Gate._fields_}

    def cfl(self, gamma=None, max_iter=20000, rtol=1e-12, seed=0):
        """(omega_max^2, iterations, converged) of K = -L_E L_B."""
        lam = ctypes.c_double()
        it = ctypes.c_int64()
        g = None if gamma is None else _f64(gamma, self.ne)
        rc = _check(lib.tyee_mesh_cfl(self._h, _ptr(g), int(max_iter), float(rtol), int(seed),
                                      ctypes.byref(lam), ctypes.byref(it)), allow=(ENOTCONVERGED,))
        return lam.value, it.value, rc == OK


    def modes(self, n_modes, gamma=None, block=0, degree=0, tol=1e-10, max_iter=200, seed=0,
              stream=None, want_vectors=True, which="lowest"):
        """Lowest (or, with which="highest", highest) n_modes eigenpairs of K = -L_E L_B on
        the device (FP64).

        Returns a dict: omega2 [n_modes] (ascending, or descending for the highest), modes
        [n_modes, n_t] (canonical triangle order, S-orthonormal; None unless want_vectors),
        residual [n_modes] (relative to the Gershgorin bound), converged, and the call's stats
        (iters, applies, lambda_bound, filter_ms, total_ms)."""
        n_modes = int(n_modes)
        om2 = np.zeros(n_modes)
        vec = np.zeros((n_modes, self.nt)) if want_vectors else None
        res = np.zeros(n_modes)
        st = _ModesStats()
        g = None if gamma is None else _f64(gamma, self.ne)
        if which not in ("lowest", "highest"):
            raise ValueError("which must be 'lowest' or 'highest'")
        rc = _check(lib.tyee_mesh_modes(self._h, _ptr(g), 0 if which == "lowest" else 1, n_modes,
                                        int(block), int(degree),
                                        float(tol), int(max_iter), int(seed),
                                        None if stream is None else int(stream), _ptr(om2),
                                        _ptr(vec), _ptr(res), ctypes.byref(st)),
                    allow=(ENOTCONVERGED,))
        out = {"omega2": om2, "modes": vec, "residual": res, "converged": rc == OK}
        out.update({n: getattr(st, n) for n, _ in _ModesStats._fields_})
        return out


    def spectrum(self, gamma=None, block=0, degree=0, tol=1e-10, max_iter=50, seed=0, stream=None,
                 want_vectors=True):
        """Every eigenpair of K = -L_E L_B on the device (FP64), window by window.

        Returns a dict: omega2 [n_t] ascending, modes [n_t, n_t] (mode-major, canonical
        triangle order, S-orthonormal; None unless want_vectors), residual [n_t] (relative to the
        Gershgorin bound), converged, and the call's stats (windows, iters, found, applies,
        below, retries, lambda_bound, filter_ms, total_ms, max_residual, min_gap, sq_launches,
        sq_ms)."""
        om2 = np.zeros(self.nt)
        vec = np.zeros((self.nt, self.nt)) if want_vectors else None
        res = np.zeros(self.nt)
        st = _SpectrumStats()
        g = None if gamma is None else _f64(gamma, self.ne)
        rc = _check(lib.tyee_mesh_spectrum(self._h, _ptr(g), int(block), int(degree), float(tol),
                                           int(max_iter), int(seed),
                                           None if stream is None else int(stream), _ptr(om2),
                                           _ptr(vec), _ptr(res), ctypes.byref(st)),
                    allow=(ENOTCONVERGED,))
        out = {"omega2": om2, "modes": vec, "residual": res, "converged": rc == OK}
        out.update({n: getattr(st, n) for n, _ in _SpectrumStats._fields_})
        return out


OPEN_FIELD = {"E": 0, "BX": 1, "BY": 2}


def pml(layers, width, sigma_max, grading=3.0):
    """PML frame parameters (tyee_pml_params)."""
    return _PmlParams(int(layers), float(width), float(sigma_max), float(grading))


def open_frame(mesh, params):
    """The mixed mesh (triangles plus the PML frame) built on the host (tyee_open_frame): a dict
    of numpy arrays in canonical order and the sizes."""
    sizes = np.zeros(5, np.int64)
    _check(lib.tyee_open_frame(mesh._h, ctypes.byref(params), _ptr(sizes), *([None] * 10)))
    nv, ne, nc = (int(v) for v in sizes[:3])
    out = {"xy": np.zeros((nv, 2)), "edge": np.zeros((ne, 2), np.int32), "cell_edge": np.zeros((nc, 4), np.int32),
           "elen": np.zeros(ne), "d": np.zeros(ne), "S": np.zeros(nc), "O": np.zeros((nc, 2)),
           "sigma_e": np.zeros(ne), "sigma_x": np.zeros(nc), "sigma_y": np.zeros(nc)}
    _check(lib.tyee_open_frame(mesh._h, ctypes.byref(params), _ptr(sizes),
                               *[_ptr(out[k]) for k in ("xy", "edge", "cell_edge", "elen", "d", "S", "O",
                                                        "sigma_e", "sigma_x", "sigma_y")]))
    out.update({"n_nodes": nv, "n_edges": ne, "n_cells": nc, "n_frame_cells": int(sizes[3]),
                "n_inner_edges": int(sizes[4])})
    return out


class Open:
    """The triangle mesh of a closed box tied to a PML frame, stepped on the device
    (tyee_open_*)."""

    def __init__(self, mesh, params, dt, prec="f32", stream=None):
        h = ctypes.c_void_p()
        _check(lib.tyee_open_create(mesh._h, ctypes.byref(params), PREC[prec], float(dt),
                                    None if stream is None else int(stream), ctypes.byref(h)))
        self._h = h
        sizes = np.zeros(5, np.int64)
        _check(lib.tyee_open_sizes(h, _ptr(sizes)))
        self.nv, self.ne, self.ncell, self.nf, self.n_inner = (int(v) for v in sizes)
        self.nt = self.ncell - self.nf
        self.dt, self.prec = float(dt), prec

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_open_destroy(h)
            self._h = None

    def _n(self, field):
        return self.ne if field == "E" else self.ncell

    def set_state(self, field, values):
        a = _f64(values, self._n(field))
        _check(lib.tyee_open_set_state(self._h, OPEN_FIELD[field], _ptr(a)))

    def get_state(self, field):
        out = np.zeros(self._n(field))
        _check(lib.tyee_open_get_state(self._h, OPEN_FIELD[field], _ptr(out)))
        return out

    def step(self, n=1):
        _check(lib.tyee_open_step(self._h, int(n)))

    def set_graph(self, steps):
        """Steps per captured HIP graph (0: eager launches; the library's default is 8)."""
        _check(lib.tyee_open_set_graph(self._h, int(steps)))

    def set_fusion(self, mesh, k=0, tile=0):
        """Fused stepping of the box (tyee_open_set_fusion): k steps per launch (0 = default,
        1 = off); mesh is the triangle mesh this handle was created from."""
        _check(lib.tyee_open_set_fusion(self._h, mesh._h, int(k), int(tile)))

    def sync(self):
        _check(lib.tyee_open_sync(self._h))

    def cfl(self, max_iter=200000, rtol=1e-12, seed=0):
        lam, it = ctypes.c_double(), ctypes.c_int64()
        rc = _check(lib.tyee_open_cfl(self._h, int(max_iter), float(rtol), int(seed), ctypes.byref(lam),
                                      ctypes.byref(it)), allow=(ENOTCONVERGED,))
        return lam.value, it.value, rc == OK

    def set_timing(self, on=True):
        _check(lib.tyee_open_set_timing(self._h, 1 if on else 0))

    def kernel_ms(self):
        out, n = np.zeros(2), ctypes.c_int64()
        _check(lib.tyee_open_kernel_ms(self._h, _ptr(out), ctypes.byref(n)))
        return {"edge_ms": float(out[0]), "cell_ms": float(out[1]), "steps": n.value}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device copy rate in GB/s (bytes read + written per second) with 16-byte non-temporal
    loads and stores: the achievable-bandwidth reference beside the HBM peak."""
    g = ctypes.c_double()
    _check(lib.tyee_copy_bandwidth(int(nbytes), int(reps), ctypes.byref(g)))
    return g.value


TET_FIELD = {"E": 0, "B": 1}


class Tet:
    """A tetrahedral mesh of a box with conducting walls (tyee_tet_*): canonical edges and
    faces, FP64 geometry and the Voronoi dual, built on the host."""

    def __init__(self, xyz, tets):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        t = np.ascontiguousarray(tets, dtype=np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 4:
            raise ValueError("xyz must be [n, 3] and tets [n, 4]")
        h = ctypes.c_void_p()
        _check(lib.tyee_tet_create(_ptr(xyz), len(xyz), _ptr(t), len(t), ctypes.byref(h)))
        self._h = h
        sizes = np.zeros(7, np.int64)
        _check(lib.tyee_tet_sizes(h, _ptr(sizes)))
        (self.nv, self.ne, self.nf, self.nt, self.n_inner_edge, self.n_inner_face,
         self.n_incidences) = (int(v) for v in sizes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_tet_destroy(h)
            self._h = None

    def view(self):
        """Canonical arrays: edge, face, face_edge, elen, dual_area, farea, d, C."""
        out = {"edge": np.zeros((self.ne, 2), np.int32), "face": np.zeros((self.nf, 3), np.int32),
               "face_edge": np.zeros((self.nf, 3), np.int32), "elen": np.zeros(self.ne),
               "dual_area": np.zeros(self.ne), "farea": np.zeros(self.nf), "d": np.zeros(self.nf),
               "C": np.zeros((self.nt, 3))}
        _check(lib.tyee_tet_view(self._h, *(_ptr(out[k]) for k in ("edge", "face", "face_edge", "elen",
                                                                  "dual_area", "farea", "d", "C"))))
        return out

    def cfl(self, max_iter=200000, rtol=1e-12, seed=0):
        """(lambda = omega_max^2, iterations, converged)."""
        lam, it = ctypes.c_double(), ctypes.c_int64()
        rc = _check(lib.tyee_tet_cfl(self._h, int(max_iter), float(rtol), int(seed), ctypes.byref(lam),
                                     ctypes.byref(it)), allow=(ENOTCONVERGED,))
        return lam.value, it.value, rc == OK


class TetSim:
    """Leap-frog stepping of E on the edges and B on the faces of a tetrahedral mesh on the
    device (tyee_tet_sim_*)."""

    def __init__(self, tet, dt, prec="f32", stream=None):
        h = ctypes.c_void_p()
        _check(lib.tyee_tet_sim_create(tet._h, PREC[prec], float(dt), None if stream is None else int(stream),
                                       ctypes.byref(h)))
        self._h = h
        self.ne, self.nf, self.dt, self.prec = tet.ne, tet.nf, float(dt), prec

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_tet_sim_destroy(h)
            self._h = None

    def set_state(self, field, values):
        a = _f64(values, self.ne if field == "E" else self.nf)
        _check(lib.tyee_tet_sim_set_state(self._h, TET_FIELD[field], _ptr(a)))

    def get_state(self, field):
        out = np.zeros(self.ne if field == "E" else self.nf)
        _check(lib.tyee_tet_sim_get_state(self._h, TET_FIELD[field], _ptr(out)))
        return out

    def step(self, n=1):
        _check(lib.tyee_tet_sim_step(self._h, int(n)))

    def set_graph(self, steps):
        _check(lib.tyee_tet_sim_set_graph(self._h, int(steps)))

    def sync(self):
        _check(lib.tyee_tet_sim_sync(self._h))

    def set_timing(self, on=True):
        _check(lib.tyee_tet_sim_set_timing(self._h, 1 if on else 0))

    def kernel_ms(self):
        out, n = np.zeros(2), ctypes.c_int64()
        _check(lib.tyee_tet_sim_kernel_ms(self._h, _ptr(out), ctypes.byref(n)))
        return {"edge_ms": float(out[0]), "face_ms": float(out[1]), "steps": n.value}


class Sim:
    """Device state of one mesh: leap-frog stepping on a HIP stream."""

    def __init__(self, mesh, dt, prec="f32", stream=None):
        h = ctypes.c_void_p()
        _check(lib.tyee_sim_create(mesh._h, PREC[prec], float(dt),
                                   None if stream is None else int(stream), ctypes.byref(h)))
        self._h = h
        self.nv, self.ne, self.nt = mesh.nv, mesh.ne, mesh.nt
        self.prec = prec
        self.dt = float(dt)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_sim_destroy(h)
            self._h = None

    def _n(self, field):
        return {"E": self.ne, "B": self.nt, "J": self.ne, "Q": self.nv}[field]

    def set_state(self, field, values):
        a = _f64(values, self._n(field))
        _check(lib.tyee_sim_set_state(self._h, FIELD[field], _ptr(a)))

    def get_state(self, field):
        out = np.zeros(self._n(field))
        _check(lib.tyee_sim_get_state(self._h, FIELD[field], _ptr(out)))
        return out

    def set_media(self, wp2_tri, nu):
        a = None if wp2_tri is None else _f64(wp2_tri, self.nt)
        _check(lib.tyee_sim_set_media(self._h, _ptr(a), float(nu)))

    def set_source(self, pairs, weights, omega, cycles):
        p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        w = _f64(weights, len(p))
        _check(lib.tyee_sim_set_source(self._h, _ptr(p), _ptr(w), len(p), float(omega),
                                       float(cycles)))

    def set_edge_scale(self, gamma):
        g = None if gamma is None else _f64(gamma, self.ne)
        _check(lib.tyee_sim_set_edge_scale(self._h, _ptr(g)))

    def set_fusion(self, k, tile=0):
        """Steps per launch (1..8; 0 = default) and tile size in triangles (0 = default)."""
        _check(lib.tyee_sim_set_fusion(self._h, int(k), int(tile)))

    def step(self, n):
        _check(lib.tyee_sim_step(self._h, int(n)))

    def sync(self):
        _check(lib.tyee_sim_sync(self._h))

    def last_step_ms(self):
        ms = ctypes.c_double()
        _check(lib.tyee_sim_last_step_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def set_profiling(self, on=True, kinds=None):
        """Time launches with HIP events: all kernel kinds, or the named ones."""
        mask = 0
        if on:
            names = KERNELS if kinds is None else kinds
            for k in names:
                mask |= 1 << KERNELS[k]
        _check(lib.tyee_sim_set_profiling(self._h, mask))

    def kernel_times(self):
        """{kind: {count, total_ms, name, steps_per_launch}} for kinds with timed launches."""
        out = {}
        for name, kind in KERNELS.items():
            c, t = ctypes.c_int64(), ctypes.c_double()
            _check(lib.tyee_sim_kernel_times(self._h, kind, ctypes.byref(c), ctypes.byref(t)))
            if c.value:
                out[name] = {"count": c.value, "total_ms": t.value, "name": KERNEL_NAMES[name],
                             "steps_per_launch": self.fusion_used() if name == "fused" else 1}
        return out

    def bind_external(self, field, buf0, buf1):
        """Use two caller-owned device buffers (torch tensors or raw device addresses) for E or
        B (device numbering, scaled E); None, None unbinds.  Tensors are kept referenced while
        bound."""
        def addr(b):
            if b is None:
                return None
            return int(b.data_ptr()) if hasattr(b, "data_ptr") else int(b)
        _check(lib.tyee_sim_bind_external(self._h, FIELD[field], addr(buf0), addr(buf1)))
        self._bound = getattr(self, "_bound", {})
        self._bound[field] = None if buf0 is None else (buf0, buf1)

    def current_buffer(self):
        """Which of the two field buffers (0 or 1) holds the current state."""
        w = ctypes.c_int32()
        _check(lib.tyee_sim_current_buffer(self._h, ctypes.byref(w)))
        return w.value

    def set_graph(self, launches):
        """Fused launches per captured HIP graph (even; 0 = eager launches)."""
        _check(lib.tyee_sim_set_graph(self._h, int(launches)))
        self.graph_launches = int(launches)

    def fusion_info(self):
        out = np.zeros(6, np.int64)
        _check(lib.tyee_sim_get_fusion(self._h, _ptr(out)))
        return dict(zip(["steps_per_launch", "tile", "tiles", "local_tris", "local_edges",
                         "special_tiles"], (int(v) for v in out)))

    def fusion_used(self):
        return self.fusion_info()["steps_per_launch"]

    def gauss(self):
        """(D E)_k - Q_k per node (canonical)."""
        out = np.zeros(self.nv)
        _check(lib.tyee_sim_gauss(self._h, _ptr(out)))
        return out

    def add_probe(self, field, ids, every, max_samples):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        pid = ctypes.c_int32()
        _check(lib.tyee_sim_add_probe(self._h, FIELD[field], _ptr(ids), len(ids), int(every),
                                      int(max_samples), ctypes.byref(pid)))
        self._probe_sizes = getattr(self, "_probe_sizes", {})
        self._probe_sizes[pid.value] = (len(ids), int(max_samples))
        return pid.value

    def read_probe(self, pid):
        n, cap = self._probe_sizes[pid]
        out = np.zeros((cap, n))
        got = ctypes.c_int64()
        _check(lib.tyee_sim_read_probe(self._h, int(pid), _ptr(out), cap, ctypes.byref(got)))
        return out[:min(cap, got.value)]

    def diagnostics(self):
        d = _Diag()
        _check(lib.tyee_sim_diagnostics(self._h, ctypes.byref(d)), allow=(EUNSTABLE,))
        return {n: getattr(d, n) for n, _ in _Diag._fields_}

    def diagnostics_noalloc(self):
        """The same diagnostics through the entry point that allocates nothing (its tables
        must have been built by one diagnostics() call since the coefficients changed)."""
        d = _Diag()
        _check(lib.tyee_sim_diagnostics_noalloc(self._h, ctypes.byref(d)), allow=(EUNSTABLE,))
        return {n: getattr(d, n) for n, _ in _Diag._fields_}

    @property
    def steps(self):
        return int(lib.tyee_sim_steps(self._h))


class _BorrowedSim(Sim):
    """Sim view of a batch's union (not owned: never destroyed from Python)."""

    def __init__(self, handle, nv, ne, nt, prec):
        self._h = handle
        self.nv, self.ne, self.nt, self.prec = nv, ne, nt, prec

    def __del__(self):
        pass


class Batch:
    """Many independent meshes stepped together in one union (see tyee_batch_create)."""

    def __init__(self, meshes, dts, prec="f32", stream=None):
        arr = (ctypes.c_void_p * len(meshes))(*[m._h.value for m in meshes])
        dt = _f64(dts, len(meshes))
        h = ctypes.c_void_p()
        _check(lib.tyee_batch_create(arr, _ptr(dt), len(meshes), PREC[prec],
                                     None if stream is None else int(stream), ctypes.byref(h)))
        self._h = h
        self.prec = prec
        self.sizes = [(m.nv, m.ne, m.nt) for m in meshes]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_batch_destroy(h)
            self._h = None

    def info(self):
        out = np.zeros(4, np.int64)
        _check(lib.tyee_batch_info(self._h, _ptr(out)))
        return dict(zip(["members", "triangles", "edges", "nodes"], (int(v) for v in out)))

    def sim(self):
        h = ctypes.c_void_p()
        _check(lib.tyee_batch_sim(self._h, ctypes.byref(h)))
        i = self.info()
        return _BorrowedSim(h, i["nodes"], i["edges"], i["triangles"], self.prec)

    def set_state(self, k, field, values):
        n = self.sizes[k][1] if field == "E" else self.sizes[k][2]
        a = _f64(values, n)
        _check(lib.tyee_batch_set_state(self._h, int(k), FIELD[field], _ptr(a)))

    def get_state(self, k, field):
        out = np.zeros(self.sizes[k][1] if field == "E" else self.sizes[k][2])
        _check(lib.tyee_batch_get_state(self._h, int(k), FIELD[field], _ptr(out)))
        return out

    def reorder(self, kind, seed=0):
        _check(lib.tyee_batch_reorder(self._h, ORDER[kind], int(seed)))

    def set_fusion(self, k, tile=0):
        _check(lib.tyee_batch_set_fusion(self._h, int(k), int(tile)))

    def set_graph(self, launches):
        _check(lib.tyee_batch_set_graph(self._h, int(launches)))

    def step(self, n):
        _check(lib.tyee_batch_step(self._h, int(n)))

    def sync(self):
        _check(lib.tyee_batch_sync(self._h))

    def tune(self, steps_per_trial=64, progress=None):
        """Autotune (tyee_batch_tune); progress(dict) is called after every trial."""
        cap = 64
        res = (_Tune * cap)()
        n = ctypes.c_int64()
        names = {v: k for k, v in ORDER.items()}
        rec = lambda r: {"order": names[r.order], "steps_per_launch": r.steps_per_launch,
                         "tile_tris": r.tile_tris, "ms_per_step": r.ms_per_step}
        cb = None
        if progress is not None:
            cb = _TUNE_PROGRESS(lambda r, user: progress(rec(r.contents)))
        _check(lib.tyee_batch_tune_progress(self._h, int(steps_per_trial), res, cap, ctypes.byref(n),
                                            cb, None))
        return [rec(r) for r in res[:min(cap, n.value)]]


class Learner:
    """Training set + MLP of the learned edge scale on the device (tyee_learner_*)."""

    def __init__(self, meshes, dts, waves, phase=2.0, stream=None):
        arr = (ctypes.c_void_p * len(meshes))(*[m._h.value for m in meshes])
        dt = _f64(dts, len(meshes))
        w = np.ascontiguousarray(waves, np.float64)
        if w.ndim != 3 or w.shape[0] != len(meshes) or w.shape[2] != 2:
            raise ValueError("waves must have shape [n_meshes, n_waves, 2]")
        h = ctypes.c_void_p()
        _check(lib.tyee_learner_create(arr, _ptr(dt), len(meshes), _ptr(w), w.shape[1],
                                       float(phase), None if stream is None else int(stream),
                                       ctypes.byref(h)))
        self._h = h
        self.n_meshes, self.n_waves = len(meshes), w.shape[1]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.tyee_learner_destroy(h)
            self._h = None

    def init(self, seed=0):
        _check(lib.tyee_learner_init(self._h, int(seed)))

    def regulariser(self, tau=0.02, beta=1e-3, target=0.9):
        _check(lib.tyee_learner_regulariser(self._h, float(tau), float(beta), float(target)))

    def params(self):
        out = np.zeros(N_PARAMS)
        _check(lib.tyee_learner_get_params(self._h, _ptr(out)))
        return out

    def set_params(self, theta):
        t = _f64(theta, N_PARAMS)
        _check(lib.tyee_learner_set_params(self._h, _ptr(t)))

    def normaliser(self, mu=None, sd=None):
        mi = None if mu is None else _f64(mu, 8)
        si = None if sd is None else _f64(sd, 8)
        mo, so = np.zeros(8), np.zeros(8)
        _check(lib.tyee_learner_normaliser(self._h, _ptr(mi), _ptr(si), _ptr(mo), _ptr(so)))
        return mo, so

    def loss_grad(self, want_grad=True, want_errors=False):
        loss = ctypes.c_double()
        g = np.zeros(N_PARAMS) if want_grad else None
        e = np.zeros((self.n_meshes, self.n_waves)) if want_errors else None
        _check(lib.tyee_learner_loss_grad(self._h, ctypes.byref(loss), _ptr(g), _ptr(e)))
        return loss.value, g, e

    def train(self, iters, lr):
        hist = np.zeros(max(1, int(iters)))
        _check(lib.tyee_learner_train(self._h, int(iters), float(lr), _ptr(hist)))
        return hist[:int(iters)]

    def gamma(self, mesh):
        out = np.zeros(mesh.ne)
        _check(lib.tyee_learner_gamma(self._h, mesh._h, _ptr(out)))
        return out

    def set_batch(self, pairs=None):
        """Active (mesh, wave) pairs [n][2] of the loss (None: all)."""
        if pairs is None or len(pairs) == 0:
            _check(lib.tyee_learner_set_batch(self._h, None, 0))
            return
        p = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        _check(lib.tyee_learner_set_batch(self._h, _ptr(p), len(p)))

    def set_path(self, path):
        """0: automatic; 1: every mesh on the multi-work-group path."""
        _check(lib.tyee_learner_set_path(self._h, int(path)))
