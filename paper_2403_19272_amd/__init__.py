"""Python binding of libcloth (include/cloth.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts numpy
arrays and torch device buffers/streams to plain pointers.  Importing it
fails if the library has not been built (python -m paper_2403_19272_amd.build).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcloth.so")

CLOTH_OK = 0
CLOTH_E_INVALID = -1
CLOTH_E_MESH = -2
CLOTH_E_OOM = -3
CLOTH_E_CAPACITY = -4
CLOTH_E_DIVERGED = -5
CLOTH_E_TANGLED = -6
CLOTH_E_DEVICE = -7
CLOTH_PLAIN_FP32 = 0
CLOTH_MIXED = 1
CLOTH_SPHERE = 0
CLOTH_CYLINDER = 1

EXPORTS = [
    "cloth_status_string", "cloth_last_error", "cloth_query_footprint", "cloth_init",
    "cloth_system_matrix", "cloth_set_basis", "cloth_add_obstacle", "cloth_set_state",
    "cloth_get_state", "cloth_step", "cloth_step_n", "cloth_destroy", "cloth_stage_broad_phase",
    "cloth_stage_toi", "cloth_stage_load_block", "cloth_stage_inner", "cloth_stage_partial_ccd",
    "cloth_stage_read_block", "cloth_set_timing", "cloth_kernel_times", "cloth_set_graph",
    "cloth_stage_outer", "cloth_stage_read_set", "cloth_step_batch", "cloth_server_create",
    "cloth_server_admit", "cloth_server_release", "cloth_server_submit", "cloth_server_poll",
    "cloth_server_wait", "cloth_server_destroy", "cloth_compute_basis", "cloth_set_step_options",
    "cloth_get_forwarded", "cloth_compute_basis_static", "cloth_set_warm_basis", "cloth_batch_create",
    "cloth_batch_step", "cloth_batch_destroy", "cloth_autotune", "cloth_set_tuning", "cloth_server_info",
    "cloth_vertex_order",
]


class Mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("tris", C.c_void_p), ("pinned", C.c_void_p)]


class Material(C.Structure):
    _fields_ = [("density", C.c_double), ("k_stretch", C.c_double), ("k_bend", C.c_double),
                ("sigma_min", C.c_double), ("sigma_max", C.c_double),
                ("k_contact", C.c_double), ("K_base", C.c_double), ("a_max", C.c_int32),
                ("d_hat", C.c_double), ("alpha", C.c_double), ("friction", C.c_double),
                ("friction_eps_v", C.c_double)]


class SolverParams(C.Structure):
    _fields_ = [("r", C.c_int32), ("iters_inner", C.c_int32), ("iters_outer", C.c_int32),
                ("tol_inner", C.c_double), ("tol_outer", C.c_double),
                ("cheb_rho", C.c_double), ("cheb_gamma", C.c_double), ("cheb_delay", C.c_int32),
                ("precision", C.c_int32), ("self_contact", C.c_int32), ("pair_capacity", C.c_int64),
                ("debug_tangles", C.c_int32), ("broad_margin", C.c_double),
                ("broad_margin_motion", C.c_double), ("r_warm", C.c_int32), ("broad_reuse", C.c_int32),
                ("uu_store", C.c_int32), ("reorder", C.c_int32), ("smoother", C.c_int32),
                ("adaptive_samples", C.c_int32)]


class Obstacle(C.Structure):
    _fields_ = [("kind", C.c_int32), ("center", C.c_double * 3), ("axis", C.c_double * 3),
                ("radius", C.c_double), ("half_length", C.c_double), ("omega", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("query_lanes", C.c_int32), ("broad_reuse", C.c_int32), ("broad_margin", C.c_double),
                ("broad_margin_motion", C.c_double), ("ms_per_step", C.c_double), ("ms_default", C.c_double),
                ("cheb_rho", C.c_double), ("cheb_gamma", C.c_double), ("trials", C.c_int32),
                ("from_cache", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepStats(C.Structure):
    _fields_ = [("inner_iters", C.c_int32), ("outer_iters", C.c_int32),
                ("n_candidates", C.c_int64), ("n_constraints", C.c_int64),
                ("dx_norm", C.c_double), ("outer_dx", C.c_double), ("min_toi", C.c_double),
                ("cheb_rho", C.c_double),
                ("cheb_gamma", C.c_double), ("peak_candidates", C.c_int64),
                ("n_contact_vertices", C.c_int64), ("n_factorizations", C.c_int64),
                ("n_broad_rebuilds", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcloth.so not built at {LIB_PATH}; run python paper_2403_19272_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    sig = {
        "cloth_status_string": (C.c_char_p, [i32]),
        "cloth_last_error": (C.c_char_p, []),
        "cloth_query_footprint": (i32, [C.POINTER(Mesh), C.POINTER(SolverParams), C.POINTER(C.c_size_t)]),
        "cloth_vertex_order": (i32, [C.POINTER(Mesh), C.POINTER(i32)]),
        "cloth_init": (i32, [C.POINTER(Mesh), P, C.POINTER(Material), f64, C.POINTER(SolverParams), P,
                             C.c_size_t, C.POINTER(P)]),
        "cloth_system_matrix": (i32, [P, C.POINTER(i64), P, P, P]),
        "cloth_set_basis": (i32, [P, P, i32]),
        "cloth_set_warm_basis": (i32, [P, P, i32]),
        "cloth_batch_create": (i32, [P, i32, P, C.POINTER(P)]),
        "cloth_batch_step": (i32, [P, i32, P]),
        "cloth_batch_destroy": (i32, [P]),
        "cloth_autotune": (i32, [P, P, i32, i32, P, C.POINTER(Tuning)]),
        "cloth_set_tuning": (i32, [P, C.POINTER(Tuning)]),
        "cloth_add_obstacle": (i32, [P, C.POINTER(Obstacle)]),
        "cloth_set_state": (i32, [P, P, P, P]),
        "cloth_get_state": (i32, [P, P, P, P]),
        "cloth_step": (i32, [P, P, P, C.POINTER(StepStats)]),
        "cloth_step_n": (i32, [P, P, i32, P, C.POINTER(StepStats)]),
        "cloth_destroy": (i32, [P]),
        "cloth_stage_broad_phase": (i32, [P, P, P, i64, P, C.POINTER(i64), P, C.POINTER(i64)]),
        "cloth_stage_toi": (i32, [P, P, P, i64, P, i64, P, P, P]),
        "cloth_stage_load_block": (i32, [P, P, P, P, P, i64, P, P, i64, P, P, P]),
        "cloth_stage_inner": (i32, [P, i32]),
        "cloth_stage_partial_ccd": (i32, [P, P]),
        "cloth_set_timing": (i32, [P, i32]),
        "cloth_set_graph": (i32, [P, i32]),
        "cloth_stage_outer": (i32, [P, P, P, i32, P, C.POINTER(f64)]),
        "cloth_stage_read_set": (i32, [P, i64, P, P, C.POINTER(i64), P, P, C.POINTER(i64), P]),
        "cloth_step_batch": (i32, [P, i32, P, P, P]),
        "cloth_server_create": (i32, [i32, C.c_size_t, C.POINTER(P)]),
        "cloth_server_admit": (i32, [P, P, C.POINTER(i32)]),
        "cloth_server_release": (i32, [P, P]),
        "cloth_server_submit": (i32, [P, P, P, C.POINTER(i64)]),
        "cloth_server_poll": (i32, [P, i64, C.POINTER(i32), C.POINTER(f64), C.POINTER(f64)]),
        "cloth_server_wait": (i32, [P, i64, C.POINTER(f64), C.POINTER(f64)]),
        "cloth_server_destroy": (i32, [P]),
        "cloth_server_info": (i32, [P, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_size_t), C.POINTER(i64)]),
        "cloth_compute_basis": (i32, [P, i32, i32, i32, f64, P, P, C.POINTER(i32), C.POINTER(f64)]),
        "cloth_compute_basis_static": (i32, [P, i32, i32, i32, f64, P, P, C.POINTER(i32), C.POINTER(f64)]),
        "cloth_set_step_options": (i32, [P, i32, i32, f64]),
        "cloth_get_forwarded": (i32, [P, P]),
        "cloth_kernel_times": (i32, [P, i32, P, P, P, C.POINTER(i32)]),
        "cloth_stage_read_block": (i32, [P, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


class ClothError(RuntimeError):
    def __init__(self, code, where):
        msg = lib.cloth_last_error().decode()
        super().__init__(f"{where}: {lib.cloth_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code, where):
    if code != CLOTH_OK:
        raise ClothError(code, where)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1, 3))


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def vertex_order(tris, nv):
    """Reverse Cuthill-McKee order of a mesh's vertices (cloth_vertex_order):
    entry i is the vertex placed at position i."""
    t = np.ascontiguousarray(tris, np.int32)
    mesh = Mesh(nv, t.shape[0], t.ctypes.data, None)
    out = np.empty(nv, np.int32)
    _check(lib.cloth_vertex_order(C.byref(mesh), out.ctypes.data_as(C.POINTER(C.c_int32))), "cloth_vertex_order")
    return out


class ClothScene:
    """One cloth scene resident on the device."""

    def __init__(self, tris, rest, *, dt, density=0.3, k_stretch=160.0, k_bend=3e-4,
                 sigma_min=1.0, sigma_max=1.0, k_contact=0.0, K_base=2.0, a_max=20, d_hat=1e-3,
                 alpha=0.8, pinned=None, r=16, iters_inner=10, iters_outer=1, tol_inner=0.0,
                 tol_outer=0.0, cheb_rho=0.0, cheb_gamma=0.0, cheb_delay=3,
                 precision=CLOTH_PLAIN_FP32, self_contact=False, pair_capacity=0,
                 debug_tangles=False, broad_margin=0.0, broad_margin_motion=0.0, r_warm=0,
                 broad_reuse=False, uu_store=False, reorder=False, friction=0.0, friction_eps_v=0.0,
                 smoother=0, adaptive_samples=False, arena=None):
        self._tris = np.ascontiguousarray(tris, np.int32)
        rest = _f32(rest)
        nv = rest.shape[0]
        self.nv = nv
        self._pinned = None if pinned is None else np.ascontiguousarray(pinned, np.uint8)
        self.mesh = Mesh(nv, self._tris.shape[0], self._tris.ctypes.data, None if self._pinned is None
                         else self._pinned.ctypes.data)
        self.mat = Material(density, k_stretch, k_bend, sigma_min, sigma_max, k_contact, K_base, a_max,
                            d_hat, alpha, friction, friction_eps_v)
        self.params = SolverParams(r, iters_inner, iters_outer, tol_inner, tol_outer, cheb_rho,
                                   cheb_gamma, cheb_delay, precision, int(bool(self_contact)),
                                   pair_capacity, int(bool(debug_tangles)), broad_margin,
                                   broad_margin_motion, r_warm, int(bool(broad_reuse)),
                                   int(bool(uu_store)), int(bool(reorder)), int(smoother),
                                   int(bool(adaptive_samples)))
        self.r = r
        self.r_warm = r_warm
        nbytes = C.c_size_t(0)
        _check(lib.cloth_query_footprint(C.byref(self.mesh), C.byref(self.params), C.byref(nbytes)),
               "cloth_query_footprint")
        self.footprint = nbytes.value
        self._arena = None
        aptr, asize = None, 0
        if arena == "torch":
            import torch
            self._arena = torch.empty(self.footprint, dtype=torch.uint8, device="cuda")
            aptr, asize = C.c_void_p(self._arena.data_ptr()), self.footprint
        self._h = C.c_void_p()
        _check(lib.cloth_init(C.byref(self.mesh), _ptr(rest), C.byref(self.mat), dt,
                              C.byref(self.params), aptr, asize, C.byref(self._h)), "cloth_init")

    # ---- setup
    def system_matrix(self):
        import scipy.sparse as sp
        nnz = C.c_int64(0)
        _check(lib.cloth_system_matrix(self._h, C.byref(nnz), None, None, None), "cloth_system_matrix")
        rp = np.empty(self.nv + 1, np.int32)
        col = np.empty(nnz.value, np.int32)
        val = np.empty(nnz.value, np.float64)
        _check(lib.cloth_system_matrix(self._h, C.byref(nnz), _ptr(rp), _ptr(col), _ptr(val)),
               "cloth_system_matrix")
        return sp.csr_matrix((val, col, rp), shape=(self.nv, self.nv))

    def set_basis(self, U: np.ndarray):
        U = np.ascontiguousarray(U, np.float64)
        _check(lib.cloth_set_basis(self._h, _ptr(U), U.shape[1]), "cloth_set_basis")

    def set_warm_basis(self, U):
        """The modal warm start's own basis (nv x r_warm)."""
        U = np.ascontiguousarray(U, np.float64)
        _check(lib.cloth_set_warm_basis(self._h, _ptr(U), U.shape[1]), "cloth_set_warm_basis")

    def autotune(self, gravity=(0.0, -9.8, 0.0), steps=5, force=False, stream=None):
        """Picks the launch settings that leave results unchanged by timing
        trials from the current state (see cloth_autotune)."""
        g = np.asarray(gravity, np.float32)
        t = Tuning()
        _check(lib.cloth_autotune(self._h, _ptr(g), steps, int(bool(force)), _stream(stream), C.byref(t)),
               "cloth_autotune")
        return t.as_dict()

    def set_tuning(self, query_lanes=8, broad_reuse=False, broad_margin=0.0, broad_margin_motion=0.0):
        t = Tuning(query_lanes, int(bool(broad_reuse)), broad_margin, broad_margin_motion, 0.0, 0.0, 0.0, 0.0, 0, 0)
        _check(lib.cloth_set_tuning(self._h, C.byref(t)), "cloth_set_tuning")

    def compute_basis(self, degree=300, max_passes=12, tol=2e-2, return_basis=False, static=False):
        """Device eigenbasis (Chebyshev-filtered subspace iteration), then set.
        static: use the entry point that allocates no device memory."""
        U = np.empty((self.nv, self.r)) if return_basis else None
        w = np.empty(self.r)
        npass = C.c_int32(0)
        res = C.c_double(0)
        name = "cloth_compute_basis_static" if static else "cloth_compute_basis"
        _check(getattr(lib, name)(self._h, self.r, degree, max_passes, tol, _ptr(U), _ptr(w),
                                  C.byref(npass), C.byref(res)), name)
        return dict(U=U, ritz=w, passes=npass.value, residual=res.value)

    def add_obstacle(self, kind, center, radius, axis=(1.0, 0.0, 0.0), half_length=0.0, omega=0.0):
        ob = Obstacle(kind, (C.c_double * 3)(*center), (C.c_double * 3)(*axis), radius,
                      half_length, omega)
        _check(lib.cloth_add_obstacle(self._h, C.byref(ob)), "cloth_add_obstacle")

    # ---- state
    def set_state(self, x, v=None, stream=None):
        x = _f32(x)
        v = None if v is None else _f32(v)
        _check(lib.cloth_set_state(self._h, _ptr(x), _ptr(v), _stream(stream)), "cloth_set_state")

    def get_state(self, stream=None):
        x = np.empty((self.nv, 3), np.float32)
        v = np.empty((self.nv, 3), np.float32)
        _check(lib.cloth_get_state(self._h, _ptr(x), _ptr(v), _stream(stream)), "cloth_get_state")
        return x, v

    def step(self, gravity=(0.0, -9.8, 0.0), n=1, stream=None, stats=True):
        g = np.asarray(gravity, np.float32)
        st = StepStats()
        _check(lib.cloth_step_n(self._h, _ptr(g), n, _stream(stream), C.byref(st) if stats else None),
               "cloth_step_n")
        return st.as_dict() if stats else None

    def set_step_options(self, warm_iters=0, rf_iters=0, rf_toi=0.5):
        _check(lib.cloth_set_step_options(self._h, warm_iters, rf_iters, rf_toi), "cloth_set_step_options")

    def forwarded(self):
        dx = np.empty((self.nv, 3), np.float32)
        _check(lib.cloth_get_forwarded(self._h, _ptr(dx)), "cloth_get_forwarded")
        return dx

    def set_graph(self, on: bool):
        _check(lib.cloth_set_graph(self._h, int(bool(on))), "cloth_set_graph")

    # ---- timing
    def set_timing(self, on: bool):
        _check(lib.cloth_set_timing(self._h, int(bool(on))), "cloth_set_timing")

    def kernel_times(self):
        """{kernel name: (total ms, launches)} since timing was switched on."""
        n = C.c_int32(0)
        names = C.create_string_buffer(32 * 32)
        ms = np.zeros(32)
        cnt = np.zeros(32, np.int64)
        _check(lib.cloth_kernel_times(self._h, 32, names, _ptr(ms), _ptr(cnt), C.byref(n)),
               "cloth_kernel_times")
        raw = names.raw
        out = {}
        for i in range(n.value):
            name = raw[32 * i:32 * i + 32].split(b"\0")[0].decode()
            out[name] = (float(ms[i]), int(cnt[i]))
        return out

    # ---- stages
    def stage_broad_phase(self, xm, xp, cap=None):
        xm, xp = _f32(xm), _f32(xp)
        cap = cap or max(1024, 64 * self.nv)
        vt = np.empty((cap, 2), np.int32)
        ee = np.empty((cap, 2), np.int32)
        nvt, nee = C.c_int64(0), C.c_int64(0)
        _check(lib.cloth_stage_broad_phase(self._h, _ptr(xm), _ptr(xp), cap, _ptr(vt), C.byref(nvt),
                                           _ptr(ee), C.byref(nee)), "cloth_stage_broad_phase")
        return vt[:nvt.value].copy(), ee[:nee.value].copy()

    def stage_toi(self, xm, xp, vt, ee):
        xm, xp = _f32(xm), _f32(xp)
        vt = np.ascontiguousarray(vt, np.int32).reshape(-1, 2)
        ee = np.ascontiguousarray(ee, np.int32).reshape(-1, 2)
        tv = np.empty(len(vt))
        te = np.empty(len(ee))
        _check(lib.cloth_stage_toi(self._h, _ptr(xm), _ptr(xp), len(vt), _ptr(vt), len(ee), _ptr(ee),
                                   _ptr(tv), _ptr(te)), "cloth_stage_toi")
        return tv, te

    def stage_load_block(self, xm, xk, xkm1, z, vt=None, a_vt=None, ee=None, a_ee=None, ob_a=None):
        vt = np.zeros((0, 2), np.int32) if vt is None else np.ascontiguousarray(vt, np.int32)
        ee = np.zeros((0, 2), np.int32) if ee is None else np.ascontiguousarray(ee, np.int32)
        a_vt = np.zeros(len(vt), np.int32) if a_vt is None else np.ascontiguousarray(a_vt, np.int32)
        a_ee = np.zeros(len(ee), np.int32) if a_ee is None else np.ascontiguousarray(a_ee, np.int32)
        ob = None if ob_a is None else np.ascontiguousarray(ob_a, np.int32)
        self._keep = (vt, ee, a_vt, a_ee, ob)
        _check(lib.cloth_stage_load_block(self._h, _ptr(_f32(xm)), _ptr(_f32(xk)), _ptr(_f32(xkm1)),
                                          _ptr(_f32(z)), len(vt), _ptr(vt), _ptr(a_vt), len(ee),
                                          _ptr(ee), _ptr(a_ee), _ptr(ob)), "cloth_stage_load_block")
        self._nvt, self._nee = len(vt), len(ee)

    def stage_inner(self, k):
        _check(lib.cloth_stage_inner(self._h, k), "cloth_stage_inner")

    def stage_outer(self, xm, xp, first=False):
        x = np.empty((self.nv, 3), np.float32)
        s = C.c_double(0)
        _check(lib.cloth_stage_outer(self._h, _ptr(_f32(xm)), _ptr(_f32(xp)), int(bool(first)), _ptr(x),
                                     C.byref(s)), "cloth_stage_outer")
        return x, s.value

    def stage_read_set(self, nob=0, cap=None):
        cap = cap or max(1024, 32 * self.nv)
        vt = np.empty((cap, 2), np.int32)
        ee = np.empty((cap, 2), np.int32)
        avt = np.empty(cap, np.int32)
        aee = np.empty(cap, np.int32)
        ob = np.empty(max(nob, 1) * self.nv, np.int32)
        nvt, nee = C.c_int64(0), C.c_int64(0)
        _check(lib.cloth_stage_read_set(self._h, cap, _ptr(vt), _ptr(avt), C.byref(nvt), _ptr(ee), _ptr(aee),
                                        C.byref(nee), _ptr(ob)), "cloth_stage_read_set")
        self._nvt, self._nee = nvt.value, nee.value
        return dict(vt=vt[:nvt.value].copy(), a_vt=avt[:nvt.value].copy(), ee=ee[:nee.value].copy(),
                    a_ee=aee[:nee.value].copy(), ob_a=ob[:nob * self.nv].reshape(nob, self.nv).copy())

    def stage_partial_ccd(self, xnew):
        _check(lib.cloth_stage_partial_ccd(self._h, _ptr(_f32(xnew))), "cloth_stage_partial_ccd")

    def stage_read_block(self, nob=0):
        xk = np.empty((self.nv, 3), np.float32)
        b = np.empty((self.nv, 3), np.float32)
        a_vt = np.empty(self._nvt, np.int32)
        a_ee = np.empty(self._nee, np.int32)
        ob = np.empty(max(nob, 1) * self.nv, np.int32)
        dx = C.c_double(0)
        Q = np.empty((self.r, 3))
        _check(lib.cloth_stage_read_block(self._h, _ptr(xk), _ptr(a_vt), _ptr(a_ee), _ptr(ob),
                                          C.byref(dx), _ptr(b), _ptr(Q)), "cloth_stage_read_block")
        return dict(xk=xk, a_vt=a_vt, a_ee=a_ee, ob_a=ob[:nob * self.nv].reshape(nob, self.nv),
                    dx=dx.value, b=b, Q=Q)

    def close(self):
        if self._h:
            lib.cloth_destroy(self._h)
            self._h = C.c_void_p()
        self._arena = None   # a torch-owned arena goes back to the caching allocator

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(scenes, gravity=(0.0, -9.8, 0.0), stream=None, stats=True):
    """One step of every scene in `scenes`, overlapping on the device."""
    n = len(scenes)
    hs = (C.c_void_p * n)(*[sc._h.value for sc in scenes])
    g = np.asarray(gravity, np.float32)
    st = (StepStats * n)()
    _check(lib.cloth_step_batch(hs, n, _ptr(g), _stream(stream), st if stats else None),
           "cloth_step_batch")
    return [s.as_dict() for s in st] if stats else None


class BatchGraph:
    """Every scene's step as one graph launch (see cloth_batch_* in cloth.h)."""

    def __init__(self, scenes, gravity=(0.0, -9.8, 0.0)):
        self.scenes = list(scenes)
        n = len(self.scenes)
        hs = (C.c_void_p * n)(*[sc._h.value for sc in self.scenes])
        g = np.asarray(gravity, np.float32)
        self._h = C.c_void_p()
        _check(lib.cloth_batch_create(hs, n, _ptr(g), C.byref(self._h)), "cloth_batch_create")

    def step(self, steps=1, stream=None):
        _check(lib.cloth_batch_step(self._h, steps, _stream(stream)), "cloth_batch_step")

    def close(self):
        if self._h:
            lib.cloth_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StepServer:
    """Continuous-batching step server (see cloth_server_* in cloth.h)."""

    def __init__(self, slots=8, hbm_budget=0):
        self._h = C.c_void_p()
        _check(lib.cloth_server_create(slots, hbm_budget, C.byref(self._h)), "cloth_server_create")

    def admit(self, scene) -> bool:
        ok = C.c_int32(0)
        _check(lib.cloth_server_admit(self._h, scene._h, C.byref(ok)), "cloth_server_admit")
        return bool(ok.value)

    def release(self, scene):
        _check(lib.cloth_server_release(self._h, scene._h), "cloth_server_release")

    def submit(self, scene, gravity=(0.0, -9.8, 0.0)) -> int:
        g = np.asarray(gravity, np.float32)
        t = C.c_int64(0)
        _check(lib.cloth_server_submit(self._h, scene._h, _ptr(g), C.byref(t)), "cloth_server_submit")
        return t.value

    def poll(self, ticket):
        done = C.c_int32(0)
        lat, svc = C.c_double(0), C.c_double(0)
        _check(lib.cloth_server_poll(self._h, ticket, C.byref(done), C.byref(lat), C.byref(svc)),
               "cloth_server_poll")
        return (lat.value, svc.value) if done.value else None

    def wait(self, ticket):
        lat, svc = C.c_double(0), C.c_double(0)
        _check(lib.cloth_server_wait(self._h, ticket, C.byref(lat), C.byref(svc)), "cloth_server_wait")
        return lat.value, svc.value

    def info(self):
        """(admitted scenes, waiting scenes, admitted footprint bytes, releases
        made to admit waiting scenes)."""
        na, nw = C.c_int32(0), C.c_int32(0)
        used, ev = C.c_size_t(0), C.c_int64(0)
        _check(lib.cloth_server_info(self._h, C.byref(na), C.byref(nw), C.byref(used), C.byref(ev)),
               "cloth_server_info")
        return na.value, nw.value, used.value, ev.value

    def close(self):
        if self._h:
            lib.cloth_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
