"""Builds and loads the oracle's plain-C geometry (geom.c) through ctypes.

Test infrastructure only: nothing in the library imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "geom.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libogeom.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile geom.c with gcc (-O2, no fast-math, no FP contraction)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.og_broad_phase.restype = C.c_int
        L.og_broad_phase.argtypes = [C.c_int, P, P, C.c_int, P, C.c_int, P, C.c_float, C.c_int,
                                     C.c_long, P, P, C.c_long, P, P]
        L.og_toi_pairs.restype = None
        L.og_toi_pairs.argtypes = [P, P, P, P, C.c_long, P, C.c_long, P, P, P, P]
        L.og_toi_vt.restype = C.c_double
        L.og_toi_vt.argtypes = [P, P, P]
        L.og_toi_ee.restype = C.c_double
        L.og_toi_ee.argtypes = [P, P, P]
        L.og_frozen_vt.restype = None
        L.og_frozen_vt.argtypes = [P, P, C.c_long, P, P, P]
        L.og_frozen_ee.restype = None
        L.og_frozen_ee.argtypes = [P, P, C.c_long, P, P, P]
        L.og_tangles.restype = C.c_long
        L.og_tangles.argtypes = [C.c_int, P, C.c_int, P, C.c_long, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def broad_phase(xm32, xp32, edges, tris, dhat, self_contact=True, cap=None):
    """Sorted VT (v, t) and EE (e1 < e2) candidate pairs: swept FP32 boxes grown
    by dhat overlap, no shared vertex."""
    L = lib()
    xm32 = np.ascontiguousarray(xm32, np.float32)
    xp32 = np.ascontiguousarray(xp32, np.float32)
    edges = np.ascontiguousarray(edges, np.int32)
    tris = np.ascontiguousarray(tris, np.int32)
    nv = xm32.shape[0]
    cap = cap or max(1024, 64 * nv)
    while True:
        vt = np.empty((cap, 2), np.int32)
        ee = np.empty((cap, 2), np.int32)
        nvt = C.c_long(0)
        nee = C.c_long(0)
        rc = L.og_broad_phase(nv, _p(xm32), _p(xp32), edges.shape[0], _p(edges), tris.shape[0],
                              _p(tris), C.c_float(np.float32(dhat)), int(bool(self_contact)),
                              cap, _p(vt), C.byref(nvt), cap, _p(ee), C.byref(nee))
        if rc == 0:
            return vt[:nvt.value].copy(), ee[:nee.value].copy()
        cap = max(nvt.value, nee.value) + 16


def toi_pairs(xm, xp, tris, edges, vt, ee):
    """FP64 time of impact (2.0 = no hit) for each VT and EE pair."""
    L = lib()
    xm = np.ascontiguousarray(xm, np.float64)
    xp = np.ascontiguousarray(xp, np.float64)
    vt = np.ascontiguousarray(vt, np.int32).reshape(-1, 2)
    ee = np.ascontiguousarray(ee, np.int32).reshape(-1, 2)
    tv = np.empty(vt.shape[0])
    te = np.empty(ee.shape[0])
    nf = C.c_long(0)
    L.og_toi_pairs(_p(xm), _p(xp), _p(np.ascontiguousarray(tris, np.int32)),
                   _p(np.ascontiguousarray(edges, np.int32)), vt.shape[0], _p(vt), ee.shape[0],
                   _p(ee), _p(tv), _p(te), C.byref(nf))
    return tv, te, int(nf.value)


def toi_vt(p0: np.ndarray, p1: np.ndarray):
    """TOI of one VT pair: rows (vertex, a, b, c) at t=0 and t=1."""
    fb = C.c_int(0)
    t = lib().og_toi_vt(_p(np.ascontiguousarray(p0, np.float64)),
                        _p(np.ascontiguousarray(p1, np.float64)), C.byref(fb))
    return t, fb.value


def toi_ee(p0: np.ndarray, p1: np.ndarray):
    """TOI of one EE pair: rows (p1, p2, p3, p4) at t=0 and t=1."""
    fb = C.c_int(0)
    t = lib().og_toi_ee(_p(np.ascontiguousarray(p0, np.float64)),
                        _p(np.ascontiguousarray(p1, np.float64)), C.byref(fb))
    return t, fb.value


def frozen_vt(xm, tris, vt):
    vt = np.ascontiguousarray(vt, np.int32).reshape(-1, 2)
    lam = np.empty((vt.shape[0], 2))
    nrm = np.empty((vt.shape[0], 3))
    lib().og_frozen_vt(_p(np.ascontiguousarray(xm, np.float64)),
                       _p(np.ascontiguousarray(tris, np.int32)), vt.shape[0], _p(vt), _p(lam),
                       _p(nrm))
    return lam, nrm


def frozen_ee(xm, edges, ee):
    ee = np.ascontiguousarray(ee, np.int32).reshape(-1, 2)
    lam = np.empty((ee.shape[0], 2))
    nrm = np.empty((ee.shape[0], 3))
    lib().og_frozen_ee(_p(np.ascontiguousarray(xm, np.float64)),
                       _p(np.ascontiguousarray(edges, np.int32)), ee.shape[0], _p(ee), _p(lam),
                       _p(nrm))
    return lam, nrm


def tangles(x32, tris, cap=4096):
    """(certain intersections, undecided pairs, first intersecting pair)."""
    x32 = np.ascontiguousarray(x32, np.float32)
    tris = np.ascontiguousarray(tris, np.int32)
    und = np.empty((cap, 2), np.int32)
    nund = C.c_long(0)
    first = np.empty(2, np.int32)
    hits = lib().og_tangles(x32.shape[0], _p(x32), tris.shape[0], _p(tris), cap, _p(und),
                            C.byref(nund), _p(first))
    return int(hits), und[:min(cap, nund.value)].copy(), int(nund.value), tuple(first)
