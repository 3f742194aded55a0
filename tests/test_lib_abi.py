"""The C-ABI library loads and exports every entry point its header declares
(no device calls: CPU only)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "cloth.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cloth_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    import paper_2403_19272_amd as P
    names = declared()
    assert "cloth_init" in names and "cloth_step" in names and len(names) >= 15
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(P.EXPORTS) <= set(names)


def test_status_strings_and_footprint_on_host():
    import paper_2403_19272_amd as P
    import scenegen
    assert P.lib.cloth_status_string(P.CLOTH_E_MESH).decode() == "invalid mesh"
    sc = scenegen.config(0)
    tris = np.ascontiguousarray(sc.tris, np.int32)
    mesh = P.Mesh(sc.nv, sc.nt, tris.ctypes.data, None)
    prm = P.SolverParams(16, 20, 1, 0.9, 0.9, 3, 0, 0, 0)
    n = ctypes.c_size_t(0)
    assert P.lib.cloth_query_footprint(ctypes.byref(mesh), ctypes.byref(prm), ctypes.byref(n)) == 0
    assert n.value > sc.nv * 100
    bad = np.array([[0, 1, 99999]], np.int32)
    mesh2 = P.Mesh(3, 1, bad.ctypes.data, None)
    assert P.lib.cloth_query_footprint(ctypes.byref(mesh2), ctypes.byref(prm), ctypes.byref(n)) == P.CLOTH_E_MESH
