"""Host-side checks of the C-ABI library that need no GPU: it loads, it
exports every function include/dg.h declares, and argument validation in
dg_create rejects bad input before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:int|const char\s*\*)\s+(dg_\w+)\s*\(", txt, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2407_19169_amd as dg

    lib = C.CDLL(dg.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 15
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert set(dg.EXPORTED) <= declared | {"dg_strerror"}


def test_strerror_codes():
    import paper_2407_19169_amd as dg

    assert dg.dg_strerror(0) == "ok"
    for code in range(-6, 0):
        assert dg.dg_strerror(code) != "unknown error"


@pytest.mark.parametrize("case", ["degree", "cells", "domain", "bc_pair", "reflect_scalar",
                                  "quad", "cfl", "dim"])
def test_create_rejects_bad_arguments(case):
    import paper_2407_19169_amd as dg

    mesh = dg.make_mesh(1, (10,), (0.0,), (1.0,), (0, 0))
    opt = dg.make_options()
    deg, eq = 2, dg.DG_EQ_BURGERS
    want = dg.DG_ERR_ARG
    if case == "degree":
        deg, want = 4, dg.DG_ERR_UNSUPPORTED
    elif case == "cells":
        mesh.n[0] = 0
    elif case == "domain":
        mesh.hi[0] = -1.0
    elif case == "bc_pair":
        mesh.bc[1] = dg.DG_BC_OUTFLOW
    elif case == "reflect_scalar":
        mesh.bc[0] = mesh.bc[1] = dg.DG_BC_REFLECT
    elif case == "quad":
        opt.quad_points, want = 5, dg.DG_ERR_UNSUPPORTED
    elif case == "cfl":
        opt.cfl = 0.0
    elif case == "dim":
        mesh.dim = 3
    h = C.c_void_p()
    rc = dg._lib.dg_create(C.byref(mesh), deg, eq, C.byref(opt), C.byref(h))
    assert rc == want
    assert not h.value
