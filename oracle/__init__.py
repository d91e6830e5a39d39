"""FP64 CPU oracle for the RKDG scheme with the jump filter (arXiv:2407.19169).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; the product package
never does.  It shares no code with the GPU library: its C source
(``dgref.c``) builds its own Legendre and Gauss tables, and the only thing the
two sides have in common is the seeded input generator in ``dg_inputs``.

The ctypes layer below only marshals numpy arrays into ``libdgref.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdgref.so")
_dp = C.POINTER(C.c_double)

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, OUTFLOW, REFLECT, DIRICHLET = 0, 1, 2, 3
FILTER_NONE, FILTER_JUMP, FILTER_HYBRID = 0, 1, 2
FLUX_LLF, FLUX_HLL, FLUX_HLLC = 0, 1, 2


_SOURCES = ("dgref.c", "dgref2d.c", "dgref_hll.c")


def build(force: bool = True, out: str | None = None, opt: tuple = ("-O2",)) -> str:
    """Compile the oracle's C sources with gcc into ``libdgref.so`` (FP64,
    OpenMP; ISO C11, so no floating-point contraction).  ``out``/``opt``: a
    copy at another path with other optimisation flags (the CPU-baseline
    timing builds one with -O3 -march=native on the host that runs it)."""
    path = out or _LIB_PATH
    if force or not os.path.exists(path):
        cmd = ["gcc", *opt, "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-o", path + ".tmp", *(os.path.join(_HERE, f) for f in _SOURCES), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)
    return path


def load_copy(path: str):
    """Load a separately built copy of the oracle (see build(out=...)) and
    set up its return types; for timing only."""
    L = C.CDLL(path)
    L.dgref_max_wavespeed1d.restype = C.c_double
    L.dgref_max_wavespeed1d.argtypes = [C.POINTER(Problem1D), _dp]
    L.dgref_max_wavespeed2d.restype = C.c_double
    return L


class Problem1D(C.Structure):
    _fields_ = [("eq", C.c_int), ("k", C.c_int), ("nq", C.c_int), ("filter", C.c_int),
                ("filter_dt", C.c_int), ("bc", C.c_int * 2), ("n", C.c_int64),
                ("lo", C.c_double), ("hi", C.c_double), ("gamma", C.c_double),
                ("adv_speed", C.c_double), ("cfl", C.c_double),
                ("dirichlet", (C.c_double * 3) * 2), ("pp", C.c_int), ("flux", C.c_int)]


class Problem2D(C.Structure):
    _fields_ = [("eq", C.c_int), ("k", C.c_int), ("nq", C.c_int), ("filter", C.c_int),
                ("filter_dt", C.c_int), ("bc", C.c_int * 4), ("nx", C.c_int64),
                ("ny", C.c_int64), ("xlo", C.c_double), ("xhi", C.c_double),
                ("ylo", C.c_double), ("yhi", C.c_double), ("gamma", C.c_double),
                ("adv_speed", C.c_double * 2), ("cfl", C.c_double),
                ("dirichlet", (C.c_double * 4) * 4), ("shock_x0", C.c_double),
                ("shock_speed", C.c_double), ("post", C.c_double * 4), ("pre", C.c_double * 4),
                ("cf_reading", C.c_int), ("basis", C.c_int), ("flux", C.c_int),
                ("pp", C.c_int)]


class Report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("ledger", C.c_double * 4),
                ("boundary_flux", C.c_double * 4), ("troubled_cells", C.c_int64),
                ("min_rho", C.c_double), ("min_p", C.c_double),
                ("max_exponent", C.c_double), ("status", C.c_int),
                ("first_bad_cell", C.c_int64), ("restarts", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.dgref_legendre_deriv.restype = C.c_double
        L.dgref_legendre_deriv.argtypes = [C.c_int, C.c_int, C.c_double]
        L.dgref_gauss.argtypes = [C.c_int, _dp, _dp]
        L.dgref_max_wavespeed1d.restype = C.c_double
        L.dgref_max_wavespeed1d.argtypes = [C.POINTER(Problem1D), _dp]
        for name in ("dgref_max_wavespeed2d",):
            if hasattr(L, name):
                getattr(L, name).restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def nvars(eq: int, dim: int = 1) -> int:
    return (3 if dim == 1 else 4) if eq == EULER else 1


def problem1d(eq, k, n, lo, hi, bc=(PERIODIC, PERIODIC), filter=FILTER_JUMP, cfl=0.1,
              gamma=1.4, adv_speed=1.0, nq=0, filter_dt=0, dirichlet=None, pp=0,
              flux=0) -> Problem1D:
    P = Problem1D()
    P.pp = pp
    P.flux = flux
    P.eq, P.k, P.nq, P.filter, P.filter_dt = eq, k, nq, filter, filter_dt
    P.bc[0], P.bc[1] = bc
    P.n, P.lo, P.hi, P.gamma, P.adv_speed, P.cfl = n, lo, hi, gamma, adv_speed, cfl
    if dirichlet is not None:
        for s in range(2):
            for v in range(3):
                P.dirichlet[s][v] = float(dirichlet[s][v]) if v < len(dirichlet[s]) else 0.0
    return P


def problem2d(eq, k, nx, ny, xlo, xhi, ylo, yhi, bc=(PERIODIC,) * 4, filter=FILTER_JUMP,
              cfl=0.1, gamma=1.4, adv_speed=(1.0, 1.0), nq=0, filter_dt=0,
              dirichlet=None, shock_x0=0.0, shock_speed=0.0, post=None, pre=None, cf_reading=0,
              basis=0, flux=0, pp=0) -> Problem2D:
    """cf_reading: mesh factors of the 2D Euler coefficient (c_fx, c_fy): 0 the
    (h_x, h_y) printed in Sec. 2.4 (default), 1 the (h_y, h_x) printed in
    Sec. 3.2, 2 none."""
    P = Problem2D()
    P.cf_reading, P.basis, P.pp = cf_reading, basis, pp
    P.flux = flux
    P.shock_x0, P.shock_speed = shock_x0, shock_speed
    for v in range(4):
        P.post[v] = float(post[v]) if post is not None else 0.0
        P.pre[v] = float(pre[v]) if pre is not None else 0.0
    P.eq, P.k, P.nq, P.filter, P.filter_dt = eq, k, nq, filter, filter_dt
    for i in range(4):
        P.bc[i] = bc[i]
    P.nx, P.ny = nx, ny
    P.xlo, P.xhi, P.ylo, P.yhi = xlo, xhi, ylo, yhi
    P.gamma, P.cfl = gamma, cfl
    P.adv_speed[0], P.adv_speed[1] = adv_speed
    if dirichlet is not None:
        for s in range(4):
            for v in range(4):
                P.dirichlet[s][v] = float(dirichlet[s][v]) if v < len(dirichlet[s]) else 0.0
    return P


def _chk(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


# ---------------------------------------------------------------- tables --
def gauss(q: int):
    x = np.zeros(q)
    w = np.zeros(q)
    _chk(lib().dgref_gauss(q, _ptr(x), _ptr(w)), "dgref_gauss")
    return x, w


def legendre_deriv(l: int, m: int, xi: float) -> float:
    return lib().dgref_legendre_deriv(l, m, float(xi))


# -------------------------------------------------------------------- 1D --
def residual1d(P: Problem1D, u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float64)
    L = np.empty_like(u)
    fh = np.empty(nvars(P.eq) * (P.n + 1))
    _chk(lib().dgref_residual1d(C.byref(P), _ptr(u), _ptr(L), _ptr(fh)), "residual1d")
    return L, fh.reshape(nvars(P.eq), P.n + 1)


def max_wavespeed1d(P: Problem1D, u: np.ndarray) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().dgref_max_wavespeed1d(C.byref(P), _ptr(u))


def stage1d(P: Problem1D, stage: int, dt: float, un: np.ndarray, us: np.ndarray | None = None):
    un = np.ascontiguousarray(un, dtype=np.float64)
    us = un if us is None else np.ascontiguousarray(us, dtype=np.float64)
    out = np.empty_like(un)
    _chk(lib().dgref_stage1d(C.byref(P), stage, C.c_double(dt), _ptr(un), _ptr(us), _ptr(out),
                             None), "stage1d")
    return out


def exponents1d(P: Problem1D, dt: float, v: np.ndarray):
    v = np.ascontiguousarray(v, dtype=np.float64)
    E = np.empty(P.n * (P.k + 1))
    eta = np.empty(P.n)
    _chk(lib().dgref_exponents1d(C.byref(P), C.c_double(dt), _ptr(v), _ptr(E), _ptr(eta)),
         "exponents1d")
    return E.reshape(P.n, P.k + 1), eta


def post1d(P: Problem1D, stage: int, dt: float, v: np.ndarray):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    tr = C.c_int64(0)
    _chk(lib().dgref_post1d(C.byref(P), stage, C.c_double(dt), _ptr(v), _ptr(out), C.byref(tr)),
         "post1d")
    return out, tr.value


def numflux1d(P: Problem1D, ul, ur) -> np.ndarray:
    """The problem's interface flux between the states ul | ur."""
    a, b = (np.ascontiguousarray(x, dtype=np.float64) for x in (ul, ur))
    f = np.zeros_like(a)
    _chk(lib().dgref_numflux1d(C.byref(P), _ptr(a), _ptr(b), _ptr(f)), "numflux1d")
    return f


def numflux2d(P: Problem2D, direction: int, ul, ur) -> np.ndarray:
    """The problem's flux across a face of normal +x (0) / +y (1)."""
    a, b = (np.ascontiguousarray(x, dtype=np.float64) for x in (ul, ur))
    f = np.zeros_like(a)
    _chk(lib().dgref_numflux2d(C.byref(P), int(direction), _ptr(a), _ptr(b), _ptr(f)), "numflux2d")
    return f


def pp_limit1d(P: Problem1D, u: np.ndarray):
    """Positivity-preserving limiter (Zhang and Shu) on every cell of u."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    _chk(lib().dgref_pp_limit1d(C.byref(P), _ptr(u)), "pp_limit1d")
    return u


def step1d_rc(P: Problem1D, dt: float, u: np.ndarray, bflux: np.ndarray | None = None):
    """One step; returns (new state or None when rejected, return code)."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    bf = np.zeros(4) if bflux is None else bflux
    tr = C.c_int64(0)
    rc = lib().dgref_step1d(C.byref(P), C.c_double(dt), _ptr(u), _ptr(bf), C.byref(tr))
    return u, rc


def step1d(P: Problem1D, dt: float, u: np.ndarray):
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    bf = np.zeros(4)
    tr = C.c_int64(0)
    _chk(lib().dgref_step1d(C.byref(P), C.c_double(dt), _ptr(u), _ptr(bf), C.byref(tr)), "step1d")
    return u


def run1d(P: Problem1D, u0: np.ndarray, t_end: float, max_steps: int = 1 << 40):
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    rep = Report()
    rc = lib().dgref_run1d(C.byref(P), C.c_double(t_end), C.c_int64(max_steps), _ptr(u),
                           C.byref(rep))
    return u, rep, rc


def check1d(P: Problem1D, u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float64)
    mr, mp = C.c_double(), C.c_double()
    bad = C.c_int64()
    rc = lib().dgref_check1d(C.byref(P), _ptr(u), C.byref(mr), C.byref(mp), C.byref(bad))
    return rc, mr.value, mp.value, bad.value


# -------------------------------------------------------------------- 2D --
def residual2d(P: Problem2D, u: np.ndarray, t: float = 0.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    L = np.empty_like(u)
    _chk(lib().dgref_residual2d(C.byref(P), C.c_double(t), _ptr(u), _ptr(L)), "residual2d")
    return L


def max_wavespeed2d(P: Problem2D, u: np.ndarray) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = lib().dgref_max_wavespeed2d
    f.restype = C.c_double
    return f(C.byref(P), _ptr(u))


def stage2d(P: Problem2D, stage: int, dt: float, un: np.ndarray, us: np.ndarray | None = None,
            t: float = 0.0):
    un = np.ascontiguousarray(un, dtype=np.float64)
    us = un if us is None else np.ascontiguousarray(us, dtype=np.float64)
    out = np.empty_like(un)
    _chk(lib().dgref_stage2d(C.byref(P), stage, C.c_double(t), C.c_double(dt), _ptr(un),
                             _ptr(us), _ptr(out)), "stage2d")
    return out


def exponents2d(P: Problem2D, dt: float, v: np.ndarray, t: float = 0.0):
    v = np.ascontiguousarray(v, dtype=np.float64)
    nc = P.nx * P.ny
    E = np.empty(nc * (2 * P.k + 1))
    eta = np.empty(nc)
    _chk(lib().dgref_exponents2d(C.byref(P), C.c_double(t), C.c_double(dt), _ptr(v), _ptr(E),
                                 _ptr(eta)), "exponents2d")
    return E.reshape(P.ny, P.nx, 2 * P.k + 1), eta.reshape(P.ny, P.nx)


def post2d(P: Problem2D, stage: int, dt: float, v: np.ndarray, t: float = 0.0):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    tr = C.c_int64(0)
    _chk(lib().dgref_post2d(C.byref(P), stage, C.c_double(t), C.c_double(dt), _ptr(v), _ptr(out),
                            C.byref(tr)), "post2d")
    return out, tr.value


def check2d(P: Problem2D, u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float64)
    mr, mp = C.c_double(), C.c_double()
    bad = C.c_int64()
    rc = lib().dgref_check2d(C.byref(P), _ptr(u), C.byref(mr), C.byref(mp), C.byref(bad))
    return rc, mr.value, mp.value, bad.value


def pp_limit2d(P: Problem2D, u: np.ndarray):
    """Positivity-preserving limiter (Zhang and Shu) on every cell of a 2D
    Euler state."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    _chk(lib().dgref_pp_limit2d(C.byref(P), _ptr(u)), "pp_limit2d")
    return u


def pp_points2d(P: Problem2D):
    """Reference coordinates (xi, eta) of the 2D limiter's test points."""
    xi = np.zeros(6 * 8 + 64)
    eta = np.zeros(6 * 8 + 64)
    n = lib().dgref_pp_points2d(C.byref(P), _ptr(xi), _ptr(eta))
    if n < 0:
        raise RuntimeError(f"pp_points2d failed with status {n}")
    return xi[:n].copy(), eta[:n].copy()


def step2d_rc(P: Problem2D, dt: float, u: np.ndarray, t: float = 0.0):
    """One step; returns (new state, or u unchanged when rejected, return code)."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    tr = C.c_int64(0)
    rc = lib().dgref_step2d(C.byref(P), C.c_double(t), C.c_double(dt), _ptr(u), C.byref(tr))
    return u, rc


def step2d(P: Problem2D, dt: float, u: np.ndarray, t: float = 0.0):
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    tr = C.c_int64(0)
    _chk(lib().dgref_step2d(C.byref(P), C.c_double(t), C.c_double(dt), _ptr(u), C.byref(tr)),
         "step2d")
    return u


def run2d(P: Problem2D, u0: np.ndarray, t_end: float, max_steps: int = 1 << 40):
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    rep = Report()
    rc = lib().dgref_run2d(C.byref(P), C.c_double(t_end), C.c_int64(max_steps), _ptr(u),
                           C.byref(rep))
    return u, rep, rc
