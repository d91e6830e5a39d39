"""paper_2407_19169_amd — MI355X (gfx950) RKDG solver with the jump filter.

Thin ctypes binding of ``libdg.so`` (C ABI in ``include/dg.h``).  Every step
of the method runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory and streams.  If the library is
not built, importing this package raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python __graft_entry__.py` "
                      "(__graft_entry__.build()) first")

_lib = C.CDLL(LIB_PATH)

# ------------------------------------------------------------- constants --
DG_OK, DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_DEVICE = 0, -1, -2, -3
DG_ERR_NONFINITE, DG_ERR_POSITIVITY, DG_ERR_STATE = -4, -5, -6
DG_EQ_ADVECTION, DG_EQ_BURGERS, DG_EQ_EULER = 0, 1, 2
DG_BC_PERIODIC, DG_BC_OUTFLOW, DG_BC_REFLECT, DG_BC_DIRICHLET = 0, 1, 2, 3
DG_BC_DMR_WALL, DG_BC_DMR_TOP = 4, 5
DG_FILTER_NONE, DG_FILTER_JUMP, DG_FILTER_HYBRID = 0, 1, 2
DG_PREC_FP64, DG_PREC_MIXED = 0, 1
DG_FLUX_LLF, DG_FLUX_HLL, DG_FLUX_HLLC = 0, 1, 2


class dg_mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64 * 2), ("lo", C.c_double * 2),
                ("hi", C.c_double * 2), ("bc", C.c_int * 4),
                ("dirichlet", (C.c_double * 4) * 4), ("shock_x0", C.c_double),
                ("shock_speed", C.c_double), ("post", C.c_double * 4), ("pre", C.c_double * 4)]


class dg_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("filter", C.c_int), ("cfl", C.c_double),
                ("gamma", C.c_double), ("adv_speed", C.c_double * 2),
                ("quad_points", C.c_int), ("stream", C.c_void_p), ("cf_reading", C.c_int),
                ("positivity", C.c_int), ("basis", C.c_int), ("flux", C.c_int)]


class dg_report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("ledger", C.c_double * 4),
                ("boundary_flux", C.c_double * 4), ("troubled_cells", C.c_int64),
                ("min_rho", C.c_double), ("min_p", C.c_double),
                ("max_exponent", C.c_double), ("status", C.c_int),
                ("first_bad_cell", C.c_int64), ("restarts", C.c_int64)]


class dg_problem1d(C.Structure):
    _fields_ = [("n", C.c_int64), ("degree", C.c_int), ("lo", C.c_double),
                ("hi", C.c_double), ("bc", C.c_int * 2), ("offset", C.c_int64)]


_vp = C.c_void_p
_sig = {
    "dg_create": [C.POINTER(dg_mesh), C.c_int, C.c_int, C.POINTER(dg_options), C.POINTER(_vp)],
    "dg_destroy": [_vp],
    "dg_buffer_sizes": [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
    "dg_bind": [_vp, _vp, _vp, _vp, _vp],
    "dg_set_state": [_vp, _vp],
    "dg_get_state": [_vp, _vp],
    "dg_max_wavespeed": [_vp, C.POINTER(C.c_double)],
    "dg_max_wavespeed_noalloc": [_vp, _vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "dg_stage": [_vp, C.c_int, C.c_double],
    "dg_jump_filter": [_vp, C.c_int, C.c_double],
    "dg_run": [_vp, C.c_double, C.c_int64, C.POINTER(dg_report)],
    "dg_report_read": [_vp, C.POINTER(dg_report)],
    "dg_last_exponents": [_vp, _vp],
    "dg_time_kernel": [_vp, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_double)],
    "dg_batch_create": [C.c_int, C.POINTER(dg_problem1d), C.c_int, C.POINTER(dg_options),
                        C.POINTER(C.c_int64), C.POINTER(_vp)],
    "dg_batch_destroy": [_vp],
    "dg_batch_buffer_sizes": [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
    "dg_batch_bind": [_vp, _vp, _vp, _vp, _vp],
    "dg_batch_set_state": [_vp, _vp],
    "dg_batch_get_state": [_vp, _vp],
    "dg_batch_run": [_vp, _vp, C.c_int64, C.POINTER(dg_report)],
    "dg_batch_tune": [_vp, C.c_int64, C.c_char_p, C.c_size_t],
    "dg_batch_set_schedule": [_vp, C.c_int, C.c_int, C.c_int],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.dg_strerror.argtypes = [C.c_int]
_lib.dg_strerror.restype = C.c_char_p

EXPORTED = tuple(_sig) + ("dg_strerror",)


class DGError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {dg_strerror(code)} ({code})")
        self.code = code


def dg_strerror(code: int) -> str:
    return _lib.dg_strerror(int(code)).decode()


def _check(rc: int, what: str) -> int:
    if rc != DG_OK:
        raise DGError(rc, what)
    return rc


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


# -------------------------------------------------- same-name functions --
def make_mesh(dim, n, lo, hi, bc, dirichlet=None, shock_x0=0.0, shock_speed=0.0, post=None,
              pre=None) -> dg_mesh:
    m = dg_mesh()
    m.shock_x0, m.shock_speed = shock_x0, shock_speed
    for v in range(4):
        m.post[v] = float(post[v]) if post is not None else 0.0
        m.pre[v] = float(pre[v]) if pre is not None else 0.0
    m.dim = dim
    for d in range(dim):
        m.n[d], m.lo[d], m.hi[d] = int(n[d]), float(lo[d]), float(hi[d])
    for i, b in enumerate(bc):
        m.bc[i] = int(b)
    if dirichlet is not None:
        for s, row in enumerate(dirichlet):
            for v, x in enumerate(row):
                m.dirichlet[s][v] = float(x)
    return m


def make_options(precision=DG_PREC_FP64, filter=DG_FILTER_JUMP, cfl=0.1, gamma=1.4,
                 adv_speed=(1.0, 0.0), quad_points=0, stream=None, cf_reading=0,
                 positivity=0, basis=0, flux=DG_FLUX_LLF) -> dg_options:
    o = dg_options()
    o.flux = flux
    o.cf_reading = cf_reading
    o.positivity = positivity
    o.basis = basis
    o.precision, o.filter, o.cfl, o.gamma = precision, filter, cfl, gamma
    o.adv_speed[0], o.adv_speed[1] = adv_speed
    o.quad_points = quad_points
    o.stream = stream
    return o


def dg_create(mesh: dg_mesh, degree: int, equation: int, options: dg_options) -> int:
    h = _vp()
    _check(_lib.dg_create(C.byref(mesh), degree, equation, C.byref(options), C.byref(h)),
           "dg_create")
    return h.value


def dg_destroy(h: int) -> None:
    _check(_lib.dg_destroy(h), "dg_destroy")


def dg_buffer_sizes(h: int):
    a, b = C.c_size_t(), C.c_size_t()
    _check(_lib.dg_buffer_sizes(h, C.byref(a), C.byref(b)), "dg_buffer_sizes")
    return a.value, b.value


def dg_bind(h, u_n, u_a, u_b, workspace) -> None:
    _check(_lib.dg_bind(h, _ptr(u_n), _ptr(u_a), _ptr(u_b), _ptr(workspace)), "dg_bind")


def dg_set_state(h, modes) -> None:
    _check(_lib.dg_set_state(h, _ptr(modes)), "dg_set_state")


def dg_get_state(h, modes) -> None:
    _check(_lib.dg_get_state(h, _ptr(modes)), "dg_get_state")


def dg_max_wavespeed(h) -> float:
    a = C.c_double()
    _check(_lib.dg_max_wavespeed(h, C.byref(a)), "dg_max_wavespeed")
    return a.value


def dg_stage(h, stage: int, dt: float) -> None:
    _check(_lib.dg_stage(h, stage, dt), "dg_stage")


def dg_jump_filter(h, stage: int, dt: float) -> None:
    _check(_lib.dg_jump_filter(h, stage, dt), "dg_jump_filter")


def dg_run(h, t_end: float, max_steps: int, check: bool = True) -> dg_report:
    rep = dg_report()
    rc = _lib.dg_run(h, t_end, max_steps, C.byref(rep))
    if check:
        _check(rc, "dg_run")
    return rep


def dg_report_read(h, check: bool = False) -> dg_report:
    rep = dg_report()
    rc = _lib.dg_report_read(h, C.byref(rep))
    if check:
        _check(rc, "dg_report_read")
    return rep


def dg_last_exponents(h, out) -> None:
    _check(_lib.dg_last_exponents(h, _ptr(out)), "dg_last_exponents")


def dg_max_wavespeed_noalloc(h, u_dev_ptr: int):
    """(alpha, first_bad, status) of the state buffer at device address
    u_dev_ptr, with the library's fixed scratch (allocates nothing); status
    is DG_OK or DG_ERR_NONFINITE (other errors raise)."""
    a = C.c_double()
    bad = C.c_int64()
    rc = _lib.dg_max_wavespeed_noalloc(h, u_dev_ptr, C.byref(a), C.byref(bad))
    if rc not in (DG_OK, DG_ERR_NONFINITE):
        _check(rc, "dg_max_wavespeed_noalloc")
    return a.value, bad.value, rc


def dg_time_kernel(h, stage: int, dt: float, reps: int) -> float:
    us = C.c_double()
    _check(_lib.dg_time_kernel(h, stage, dt, reps, C.byref(us)), "dg_time_kernel")
    return us.value


# ------------------------------------------------------- torch plumbing --
class Solver:
    """Owns a handle plus torch-allocated state buffers and workspace."""

    def __init__(self, mesh: dg_mesh, degree: int, equation: int, options: dg_options,
                 device="cuda"):
        import torch

        self.torch = torch
        self.mesh, self.degree, self.equation, self.options = mesh, degree, equation, options
        self.h = dg_create(mesh, degree, equation, options)
        sb, wb = dg_buffer_sizes(self.h)
        self.state_bytes, self.ws_bytes = sb, wb
        alloc = lambda nbytes: torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._raw = [alloc(sb) for _ in range(3)] + [alloc(wb)]
        self._ptrs = [((t.data_ptr() + 255) // 256) * 256 for t in self._raw]
        dg_bind(self.h, *self._ptrs)
        self.nv = (3 if mesh.dim == 1 else 4) if equation == DG_EQ_EULER else 1
        self.nmodes = (degree + 1) if mesh.dim == 1 else (degree + 1) ** 2
        # modes stored per variable: the 2D P^k space keeps p + q <= k only
        self.nmodes_stored = ((degree + 1) * (degree + 2) // 2
                              if mesh.dim == 2 and options.basis == 1 and degree > 0 else self.nmodes)
        self.ncell = mesh.n[0] if mesh.dim == 1 else mesh.n[0] * mesh.n[1]

    def shape(self):
        if self.mesh.dim == 1:
            return (self.nv, self.nmodes, self.ncell)
        return (self.nv, self.nmodes, self.mesh.n[1], self.mesh.n[0])

    def set_state(self, u) -> None:
        t = self.torch.as_tensor(u, dtype=self.torch.float64).to("cuda").contiguous()
        assert tuple(t.shape) == self.shape(), (t.shape, self.shape())
        dg_set_state(self.h, t)
        self.torch.cuda.synchronize()

    def get_state(self):
        out = self.torch.empty(self.shape(), dtype=self.torch.float64, device="cuda")
        dg_get_state(self.h, out)
        self.torch.cuda.synchronize()
        return out

    def exponents(self):
        lmax = self.degree if self.mesh.dim == 1 else 2 * self.degree
        out = self.torch.empty((self.ncell, lmax + 1), dtype=self.torch.float64, device="cuda")
        dg_last_exponents(self.h, out)
        self.torch.cuda.synchronize()
        return out

    def close(self) -> None:
        if self.h:
            dg_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def buffer_view(solver: Solver, i: int):
    """FP64-layout view of state buffer i (0 = u_n, 1 = u_a, 2 = u_b) of a
    DG_PREC_FP64 solver (the caller owns these buffers).  The mode axis has
    the stored modes: for the 2D P^k space the modes p + q <= k in p-major
    order (`pk_modes`)."""
    torch = solver.torch
    t = solver._raw[i]
    off = solver._ptrs[i] - t.data_ptr()
    shape = list(solver.shape())
    shape[1] = solver.nmodes_stored
    nel = 1
    for d in shape:
        nel *= d
    return t[off:off + nel * 8].view(torch.float64).view(shape)


def pk_modes(k: int):
    """Q^k mode indices p*(k+1)+q of the P^k modes (p + q <= k), in the order
    the device stores them."""
    return [p * (k + 1) + q for p in range(k + 1) for q in range(k + 1) if p + q <= k]


# ----------------------------------------------------------------- batch --
def dg_batch_create(problems, equation: int, options: dg_options):
    """problems: sequence of (n, degree, lo, hi, bc_lo, bc_hi).  Returns
    (handle, offsets, total_elems)."""
    arr = (dg_problem1d * len(problems))()
    for i, (n, k, lo, hi, b0, b1) in enumerate(problems):
        arr[i].n, arr[i].degree, arr[i].lo, arr[i].hi = int(n), int(k), float(lo), float(hi)
        arr[i].bc[0], arr[i].bc[1] = int(b0), int(b1)
    total = C.c_int64()
    h = _vp()
    _check(_lib.dg_batch_create(len(problems), arr, equation, C.byref(options), C.byref(total),
                                C.byref(h)), "dg_batch_create")
    return h.value, [arr[i].offset for i in range(len(problems))], total.value


def dg_batch_destroy(h) -> None:
    _check(_lib.dg_batch_destroy(h), "dg_batch_destroy")


def dg_batch_buffer_sizes(h):
    a, b = C.c_size_t(), C.c_size_t()
    _check(_lib.dg_batch_buffer_sizes(h, C.byref(a), C.byref(b)), "dg_batch_buffer_sizes")
    return a.value, b.value


def dg_batch_bind(h, u_n, u_a, u_b, workspace) -> None:
    _check(_lib.dg_batch_bind(h, _ptr(u_n), _ptr(u_a), _ptr(u_b), _ptr(workspace)), "dg_batch_bind")


def dg_batch_set_state(h, packed) -> None:
    _check(_lib.dg_batch_set_state(h, _ptr(packed)), "dg_batch_set_state")


def dg_batch_get_state(h, packed) -> None:
    _check(_lib.dg_batch_get_state(h, _ptr(packed)), "dg_batch_get_state")


def dg_batch_run(h, nprob: int, steps: int, t_end=None, check: bool = True):
    reps = (dg_report * nprob)()
    te = None
    if t_end is not None:
        te = (C.c_double * nprob)(*[float(x) for x in t_end])
    rc = _lib.dg_batch_run(h, te, steps, reps)
    if check:
        _check(rc, "dg_batch_run")
    return list(reps)


def dg_batch_tune(h, trial_steps: int) -> str:
    buf = C.create_string_buffer(8192)
    _check(_lib.dg_batch_tune(h, trial_steps, buf, 8192), "dg_batch_tune")
    return buf.value.decode()


def _batch_key(problems) -> str:
    """The autotuner's cache key of a batch: the fractions of degrees 0..3
    and round(log2(mean cells)), as dg_batch_tune reports them."""
    import math

    n = len(problems)
    kf = [sum(1 for p in problems if int(p[1]) == k) / n for k in range(4)]
    mean_n = sum(int(p[0]) for p in problems) / n
    return "k%s_n%d" % ("-".join(f"{x:.2f}" for x in kf), round(math.log2(max(mean_n, 1.0))))


class Batch:
    """Owns a batch handle plus torch-allocated buffers."""

    def __init__(self, problems, options: dg_options, equation: int = DG_EQ_EULER):
        import torch

        self.torch = torch
        self.problems = list(problems)
        self.h, self.offsets, self.total = dg_batch_create(self.problems, equation, options)
        sb, wb = dg_batch_buffer_sizes(self.h)
        alloc = lambda nbytes: torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self._raw = [alloc(sb) for _ in range(3)] + [alloc(wb)]
        self._ptrs = [((t.data_ptr() + 255) // 256) * 256 for t in self._raw]
        dg_batch_bind(self.h, *self._ptrs)

    def set_state(self, states) -> None:
        flat = self.torch.cat([self.torch.as_tensor(s, dtype=self.torch.float64).reshape(-1)
                               for s in states]).to("cuda")
        assert flat.numel() == self.total
        dg_batch_set_state(self.h, flat)
        self.torch.cuda.synchronize()

    def get_state(self):
        flat = self.torch.empty(self.total, dtype=self.torch.float64, device="cuda")
        dg_batch_get_state(self.h, flat)
        self.torch.cuda.synchronize()
        flat = flat.cpu().numpy()
        out = []
        for (n, k, *_), off in zip(self.problems, self.offsets):
            out.append(flat[off:off + 3 * (k + 1) * n].reshape(3, k + 1, n))
        return out

    def run(self, steps: int, t_end=None, check: bool = True):
        return dg_batch_run(self.h, len(self.problems), steps, t_end, check)

    def tune(self, trial_steps: int = 5, cache: str | None = None) -> str:
        """Autotune the schedule (JSON summary).  With `cache` (a JSON file
        path), a schedule stored there under this batch's key (degree mix,
        size bucket) is applied without timing, and a new one is stored."""
        import json
        import os

        key = _batch_key(self.problems)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if key in table:
            best = table[key]
            _check(_lib.dg_batch_set_schedule(self.h, best["block_size"], best["wg_per_cu"],
                                              1 if best["order"] == "lpt" else 0),
                   "dg_batch_set_schedule")
            return json.dumps({"key": key, "cached": True, "best": best})
        out = dg_batch_tune(self.h, trial_steps)
        if cache:
            table[key] = json.loads(out)["best"]
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return out

    def set_schedule(self, block_size: int, wg_per_cu: int, lpt: bool = True) -> None:
        _check(_lib.dg_batch_set_schedule(self.h, block_size, wg_per_cu, int(lpt)),
               "dg_batch_set_schedule")

    def close(self) -> None:
        if self.h:
            dg_batch_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
