"""Seeded, synthetic inputs shared by the GPU library's tests and benchmark and
by the CPU oracle.

This module holds no arithmetic of the method itself: it builds initial
states (the paper's analytic initial data, or seeded random draws shaped like
the paper's workloads) and projects them onto the modal Legendre space with
NumPy's own Gauss–Legendre routines (``numpy.polynomial.legendre``).  Both
sides of every parity check receive the same arrays from here.

State layout: 1D ``u[var, mode, cell]``; 2D ``u[var, p*(k+1)+q, iy, ix]``
(x fastest), FP64, C-contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as npleg

GAMMA = 1.4


# ------------------------------------------------------------ projection --
def _legendre_values(k: int, x: np.ndarray) -> np.ndarray:
    """P_l(x) for l = 0..k, shape (k+1, len(x)), via numpy.polynomial."""
    out = np.empty((k + 1,) + np.shape(x))
    for l in range(k + 1):
        c = np.zeros(l + 1)
        c[l] = 1.0
        out[l] = npleg.legval(x, c)
    return out


def project1d(func, k: int, n: int, lo: float, hi: float, nquad: int = 8,
              sub: int = 1) -> np.ndarray:
    """L2 projection of ``func(x) -> (nvars, ...)`` onto P^k on a uniform mesh.

    ``sub`` splits each cell into that many sub-intervals for the quadrature,
    which keeps the projection of data with a kink or jump inside a cell
    accurate."""
    h = (hi - lo) / n
    xg, wg = npleg.leggauss(nquad)
    # sub-interval Gauss points in reference coordinates
    xs = np.concatenate([(-1.0 + (2.0 * s + 1.0 + xg) / sub) for s in range(sub)])
    ws = np.concatenate([wg / sub for _ in range(sub)])
    P = _legendre_values(k, xs)                                   # (k+1, Q)
    xc = lo + (np.arange(n) + 0.5) * h
    X = xc[:, None] + 0.5 * h * xs[None, :]                       # (n, Q)
    F = np.asarray(func(X), dtype=np.float64)
    if F.ndim == 2:
        F = F[None]
    nv = F.shape[0]
    u = np.empty((nv, k + 1, n))
    for l in range(k + 1):
        u[:, l, :] = (2 * l + 1) / 2.0 * np.einsum("vnq,q->vn", F, ws * P[l])
    return np.ascontiguousarray(u)


def project2d(func, k: int, nx: int, ny: int, xlo: float, xhi: float, ylo: float,
              yhi: float, nquad: int = 8, sub: int = 1) -> np.ndarray:
    """L2 projection of ``func(X, Y) -> (nvars, ...)`` onto Q^k (tensor
    Legendre, mode index p*(k+1)+q with p the x-degree)."""
    hx, hy = (xhi - xlo) / nx, (yhi - ylo) / ny
    xg, wg = npleg.leggauss(nquad)
    xs = np.concatenate([(-1.0 + (2.0 * s + 1.0 + xg) / sub) for s in range(sub)])
    ws = np.concatenate([wg / sub for _ in range(sub)])
    P = _legendre_values(k, xs)                                   # (k+1, Q)
    xc = xlo + (np.arange(nx) + 0.5) * hx
    yc = ylo + (np.arange(ny) + 0.5) * hy
    nm = (k + 1) ** 2
    out = None
    # row by row to bound memory: X,Y of shape (nx, Q, Q)
    for iy in range(ny):
        X = xc[:, None, None] + 0.5 * hx * xs[None, :, None]
        Y = yc[iy] + 0.5 * hy * xs[None, None, :]
        X, Y = np.broadcast_arrays(X, Y)
        F = np.asarray(func(X, Y), dtype=np.float64)
        if F.ndim == 3:
            F = F[None]
        nv = F.shape[0]
        if out is None:
            out = np.empty((nv, nm, ny, nx))
        for p in range(k + 1):
            for q in range(k + 1):
                wgt = (ws * P[p])[:, None] * (ws * P[q])[None, :]
                out[:, p * (k + 1) + q, iy, :] = ((2 * p + 1) * (2 * q + 1) / 4.0 *
                                                  np.einsum("vnab,ab->vn", F, wgt))
    return np.ascontiguousarray(out)


# -------------------------------------------------------- gas dynamics IC --
def conserved(rho, u, p, gamma=GAMMA):
    rho, u, p = np.broadcast_arrays(np.asarray(rho, float), np.asarray(u, float),
                                    np.asarray(p, float))
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def conserved2d(rho, u, v, p, gamma=GAMMA):
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, float) for a in (rho, u, v, p)))
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def rankine_hugoniot(mach: float, rho0: float, p0: float, gamma: float = GAMMA):
    """Post-shock (rho, u, p) and shock speed for a shock of Mach ``mach``
    running into gas at rest (rho0, p0) — the textbook normal-shock
    relations."""
    c0 = math.sqrt(gamma * p0 / rho0)
    S = mach * c0
    M2 = mach * mach
    rho1 = rho0 * (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
    p1 = p0 * (2.0 * gamma * M2 - (gamma - 1.0)) / (gamma + 1.0)
    u1 = S * (1.0 - rho0 / rho1)
    return rho1, u1, p1, S


# --------------------------------------------------------------- workloads --
@dataclass
class Workload1D:
    name: str
    eq: int                  # 0 advection, 1 Burgers, 2 Euler
    k: int
    n: int
    lo: float
    hi: float
    bc: tuple
    u0: np.ndarray
    cfl: float = 0.1
    gamma: float = GAMMA
    t_end: float = 0.0
    filter: int = 1          # 0 none, 1 jump, 2 hybrid
    extra: dict = field(default_factory=dict)


def burgers_sine(n: int = 200, k: int = 2) -> Workload1D:
    """Periodic Burgers on [0,2], u0 = 0.5 + sin(pi x), run to t = 1.5."""
    u0 = project1d(lambda x: 0.5 + np.sin(np.pi * x), k, n, 0.0, 2.0)
    return Workload1D("burgers_sine", 1, k, n, 0.0, 2.0, (0, 0), u0, 0.1, GAMMA, 1.5, 1)


def burgers_table(n: int, k: int) -> Workload1D:
    """Burgers on (-pi, pi), u0 = 1/2 + sin x, smooth up to t = 0.5."""
    u0 = project1d(lambda x: 0.5 + np.sin(x), k, n, -math.pi, math.pi)
    return Workload1D("burgers_table", 1, k, n, -math.pi, math.pi, (0, 0), u0, 0.1, GAMMA,
                      0.5, 1)


def advection_sine(n: int, k: int, a: float = 1.0) -> Workload1D:
    u0 = project1d(lambda x: np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x), k, n, 0.0, 1.0)
    return Workload1D("advection_sine", 0, k, n, 0.0, 1.0, (0, 0), u0, 0.1, GAMMA, 1.0, 1,
                      {"adv_speed": a})


def shu_osher(n: int = 20000, k: int = 2, gamma: float = GAMMA) -> Workload1D:
    """Mach-3 shock at x = -4 into rho = 1 + 0.2 sin 5x, u = 0, p = 1 on
    [-5, 5], outflow; post-shock state from the normal-shock relations."""
    r1, u1, p1, _ = rankine_hugoniot(3.0, 1.0, 1.0, gamma)

    def f(x):
        left = x < -4.0
        rho = np.where(left, r1, 1.0 + 0.2 * np.sin(5.0 * x))
        vel = np.where(left, u1, 0.0)
        p = np.where(left, p1, 1.0)
        return conserved(rho, vel, p, gamma)

    u0 = project1d(f, k, n, -5.0, 5.0)
    return Workload1D("shu_osher", 2, k, n, -5.0, 5.0, (1, 1), u0, 0.1, gamma, 1.8, 2)


def riemann1d(left, right, n: int, k: int, lo=-1.0, hi=1.0, x0=0.0, gamma=GAMMA,
              name="riemann") -> Workload1D:
    """Piecewise-constant Riemann data, (rho, u, p) left/right of x0."""

    def f(x):
        L = x < x0
        return conserved(np.where(L, left[0], right[0]), np.where(L, left[1], right[1]),
                         np.where(L, left[2], right[2]), gamma)

    u0 = project1d(f, k, n, lo, hi)
    return Workload1D(name, 2, k, n, lo, hi, (1, 1), u0, 0.1, gamma, 0.0, 1,
                      {"left": left, "right": right, "x0": x0})


def lax(n: int = 200, k: int = 2) -> Workload1D:
    w = riemann1d((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), n, k, -1.0, 1.0, 0.0, name="lax")
    w.t_end = 0.13
    return w


def random_state_1d(seed: int, n: int, k: int, nvars: int = 3, amp: float = 0.1) -> np.ndarray:
    """A positive smooth-ish random Euler state (for per-call parity)."""
    rng = np.random.default_rng(seed)
    u = np.zeros((nvars, k + 1, n))
    rho = 1.0 + 0.5 * rng.random(n)
    vel = rng.uniform(-0.5, 0.5, n)
    p = 1.0 + 0.5 * rng.random(n)
    u[:, 0, :] = conserved(rho, vel, p)
    for l in range(1, k + 1):
        u[:, l, :] = amp / (l + 1) * rng.standard_normal((nvars, n)) * np.abs(u[:, :1, :]).squeeze(1)
    return u


# ----------------------------------------------------------- batched set --
@dataclass
class BatchSpec:
    n: np.ndarray        # cells per problem
    k: np.ndarray        # degree per problem
    left: np.ndarray     # (nprob, 3) rho, u, p
    right: np.ndarray    # (nprob, 3)


def batched_riemann_spec(nprob: int = 4096, seed: int = 4001, nmin: int = 256,
                         nmax: int = 8192, kmin: int = 1, kmax: int = 3,
                         gamma: float = GAMMA) -> BatchSpec:
    """Seeded random Riemann problems: rho log-uniform [0.1, 10], p
    log-uniform [0.01, 1000], u uniform [-2, 2]; cell counts uniform (even)
    in [nmin, nmax]; degrees uniform in [kmin, kmax].  Draws whose exact
    solution would open a vacuum (pressure-positivity condition of the
    exact Riemann problem) are redrawn from the same stream."""
    rng = np.random.default_rng(seed)
    n = (rng.integers(nmin // 2, nmax // 2 + 1, nprob) * 2).astype(np.int64)
    k = rng.integers(kmin, kmax + 1, nprob).astype(np.int32)
    L = np.empty((nprob, 3))
    R = np.empty((nprob, 3))
    for i in range(nprob):
        while True:
            rl, rr = 10.0 ** rng.uniform(-1, 1, 2)
            ul, ur = rng.uniform(-2, 2, 2)
            pl, pr = 10.0 ** rng.uniform(-2, 3, 2)
            cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
            # vacuum forms when the velocity difference exceeds this bound
            if (ur - ul) < 2.0 * (cl + cr) / (gamma - 1.0) * 0.5:
                break
        L[i] = (rl, ul, pl)
        R[i] = (rr, ur, pr)
    return BatchSpec(n, k, L, R)


def batched_riemann_states(spec: BatchSpec, lo=-1.0, hi=1.0, gamma=GAMMA):
    """Per-problem projected initial states (list of (3, k+1, n) arrays)."""
    out = []
    for i in range(len(spec.n)):
        w = riemann1d(tuple(spec.left[i]), tuple(spec.right[i]), int(spec.n[i]), int(spec.k[i]),
                      lo, hi, 0.0, gamma)
        out.append(w.u0)
    return out


# -------------------------------------------------------------------- 2D --
@dataclass
class Workload2D:
    name: str
    k: int
    nx: int
    ny: int
    xlo: float
    xhi: float
    ylo: float
    yhi: float
    bc: tuple                # x-lo, x-hi, y-lo, y-hi
    u0: np.ndarray
    cfl: float = 0.1
    gamma: float = GAMMA
    t_end: float = 0.0
    filter: int = 1
    extra: dict = field(default_factory=dict)


def vortex_exact(X, Y, t, x0=5.0, y0=0.0, beta=5.0, gamma=GAMMA, period=10.0):
    """Isentropic vortex advected by the mean flow (1, 0): centre at
    (x0 + t, y0); the x-offset is wrapped to the periodic box."""
    dx = X - x0 - t
    dx = dx - period * np.round(dx / period)
    dy = Y - y0
    r2 = dx * dx + dy * dy
    e = np.exp(1.0 - r2)
    u = 1.0 - beta * e * dy / (2.0 * math.pi)
    v = beta * e * dx / (2.0 * math.pi)
    rho = (1.0 - (gamma - 1.0) / (16.0 * gamma * math.pi ** 2) * beta ** 2 * e * e) ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return conserved2d(rho, u, v, p, gamma)


def vortex2d(n: int = 1024, k: int = 2, seed: int | None = 3001) -> Workload2D:
    """Isentropic vortex on [0,10] x [-5,5], periodic; centre drawn from
    ``seed`` in [4.5,5.5] x [-0.5,0.5] (seed None: the centre (5, 0))."""
    if seed is None:
        x0, y0 = 5.0, 0.0
    else:
        rng = np.random.default_rng(seed)
        x0, y0 = rng.uniform(4.5, 5.5), rng.uniform(-0.5, 0.5)
    u0 = project2d(lambda X, Y: vortex_exact(X, Y, 0.0, x0, y0), k, n, n, 0.0, 10.0, -5.0, 5.0,
                   nquad=k + 3)
    return Workload2D("vortex", k, n, n, 0.0, 10.0, -5.0, 5.0, (0, 0, 0, 0), u0, 0.1, GAMMA,
                      10.0, 1, {"x0": x0, "y0": y0})


def quadrant2d(n: int = 1024, k: int = 2, seed: int = 3002) -> Workload2D:
    """Four-quadrant Riemann problem on [0,10] x [-5,5], periodic, split at
    the centre; states drawn from ``seed``: rho U[0.1,2], u,v U[-1,1],
    p U[0.03,1.5]."""
    rng = np.random.default_rng(seed)
    S = np.stack([rng.uniform(0.1, 2.0, 4), rng.uniform(-1, 1, 4), rng.uniform(-1, 1, 4),
                  rng.uniform(0.03, 1.5, 4)], axis=1)

    def f(X, Y):
        q = (X >= 5.0).astype(int) + 2 * (Y >= 0.0).astype(int)
        return conserved2d(S[q, 0], S[q, 1], S[q, 2], S[q, 3])

    u0 = project2d(f, k, n, n, 0.0, 10.0, -5.0, 5.0, nquad=k + 2)
    return Workload2D("quadrant", k, n, n, 0.0, 10.0, -5.0, 5.0, (0, 0, 0, 0), u0, 0.1, GAMMA,
                      0.0, 1, {"states": S})


def double_mach(nx: int = 4096, ny: int = 1024, k: int = 3) -> Workload2D:
    """Mach-10 shock at x = 1/6 on the wall, inclined 60 degrees, into
    (rho, u, v, p) = (1.4, 0, 0, 1) on [0,4] x [0,1]."""
    r1, s1, p1, S = rankine_hugoniot(10.0, 1.4, 1.0)
    ang = math.pi / 6.0
    post = (r1, s1 * math.cos(ang), -s1 * math.sin(ang), p1)

    def f(X, Y):
        behind = X < 1.0 / 6.0 + Y / math.sqrt(3.0)
        return conserved2d(np.where(behind, post[0], 1.4), np.where(behind, post[1], 0.0),
                           np.where(behind, post[2], 0.0), np.where(behind, post[3], 1.0))

    # Piecewise constant data: cells the shock line misses hold a constant
    # (mode 0 only); the cells it cuts start from their exact cell average
    # with all higher modes zero (an L2 projection of the Mach-10 jump onto
    # Q^k overshoots to negative density and pressure inside those cells).
    hx, hy = 4.0 / nx, 1.0 / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    xs = 1.0 / 6.0 + yc / math.sqrt(3.0)                       # shock x at row centres
    d = xc[None, :] - xs[:, None]
    reach = 0.5 * hx + 0.5 * hy / math.sqrt(3.0) + 1e-12
    nm = (k + 1) ** 2
    u0 = np.zeros((4, nm, ny, nx))
    Upost = conserved2d(*post)
    Upre = conserved2d(1.4, 0.0, 0.0, 1.0)
    for v in range(4):
        u0[v, 0] = np.where(d < 0, Upost[v], Upre[v])
    for jy in range(ny):
        cut = np.nonzero(np.abs(d[jy]) <= reach)[0]
        if len(cut) == 0:
            continue
        i0, i1 = int(cut.min()), int(cut.max()) + 1
        part = project2d(f, 0, i1 - i0, 1, i0 * hx, i1 * hx, jy * hy, (jy + 1) * hy,
                         nquad=8, sub=4)
        u0[:, 0, jy, i0:i1] = part[:, 0, 0, :]
    return Workload2D("double_mach", k, nx, ny, 0.0, 4.0, 0.0, 1.0, (3, 1, 4, 5), u0, 0.1, GAMMA,
                      0.2, 2, {"post": post, "shock_speed": S})
