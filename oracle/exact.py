"""Exact solutions used to pin the oracle (test infrastructure only).

* ``riemann_exact`` — the exact solution of the Riemann problem for the 1D
  Euler equations of an ideal gas (pressure-function method with Newton
  iteration for the star pressure, then self-similar sampling; the textbook
  construction the paper compares its Lax-problem result against).
* ``burgers_smooth`` — the characteristic solution u = u0(x - u t) of the
  inviscid Burgers equation before shock formation.
* ``burgers_sine_shock`` — the entropy solution of u_t + (u^2/2)_x = 0 with
  u0 = 1/2 + sin(pi x) on [0, 2] periodic after the shock has formed,
  by brute-force characteristics on the branch not yet absorbed by the shock.
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------- Euler Riemann --
def _pressure_function(p, rho, pK, cK, gamma):
    """f_K(p) and f_K'(p) for one side (shock branch if p > pK, else
    rarefaction)."""
    if p > pK:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        sq = math.sqrt(A / (p + B))
        f = (p - pK) * sq
        df = sq * (1.0 - 0.5 * (p - pK) / (B + p))
    else:
        r = p / pK
        f = 2.0 * cK / (gamma - 1.0) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * cK) * r ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma=1.4):
    """(p*, u*) of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if ur - ul >= 2.0 * (cl + cr) / (gamma - 1.0):
        raise ValueError("vacuum is generated")
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _pressure_function(p, rl, pl, cl, gamma)
        fr, dfr = _pressure_function(p, rr, pr, cr, gamma)
        g = fl + fr + (ur - ul)
        pn = p - g / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_function(p, rl, pl, cl, gamma)
    fr, _ = _pressure_function(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_exact(left, right, x, t, x0=0.0, gamma=1.4):
    """Primitive (rho, u, p) at positions ``x`` and time ``t``."""
    x = np.asarray(x, dtype=float)
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    S = (x - x0) / t if t > 0 else np.sign(x - x0) * np.inf
    rho = np.empty_like(x)
    vel = np.empty_like(x)
    p = np.empty_like(x)
    for i, s in enumerate(np.ravel(S)):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    st = (rl, ul, pl)
                else:
                    st = (rl * (ps / pl + g1) / (g1 * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                cs = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                if s <= ul - cl:
                    st = (rl, ul, pl)
                elif s >= us - cs:
                    st = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cl + 0.5 * (gamma - 1) * (ul - s))
                    v = 2.0 / (gamma + 1) * (cl + 0.5 * (gamma - 1) * ul + s)
                    st = (rl * (c / cl) ** (2.0 / (gamma - 1)), v, pl * (c / cl) ** (2 * gamma / (gamma - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    st = (rr, ur, pr)
                else:
                    st = (rr * (ps / pr + g1) / (g1 * ps / pr + 1.0), us, ps)
            else:  # right rarefaction
                cs = cr * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                if s >= ur + cr:
                    st = (rr, ur, pr)
                elif s <= us + cs:
                    st = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cr - 0.5 * (gamma - 1) * (ur - s))
                    v = 2.0 / (gamma + 1) * (-cr + 0.5 * (gamma - 1) * ur + s)
                    st = (rr * (c / cr) ** (2.0 / (gamma - 1)), v, pr * (c / cr) ** (2 * gamma / (gamma - 1)))
        rho.flat[i], vel.flat[i], p.flat[i] = st
    return rho, vel, p


def riemann_waves(left, right, gamma=1.4):
    """Speeds of the outermost left and right waves (shock speed or
    rarefaction head) and the contact speed."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    if ps > pl:
        sl = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
    else:
        sl = ul - cl
    if ps > pr:
        sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
    else:
        sr = ur + cr
    return sl, us, sr


# ------------------------------------------------------------------ Burgers --
def burgers_smooth(u0, du0, x, t, iters=100):
    """u(x, t) = u0(x - u t) by Newton's method (valid before the shock)."""
    x = np.asarray(x, dtype=float)
    u = u0(x)
    for _ in range(iters):
        xi = x - u * t
        g = u - u0(xi)
        dg = 1.0 + du0(xi) * t
        u = u - g / dg
    return u


def burgers_sine_shock(x, t):
    """Entropy solution for u0 = 1/2 + sin(pi x) on [0, 2] (periodic) for
    t > 1/pi: in the frame moving with speed 1/2 the data sin(pi y) is odd
    about y = 1, so the shock sits at y = 1, i.e. x = 1 + t/2 (mod 2).  For
    each x the foot xi of the characteristic is found by bisection on the
    side of the shock that x lies on."""
    x = np.asarray(x, dtype=float)
    y = np.mod(x - 0.5 * t, 2.0)             # moving frame, in [0, 2)
    out = np.empty_like(y)
    for i, yy in enumerate(np.ravel(y)):
        # w(y, t) = sin(pi xi) with y = xi + t sin(pi xi); on [0,1) the foot
        # lies in [0, 1), on (1, 2) in (1, 2]: the map is monotone on each.
        if yy == 1.0:
            out.flat[i] = 0.0
            continue
        lo_, hi_ = (0.0, 1.0) if yy < 1.0 else (1.0, 2.0)
        g = lambda xi: xi + t * math.sin(math.pi * xi) - yy
        a, b = lo_, hi_
        ga = g(a)
        for _ in range(200):
            m = 0.5 * (a + b)
            gm = g(m)
            if (gm > 0) == (ga > 0):
                a, ga = m, gm
            else:
                b = m
        xi = 0.5 * (a + b)
        out.flat[i] = math.sin(math.pi * xi)
    return 0.5 + out
