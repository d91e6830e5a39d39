"""The device positivity limiter first screens each cell: with |P_l| <= 1 on
[-1, 1], rho_bar - sum_l |rho_l| and (gamma - 1) (E_lo - M_hi^2 / (2 rho_lo))
bound the density and the pressure from below, and a cell whose bounds
exceed twice every threshold and rounding margin the limiter could apply is
skipped.  Skipping must change nothing, so this test restates the screen
and checks, on many seeded cells near and far from vacuum, that every cell
it skips is one the oracle's limiter (Zhang and Shu, FP64) leaves bitwise
unchanged (a screen without the margins fails this), and, as a sanity
check, that the modes' own precision (FP32 for the mixed form) keeps every
test-point density and pressure positive there as well.  (The device forms
1/rho_lo by a Newton-refined reciprocal, within about an ulp of the quotient
restated here; the two-fold margins cover that.)"""
import numpy as np
from numpy.polynomial import legendre as npleg

import oracle as O

GAMMA = 1.4


def _screen(u, ur):
    """Boolean per cell: the device screen's verdict (u: (3, k+1, n))."""
    sa = np.abs(u[:, 1:, :]).sum(axis=1)
    rlo = u[0, 0] - sa[0]
    sr = np.abs(u[0, 0]) + sa[0]
    mhi = np.abs(u[1, 0]) + sa[1]
    elo = u[2, 0] - sa[2]
    se = np.abs(u[2, 0]) + sa[2]
    with np.errstate(all="ignore"):
        kin = 0.5 * mhi * mhi / rlo
        plo = (GAMMA - 1.0) * (elo - kin)
        mmax = 8.0 * ur * (se + 2.0 * kin + kin * sr / rlo)
        return (rlo > 2.0 * (1e-13 + 8.0 * ur * sr)) & (plo > 2.0 * (1e-13 + mmax))


def _cells(rng, k, n, dtype):
    rho = 10.0 ** rng.uniform(-8, 1, n)
    vel = rng.uniform(-50, 50, n) * rng.choice([0.0, 1.0, 1e-3], n)
    p = 10.0 ** rng.uniform(-12, 3, n)
    avg = np.stack([rho, rho * vel, p / (GAMMA - 1.0) + 0.5 * rho * vel * vel])
    scale = rng.choice([1e-6, 1e-3, 0.1, 0.3, 0.6, 1.0, 2.0], (3, n))
    u = np.zeros((3, k + 1, n))
    u[:, 0, :] = avg
    u[:, 1:, :] = (rng.uniform(-1, 1, (3, k, n)) * np.abs(avg)[:, None, :] * scale[:, None, :] / k)
    u[:, 1:, :] = u[:, 1:, :].astype(dtype).astype(np.float64)  # modes as stored
    return u


def _test_points(k):
    n_gl = (k + 4) // 2
    gl = [-1.0, 1.0] + ([0.0] if n_gl == 3 else [])
    return np.array(gl + list(npleg.leggauss(k + 1)[0]))


def test_screened_cells_are_left_unchanged():
    rng = np.random.default_rng(2024)
    for k in (1, 2, 3):
        u = _cells(rng, k, 60000, np.float64)
        P = O.problem1d(O.EULER, k, u.shape[2], 0.0, 1.0, bc=(O.OUTFLOW, O.OUTFLOW), pp=1)
        lim = O.pp_limit1d(P, u)
        skip = _screen(u, 2.0 ** -52)
        assert skip.sum() > 10000 and (~skip).sum() > 10000
        same = np.all(lim == u, axis=(0, 1))
        assert np.all(same[skip]), (k, np.flatnonzero(skip & ~same)[:5])


def test_screened_cells_positive_in_fp32():
    rng = np.random.default_rng(2025)
    for k in (1, 2, 3):
        u = _cells(rng, k, 60000, np.float32)
        skip = _screen(u, 2.0 ** -23)
        assert skip.sum() > 10000
        f = np.float32
        pts = _test_points(k)
        for x in pts:
            leg = np.array([npleg.legval(x, np.eye(k + 1)[l]) for l in range(k + 1)])
            w = [u[v, 0].astype(f) + sum(u[v, l].astype(f) * f(leg[l]) for l in range(1, k + 1))
                 for v in range(3)]
            w = [np.asarray(a, dtype=f) for a in w]
            with np.errstate(all="ignore"):
                vel = (w[1] / w[0]).astype(f)
                pr = ((f(GAMMA) - f(1)) * (w[2] - f(0.5) * w[1] * vel)).astype(f)
            assert np.all(w[0][skip] > 0) and np.all(pr[skip] > 0), (k, x)
