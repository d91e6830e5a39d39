"""Pins of the oracle's 2D positivity-preserving limiter (Zhang and Shu on
rectangles; the paper applies it after the jump filter in its Sec. 3.2
examples with extreme positivity demands) and of the step rejection that goes
with it.

* The test-point set: (Gauss-Lobatto x Gauss) u (Gauss x Gauss-Lobatto) with
  N = ceil((k+3)/2) Lobatto points, plus the volume Gauss points.  Checked
  against numpy's Gauss rules, and against the property the limiter rests
  on: the Q^k cell average is a convex combination of the values at the
  first set (checked here with numpy's Legendre series on random cells).
* Closed forms: a cell whose only negative pressure is at an edge Gauss point
  (xi, eta) = (+-1, +-1/sqrt(3)) of Q^1 -- a point outside the Gauss x Gauss
  set -- gives the limiting factor in closed form.
* Invariants: admissible cells untouched, cell averages untouched, density
  and pressure positive at every test point afterwards (evaluated with
  numpy), a rejected step leaves the state unchanged.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import dg_inputs as I

GAMMA = 1.4
EPS = 1e-13


def _problem(ref, k, nx=1, ny=1, **kw):
    return ref.problem2d(2, k, nx, ny, 0.0, 1.0, 0.0, 1.0, bc=(1, 1, 1, 1), filter=1, pp=1, **kw)


def _leg(k, x):
    return np.array([npleg.legval(x, np.eye(k + 1)[l]) for l in range(k + 1)])


def _point_values(u, xi, eta):
    """(4, npts, ny, nx) point values of a modal Q^k state, with numpy."""
    k = int(round(math.sqrt(u.shape[1]))) - 1
    out = np.zeros((u.shape[0], len(xi)) + u.shape[2:])
    for i, (x, y) in enumerate(zip(xi, eta)):
        px, py = _leg(k, x), _leg(k, y)
        w = np.outer(px, py).reshape(-1)
        out[:, i] = np.einsum("m,vmyx->vyx", w, u)
    return out


def _pressure(w):
    return (GAMMA - 1.0) * (w[3] - 0.5 * (w[1] ** 2 + w[2] ** 2) / w[0])


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_point_set_is_lobatto_gauss_tensor(ref, k):
    xi, eta = ref.pp_points2d(_problem(ref, k))
    N = (k + 4) // 2
    lob = {2: [-1.0, 1.0], 3: [-1.0, 0.0, 1.0]}[N]
    g, _ = npleg.leggauss(k + 1)
    want = {(x, y) for x in lob for y in g} | {(x, y) for x in g for y in lob} | \
           {(x, y) for x in g for y in g}
    got = {(round(a, 14), round(b, 14)) for a, b in zip(xi, eta)}
    assert got == {(round(a, 14), round(b, 14)) for a, b in want}
    assert len(xi) == 2 * N * (k + 1) + (k + 1) ** 2


@pytest.mark.parametrize("k", [1, 2, 3])
def test_average_is_convex_combination_of_lobatto_gauss_values(k):
    """Zhang-Shu decomposition on rectangles: with Lobatto weights w^L (N
    points, exact to degree 2N-3 >= k) in xi and Gauss weights w^G in eta,
    u_bar = sum_i sum_b (w^L_i / 2)(w^G_b / 2) u(x^L_i, y^G_b) for every Q^k
    polynomial, all weights positive."""
    N = (k + 4) // 2
    lob, wl = {2: ([-1.0, 1.0], [1.0, 1.0]), 3: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3])}[N]
    g, wg = npleg.leggauss(k + 1)
    rng = np.random.default_rng(40 + k)
    u = rng.standard_normal((1, (k + 1) ** 2, 1, 1))
    xi = np.repeat(lob, k + 1)
    eta = np.tile(g, N)
    vals = _point_values(u, xi, eta)[0, :, 0, 0]
    wts = np.outer(np.array(wl) / 2, wg / 2).reshape(-1)
    assert np.all(wts > 0)
    assert np.dot(wts, vals) == pytest.approx(u[0, 0, 0, 0], abs=1e-14)


def test_pressure_factor_closed_form_edge_gauss_point(ref):
    """rho = 1, m = 0, E = 1 + 2 xi eta (mode (1,1) = 2), Q^1.  Over the test
    points xi*eta >= -1/sqrt(3) (the edge points (+-1, -+1/sqrt(3)); at the
    volume Gauss points xi*eta >= -1/3, where E stays positive), so the
    pressure 0.4 (1 - 2 t/sqrt(3)) of the limited cell reaches eps there:
    t = (1 - eps/0.4) sqrt(3)/2."""
    u = np.zeros((4, 4, 1, 1))
    u[0, 0] = 1.0
    u[3, 0] = 1.0
    u[3, 3] = 2.0
    out = ref.pp_limit2d(_problem(ref, 1), u)
    theta = (1.0 - EPS / (GAMMA - 1.0)) * math.sqrt(3.0) / 2.0
    assert out[3, 3, 0, 0] == pytest.approx(2.0 * theta, abs=2e-15)
    assert np.array_equal(out[:, 0], u[:, 0])
    # without the edge points (Gauss x Gauss only) the cell would be admissible
    assert 1.0 - 2.0 / 3.0 > 0


def test_density_factor_closed_form(ref):
    """rho = 1 + 2 xi (mode (1,0) = 2), E = 10: rho(-1, .) = -1 at the
    Lobatto points xi = -1: theta = (1 - eps)/(1 - (-1))."""
    u = np.zeros((4, 4, 1, 1))
    u[0, 0] = 1.0
    u[0, 2] = 2.0   # mode (p, q) = (1, 0)
    u[3, 0] = 10.0
    out = ref.pp_limit2d(_problem(ref, 1), u)
    assert out[0, 2, 0, 0] == pytest.approx(1.0 - EPS, rel=0, abs=4e-16)
    assert np.array_equal(out[:, 0], u[:, 0])


def test_admissible_cells_untouched(ref):
    rng = np.random.default_rng(7)
    for k in (1, 2, 3):
        nx, ny = 8, 4
        u = np.zeros((4, (k + 1) ** 2, ny, nx))
        u[:, 0] = I.conserved2d(rng.uniform(0.5, 2.0, (ny, nx)), rng.uniform(-1, 1, (ny, nx)),
                                rng.uniform(-1, 1, (ny, nx)), rng.uniform(1.0, 2.0, (ny, nx)))
        u[:, 1:] = 0.005 * rng.standard_normal((4, (k + 1) ** 2 - 1, ny, nx))
        out = ref.pp_limit2d(_problem(ref, k, nx, ny), u)
        assert np.array_equal(out, u)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_random_cells_become_positive(ref, k):
    rng = np.random.default_rng(8 + k)
    nx, ny = 20, 10
    nm = (k + 1) ** 2
    u = np.zeros((4, nm, ny, nx))
    rho = rng.uniform(0.01, 2.0, (ny, nx))
    u[:, 0] = I.conserved2d(rho, rng.uniform(-2, 2, (ny, nx)), rng.uniform(-2, 2, (ny, nx)),
                            10.0 ** rng.uniform(-6, 0, (ny, nx)))
    u[:, 1:] = rng.standard_normal((4, nm - 1, ny, nx)) * u[:, :1] * 0.6
    P = _problem(ref, k, nx, ny)
    out = ref.pp_limit2d(P, u)
    np.testing.assert_array_equal(out[:, 0], u[:, 0])
    xi, eta = ref.pp_points2d(P)
    w = _point_values(out, xi, eta)
    # positive at every test point, up to the rounding of this evaluation
    scale = _point_values(np.abs(out), xi, eta)
    assert np.all(w[0] > -1e-14 * scale[0])
    p = _pressure(w)
    assert np.all(p > -1e-12 * (scale[3] + 1.0))
    # the limiter scaled the higher modes of some cells, by a factor in [0, 1]
    changed = np.any(out[:, 1:] != u[:, 1:], axis=(0, 1))
    assert changed.sum() > 10
    ratio = np.where(u[:, 1:] != 0, out[:, 1:] / np.where(u[:, 1:] != 0, u[:, 1:], 1), 1)
    assert np.all(ratio >= -1e-15) and np.all(ratio <= 1 + 1e-15)


def test_rejected_step_leaves_state(ref):
    """A time step far beyond the CFL bound drives cell averages negative:
    the step is rejected and the state is left as it was."""
    w = I.double_mach(32, 8, 1)
    post = I.conserved2d(*w.extra["post"])
    pre = I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = w.extra["shock_speed"] / math.sin(math.pi / 3)
    P = ref.problem2d(2, 1, 32, 8, 0.0, 4.0, 0.0, 1.0, bc=(3, 1, 4, 5), filter=1,
                      dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed, post=post,
                      pre=pre, pp=1)
    alpha = ref.max_wavespeed2d(P, w.u0)
    out, rc = ref.step2d_rc(P, 20.0 / alpha, w.u0)
    assert rc == -5
    assert np.array_equal(out, w.u0)
    # at the CFL step the same state advances
    out, rc = ref.step2d_rc(P, 0.1 / alpha, w.u0)
    assert rc == 0 and not np.array_equal(out, w.u0)


@pytest.mark.slow
def test_double_mach_printed_coefficient_with_limiter_runs(ref):
    """The double Mach reflection (Sec. 3.2) with the printed coefficient,
    Q^3, 64 x 16, filter then limiter: 150 steps with every cell average
    admissible and every value finite.  Without the limiter the printed
    coefficient leaves the linear modes of the shock cells nearly undamped
    (E^1 < 1 there) and the pressure at edge points goes negative in the
    first stage."""
    w = I.double_mach(64, 16, 3)
    post = I.conserved2d(*w.extra["post"])
    pre = I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = w.extra["shock_speed"] / math.sin(math.pi / 3)
    kw = dict(bc=(3, 1, 4, 5), dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
              post=post, pre=pre)
    P = ref.problem2d(2, 3, 64, 16, 0.0, 4.0, 0.0, 1.0, filter=1, pp=1, **kw)
    u, rep, rc = ref.run2d(P, w.u0, 1.0, 150)
    assert rc == 0 and rep.steps == 150 and np.all(np.isfinite(u))
    rho, p = u[0, 0], _pressure(u[:, 0])
    assert rho.min() > 0 and p.min() > 0
    Pn = ref.problem2d(2, 3, 64, 16, 0.0, 4.0, 0.0, 1.0, filter=1, pp=0, **kw)
    alpha = ref.max_wavespeed2d(Pn, w.u0)
    s0 = ref.stage2d(Pn, 0, 0.1 / alpha, w.u0)
    f0, _ = ref.post2d(Pn, 0, 0.1 / alpha, s0, t=0.1 / alpha)
    assert ref.check2d(Pn, f0)[0] == -5
