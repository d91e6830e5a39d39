"""Pins of the oracle's positivity-preserving limiter (Zhang and Shu, used
after the filter for the extreme cases of Sec. 3.2) and of the step
rejection / half-dt retry that goes with it.

Closed forms: cells whose only negative point value sits at a known test
point give the limiting factor in closed form; the Gauss-Lobatto set of
each degree is pinned by a P3 cell whose only negative pressure is at the
cell centre (a Gauss-Lobatto point of N = 3, not a Gauss point of Q = 4).
Invariants: admissible cells untouched, cell averages untouched, positivity
at every test point afterwards (evaluated here with numpy's Legendre
series, not the oracle's), conservation over rejected steps."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import dg_inputs as I

GAMMA = 1.4
EPS = 1e-13


def _cell_state(rho, mom, ener, n=1):
    """(3, k+1, n) modal state repeating one cell's modes n times."""
    k = len(rho) - 1
    u = np.zeros((3, k + 1, n))
    for v, modes in enumerate((rho, mom, ener)):
        u[v, :, :] = np.asarray(modes, float)[:, None]
    return u


def _problem(ref, k, n, **kw):
    return ref.problem1d(2, k, n, -1.0, 1.0, bc=(1, 1), filter=1, cfl=0.1, pp=1, **kw)


def _test_points(k):
    N = (k + 4) // 2
    gl = {2: [-1.0, 1.0], 3: [-1.0, 0.0, 1.0]}[N]
    xg, _ = npleg.leggauss(k + 1)
    return np.array(gl + list(xg))


def _point_values(u, xs):
    """Point values (3, npts, n) of a modal state at reference points."""
    k = u.shape[1] - 1
    V = np.array([[npleg.legval(x, np.eye(k + 1)[l]) for l in range(k + 1)] for x in xs])
    return np.einsum("pl,vln->vpn", V, u)


def test_pressure_factor_closed_form_p1(ref):
    # rho = 1, m = 0, E = 1 + 2 xi: p(-1) = 0.4 (1 - 2) < 0; the factor on
    # the energy slope solves 0.4 (1 - 2 theta) = eps
    u = _cell_state([1.0, 0.0], [0.0, 0.0], [1.0, 2.0])
    out = ref.pp_limit1d(_problem(ref, 1, 1), u)
    theta = (1.0 - EPS / (GAMMA - 1.0)) / 2.0
    assert out[2, 1, 0] == pytest.approx(2.0 * theta, abs=1e-15)
    assert out[2, 1, 0] <= 2.0 * theta + 2e-16
    assert np.array_equal(out[:, 0], u[:, 0])
    assert out[0, 1, 0] == 0.0 and out[1, 1, 0] == 0.0


def test_density_factor_closed_form_p1(ref):
    # rho = 1 + 2 xi: rho(-1) = -1; theta = (1 - eps) / (1 - (-1))
    u = _cell_state([1.0, 2.0], [0.0, 0.0], [10.0, 0.0])
    out = ref.pp_limit1d(_problem(ref, 1, 1), u)
    assert out[0, 1, 0] == pytest.approx(1.0 - EPS, rel=0, abs=4e-16)
    assert np.array_equal(out[:, 0], u[:, 0])
    assert out[2, 1, 0] == 0.0


def test_centre_point_p2(ref):
    # E = 1 + 4 P2(xi): E(0) = -1 (the centre is a Gauss-Lobatto point and,
    # for Q = 3, a Gauss point), E(+-1) = 5
    u = _cell_state([1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 4.0])
    out = ref.pp_limit1d(_problem(ref, 2, 1), u)
    theta = (1.0 - EPS / (GAMMA - 1.0)) / 2.0
    assert out[2, 2, 0] == pytest.approx(4.0 * theta, abs=2e-15)


def test_gauss_lobatto_set_p3(ref):
    # Degree 3 uses N = ceil((3+3)/2) = 3 Gauss-Lobatto points {-1, 0, 1}.
    # E = 1 + e2 P2 with e2 = 2.2: E(0) = -0.1 < 0, the only negative value
    # among the test points (at the 4 Gauss points P2 >= -0.33, E >= 0.27),
    # so the factor comes from the centre: 0.4 (1 - 1.1 theta) = eps
    e2 = 2.2
    xs = _test_points(3)
    vals = 1.0 + e2 * npleg.legval(xs, [0, 0, 1])
    assert (vals[np.abs(xs) > 1e-12] > 0).all() and 1.0 - e2 / 2 < 0
    u = _cell_state([1.0, 0.0, 0.0, 0.0], [0.0] * 4, [1.0, 0.0, e2, 0.0])
    out = ref.pp_limit1d(_problem(ref, 3, 1), u)
    theta = (1.0 - EPS / (GAMMA - 1.0)) / (e2 / 2.0)
    assert out[2, 2, 0] == pytest.approx(e2 * theta, abs=2e-15)


def test_admissible_cells_untouched(ref):
    rng = np.random.default_rng(5)
    for k in (1, 2, 3):
        n = 64
        u = np.zeros((3, k + 1, n))
        u[0, 0] = rng.uniform(0.5, 2.0, n)
        u[1, 0] = rng.uniform(-1.0, 1.0, n)
        u[2, 0] = rng.uniform(3.0, 5.0, n)
        u[:, 1:] = 0.01 * rng.standard_normal((3, k, n))
        out = ref.pp_limit1d(_problem(ref, k, n), u)
        assert np.array_equal(out, u)


def test_random_cells_become_positive(ref):
    rng = np.random.default_rng(6)
    for k in (1, 2, 3):
        n = 400
        u = np.zeros((3, k + 1, n))
        rho = 10.0 ** rng.uniform(-2, 1, n)
        vel = rng.uniform(-3, 3, n)
        p = 10.0 ** rng.uniform(-3, 2, n)
        u[0, 0], u[1, 0], u[2, 0] = I.conserved(rho, vel, p)
        u[:, 1:] = u[:, :1] * rng.uniform(-1.5, 1.5, (3, k, n))
        P = _problem(ref, k, n)
        out = ref.pp_limit1d(P, u)
        assert np.array_equal(out[:, 0], u[:, 0])
        w = _point_values(out, _test_points(k))
        pmin = (GAMMA - 1.0) * (w[2] - 0.5 * w[1] ** 2 / w[0])
        eps = np.minimum(EPS, np.minimum(rho, p))
        assert (w[0] >= eps * (1 - 1e-9) - 1e-18).all()
        # the pressure at a point cancels E against m^2/(2 rho): allow the
        # rounding of that difference and of the point density (evaluated
        # here in another summation order than the limiter's)
        kin = 0.5 * w[1] ** 2 / w[0]
        rho_err = 1e-15 * np.abs(out[0]).sum(axis=0)[None, :]
        e_err = 1e-15 * np.abs(out[2]).sum(axis=0)[None, :]
        tol = 1e-13 * kin + 4.0 * (e_err + kin * rho_err / w[0])
        assert (pmin >= eps * (1 - 1e-6) - tol).all()
        # modes >= 1 are only scaled down, by one factor per variable
        ratio = np.where(u[:, 1:] != 0, out[:, 1:] / np.where(u[:, 1:] != 0, u[:, 1:], 1), np.nan)
        assert np.nanmax(ratio) <= 1.0 + 1e-15 and np.nanmin(ratio) >= 0.0
        for v in range(3):
            spread = np.nanmax(ratio[v], axis=0) - np.nanmin(ratio[v], axis=0)
            assert np.nanmax(spread) <= 1e-12


def test_rejected_step_leaves_state(ref):
    # an absurd time step drives a stage average negative: the step is
    # rejected and nothing is written
    w = I.riemann1d((1.0, 0.0, 1000.0), (0.1, 0.0, 0.01), 64, 2)
    P = _problem(ref, 2, 64)
    bf = np.zeros(4)
    out, rc = ref.step1d_rc(P, 0.5, w.u0, bf)
    assert rc == -5
    assert np.array_equal(out, w.u0) and (bf == 0).all()


@pytest.mark.parametrize("cfl", [0.1, 0.2])
def test_random_riemann_survive_with_restarts_conserving(ref, cfl):
    """Seeded draws with the batched workload's ranges (rho in [0.1, 10],
    p in [0.01, 1000], |u| <= 2): with the limiter every problem reaches
    200 steps, finite and positive, and the FP64 ledger closes over the
    rejected and retried steps (at CFL 0.2 some stages break the CFL bound
    of the positivity argument and are retried)."""
    spec = I.batched_riemann_spec(24, 4001, 96, 160, 1, 3)
    states = I.batched_riemann_states(spec)
    total_restarts = 0
    for i in range(24):
        n, k = int(spec.n[i]), int(spec.k[i])
        P = ref.problem1d(2, k, n, -1.0, 1.0, bc=(1, 1), filter=1, cfl=cfl, pp=1)
        u, rep, rc = ref.run1d(P, states[i], 1e30, 200)
        assert rc == 0 and rep.steps == 200, (i, rc, rep.steps)
        assert ref.check1d(P, u)[0] == 0
        h = 2.0 / n
        for v in range(3):
            q0 = h * states[i][v, 0].sum()
            assert abs(rep.ledger[v] + rep.boundary_flux[v] - q0) < 1e-12 * max(1.0, abs(q0))
        total_restarts += rep.restarts
    if cfl == 0.2:
        assert total_restarts > 0  # the draw exercises the retry path
