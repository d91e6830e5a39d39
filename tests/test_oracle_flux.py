"""Pins of the oracle's interface fluxes for the Euler equations: local
Lax-Friedrichs (the paper's choice, Sec. 3) and the HLL / HLLC fluxes that
Sec. 3 names as alternatives (Davis wave-speed estimates).

What fixes them, independently of their code:
  * consistency, F(U, U) = f(U), for every flux, in 1D and across x and y
    faces in 2D;
  * upwinding: with every wave moving right (u - c > 0 on both sides) HLL and
    HLLC return f(U_L) exactly, and f(U_R) when every wave moves left;
  * HLL equals LLF exactly when the wave-speed bounds are -c and +c (both
    states at rest with the same sound speed);
  * HLLC resolves contact waves exactly: across a stationary contact (equal
    pressure, no normal velocity, any density and tangential-velocity jump)
    its mass flux is zero and its momentum flux is the pressure, where HLL
    and LLF diffuse; across a contact moving right it is f(U_L);
  * mirror symmetry: reflecting x and swapping the sides flips the sign of
    the mass and energy fluxes;
  * the exact Riemann solution: a run with HLLC puts the Lax shock where the
    exact solution does.  (Single fluxes are not compared with the Godunov
    flux: with Davis's speed bounds HLLC's contact speed on the Sod problem
    is 0.68 against the exact 0.93, a property of the method.)"""
import os

import numpy as np
import pytest

import dg_inputs as I
import oracle as O
from oracle import exact

GAMMA = 1.4
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cons1d(rho, u, p):
    return np.array([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u])


def phys1d(U):
    rho, m, E = U
    u = m / rho
    p = (GAMMA - 1) * (E - 0.5 * m * u)
    return np.array([m, m * u + p, u * (E + p)])


def _p1(flux):
    return O.problem1d(O.EULER, 1, 4, 0.0, 1.0, flux=flux)


def _p2(flux):
    return O.problem2d(O.EULER, 1, 4, 4, 0.0, 1.0, 0.0, 1.0, flux=flux)


def _random_states(rng, n):
    rho = 10 ** rng.uniform(-1, 1, n)
    u = rng.uniform(-3, 3, n)
    v = rng.uniform(-3, 3, n)
    p = 10 ** rng.uniform(-1, 2, n)
    return rho, u, v, p


@pytest.mark.parametrize("flux", [O.FLUX_LLF, O.FLUX_HLL, O.FLUX_HLLC])
def test_consistency(flux):
    rng = np.random.default_rng(11)
    P1, P2 = _p1(flux), _p2(flux)
    for rho, u, v, p in zip(*_random_states(rng, 200)):
        U = cons1d(rho, u, p)
        np.testing.assert_allclose(O.numflux1d(P1, U, U), phys1d(U), rtol=1e-14, atol=1e-14)
        U2 = I.conserved2d(rho, u, v, p)
        for d, (un, ut) in enumerate(((u, v), (v, u))):
            F = O.numflux2d(P2, d, U2, U2)
            E = U2[3]
            want = np.zeros(4)
            want[0] = rho * un
            want[1] = rho * u * un + (p if d == 0 else 0.0)
            want[2] = rho * v * un + (p if d == 1 else 0.0)
            want[3] = un * (E + p)
            np.testing.assert_allclose(F, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("flux", [O.FLUX_HLL, O.FLUX_HLLC])
def test_supersonic_upwinding(flux):
    P = _p1(flux)
    UL, UR = cons1d(1.0, 3.0, 1.0), cons1d(0.5, 2.5, 0.4)   # u - c > 0 on both sides
    assert np.array_equal(O.numflux1d(P, UL, UR), phys1d(UL))
    UL, UR = cons1d(1.0, -3.0, 1.0), cons1d(0.5, -2.5, 0.4)
    assert np.array_equal(O.numflux1d(P, UL, UR), phys1d(UR))


def test_hll_reduces_to_llf_for_symmetric_speed_bounds():
    # both at rest with c = sqrt(1.4): S_L = -c, S_R = +c, the LLF alpha
    UL, UR = cons1d(2.0, 0.0, 2.0), cons1d(1.0, 0.0, 1.0)
    np.testing.assert_allclose(O.numflux1d(_p1(O.FLUX_HLL), UL, UR),
                               O.numflux1d(_p1(O.FLUX_LLF), UL, UR), rtol=1e-15, atol=1e-15)


def test_hllc_resolves_contacts():
    UL, UR = cons1d(1.0, 0.0, 1.0), cons1d(0.125, 0.0, 1.0)
    F = O.numflux1d(_p1(O.FLUX_HLLC), UL, UR)
    np.testing.assert_allclose(F, [0.0, 1.0, 0.0], atol=1e-15)
    assert abs(O.numflux1d(_p1(O.FLUX_HLL), UL, UR)[0]) > 1e-2
    assert abs(O.numflux1d(_p1(O.FLUX_LLF), UL, UR)[0]) > 1e-2
    # 2D: a shear layer (tangential velocity jump) at rest across an x face
    A, B = I.conserved2d(1.0, 0.0, 0.7, 1.0), I.conserved2d(0.3, 0.0, -0.4, 1.0)
    F2 = O.numflux2d(_p2(O.FLUX_HLLC), 0, A, B)
    np.testing.assert_allclose(F2, [0.0, 1.0, 0.0, 0.0], atol=1e-15)
    # the same across a y face (normal momentum is the y component)
    A, B = I.conserved2d(1.0, 0.7, 0.0, 1.0), I.conserved2d(0.3, -0.4, 0.0, 1.0)
    np.testing.assert_allclose(O.numflux2d(_p2(O.FLUX_HLLC), 1, A, B), [0.0, 0.0, 1.0, 0.0],
                               atol=1e-15)
    # a contact moving right: the face sees the left state
    UL, UR = cons1d(1.0, 0.5, 1.0), cons1d(0.2, 0.5, 1.0)
    np.testing.assert_allclose(O.numflux1d(_p1(O.FLUX_HLLC), UL, UR), phys1d(UL), rtol=1e-14)


@pytest.mark.parametrize("flux", [O.FLUX_LLF, O.FLUX_HLL, O.FLUX_HLLC])
def test_mirror_symmetry(flux):
    rng = np.random.default_rng(12)
    P = _p1(flux)
    r, u, _, p = _random_states(rng, 100)
    for i in range(50):
        UL, UR = cons1d(r[2 * i], u[2 * i], p[2 * i]), cons1d(r[2 * i + 1], u[2 * i + 1], p[2 * i + 1])
        F = O.numflux1d(P, UL, UR)
        M = np.array([1.0, -1.0, 1.0])
        G = O.numflux1d(P, M * UR, M * UL)
        np.testing.assert_allclose(F * np.array([-1.0, 1.0, -1.0]), G, rtol=1e-12, atol=1e-12)


def test_hllc_run_puts_the_lax_shock_where_the_exact_solution_does():
    states = np.loadtxt(os.path.join(GOLD, "lax_states.txt"))
    left, right = tuple(states[0]), tuple(states[1])
    w = I.lax(200, 2)
    P = O.problem1d(O.EULER, 2, 200, -1.0, 1.0, bc=(1, 1), filter=O.FILTER_JUMP, cfl=0.1,
                    flux=O.FLUX_HLLC)
    u, rep, rc = O.run1d(P, w.u0, 0.13)
    assert rc == 0 and rep.t == 0.13
    h = 0.01
    xc = -1.0 + (np.arange(200) + 0.5) * h
    rho_ex, _, _ = exact.riemann_exact(left, right, xc, 0.13)
    rho = u[0, 0]
    assert np.sum(np.abs(rho - rho_ex)) * h < 0.02
    _, _, sr = exact.riemann_waves(left, right)
    jump = np.abs(np.diff(rho))
    jj = int(np.argmax(np.where(xc[:-1] > 0.3, jump, 0.0)))
    assert abs(0.5 * (xc[jj] + xc[jj + 1]) - sr * 0.13) < 2 * h
