"""Hand-worked pins of the oracle's damping exponents.

Each expected value below is worked out by hand in the test's docstring from
the paper's formulas, with numbers chosen so that every intermediate is exact
in a few digits; the literals are those hand results, not re-evaluations of
the oracle's own formula.

* Euler, 1D (Sec. 2.4, (para:dampsystems1d) with (para:damp21)): the
  spectral radius beta = |u| + c and the average enthalpy H = (E + p)/rho of
  each cell's average state, the jump sums of every component and the
  maximum over components.  A dropped sound speed, an enthalpy taken as E/rho,
  a sum instead of a maximum over components, or a wrong derivative weight
  each changes the result.
* 2D (Sec. 2.3, (para:damp22d)-(para:damp22d1) with the Euler coefficient of
  Sec. 2.4 / Sec. 3.2): a Q^1 state whose only non-zero mode is the mixed
  mode xi*eta, on non-square cells, so that the mixed derivative d_x d_y and
  the trapezoidal edge averages at the cell corners carry the result, and the
  three readings of the mesh factors of (c_fx, c_fy) give three different
  exponents.
* 2D hybrid indicator (Algorithm 1 in two dimensions): value jumps of
  different size across the two face directions of non-square cells, so
  the sum of the two directions' terms and their mesh widths carry eta.
"""
import numpy as np
import pytest


def test_euler_two_cell_exponent_worked_example(ref):
    """Two periodic cells of width h = 1 on [0, 2], P^1, gamma = 1.4, with
    modes (average, slope) per variable (rho, m, E):

      cell A: rho (1.4, 0.1),  m (0, 0.2),   E (2.5, 0)
      cell B: rho (1.4, -0.1), m (0.7, 0),   E (2.675, 0.4)

    Averages: A has u = 0, p = 0.4 * 2.5 = 1, c = sqrt(1.4 / 1.4) = 1, so
    beta = 1 and H = (2.5 + 1)/1.4 = 2.5.  B has u = 0.5, p = 0.4 (2.675 -
    0.5 * 0.7 * 0.5) = 1, c = 1, beta = 1.5, H = (2.675 + 1)/1.4 = 2.625.

    Traces u(-1) = u0 - u1, u(+1) = u0 + u1; slopes d_x u = (2/h) u1.
    Both cells share the interfaces x = 1 (A | B) and x = 0 = 2 (B | A):
      rho: values 1.5|1.5 and 1.3|1.3 -> J0 = 0;    slopes 0.2, -0.2 -> J1 = 0.8
      m:   values 0.2|0.7 and 0.7|-0.2 -> J0 = 1.4; slopes 0.4, 0     -> J1 = 0.8
      E:   values 2.5|2.275, 3.075|2.5 -> J0 = 0.8; slopes 0, 0.8     -> J1 = 1.6
    The l = 1 sum J0 + 1*2*h*J1 per component: rho 1.6, m 3.0, E 4.0; the
    maximum over components is 4.0 (E).  Exponent (c_f^1 = beta/(4*2*H),
    sigma^1 = c_f^1 (2/h)^2 * 2 * h * sum): E^1 = beta dt / (h H) * 4.0, so
    with dt = 0.1: A: 0.1/2.5 * 4 = 0.16; B: 0.15/2.625 * 4 = 8/35.
    Hybrid indicator eta = max_s J0_s / (2h) = 1.4 / 2 = 0.7 in both cells.
    """
    u = np.zeros((3, 2, 2))
    u[:, :, 0] = [[1.4, 0.1], [0.0, 0.2], [2.5, 0.0]]
    u[:, :, 1] = [[1.4, -0.1], [0.7, 0.0], [2.675, 0.4]]
    P = ref.problem1d(2, 1, 2, 0.0, 2.0, bc=(0, 0), filter=1)
    E, eta = ref.exponents1d(P, 0.1, u)
    assert E[0, 0] == 0.0 and E[1, 0] == 0.0
    assert E[0, 1] == pytest.approx(0.16, rel=1e-13)
    assert E[1, 1] == pytest.approx(8.0 / 35.0, rel=1e-13)
    np.testing.assert_allclose(eta, [0.7, 0.7], rtol=1e-13)
    # the filter multiplies each cell's slope by exp(-E^1) and keeps averages
    out, _ = ref.post1d(P, 0, 0.1, u)
    np.testing.assert_array_equal(out[:, 0], u[:, 0])
    np.testing.assert_allclose(out[:, 1, 0], np.exp(-0.16) * u[:, 1, 0], rtol=1e-14)
    np.testing.assert_allclose(out[:, 1, 1], np.exp(-8.0 / 35.0) * u[:, 1, 1], rtol=1e-14)


# (reading, E^1 / dt, E^2 / dt) worked out in the docstring below
MIXED_CASES = [(0, 3.6, 43.2), (1, 2.4, 24.0), (2, 2.0, 22.4)]


@pytest.mark.parametrize("reading,e1,e2", MIXED_CASES)
def test_2d_mixed_derivative_worked_example(ref, reading, e1, e2):
    """Advection u_t + u_x - 0.5 u_y = 0 (beta^x = 1, beta^y = 0.5, H = 1) on
    [0, 4] x [0, 2] with 2 x 2 periodic cells: h_x = 2, h_y = 1 (non-square).
    Q^1 state u = +-s xi eta (s = 0.1) in a checkerboard: + in cells (0, 0)
    and (1, 1), - in the other two; every face neighbour has the other sign.

    Across a vertical face (xi = +1 on one side, -1 on the other) the value
    s xi eta and d_y u = (2/h_y) s xi agree on both sides; d_x u = (2/h_x) s
    eta jumps by (4/h_x) s |eta| = 0.2 at the corners (eta = +-1), and
    d_x d_y u = (2/h_x)(2/h_y) (+-s) = +-0.2 jumps by 0.4.  Trapezoid edge
    average over the two corners, summed over the two vertical faces:
    Jx(1,0) = 0.4, Jx(1,1) = 0.8, all other Jx zero.  Horizontal faces
    likewise: d_y u jumps by (4/h_y) s = 0.4, so Jy(0,1) = 0.8, Jy(1,1) =
    0.8.

    Jump sums of (para:damp22d1), per direction:
      Sx(1) = 2 h_x^2 (Jx(1,0) + Jx(0,1)) = 2 * 4 * 0.4 = 3.2
      Sx(2) = Sx(1) + 6 h_x^3 (Jx(2,0) + Jx(1,1) + Jx(0,2)) = 3.2 + 38.4 = 41.6
      Sy(1) = 2 h_y^2 * 0.8 = 1.6;  Sy(2) = 1.6 + 6 * 0.8 = 6.4
    With (c_fx, c_fy) = (m_x beta^x, m_y beta^y)/(4 lambda H) and sigma^l =
    sigma_l (2/h_x)(2/h_y) lambda, lambda cancels:
      E^l / dt = [m_x beta^x Sx(l) + m_y beta^y Sy(l)] / (h_x h_y)
      (m_x, m_y) = (h_x, h_y) = (2, 1) (Sec. 2.4): (6.4 + 0.8)/2 = 3.6,
                                                  (83.2 + 3.2)/2 = 43.2
      (m_x, m_y) = (h_y, h_x) = (1, 2) (Sec. 3.2): (3.2 + 1.6)/2 = 2.4,
                                                  (41.6 + 6.4)/2 = 24.0
      (m_x, m_y) = (1, 1):                        (3.2 + 0.8)/2 = 2.0,
                                                  (41.6 + 3.2)/2 = 22.4
    The value jumps are zero, so the hybrid indicator is 0.
    """
    s, k = 0.1, 1
    u = np.zeros((1, 4, 2, 2))
    u[0, 0] = 1.0
    for jy in range(2):
        for ix in range(2):
            u[0, 3, jy, ix] = s if (ix + jy) % 2 == 0 else -s   # mode (p, q) = (1, 1)
    P = ref.problem2d(0, k, 2, 2, 0.0, 4.0, 0.0, 2.0, bc=(0, 0, 0, 0), filter=1,
                      adv_speed=(1.0, -0.5), cf_reading=reading)
    dt = 0.01
    E, eta = ref.exponents2d(P, dt, u)
    for jy in range(2):
        for ix in range(2):
            assert E[jy, ix, 0] == 0.0
            assert E[jy, ix, 1] == pytest.approx(e1 * dt, rel=1e-13)
            assert E[jy, ix, 2] == pytest.approx(e2 * dt, rel=1e-13)
    assert np.all(eta == 0.0)


def test_2d_reading_default_is_printed_sec_2_4(ref):
    """The oracle's default mesh factors are the (h_x, h_y) printed in
    Sec. 2.4 (reading 0)."""
    P0 = ref.problem2d(0, 1, 2, 2, 0.0, 4.0, 0.0, 2.0, filter=1, adv_speed=(1.0, -0.5))
    assert P0.cf_reading == 0


def test_2d_hybrid_indicator_worked_example(ref):
    """2D hybrid indicator (Algorithm 1 with the 2D reading: the value jumps
    averaged over each face by the trapezoid rule at its two corners, summed
    over the two faces of each direction, eta = Jx0/(2 h_x) + Jy0/(2 h_y)).

    Advection on [0, 4] x [0, 2] with 2 x 2 periodic P^0 cells (h_x = 2,
    h_y = 1) holding u = 1 + a (-1)^ix + b (-1)^jy, a = 0.3, b = 0.05.  Every
    vertical face separates ix = 0 from ix = 1 (a jump of 2a = 0.6 at both
    corners), every horizontal face jy = 0 from jy = 1 (2b = 0.1).  Per
    cell Jx0 = 0.6 + 0.6 = 1.2 and Jy0 = 0.1 + 0.1 = 0.2, so
    eta = 1.2/4 + 0.2/2 = 0.3 + 0.1 = 0.4 in every cell.  (A maximum of the
    two terms would give 0.3, swapped mesh widths 0.65.)
    """
    a, b = 0.3, 0.05
    u = np.zeros((1, 1, 2, 2))
    for jy in range(2):
        for ix in range(2):
            u[0, 0, jy, ix] = 1.0 + a * (-1) ** ix + b * (-1) ** jy
    P = ref.problem2d(0, 0, 2, 2, 0.0, 4.0, 0.0, 2.0, bc=(0, 0, 0, 0), filter=2,
                      adv_speed=(1.0, -0.5))
    _, eta = ref.exponents2d(P, 0.01, u)
    np.testing.assert_allclose(eta, np.full((2, 2), 0.4), rtol=1e-14)
