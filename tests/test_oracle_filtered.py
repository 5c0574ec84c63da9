"""Pins for the oracle's cell-averaged two-point function (App. A: eqs. exactformula, xibar,
CoolEq) and the lognormal target (eq. Lncov).  CPU only."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import embedding, filtered

POWEXP = dict(kind="powexp", sigma2=0.2, r0=2.0, gamma=1.8, rc=300.0)


def om(xi):
    return lambda r: float(embedding.eval_xi(xi, r))


@pytest.mark.parametrize("theta,h", [((0.0, 0.0), (1.0, 1.0)), ((1.0, 0.0), (1.0, 1.0)), ((3.0, 2.1), (1.5, 0.7))])
def test_constant_and_quadratic(theta, h):
    """The triangular overlap weights integrate to 1 and have second moment 1/6 per axis:
    a constant is unchanged and a - b r^2 becomes a - b (theta^2 + (h_0^2 + h_1^2) / 6)."""
    assert abs(filtered.cell_average_exact(lambda r: 0.7, theta, h) - 0.7) < 1e-13
    a, b = 2.0, 0.3
    got = filtered.cell_average_exact(lambda r: a - b * r * r, theta, h)
    want = a - b * (theta[0] ** 2 + theta[1] ** 2 + (h[0] ** 2 + h[1] ** 2) / 6.0)
    assert abs(got - want) < 1e-12


@pytest.mark.parametrize("theta,h", [((0.0, 0.0), (1.0, 1.0)), ((1.0, 0.0), (1.0, 0.7)), ((2.0, 3.0), (1.0, 0.7))])
def test_separable_gaussian(theta, h):
    """exp(-r^2 / 2 s^2) factorises over the axes, so the 2-D average is the product of two 1-D
    averages with the triangular weight."""
    s = 1.3

    def g1(t, hh):
        v, _ = integrate.quad(lambda e: (1 - abs(e)) * math.exp(-(t + hh * e) ** 2 / (2 * s * s)), -1, 1,
                              points=[0.0], epsabs=1e-15, epsrel=1e-13)
        return v

    got = filtered.cell_average_exact(lambda r: math.exp(-r * r / (2 * s * s)), theta, h)
    assert abs(got - g1(theta[0], h[0]) * g1(theta[1], h[1])) < 1e-12


@pytest.mark.parametrize("xi", [dict(kind="exp", sigma2=1.0, a=3.0), POWEXP,
                                dict(kind="powexp", sigma2=1.0, r0=0.5, gamma=1.7, rc=0.0)])
@pytest.mark.parametrize("ell", [1.0, 2.3])
def test_zero_lag_reduction(xi, ell):
    """The paper's radial reduction eq. xibar equals the direct integral eq. exactformula at 0."""
    a = filtered.cell_average_zero(om(xi), ell)
    b = filtered.cell_average_exact(om(xi), (0.0, 0.0), (ell, ell))
    assert abs(a - b) < 1e-11 * abs(b)


def test_xibar_kernel_continuity():
    f = filtered.xibar_kernel
    assert abs(f(1.0 - 1e-12) - f(1.0 + 1e-12)) < 1e-10
    assert abs(f(math.sqrt(2.0))) < 1e-14
    assert abs(f(0.0) - math.pi / 2) < 1e-15


@pytest.mark.parametrize("theta,h", [((15.0, 0.0), (1.0, 1.0)), ((20.0, 0.0), (1.0, 1.0)),
                                     ((11.0, 11.0), (1.0, 1.0)), ((18.0, 9.0), (1.0, 0.6))])
def test_expansion_matches_direct_integral_far_away(theta, h):
    """Eq. CoolEq against eq. exactformula beyond 15 cells: the O((l/theta)^4) remainder is
    far below the correction itself."""
    w = om(POWEXP)
    ex = filtered.cell_average_exact(w, theta, h)
    far = filtered.cell_average_far(w, theta, h)
    unf = w(math.hypot(*theta))
    assert abs(far - ex) < 3e-6 * abs(ex)
    assert abs(far - ex) < 0.05 * abs(ex - unf)


def test_power_law_correction():
    """For omega proportional to theta^-g the correction is (1/12)(l/theta)^2 g^2 (App. A)."""
    g = 0.7
    xi = dict(kind="powexp", sigma2=1.0, r0=1e-3, gamma=g, rc=0.0)
    w = om(xi)
    for theta in (40.0, 80.0):
        ratio = filtered.cell_average_far(w, (theta, 0.0), (1.0, 1.0)) / w(theta) - 1.0
        assert abs(ratio / ((1.0 / 12.0) * (1.0 / theta) ** 2 * g * g) - 1.0) < 1e-3


def test_octant_switches_at_fifteen_cells_and_lognormal():
    n, h = (20, 20), (1.0, 1.0)
    xi = dict(POWEXP, cell_average=True)
    tab = embedding.lag_octant(n, h, xi)
    w = om(POWEXP)
    assert tab[3, 4] == filtered.cell_average_exact(w, (3.0, 4.0), h)
    assert tab[14, 5] == filtered.cell_average_exact(w, (14.0, 5.0), h)   # |theta| = 14.9
    assert tab[15, 0] == filtered.cell_average_far(w, (15.0, 0.0), h)
    assert tab[20, 20] == filtered.cell_average_far(w, (20.0, 20.0), h)
    ln = embedding.lag_octant(n, h, dict(xi, lognormal=True))
    assert np.array_equal(ln, np.log1p(tab))
    # averaging lowers the variance of a cell below the point variance
    assert tab[0, 0] < POWEXP["sigma2"]


def test_lognormal_target_plan():
    """A plan built from ln(1 + omega^h) embeds (the cell average keeps the table positive
    definite) and its cell variance is sigma_A^2 = ln(1 + omega^h(0))."""
    n, h = (16, 16), (1.0, 1.0)
    xi = dict(POWEXP, cell_average=True, lognormal=True)
    p = embedding.plan(n, h, xi)
    w0 = filtered.cell_average_exact(om(POWEXP), (0.0, 0.0), h)
    assert abs(p["sigma2"] - math.log1p(w0)) < 1e-15
    assert p["lambda_min"] >= -1e-13 * p["lambda_max"]
