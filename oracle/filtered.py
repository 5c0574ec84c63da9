"""Cell-averaged (square top-hat filtered) two-point function and the lognormal target.
Test infrastructure only.

Sec. 3.1 of the paper takes the density in each cell to be the cell integral of
a continuous field, so the covariance of the cell values is the two-point
function omega averaged over pairs of points of the two cells: the square
top-hat filtered function of App. A.  For cells of sides (h_0, h_1) the overlap
of two box filters leaves (eq. exactformula, with the paper's square cell
h_0 = h_1 = l)

    omega^h(theta) = int_{[-1,1]^2} (1 - |e_0|)(1 - |e_1|) omega(|theta + (h_0 e_0, h_1 e_1)|) d^2e.

At theta = 0 and square cells it reduces to a radial integral (eq. xibar)

    omega^l(0) = 4 int_0^sqrt(2) x omega(l x) F(x) dx,
    F(x) = pi/2 + x^2/2 - 2x (x <= 1);  pi/2 - x^2/2 - 2 acos(1/x) + 2 sqrt(x^2 - 1) - 1 (x >= 1).

Far from the origin the paper uses the derivative expansion (eq. CoolEq)
omega^l ~ omega + (1/12)(l/theta)^2 d^2 omega / d(ln theta)^2, the second
logarithmic derivative from O(h^4) finite differences on an equidistant
logarithmic grid.  The Gaussian log-density then has covariance
omega_A = ln(1 + omega^h) (eq. Lncov).

Readings taken here:

* The paper switches to the expansion at theta / l ~ 15.  Here a lag uses the
  direct integral when |theta| < 15 max(h_0, h_1) and the expansion otherwise.
* Rectangular cells: the exact integral takes (h_0 e_0, h_1 e_1) as above; the
  expansion is the second-order term of the same average for any cell,
  (1/12) sum_i h_i^2 d^2 omega / d theta_i^2, written with the logarithmic
  derivatives D1 = d omega / d ln theta and D2 = d^2 omega / d(ln theta)^2 of
  the isotropic omega:
  (1 / (12 theta^2)) [ (sum_i h_i^2 theta_i^2 / theta^2)(D2 - 2 D1) + D1 sum_i h_i^2 ].
  For square cells this is eq. CoolEq exactly.
* The finite differences are the 5-point central stencils (the four
  neighbours plus the centre) on ln theta with step 2e-3:
  D1 = (f_-2 - 8 f_-1 + 8 f_1 - f_2) / (12 s), D2 = (-f_-2 + 16 f_-1 - 30 f_0 + 16 f_1 - f_2) / (12 s^2).
* The filter is defined for 2-D maps (the paper's angular cells); it needs an
  analytic omega (not a table).

Parity: the direct integral is pinned by a constant and a quadratic omega
(closed forms: the triangular weights integrate to 1 and have second moment 1/6
per axis), by a separable Gaussian omega (product of two 1-D integrals), and by
the paper's own reduction eq. xibar at theta = 0; the expansion by the direct
integral at theta = 15 and 20 cells and by the paper's power-law correction
(1/12)(l/theta)^2 (slope)^2.  See ``tests/test_oracle_filtered.py``.
"""

import math
import warnings

import numpy as np
from scipy import integrate

NEAR_CELLS = 15.0
LOG_STEP = 2e-3


def cell_average_exact(omega, theta, h):
    """Eq. exactformula at the lag vector theta for cells of sides h (2-D), by adaptive
    quadrature split at the kinks of the weights and of the distance."""
    t0, t1 = float(theta[0]), float(theta[1])
    h0, h1 = float(h[0]), float(h[1])

    def f(e0, e1):
        return (1.0 - abs(e0)) * (1.0 - abs(e1)) * omega(math.hypot(t0 + h0 * e0, t1 + h1 * e1))

    def pts(t, hh):
        p = {0.0}
        if abs(t / hh) < 1.0:
            p.add(-t / hh)
        return sorted(p)

    opts = [dict(points=pts(t0, h0), epsabs=1e-15, epsrel=1e-13, limit=200),
            dict(points=pts(t1, h1), epsabs=1e-15, epsrel=1e-13, limit=200)]
    # nquad integrates the first argument innermost; the options follow the same order.
    # (quadpack warns when FP64 round-off stops it short of the requested 1e-13)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        v, _ = integrate.nquad(f, [[-1.0, 1.0], [-1.0, 1.0]], opts=opts)
    return v


def xibar_kernel(x):
    """F(x) of eq. xibar."""
    if x <= 1.0:
        return math.pi / 2 + 0.5 * x * x - 2.0 * x
    return math.pi / 2 - 0.5 * x * x - 2.0 * math.acos(1.0 / x) + 2.0 * math.sqrt(x * x - 1.0) - 1.0


def cell_average_zero(omega, ell):
    """omega^l(0) for square cells of side ell by eq. xibar."""
    g = lambda x: x * omega(ell * x) * xibar_kernel(x)  # noqa: E731
    a, _ = integrate.quad(g, 0.0, 1.0, epsabs=1e-15, epsrel=1e-13, limit=200)
    b, _ = integrate.quad(g, 1.0, math.sqrt(2.0), epsabs=1e-15, epsrel=1e-13, limit=200)
    return 4.0 * (a + b)


def log_derivatives(omega, theta, step=LOG_STEP):
    """D1 = d omega / d ln theta and D2 = d^2 omega / d(ln theta)^2 at the distance theta."""
    lt = math.log(theta)
    f = [float(omega(math.exp(lt + k * step))) for k in (-2, -1, 0, 1, 2)]
    d1 = (f[0] - 8.0 * f[1] + 8.0 * f[3] - f[4]) / (12.0 * step)
    d2 = (-f[0] + 16.0 * f[1] - 30.0 * f[2] + 16.0 * f[3] - f[4]) / (12.0 * step * step)
    return f[2], d1, d2


def cell_average_far(omega, theta, h):
    """Eq. CoolEq (second-order derivative expansion), for cells of sides h."""
    t0, t1 = float(theta[0]), float(theta[1])
    t2 = t0 * t0 + t1 * t1
    w, d1, d2 = log_derivatives(omega, math.sqrt(t2))
    hh = h[0] * h[0] + h[1] * h[1]
    aniso = (h[0] * h[0] * t0 * t0 + h[1] * h[1] * t1 * t1) / t2
    return w + (aniso * (d2 - 2.0 * d1) + d1 * hh) / (12.0 * t2)


def is_near(theta, h):
    t2 = float(theta[0]) ** 2 + float(theta[1]) ** 2
    r = NEAR_CELLS * max(float(h[0]), float(h[1]))
    return t2 < r * r


def cell_averaged_octant(n, h, omega):
    """omega^h on the lag octant l_i in [0, N_i] (shape (N_0+1, N_1+1)): the direct integral
    for lags shorter than 15 cells, the expansion beyond."""
    if len(n) != 2:
        raise ValueError("the cell average is defined for 2-D maps")
    out = np.empty((int(n[0]) + 1, int(n[1]) + 1))
    for l0 in range(out.shape[0]):
        for l1 in range(out.shape[1]):
            th = (h[0] * l0, h[1] * l1)
            out[l0, l1] = cell_average_exact(omega, th, h) if is_near(th, h) else cell_average_far(omega, th, h)
    return out


def lognormal_target(table):
    """omega_A = ln(1 + omega) (eq. Lncov)."""
    return np.log1p(np.asarray(table, dtype=np.float64))
