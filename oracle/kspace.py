"""The k-space sampling comparator: a periodic box whose modes follow the continuous
spectrum.  Test infrastructure only.

Sec. 3.3 of the paper compares the exact method with the classical construction: A is
simulated on a periodic box of side M cells (128, 256 or 512 for the 128^2 map) whose
Fourier modes have the variance of the continuous field, the Fourier integral of
ln(1 + omega) over the whole plane (eq. Periodicboxmodes), with the DC mode set to zero;
the survey is a 128^2 corner of the box.

For an isotropic two-point function the Fourier integral is a Hankel transform,

    2-D:  P(k) = 2 pi int_0^inf r J0(k r) xi(r) dr,
    3-D:  P(k) = 4 pi int_0^inf r^2 (sin(k r) / (k r)) xi(r) dr.

On a periodic box of M^d cells of side h the DFT amplitudes of the sampled field then have
variance M^d lambda(q) with lambda(q) = P(|k_q|) / h^d, k_q = 2 pi q~ / (M h) (q~ the signed
frequency), the same normalisation as the circulant eigenvalues of eq. Specd, so the
generator of ``fields`` runs unchanged on the box.

Readings taken here:

* Square / cubic boxes with equal h on every axis; the survey is cells [0, N)^d of the box.
* The xi fed to the transform is the spec's function after its lognormal transform
  (ln(1 + omega)); the cell average of App. A does not enter (the k-space method samples
  the continuous field at the cell centres).
* lambda(0) = 0 (the DC mode is zeroed, as stated).
* Both transforms are integrated between consecutive zeros of the oscillating factor (J0 from
  scipy in 2-D, sin(k r) in 3-D) up to the radius where the exponential cut-off of xi has
  reached e^-40.

Parity: pinned by the closed forms of the exponential two-point function in 2-D,
2 pi s a^2 / (1 + k^2 a^2)^(3/2), and 3-D, 8 pi s a^3 / (1 + k^2 a^2)^2, and of a 2-D
Gaussian; the box plan by those closed forms on chosen modes (signed frequencies, the
Nyquist corner), its zeroed DC mode and its cell variance.  See
``tests/test_oracle_kspace.py``.
"""

import math
import warnings

import numpy as np
from scipy import integrate, special

from . import embedding


def hankel_2d(xi_fn, k, rmax):
    """2 pi int_0^inf r J0(k r) xi(r) dr, integrated between zeros of J0 up to rmax."""
    if k == 0:
        edges = np.linspace(0.0, rmax, 2001)
    else:
        nz = int(k * rmax / math.pi) + 2
        zeros = special.jn_zeros(0, nz) / k
        edges = np.concatenate([[0.0], zeros[zeros < rmax], [rmax]])
    tot = 0.0
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        for a, b in zip(edges[:-1], edges[1:]):
            v, _ = integrate.quad(lambda r: r * special.j0(k * r) * xi_fn(r), a, b, epsabs=0.0, epsrel=1e-13,
                                  limit=200)
            tot += v
    return 2.0 * math.pi * tot


def hankel_3d(xi_fn, k, rmax):
    """4 pi int_0^inf r^2 sinc(k r) xi(r) dr = (4 pi / k) int_0^inf r xi(r) sin(k r) dr, integrated
    between consecutive zeros of sin(k r) up to rmax."""
    if k == 0:
        edges = np.linspace(0.0, rmax, 2001)
    else:
        nz = int(k * rmax / math.pi) + 1
        zeros = math.pi * np.arange(1, nz + 1) / k
        edges = np.concatenate([[0.0], zeros[zeros < rmax], [rmax]])
    tot = 0.0
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        for a, b in zip(edges[:-1], edges[1:]):
            if k == 0:
                f = lambda r: r * r * xi_fn(r)  # noqa: E731
            else:
                f = lambda r: r * math.sin(k * r) * xi_fn(r) / k  # noqa: E731
            v, _ = integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=200)
            tot += v
    return 4.0 * math.pi * tot


def xi_of(xi):
    """The spec's function of r after its lognormal transform (no cell average)."""
    base = {k: v for k, v in xi.items() if k not in ("cell_average", "lognormal")}
    if xi.get("lognormal"):
        return lambda r: math.log1p(float(embedding.eval_xi(base, r)))
    return lambda r: float(embedding.eval_xi(base, r))


def cutoff_radius(xi):
    """Radius beyond which the exponential cut-off leaves xi below e^-40 of its scale."""
    if xi["kind"] == "exp":
        return 40.0 * xi["a"]
    if xi["kind"] == "powexp" and xi.get("rc", 0.0) > 0:
        return 40.0 * xi["rc"]
    raise ValueError("the periodic box needs a two-point function with an exponential cut-off")


def box_plan(n, M, h, xi):
    """lambda on the periodic box of side M (square / cubic, cell side h), survey n in its corner.

    Returns a plan dict accepted by ``fields.generate_fields`` (lam, M, n, sigma2)."""
    d = len(n)
    M = int(M)
    fn = xi_of(xi)
    rmax = cutoff_radius(xi)
    q = np.arange(M)
    qt = np.where(q <= M // 2, q, q - M).astype(np.int64)
    grids = np.meshgrid(*([qt] * d), indexing="ij")
    s = sum(g * g for g in grids)
    lam = np.zeros(s.shape)
    cache = {}
    for val in np.unique(s):
        if val == 0:
            continue
        k = 2.0 * math.pi * math.sqrt(float(val)) / (M * h)
        cache[int(val)] = (hankel_2d(fn, k, rmax) if d == 2 else hankel_3d(fn, k, rmax)) / h ** d
    for val, p in cache.items():
        lam[s == val] = p
    return dict(lam=lam, M=(M,) * d, n=tuple(int(x) for x in n), h=(float(h),) * d,
                sigma2=float(lam.sum() / lam.size))
