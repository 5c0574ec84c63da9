"""Counts-in-cells histogram, its Poisson-lognormal prediction and the A* map.
Test infrastructure only.

Sec. 3.4 of the paper checks statistics of the counts beyond the spectrum:

* The counts-in-cells histogram P^(N): the number of cells with count N among
  the cells with f_i != 0 (fully masked cells are ignored), N = 0 .. 41 for
  the W1 map.
* Its mean under the model is a Poisson-lognormal mixture: the log-density A
  of a cell is Gaussian with mean -sigma_A^2 / 2 and variance sigma_A^2, and
  given A the count is Poisson with rate N_bar_i e^A, N_bar_i = N_bar f_i.
  Hence <P^(N)> = int dA G(A) sum_{f_i != 0} Pois(N; N_bar_i e^A).
* The A* map: in each cell, A*(N) is the root of
  e^{A*} N_bar_i sigma_A^2 + A* = sigma_A^2 (N - 1/2) (eq. As), with
  sigma_A^2 = ln(1 + sigma_delta^2) the same in every cell and N_bar_i =
  N_bar f_i the cell's Poisson intensity.  Its spectrum is then estimated.

Readings taken here:

* Counts at or above the histogram length nhist are in no bin (the paper uses
  the range of the data map).
* The left side of eq. As is strictly increasing in A* (its derivative is
  N_bar_i sigma_A^2 e^{A*} + 1 > 0), so the root exists and is unique; it is
  found here by bisection in FP64 until the bracket cannot shrink.  The
  bracket is [d - ln(1 + c e^d) - 1, d] with c = N_bar_i sigma_A^2 and
  d = sigma_A^2 (N - 1/2): the left side minus the right side is positive at
  d and negative at the lower end, because the root is d - W(c e^d) with W
  the principal Lambert function and 0 < W(x) <= ln(1 + x).
* A* is evaluated on cells with f_i != 0 only; masked cells hold 0.  For the
  spectrum the map is A* minus its mean over the unmasked cells, 0 on masked
  cells (the same convention as the galaxy contrast), and it is passed to the
  spectrum estimator of ``pk`` as a plain map.

Parity: the histogram is pinned by a hand-counted fixture and by its sum;
the prediction by its sum rules (total = number of unmasked cells, first
moment = sum of N_bar_i), its Poisson limit at sigma_A^2 -> 0 and a Monte
Carlo draw of the mixture; A* by the Lambert-function closed form
(scipy.special.lambertw), the small-sigma_A^2 expansion, the large-N limit
ln(N / N_bar) stated in the paper, and the residual of eq. As.  See
``tests/test_oracle_cic.py``.
"""

import math

import numpy as np
from scipy import integrate, special


def histogram(counts, mask_f=None, nhist=42):
    """P^(N) for N = 0 .. nhist-1 over cells with f != 0, one row per map (Sec. 3.4).

    counts: (R,) + n integers.  mask_f: n, or None for f = 1.  Returns (R, nhist) int64.
    """
    counts = np.asarray(counts)
    R = counts.shape[0]
    flat = counts.reshape(R, -1)
    keep = np.ones(flat.shape[1], bool) if mask_f is None else (np.asarray(mask_f).reshape(-1) != 0)
    out = np.zeros((R, nhist), np.int64)
    for r in range(R):
        c = flat[r][keep]
        c = c[(c >= 0) & (c < nhist)]
        out[r] = np.bincount(c, minlength=nhist)[:nhist]
    return out


def predicted_histogram(nbar, sigma2_A, mask_f, n=None, nhist=42):
    """<P^(N)>, N = 0 .. nhist-1: the Poisson-lognormal mixture of Sec. 3.4, integrated over
    the Gaussian log-density with scipy.integrate.quad.

    mask_f: the survey's f (any shape), or None together with n (the grid shape) for f = 1.
    """
    f = np.ones(int(np.prod(n))) if mask_f is None else np.asarray(mask_f, np.float64).reshape(-1)
    rates = nbar * f[f != 0]
    s = math.sqrt(sigma2_A)
    mean = -0.5 * sigma2_A
    out = np.zeros(nhist)
    for N in range(nhist):
        lg = math.lgamma(N + 1)

        def integrand(A):
            g = math.exp(-0.5 * ((A - mean) / s) ** 2) / math.sqrt(2 * math.pi * sigma2_A)
            lam = rates * math.exp(A)
            return g * float(np.sum(np.exp(N * np.log(lam) - lam - lg)))

        val, _ = integrate.quad(integrand, mean - 12 * s, mean + 12 * s, limit=200,
                                epsabs=0.0, epsrel=1e-12)
        out[N] = val
    return out


def astar_root(N, nbar_i, sigma2_A):
    """A* of one cell: the root of e^A c + A = d, c = nbar_i sigma2_A, d = sigma2_A (N - 1/2)
    (eq. As), by bisection in FP64."""
    c = float(nbar_i) * sigma2_A
    d = sigma2_A * (float(N) - 0.5)
    y = math.log(c) + d  # ln(c e^d)
    log1p_x = y + math.log1p(math.exp(-y)) if y > 0 else math.log1p(math.exp(y))
    lo, hi = d - log1p_x - 1.0, d

    lnc = math.log(c)

    def g(A):
        if A + lnc > 700.0:  # c e^A beyond FP64 range: far above the root
            return math.inf
        e = c * math.exp(A) if A < 700.0 else math.exp(A + lnc)
        return e + (A - d)

    assert g(lo) < 0 <= g(hi)
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if g(mid) < 0:
            lo = mid
        else:
            hi = mid
    return lo if abs(g(lo)) <= abs(g(hi)) else hi


def astar_map(counts, nbar, sigma2_A, mask_f=None, subtract_mean=False):
    """A* in every cell with f != 0 (0 where f = 0), one map per row of counts (eq. As).

    subtract_mean: subtract the mean of A* over the unmasked cells of each map (the form whose
    spectrum is estimated).  Returns float64 of the shape of counts.
    """
    counts = np.asarray(counts)
    R = counts.shape[0]
    flat = counts.reshape(R, -1)
    f = np.ones(flat.shape[1]) if mask_f is None else np.asarray(mask_f, np.float64).reshape(-1)
    out = np.zeros(flat.shape, np.float64)
    keep = np.nonzero(f != 0)[0]
    memo = {}
    for r in range(R):
        for i in keep:
            key = (int(flat[r, i]), f[i])
            if key not in memo:
                memo[key] = astar_root(key[0], nbar * f[i], sigma2_A)
            out[r, i] = memo[key]
        if subtract_mean and keep.size:
            out[r, keep] -= out[r, keep].mean()
    return out.reshape(counts.shape)


def astar_lambert(N, nbar_i, sigma2_A):
    """A* = d - W0(c e^d): the closed form of the root through the principal Lambert
    function (used only to pin ``astar_root``)."""
    c = nbar_i * sigma2_A
    d = sigma2_A * (N - 0.5)
    return d - special.lambertw(c * math.exp(d)).real
