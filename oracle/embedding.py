"""Embedding plan: lag table, circulant eigenvalues, non-negativity check.
Test infrastructure only (see package doc).

Sec. 2 of the paper enlarges the survey grid x = h (i, j), i, j = 0..N-1 to
i, j = -N..N-1 (eq. grid), i.e. a periodic grid of side M = 2N per axis, and
defines the ad-hoc spectrum as the DFT of the two-point function sampled on
that grid (eq. Specd):

    P~(k) = h^n sum_{x in grid} xi(x) exp(-i k.x),  k = (2 pi / 2L) n,  n_i = 0..2N-1.

With x = h * l and k.x = 2 pi n.l / M this is h^n times the plain DFT
lambda(q) = sum_m c(m) exp(-2 pi i q.m / M) of the lag table c, where grid
index m in [0, M) stands for the lag l = m (m < N) or m - M (m >= N).  The
method requires P~ >= 0 for every mode (eq. condition); it fails otherwise
(text after eq. Papos2).

Readings of the paper taken here:

* Eq. Specd is written for n = 2 with prefactor (L/N)^2; for n dimensions the
  prefactor is h^n (it cancels in the field, since the field only needs
  lambda and the DFT normalisation).
* Index m = N stands for lag -N; because xi is even that equals the minimum
  image |l_i| = min(m_i, M_i - m_i) on every axis.
* Tabulated two-point functions are given on the lag octant l_i in [0, N_i]
  and must be even in every axis separately (true of isotropic functions and
  of the square top-hat filtered function of the appendix).
* Round-off can leave eigenvalues slightly below zero even when the exact
  spectrum is non-negative.  A plan is rejected when
  lambda_min < -tol * lambda_max (tol = 1e-13 by default); otherwise negative
  values are set to zero and counted.

Parity: pinned by (1) brute force on tiny grids -- the covariance of the
restricted field, formed from the explicit linear map, equals the target
matrix xi(x - y) (the exactness claim after eq. Specd); (2) the closed form of
the 1-D exponential kernel's spectrum (geometric series); (3) trace and sum
identities of the DFT.  See ``tests/test_oracle_embedding.py``.
"""

import numpy as np

DEFAULT_NEG_TOL = 1e-13


class NotPSD(Exception):
    """The ad-hoc spectrum has a negative mode beyond round-off (eq. condition fails)."""

    def __init__(self, info):
        super().__init__("embedding spectrum is not non-negative: lambda_min=%g lambda_max=%g"
                         % (info["lambda_min"], info["lambda_max"]))
        self.info = info


def xi_exp(r, sigma2, a):
    """Exponential two-point function sigma2 * exp(-r / a)."""
    return sigma2 * np.exp(-np.asarray(r, dtype=np.float64) / a)


def xi_powexp(r, sigma2, r0, gamma=1.8, rc=0.0):
    """sigma2 * (1 + r/r0)^-gamma * exp(-r/rc); rc <= 0 means no cut-off."""
    r = np.asarray(r, dtype=np.float64)
    out = sigma2 * np.power(1.0 + r / r0, -gamma)
    if rc > 0:
        out = out * np.exp(-r / rc)
    return out


def eval_xi(xi, r):
    """Evaluate an isotropic two-point function spec at distances r."""
    kind = xi["kind"]
    if kind == "exp":
        return xi_exp(r, xi["sigma2"], xi["a"])
    if kind == "powexp":
        return xi_powexp(r, xi["sigma2"], xi["r0"], xi.get("gamma", 1.8), xi.get("rc", 0.0))
    raise ValueError("not an isotropic kind: %r" % kind)


def embedding_shape(n):
    """Side of the periodic embedding per axis: M_i = 2 N_i (eq. grid)."""
    return tuple(2 * int(x) for x in n)


def lag_octant(n, h, xi):
    """xi on the lag octant l_i in [0, N_i] (shape (N_0+1, ..., N_{d-1}+1)).

    Optional flags of the spec: ``cell_average`` (xi is the unfiltered omega; the table holds
    its square top-hat cell average, App. A) and ``lognormal`` (the table holds
    ln(1 + value), eq. Lncov), applied in that order.
    """
    n = tuple(int(x) for x in n)
    if xi["kind"] == "table":
        if xi.get("cell_average"):
            raise ValueError("the cell average needs an analytic two-point function")
        tab = np.asarray(xi["table"], dtype=np.float64)
        if tab.shape != tuple(x + 1 for x in n):
            raise ValueError("table must have shape (N_i + 1)")
        out = tab.copy()
    elif xi.get("cell_average"):
        from . import filtered
        out = filtered.cell_averaged_octant(n, h, lambda r: float(eval_xi(xi, r)))
    else:
        axes = np.meshgrid(*[h[i] * np.arange(n[i] + 1, dtype=np.float64) for i in range(len(n))],
                           indexing="ij")
        r = np.sqrt(sum(a * a for a in axes))
        out = eval_xi(xi, r)
    if xi.get("lognormal"):
        from . import filtered
        out = filtered.lognormal_target(out)
    return out


def lag_table(n, h, xi):
    """c(m) = xi(lag(m)) on the full periodic grid [0, M)^d (eq. grid)."""
    octant = lag_octant(n, h, xi)
    M = embedding_shape(n)
    idx = [np.minimum(np.arange(M[i]), M[i] - np.arange(M[i])) for i in range(len(n))]
    return octant[np.ix_(*idx)]


def eigenvalues(c):
    """lambda(q) = sum_m c(m) exp(-2 pi i q.m / M): the circulant eigenvalues (eq. Specd / h^n).

    c is even, so lambda is real; the imaginary part is checked to be round-off.
    """
    lam = np.fft.fftn(c)
    scale = max(np.max(np.abs(lam.real)), 1e-300)
    if np.max(np.abs(lam.imag)) > 1e-12 * scale:
        raise ValueError("lag table is not even: spectrum has an imaginary part")
    return lam.real.copy()


def plan(n, h, xi, neg_tol=DEFAULT_NEG_TOL):
    """Build the embedding plan: lambda >= 0 on the (2N)^d grid, plus diagnostics.

    Raises NotPSD when the spectrum violates eq. condition beyond round-off.
    Returns dict(lam, sigma2, lambda_min, lambda_max, n_negative, n_clamped, n, h, M).
    """
    if neg_tol < 0:
        neg_tol = DEFAULT_NEG_TOL
    c = lag_table(n, h, xi)
    lam = eigenvalues(c)
    lmin, lmax = float(lam.min()), float(lam.max())
    nneg = int(np.count_nonzero(lam < 0))
    info = dict(lambda_min=lmin, lambda_max=lmax, n_negative=nneg, sigma2=float(c.flat[0]))
    if lmin < -neg_tol * lmax:
        raise NotPSD(info)
    lam = np.maximum(lam, 0.0)
    info.update(lam=lam, n_clamped=nneg, n=tuple(int(x) for x in n),
                h=tuple(float(x) for x in h), M=embedding_shape(n))
    return info
