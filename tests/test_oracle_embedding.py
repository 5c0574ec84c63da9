"""Pins for the oracle's embedding plan and linear field map (CPU only).

The exactness claim of Sec. 2 (the restricted field has covariance xi(x - y)
on the survey grid) is checked by forming the explicit linear map from the
noise to the kept cells and comparing A A^T with the target matrix built here
directly from the two-point function -- not from the oracle's lag table.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import embedding, fields


def target_matrix(n, h, xi_fn):
    """xi(|x - y|) on the survey grid, built from explicit coordinates."""
    cells = list(itertools.product(*[range(x) for x in n]))
    T = np.empty((len(cells), len(cells)))
    for a, x in enumerate(cells):
        for b, y in enumerate(cells):
            T[a, b] = xi_fn(tuple(abs(x[i] - y[i]) for i in range(len(n))), h)
    return T


def linear_map(plan):
    """Columns = kept field for unit real / unit imaginary noise in each mode."""
    M = plan["M"]
    modes = int(np.prod(M))
    cols_re, cols_im = [], []
    for part in (1.0, 1j):
        for k in range(modes):
            eps = np.zeros(modes, dtype=np.complex128)
            eps[k] = part
            Z = fields.field_pair_from_noise(plan, eps.reshape(M)).ravel()
            cols_re.append(Z.real)
            cols_im.append(Z.imag)
    return np.array(cols_re).T, np.array(cols_im).T


def iso(fn):
    return lambda lag, h: fn(math.sqrt(sum((lag[i] * h[i]) ** 2 for i in range(len(lag)))))


CASES = [
    ((5,), (1.0,), dict(kind="exp", sigma2=0.5, a=2.0), iso(lambda r: 0.5 * math.exp(-r / 2.0))),
    ((3, 4), (1.0, 1.0), dict(kind="exp", sigma2=1.3, a=1.5), iso(lambda r: 1.3 * math.exp(-r / 1.5))),
    ((3, 4), (1.0, 0.7), dict(kind="powexp", sigma2=1.0, r0=2.0, gamma=1.8, rc=30.0),
     iso(lambda r: (1 + r / 2.0) ** -1.8 * math.exp(-r / 30.0))),
    ((2, 2, 3), (1.0, 1.0, 1.0), dict(kind="exp", sigma2=0.8, a=1.0), iso(lambda r: 0.8 * math.exp(-r / 1.0))),
]


@pytest.mark.parametrize("n,h,xi,xi_fn", CASES)
def test_restricted_covariance_is_exact(n, h, xi, xi_fn):
    plan = embedding.plan(n, h, xi)
    A_re, A_im = linear_map(plan)
    T = target_matrix(n, h, xi_fn)
    scale = T[0, 0]
    assert np.max(np.abs(A_re @ A_re.T - T)) <= 1e-13 * scale
    assert np.max(np.abs(A_im @ A_im.T - T)) <= 1e-13 * scale
    # the two fields of a pair are independent
    assert np.max(np.abs(A_re @ A_im.T)) <= 1e-13 * scale


def test_restricted_covariance_table_anisotropic():
    # separable (per-axis even) table: xi = exp(-|lx|/2 - |ly|/0.8)
    n = (3, 3)
    tab = np.exp(-np.arange(4)[:, None] / 2.0 - np.arange(4)[None, :] / 0.8)
    plan = embedding.plan(n, (1.0, 1.0), dict(kind="table", table=tab))
    A_re, A_im = linear_map(plan)
    T = target_matrix(n, (1.0, 1.0), lambda lag, h: math.exp(-lag[0] / 2.0 - lag[1] / 0.8))
    assert np.max(np.abs(A_re @ A_re.T - T)) <= 1e-13
    assert np.max(np.abs(A_im @ A_im.T - T)) <= 1e-13


def test_wrong_lag_at_N_would_fail():
    """Guard that the brute-force pin is sensitive: a perturbed plan breaks it."""
    n, h = (3, 4), (1.0, 1.0)
    xi = dict(kind="exp", sigma2=1.3, a=1.5)
    plan = embedding.plan(n, h, xi)
    plan = dict(plan, lam=plan["lam"] * 1.001)
    A_re, _ = linear_map(plan)
    T = target_matrix(n, h, iso(lambda r: 1.3 * math.exp(-r / 1.5)))
    assert np.max(np.abs(A_re @ A_re.T - T)) > 1e-6


@pytest.mark.parametrize("N,a,h", [(8, 3.0, 1.0), (64, 8.0, 1.0), (33, 5.0, 0.5)])
def test_1d_exponential_closed_form(N, a, h):
    """1-D exp kernel: the doubled-grid DFT is a geometric series (Dietrich-Newsam case)."""
    sigma2 = 0.7
    plan = embedding.plan((N,), (h,), dict(kind="exp", sigma2=sigma2, a=a))
    M = 2 * N
    rho = math.exp(-h / a)
    lam = []
    for q in range(M):
        z = rho * complex(math.cos(2 * math.pi * q / M), math.sin(2 * math.pi * q / M))
        s = 1 + 2 * (z * (1 - z ** (N - 1)) / (1 - z)).real + rho ** N * (-1) ** q
        lam.append(sigma2 * s)
    lam = np.array(lam)
    assert np.max(np.abs(plan["lam"] - lam)) <= 1e-12 * lam.max()
    # the 1-D exponential embedding is non-negative (no clamping needed)
    assert lam.min() > 0 and plan["n_clamped"] == 0


def test_dft_identities():
    n, h = (16, 12), (1.0, 1.0)
    xi = dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0)
    c = embedding.lag_table(n, h, xi)
    plan = embedding.plan(n, h, xi)
    lam = plan["lam"]
    assert abs(lam.mean() - 1.0) < 1e-13          # mean eigenvalue = xi(0)
    assert abs(lam.flat[0] - c.sum()) < 1e-11      # DC eigenvalue = sum of lags
    assert plan["sigma2"] == 1.0


def test_not_psd_is_rejected():
    # a top-hat correlation is not positive definite
    n = (16, 16)
    tab = (np.hypot(*np.meshgrid(np.arange(17), np.arange(17), indexing="ij")) < 2.5).astype(float)
    with pytest.raises(embedding.NotPSD) as err:
        embedding.plan(n, (1.0, 1.0), dict(kind="table", table=tab))
    assert err.value.info["lambda_min"] < 0
    assert err.value.info["n_negative"] > 0


def test_3d_powerlaw_large_r0_is_rejected():
    # long-range 3-D correlations at a small side violate the condition
    with pytest.raises(embedding.NotPSD):
        embedding.plan((32, 32, 32), (1.0,) * 3, dict(kind="powexp", sigma2=1.0, r0=10.0, gamma=1.8, rc=0.0))


def test_roundoff_negatives_are_clamped():
    # Gaussian kernel: exact spectrum is positive but tiny; round-off goes slightly negative
    n = (64, 64)
    g = np.meshgrid(np.arange(65.0), np.arange(65.0), indexing="ij")
    tab = np.exp(-(g[0] ** 2 + g[1] ** 2) / (2 * 8.0 ** 2))
    plan = embedding.plan(n, (1.0, 1.0), dict(kind="table", table=tab))
    assert plan["lam"].min() >= 0
    assert plan["n_clamped"] > 0
    assert plan["lambda_min"] > -1e-13 * plan["lambda_max"]


@pytest.mark.parametrize("cfg", ["small_2d", "batched_2d", "volume_3d"])
def test_named_workloads_are_psd(cfg):
    from synth import workloads
    w = workloads.WORKLOADS[cfg]
    if cfg == "volume_3d":
        pytest.skip("512^3 FP64 FFT is covered by the GPU plan test")
    plan = embedding.plan(w["n"], w["h"], w["xi"])
    assert plan["lambda_min"] > 0
