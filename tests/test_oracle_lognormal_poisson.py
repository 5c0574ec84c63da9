"""Pins for the oracle's lognormal map and Poisson sampler (CPU only)."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import embedding, fields, lognormal_poisson as lp


@pytest.mark.parametrize("m", [0.1, 0.3, 1.0, 5.0, 17.5, 64.0])
def test_chunk_inversion_is_the_poisson_quantile(m):
    """Sequential inversion equals scipy's Poisson quantile function for every u."""
    rng = np.random.default_rng(11)
    u = rng.random(20000)
    u = u[np.abs(stats.poisson.cdf(stats.poisson.ppf(u, m), m) - u) > 1e-12]  # avoid CDF ties
    k = lp.poisson_inverse(u, m)
    assert np.array_equal(k, stats.poisson.ppf(u, m).astype(np.int64))


@pytest.mark.parametrize("mu", [0.1, 0.3, 5.0, 150.0])
def test_counts_mean_equals_variance(mu):
    counts = lp.poisson_counts(np.full(200000, mu), seed=3, request_id=0, realization=5)
    n = counts.size
    assert abs(counts.mean() - mu) < 5 * math.sqrt(mu / n)
    assert abs(counts.var() - mu) < 5 * mu * math.sqrt((2 + 1 / mu) / n)
    assert abs(np.mean(counts == 0) - math.exp(-mu)) < 5 * math.sqrt(math.exp(-mu) / n) + 1e-12


def test_counts_pmf_chisquare():
    mu = 3.7
    counts = lp.poisson_counts(np.full(100000, mu), seed=9, request_id=2, realization=0)
    kmax = 12
    obs = np.bincount(np.minimum(counts, kmax), minlength=kmax + 1)
    p = stats.poisson.pmf(np.arange(kmax), mu)
    p = np.append(p, 1 - p.sum())
    assert stats.chisquare(obs, p * counts.size).pvalue > 1e-4


def test_even_odd_realizations_use_independent_words():
    a = lp.poisson_counts(np.full(50000, 2.0), seed=1, request_id=0, realization=4)
    b = lp.poisson_counts(np.full(50000, 2.0), seed=1, request_id=0, realization=5)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


def test_zero_intensity_gives_zero():
    counts = lp.poisson_counts(np.array([0.0, 0.0, 1e-300]), seed=0, request_id=0, realization=0)
    assert counts[0] == 0 and counts[1] == 0


def test_lognormal_closed_forms():
    s2 = 0.5
    rng = np.random.default_rng(2)
    g = rng.normal(0.0, math.sqrt(s2), 400000)
    d = lp.lognormal_delta(g, s2)
    assert abs(d.mean()) < 5 * math.sqrt((math.exp(s2) - 1) / g.size)
    assert abs(d.var() / (math.exp(s2) - 1) - 1) < 0.03
    assert lp.lognormal_delta(np.array([s2 / 2]), s2)[0] == 0.0


def test_pipeline_moments():
    """E N = nbar and Var N = nbar + nbar^2 (exp(s2) - 1) for a lognormal-Poisson cell."""
    plan = embedding.plan((8, 8), (1.0, 1.0), dict(kind="exp", sigma2=0.5, a=2.0))
    g = fields.generate_fields(plan, seed=0, request_id=0, first_realization=0, count=400)
    nbar = 5.0
    _, counts, ntot = lp.lognormal_poisson(g, plan["sigma2"], nbar, seed=1, request_id=0, first_realization=0)
    c = counts.ravel().astype(float)
    var_th = nbar + nbar ** 2 * (math.exp(0.5) - 1)
    assert abs(c.mean() - nbar) < 6 * math.sqrt(var_th / 400 / 4)  # cells are correlated; loose
    assert abs(c.var() / var_th - 1) < 0.1
    assert np.array_equal(ntot, counts.reshape(400, -1).sum(axis=1))


def test_lognormal_variance_relation_matches_paper_numbers():
    """Sec. 3.4: sigma_A^2 = ln(1 + sigma_delta^2) ~ 0.13 for sigma_delta^2 = 0.14 (Fig. 2)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    s2d = gold["sigma2_delta"]["value"]
    s2a = gold["sigma2_A"]["value"]
    assert abs(math.log(1 + s2d) - s2a) < 0.005
    # and our lognormal map reproduces that variance of delta for Gaussian variance ln(1 + s2d)
    rng = np.random.default_rng(3)
    g = rng.normal(0.0, math.sqrt(math.log(1 + s2d)), 1000000)
    assert abs(lp.lognormal_delta(g, math.log(1 + s2d)).var() - s2d) < 0.003


def test_masked_rate_is_nbar_times_f():
    """Eq. sampling: with the surface fraction f fixed per cell (and rho = 1), counts of every cell
    have mean = variance = nbar f; cells with f = 0 draw nothing.  A rate that ignored f (nbar)
    or applied it twice (nbar f^2) fails every partially covered group by tens of standard errors."""
    nbar, R = 4.0, 120
    fs = np.array([0.0, 0.25, 0.5, 0.85, 1.0])
    mask = np.repeat(fs, 16 * 64).reshape(80, 64).astype(np.float32)   # stripes of 16 rows per value
    delta = np.zeros((R,) + mask.shape)
    _, counts, ntot = lp.lognormal_poisson(delta, 0.0, nbar, seed=8, request_id=3, first_realization=0,
                                           mask=mask, delta=delta)
    assert np.array_equal(ntot, counts.reshape(R, -1).sum(axis=1))
    for f in fs:
        c = counts[:, mask == np.float32(f)].astype(np.float64).ravel()
        mu = nbar * float(np.float32(f))
        if f == 0:
            assert not c.any()
            continue
        n = c.size
        assert abs(c.mean() - mu) < 5 * math.sqrt(mu / n), (f, c.mean(), mu)
        assert abs(c.var() - mu) < 5 * math.sqrt((mu + 2 * mu * mu) / n), (f, c.var(), mu)
        for wrong in (nbar, nbar * float(np.float32(f)) ** 2):
            if abs(wrong - mu) > 1e-12:
                assert abs(c.mean() - wrong) > 20 * math.sqrt(mu / n)
