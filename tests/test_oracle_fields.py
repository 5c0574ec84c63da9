"""Pins for the oracle's noise -> field composition (CPU only).

The exact linear map is pinned in test_oracle_embedding; here the full
Philox -> Box-Muller -> scaling -> inverse DFT -> crop path is checked
statistically against the target covariance xi(x - y) over many draws, with
Re and Im of each pair independent.
"""

import itertools
import math

import numpy as np

from oracle import embedding, fields


def test_empirical_covariance_matches_target():
    n, h = (3, 3), (1.0, 1.0)
    xi = dict(kind="exp", sigma2=0.5, a=2.0)
    plan = embedding.plan(n, h, xi)
    R = 20000
    g = fields.generate_fields(plan, seed=7, request_id=3, first_realization=0, count=R)
    g = g.reshape(R, -1)
    emp = g.T @ g / R
    cells = list(itertools.product(range(3), range(3)))
    T = np.array([[0.5 * math.exp(-math.dist(x, y) / 2.0) for y in cells] for x in cells])
    sigma = np.sqrt((T[0, 0] ** 2 + T ** 2) / R)
    assert np.all(np.abs(emp - T) < 5 * sigma)
    assert np.all(np.abs(g.mean(axis=0)) < 5 * math.sqrt(0.5 / R))
    # Re/Im of a pair are independent: cross-covariance of even vs odd realizations
    cross = g[0::2].T @ g[1::2] / (R // 2)
    assert np.all(np.abs(cross) < 5 * np.sqrt(T[0, 0] ** 2 / (R // 2)))


def test_realization_numbering_is_consistent():
    plan = embedding.plan((4, 4), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=1.0))
    a = fields.generate_fields(plan, seed=1, request_id=0, first_realization=0, count=6)
    b = fields.generate_fields(plan, seed=1, request_id=0, first_realization=2, count=3)
    assert np.array_equal(a[2:5], b)
    c = fields.generate_fields(plan, seed=1, request_id=1, first_realization=0, count=2)
    assert not np.allclose(a[:2], c)
