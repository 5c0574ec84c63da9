"""Pins for the oracle's k-space comparator (Sec. 3.3, eq. Periodicboxmodes) and the cumulative
information (eq. cuminfo).  CPU only."""

import math

import numpy as np
import pytest

from oracle import kspace, pk


def exp_2d(k, s, a):
    return 2 * math.pi * s * a * a / (1 + (k * a) ** 2) ** 1.5


def exp_3d(k, s, a):
    return 8 * math.pi * s * a ** 3 / (1 + (k * a) ** 2) ** 2


@pytest.mark.parametrize("k", [0.05, 0.7, 2.0, 4.4])
def test_hankel_2d_exponential(k):
    s, a = 0.5, 2.0
    got = kspace.hankel_2d(lambda r: s * math.exp(-r / a), k, 40 * a)
    assert abs(got / exp_2d(k, s, a) - 1) < 1e-9


@pytest.mark.parametrize("k", [0.1, 1.0, 2.5])
def test_hankel_2d_gaussian(k):
    sg = 1.7
    got = kspace.hankel_2d(lambda r: math.exp(-r * r / (2 * sg * sg)), k, 14 * sg)
    want = 2 * math.pi * sg * sg * math.exp(-k * k * sg * sg / 2)
    assert abs(got - want) < 1e-10 * 2 * math.pi * sg * sg


@pytest.mark.parametrize("k", [0.0, 0.3, 2 * math.pi * 2 / 16, 2 * math.pi * math.sqrt(5) / 16, 1.1, 3.0])
def test_hankel_3d_exponential(k):
    s, a = 0.8, 1.5
    got = kspace.hankel_3d(lambda r: s * math.exp(-r / a), k, 40 * a)
    assert abs(got / exp_3d(k, s, a) - 1) < 1e-11


@pytest.mark.parametrize("d,M,h", [(2, 16, 0.5), (3, 8, 2.0)])
def test_box_plan_modes(d, M, h):
    """lambda(q) = P(2 pi |q~| / (M h)) / h^d on every mode (signed frequencies, Nyquist
    included), DC zeroed, non-negative; the cell variance is sum(lambda) / M^d."""
    s, a = 0.6, 1.3
    xi = dict(kind="exp", sigma2=s, a=a)
    p = kspace.box_plan((M // 2,) * d, M, h, xi)
    lam = p["lam"]
    assert lam.shape == (M,) * d and lam.flat[0] == 0.0 and lam.min() >= 0
    f = exp_2d if d == 2 else exp_3d
    for q in [(1,) + (0,) * (d - 1), (3, M - 4) + (0,) * (d - 2), (M // 2,) * d, (M - 1,) * d]:
        qt = [x if x <= M // 2 else x - M for x in q]
        k = 2 * math.pi * math.sqrt(sum(x * x for x in qt)) / (M * h)
        assert abs(lam[q] / (f(k, s, a) / h ** d) - 1) < 1e-9
    assert p["sigma2"] == lam.sum() / lam.size


def test_box_plan_lognormal_transform():
    xi = dict(kind="powexp", sigma2=0.2, r0=1.0, gamma=0.7, rc=3.0, lognormal=True)
    p = kspace.box_plan((8, 8), 16, 1.0, xi)
    k = 2 * math.pi / 16
    want = kspace.hankel_2d(lambda r: math.log1p(0.2 * (1 + r) ** -0.7 * math.exp(-r / 3.0)), k, 120.0)
    assert abs(p["lam"][1, 0] - want) < 1e-12 * abs(want)
    with pytest.raises(ValueError):
        kspace.box_plan((8, 8), 16, 1.0, dict(kind="powexp", sigma2=0.2, r0=1.0, gamma=0.7, rc=0.0))


def test_cumulative_information_closed_forms():
    """Independent shells of N_b modes (C = diag(2 / N_b), the Gaussian case) give half the
    number of modes; a 2x2 block gives (a + c - 2b) / (ac - b^2); scaling C scales I by 1/s."""
    nb = np.array([4, 8, 12, 20, 28])
    info = pk.cumulative_information(np.diag(2.0 / nb))
    assert np.allclose(info, np.cumsum(nb) / 2.0, rtol=1e-14)
    a, b, c = 0.3, 0.1, 0.5
    info = pk.cumulative_information(np.array([[a, b], [b, c]]))
    assert abs(info[0] - 1 / a) < 1e-14 and abs(info[1] - (a + c - 2 * b) / (a * c - b * b)) < 1e-13
    rng = np.random.default_rng(0)
    X = rng.normal(size=(50, 6))
    C = X.T @ X / 50 + 0.1 * np.eye(6)
    assert np.allclose(pk.cumulative_information(3.0 * C), pk.cumulative_information(C) / 3.0, rtol=1e-12)
