"""Pins for the oracle's counts-in-cells histogram, its Poisson-lognormal prediction and the
A* map (Sec. 3.4, eq. As).  CPU only."""

import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import cic

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
S2A = GOLD["sigma2_A"]["value"]
NBAR = GOLD["nbar_sim"]["value"]
NHIST = GOLD["cic_n_range"]["value"][1] + 1


# --------------------------------------------------------------------------- histogram

def test_histogram_hand_counted():
    """Two 3x3 maps counted by hand; the masked centre cell and counts >= nhist are in no bin."""
    counts = np.array([[[0, 1, 1], [2, 9, 0], [5, 1, 0]],
                       [[3, 3, 3], [3, 0, 7], [1, 2, 4]]])
    f = np.array([[1.0, 0.5, 1.0], [1.0, 0.0, 1.0], [0.25, 1.0, 1.0]], np.float32)
    h = cic.histogram(counts, f, nhist=5)
    # map 0 without the centre: 0,1,1,2,0,5,1,0 -> N=0:3, N=1:3, N=2:1, 5 out of range
    assert h[0].tolist() == [3, 3, 1, 0, 0]
    # map 1 without the centre: 3,3,3,3,7,1,2,4 -> N=1:1, N=2:1, N=3:4, N=4:1, 7 out of range
    assert h[1].tolist() == [0, 1, 1, 4, 1]
    assert cic.histogram(counts, None, nhist=10)[0].tolist() == [3, 3, 1, 0, 0, 1, 0, 0, 0, 1]


# --------------------------------------------------------------------------- prediction

def survey_f(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.2, 1.0, size=n)
    f[rng.uniform(size=n) < 0.1] = 0.0
    return f.astype(np.float32)


def test_prediction_sum_rules():
    """Summed over all N the mixture counts every unmasked cell once; its first moment is
    sum_i N_bar_i, since the log-density has <e^A> = 1."""
    f = survey_f((6, 7), 3)
    nh = 120
    p = cic.predicted_histogram(NBAR, S2A, f, nhist=nh)
    keep = f[f != 0].astype(np.float64)
    assert abs(p.sum() - keep.size) < 1e-8 * keep.size
    assert abs((np.arange(nh) * p).sum() - NBAR * keep.sum()) < 1e-8 * NBAR * keep.sum()


def test_prediction_poisson_limit():
    """sigma_A^2 -> 0: the mixture collapses to a Poisson law with rate N_bar_i per cell."""
    f = survey_f((5, 5), 4)
    p = cic.predicted_histogram(4.0, 1e-10, f, nhist=30)
    keep = f[f != 0].astype(np.float64)
    want = np.array([stats.poisson.pmf(N, 4.0 * keep).sum() for N in range(30)])
    assert np.allclose(p, want, rtol=1e-6, atol=1e-12)


def test_prediction_matches_monte_carlo():
    """Draw A ~ Normal(-s2/2, s2) and N ~ Poisson(N_bar e^A) per cell; the mean histogram of
    many draws agrees with the mixture within its sampling error."""
    rng = np.random.default_rng(11)
    n = (64, 64)
    nh = NHIST
    p = cic.predicted_histogram(NBAR, S2A, None, n=n, nhist=nh)
    R = 40
    A = rng.normal(-0.5 * S2A, math.sqrt(S2A), size=(R,) + n)
    N = rng.poisson(NBAR * np.exp(A))
    h = cic.histogram(N, None, nhist=nh).mean(axis=0)
    cells = np.prod(n)
    sd = np.sqrt(p * (1 - p / cells) / R)
    big = p > 20
    assert np.all(np.abs(h[big] - p[big]) < 5 * sd[big])


# --------------------------------------------------------------------------- A*

@pytest.mark.parametrize("N", [0, 1, 2, 5, 10, 41, 200])
@pytest.mark.parametrize("nbar_i", [0.3, 1.0, 5.0, NBAR])
def test_astar_matches_lambert_closed_form(N, nbar_i):
    a = cic.astar_root(N, nbar_i, S2A)
    b = cic.astar_lambert(N, nbar_i, S2A)
    assert abs(a - b) <= 4e-15 * max(1.0, abs(b))


@pytest.mark.parametrize("N", [0, 3, 17])
def test_astar_residual(N):
    a = cic.astar_root(N, NBAR, S2A)
    lhs = math.exp(a) * NBAR * S2A + a
    assert abs(lhs - S2A * (N - 0.5)) <= 4e-16 * max(1.0, abs(S2A * (N - 0.5)))


def test_astar_small_variance_expansion():
    """For sigma_A^2 -> 0 the root is sigma_A^2 (N - 1/2 - N_bar) + O(sigma_A^4): the
    linearisation of eq. As about A* = 0 (sign and offset of every term)."""
    s2 = 1e-7
    for N in (0, 4, 12):
        for nb in (1.0, 5.0, 9.0):
            a = cic.astar_root(N, nb, s2)
            assert abs(a / s2 - (N - 0.5 - nb)) < 1e-4 * (1 + abs(N - nb)) + 1e-5 * nb * nb


def test_astar_large_n_is_log_map():
    """For large N the transform approaches ln(1 + delta_g) = ln(N / N_bar) (Sec. 3.4)."""
    for nb in (1.0, 5.0, NBAR):
        gaps = [abs(cic.astar_root(N, nb, S2A) - math.log(N / nb)) for N in (10 ** 3, 10 ** 5, 10 ** 7)]
        assert gaps[0] > gaps[1] > gaps[2]
        assert gaps[2] < 1e-4


def test_astar_monotone():
    """A*(N) increases with N and decreases with the intensity (the curves of Fig. 3, lower
    panel: N_bar = 1, 5, 9.68 from top to bottom)."""
    for nb in (1.0, 5.0, NBAR):
        a = [cic.astar_root(N, nb, S2A) for N in range(NHIST)]
        assert all(x < y for x, y in zip(a, a[1:]))
    for N in range(0, NHIST, 7):
        a = [cic.astar_root(N, nb, S2A) for nb in (1.0, 5.0, NBAR)]
        assert a[0] > a[1] > a[2]


def test_astar_map_masks_and_mean():
    rng = np.random.default_rng(5)
    counts = rng.poisson(6.0, size=(3, 5, 6)).astype(np.int32)
    f = survey_f((5, 6), 8)
    m = cic.astar_map(counts, NBAR, S2A, f)
    keep = f != 0
    assert np.all(m[:, ~keep] == 0.0)
    for r in range(3):
        for i in zip(*np.nonzero(keep)):
            assert m[(r,) + i] == cic.astar_root(int(counts[(r,) + i]), NBAR * float(f[i]), S2A)
    c = cic.astar_map(counts, NBAR, S2A, f, subtract_mean=True)
    assert np.all(c[:, ~keep] == 0.0)
    assert np.allclose(c[:, keep].mean(axis=1), 0.0, atol=1e-14)
    assert np.allclose(c[:, keep], m[:, keep] - m[:, keep].mean(axis=1, keepdims=True), atol=1e-15)
