"""Pins for the oracle's spectrum estimator, shells and covariance (CPU only)."""

import itertools
import math

import numpy as np
import pytest

from oracle import embedding, fields, pk


def brute_shell_rect(q, n, nbins):
    """Smallest s >= 0 with s >= nb |k| / k_Ny, |k| / k_Ny = 2 sqrt(sum (q~_i / N_i)^2), compared
    as exact rationals."""
    from fractions import Fraction
    u = sum(Fraction(x if x <= N // 2 else x - N, N) ** 2 for x, N in zip(q, n)) * 4 * nbins * nbins
    s = 0
    while s * s < u:
        s += 1
    b = s - 1
    return b if 0 <= b < nbins else -1


@pytest.mark.parametrize("n,nbins", [((12, 20), 7), ((16, 24), 8), ((6, 10, 8), 4), ((18, 12), 9)])
def test_rectangular_shells_match_rational_enumeration(n, nbins):
    b = pk.shell_index(n, nbins)
    for q in itertools.product(*[range(x) for x in n]):
        assert b[q] == brute_shell_rect(q, n, nbins), q


def test_rectangular_shell_stats():
    """Mean |k| of a shell lies inside it; the modes of all shells are those with |k| <= k_Ny."""
    n, h, nb = (24, 40), 0.5, 10
    nm, km = pk.shell_stats(n, h, nb)
    kny = math.pi / h
    for b in range(nb):
        assert b * kny / nb < km[b] <= (b + 1) * kny / nb
    q0 = np.minimum(np.arange(24), 24 - np.arange(24)) / 24.0
    q1 = np.minimum(np.arange(40), 40 - np.arange(40)) / 40.0
    kk = 2 * np.sqrt(q0[:, None] ** 2 + q1[None, :] ** 2)
    assert nm.sum() == np.count_nonzero((kk > 0) & (kk <= 1 + 1e-12))


def brute_shell(q, N, nbins):
    """Smallest s >= 0 with s^2 N^2 >= 4 nb^2 |q~|^2, by counting up in Python integers."""
    qt = [x if x <= N // 2 else x - N for x in q]
    t = 4 * nbins * nbins * sum(x * x for x in qt)
    s = 0
    while s * s * N * N < t:
        s += 1
    b = s - 1
    return b if 0 <= b < nbins else -1


@pytest.mark.parametrize("N,d,nbins", [(16, 2, 8), (12, 2, 5), (8, 3, 4), (10, 1, 3)])
def test_shells_match_integer_enumeration(N, d, nbins):
    b = pk.shell_index((N,) * d, nbins)
    for q in itertools.product(range(N), repeat=d):
        assert b[q] == brute_shell(q, N, nbins), q


def test_shell_edges_follow_pixel_scale():
    """Outer edge of the last shell is k_Ny = pi / h, the pixel scale pi N / L of Sec. 3.3."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    N = gold["survey_cells_per_side"]["value"]
    L = math.radians(gold["survey_side_deg"]["value"])
    h = L / N
    nmodes, kmean = pk.shell_stats((N, N), h, 20)
    kny = math.pi * N / L
    assert abs(kny - 3088) < 1          # pixel scale of the 128^2 W1 map
    assert kmean[-1] <= kny and kmean[-1] > kny * 0.9
    # the axis Nyquist mode (|q~| = N/2) lies in the last shell
    assert pk.shell_index((N, N), 20)[N // 2, 0] == 19


def test_plane_wave_closed_form():
    N, nb, h = 16, 8, 0.5
    q0 = (3, 1)
    x = np.arange(N)
    phi = np.cos(2 * np.pi * (q0[0] * x[:, None] + q0[1] * x[None, :]) / N)
    P = pk.power_spectrum(phi, h, nb)
    b = pk.shell_index((N, N), nb)
    nmodes, _ = pk.shell_stats((N, N), h, nb)
    expect = np.zeros(nb)
    bb = b[q0]
    expect[bb] = (h ** 2 / N ** 2) * 2 * (N * N / 2) ** 2 / nmodes[bb]
    assert np.allclose(P, expect, atol=1e-12)


def test_white_noise_level():
    rng = np.random.default_rng(0)
    N, nb, h, s2 = 64, 16, 2.0, 0.7
    maps = rng.normal(0, math.sqrt(s2), (200, N, N))
    P = pk.estimate_pk(maps, h, nb).mean(axis=0)
    assert np.all(np.abs(P / (s2 * h * h) - 1) < 0.05)


def test_expected_survey_power_closed_form():
    """<|F(q)|^2> = sum_d prod(N - |d_i|) xi(d) exp(-2 pi i q.d / N) for the exact Gaussian field."""
    N, nb = 12, 6
    xi = dict(kind="exp", sigma2=1.0, a=2.0)
    plan = embedding.plan((N, N), (1.0, 1.0), xi)
    R = 3000
    g = fields.generate_fields(plan, seed=2, request_id=0, first_realization=0, count=R)
    Pm = pk.estimate_pk(g, 1.0, nb)
    # closed form per mode
    d = np.arange(-N + 1, N)
    w = (N - np.abs(d))[:, None] * (N - np.abs(d))[None, :]
    r = np.hypot(d[:, None], d[None, :])
    K = w * np.exp(-r / 2.0)
    q = np.arange(N)
    E = np.exp(-2j * np.pi * np.outer(q, d) / N)
    F2 = (E @ K @ E.T).real
    b = pk.shell_index((N, N), nb)
    nmodes = np.bincount(b[b >= 0], minlength=nb)
    expect = np.bincount(b[b >= 0], weights=F2[b >= 0], minlength=nb) / nmodes / N ** 2
    se = Pm.std(axis=0) / math.sqrt(R)
    assert np.all(np.abs(Pm.mean(axis=0) - expect) < 5 * se)


def test_contrast_from_counts_hand_example():
    c = np.array([[2, 0], [4, 2]])
    assert np.array_equal(pk.contrast_from_counts(c), np.array([[0.0, -1.0], [1.0, 0.0]]))
    f = np.array([[1.0, 0.0], [0.5, 1.0]])
    # N^ = 8 / 2.5 = 3.2; masked cell -> 0
    out = pk.contrast_from_counts(c, mask=f)
    assert np.allclose(out, [[(2 - 3.2) / 3.2, 0.0], [(8 - 3.2) / 3.2, (2 - 3.2) / 3.2]])


def test_covariance_matches_numpy_and_paper_form():
    rng = np.random.default_rng(4)
    P = rng.gamma(5.0, 1.0, (300, 7))
    cov, cp = pk.covariance(P)
    assert np.allclose(cov, np.cov(P, rowvar=False), rtol=1e-13, atol=1e-14)
    m = P.mean(axis=0)
    assert np.allclose(cp, np.mean(P[:, :, None] * P[:, None, :], axis=0) / np.outer(m, m) - 1, rtol=1e-12)


@pytest.mark.parametrize("n,nb,h", [((64, 64), 32, 1.0), ((48, 80), 12, 0.7), ((16, 24, 12), 5, 2.0)])
def test_linear_edges_reproduce_integer_rule(n, nb, h):
    e = np.linspace(0.0, math.pi / h, nb + 1)
    assert np.array_equal(pk.shell_index(n, nb, e, h), pk.shell_index(n, nb))


@pytest.mark.parametrize("n,h", [((128, 128), 1.0), ((96, 64), 0.5), ((20, 16, 24), 1.0)])
def test_log_edges_match_direct_classification(n, h):
    """Shells equally spaced in ln k (the paper's binning): every mode not within 1e-9 of an
    edge is in the shell with e_b < |k| <= e_{b+1}, |k| from its signed frequencies."""
    nb = 20
    kny = math.pi / h
    e = np.exp(np.linspace(math.log(kny / 40.0), math.log(kny), nb + 1))
    b = pk.shell_index(n, nb, e, h)
    grids = np.meshgrid(*[pk.signed_freq(x).astype(np.float64) / x for x in n], indexing="ij")
    k = 2 * math.pi * np.sqrt(sum(g * g for g in grids)) / h
    direct = np.searchsorted(e, k, side="left") - 1
    direct = np.where((direct >= 0) & (direct < nb), direct, -1)
    far = np.min(np.abs(k[..., None] - e), axis=-1) > 1e-9 * k.max()
    assert np.array_equal(b[far], direct[far])
    assert (b >= 0).sum() > 0


def test_kmax_edges_take_the_corners():
    """Edges on (0, pi sqrt(2) / h] (the variant that includes the corners) bin every mode
    but DC."""
    n, nb, h = (32, 32), 10, 1.0
    e = np.linspace(0.0, math.pi * math.sqrt(2.0) / h, nb + 1)
    nm, km = pk.shell_stats(n, h, nb, e)
    assert nm.sum() == 32 * 32 - 1


# rectangular cells (h_i differ): shells in |k| = 2 pi sqrt(sum (q~_i / (N_i h_i))^2) up to
# pi / max h_i

@pytest.mark.parametrize("n,h,nb", [((16, 32), (2.0, 1.0), 10), ((24, 20), (0.5, 0.75), 12),
                                    ((12, 16, 10), (1.0, 0.5, 1.5), 7), ((30, 18), (1.0, 1.0 / 3.0), 9)])
def test_rectangular_cells_match_direct_classification(n, h, nb):
    """Every mode away from an edge lands where the plain FP64 |k| puts it."""
    b = pk.shell_index(n, nb, h=h)
    grids = np.meshgrid(*[pk.signed_freq(x) for x in n], indexing="ij")
    k = 2 * math.pi * np.sqrt(sum((g / (x * hi)) ** 2 for g, x, hi in zip(grids, n, h)))
    u = nb * k / (math.pi / max(h))
    clear = np.abs(u - np.round(u)) > 1e-9
    want = np.where(u > 0, np.ceil(u) - 1, -1).astype(np.int64)
    want = np.where(want < nb, want, -1)
    assert clear.sum() > 0.5 * clear.size
    assert np.array_equal(b[clear], want[clear])
    nm, km = pk.shell_stats(n, h, nb)
    ok = nm > 0
    assert nm.sum() == np.count_nonzero((u > 0) & (u <= nb + 1e-12))
    # mean |k| of every shell lies inside it
    assert np.all(km[ok] > (np.arange(nb)[ok]) * math.pi / max(h) / nb - 1e-12)
    assert np.all(km[ok] <= (np.arange(nb)[ok] + 1) * math.pi / max(h) / nb + 1e-12)


def test_rectangular_cells_reduce_to_a_square_grid():
    """16 x 32 cells of 2 x 1 have the same |k| as the 32 x 32 unit grid on the shared modes
    and shells of the same width (pi / 2 over nb against pi over 2 nb): identical shells."""
    nb = 8
    rect = pk.shell_index((16, 32), nb, h=(2.0, 1.0))
    sq = pk.shell_index((32, 32), 2 * nb)
    for q0 in range(16):
        s0 = q0 if q0 <= 8 else q0 - 16
        for q1 in range(32):
            want = sq[s0 % 32, q1]
            assert rect[q0, q1] == (want if want < nb else -1)
    with pytest.raises(ValueError):
        pk.shell_index((16, 16), 4, h=(1.0, math.sqrt(0.5)))


def test_rectangular_cells_parseval():
    """Shells that take every nonzero mode: sum_b P_b N_b = (prod h_i)(sum phi^2 - (sum phi)^2 / N)."""
    rng = np.random.default_rng(3)
    n, h, nb = (24, 16), (0.5, 1.5), 5
    phi = rng.normal(size=n)
    edges = np.linspace(0.0, 2 * math.pi * math.sqrt(sum((0.5 / x) ** 2 for x in h)) * 1.01, nb + 1)
    p = pk.power_spectrum(phi, h, nb, edges)
    nm, _ = pk.shell_stats(n, h, nb, edges)
    assert nm.sum() == phi.size - 1
    want = h[0] * h[1] * (np.sum(phi ** 2) - phi.sum() ** 2 / phi.size)
    assert abs(np.nansum(p * nm) / want - 1) < 1e-12
