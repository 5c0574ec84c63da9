"""Counts-in-cells statistics on the GPU through the C ABI (Sec. 3.4): the histogram over
unmasked cells (bit-exact against the oracle), the A* map of eq. As (FP64 solve, against the
oracle's bisection) and its spectrum, and the mean histogram of simulated maps against the
Poisson-lognormal mixture."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cic as ocic, pk as opk  # noqa: E402
from synth import workloads  # noqa: E402

S2A, NBAR = 0.13, 9.68
# A* from the FP64 Newton solve differs from the bisection root by rounding only; the map is
# rounded once to the output precision
TOL_ASTAR = {1: 1e-13, 0: 2e-7}


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


def seeded_counts(count, n, seed, nbar=NBAR, s2=S2A, mask=None, extra=()):
    """Poisson counts with an iid lognormal rate (seeded numpy draws: test input only), plus
    optional planted values."""
    rng = np.random.default_rng(seed)
    A = rng.normal(-0.5 * s2, math.sqrt(s2), size=(count,) + tuple(n))
    f = 1.0 if mask is None else mask.astype(np.float64)
    c = rng.poisson(nbar * f * np.exp(A)).astype(np.int32)
    flat = c.reshape(-1)
    for i, v in extra:
        flat[i] = v
    return c


def status_of(b, fn, *args, **kw):
    try:
        fn(*args, **kw)
    except b.CeError as e:
        return e.status
    return b.OK


@pytest.mark.parametrize("n,masked,nhist", [((37, 41), False, 42), ((64, 64), True, 42), ((12, 10, 14), True, 7),
                                            ((300, 260), True, 1), ((129, 127), False, 4096)])
def test_histogram_matches_oracle(ce, n, masked, nhist):
    b, ctx = ce
    print("histogram", n, masked, nhist, flush=True)
    count = 5
    mask = workloads.survey_mask(n, seed=2) if masked else None
    # planted values: counts past the last bin and a negative count are in no bin
    c = seeded_counts(count, n, 1, mask=mask, extra=[(3, nhist), (17, nhist + 1000), (29, -1)])
    cells = int(np.prod(n))
    out = torch.full((count * nhist,), -5, dtype=torch.int64, device="cuda")
    b.cic_histogram(ctx, torch.from_numpy(c.ravel()).cuda(), cells, count,
                    None if mask is None else torch.from_numpy(mask.ravel()).cuda(), nhist, out)
    torch.cuda.synchronize()
    want = ocic.histogram(c, mask, nhist=nhist)
    assert np.array_equal(out.cpu().numpy().reshape(count, nhist), want)


@pytest.mark.parametrize("n,masked,prec", [((37, 41), False, 1), ((64, 64), True, 1), ((64, 64), True, 0),
                                           ((12, 10, 14), True, 1), ((48, 40), False, 0), ((33, 30), True, 0)])
@pytest.mark.parametrize("subtract", [False, True])
def test_astar_matches_oracle(ce, n, masked, prec, subtract):
    b, ctx = ce
    print("astar", n, masked, prec, subtract, flush=True)
    count = 3
    mask = workloads.survey_mask(n, seed=2) if masked else None
    cells = int(np.prod(n))
    if masked:
        # tiny surface fractions, down to an FP32 denormal
        flat = mask.reshape(-1)
        for i, v in zip((cells // 3, cells // 3 + 1, cells // 3 + 2, cells // 3 + 3), (1e-20, 1e-38, 1.4e-45, 1e-3)):
            flat[i] = v
    # large counts (up to the int32 maximum) and N = 0 everywhere in the first row of the first map
    big = [(cells // 3 + k, v) for k, v in enumerate((5000, 10 ** 6, 2 ** 31 - 1, 77))]
    c = seeded_counts(count, n, 4, mask=mask, extra=big + [(5, 5000)] + [(i, 0) for i in range(n[-1])])
    dt = torch.float64 if prec == 1 else torch.float32
    out = torch.full((count * cells,), 7.0, dtype=dt, device="cuda")
    mean = torch.empty(count, dtype=torch.float64, device="cuda")
    mk = None if mask is None else torch.from_numpy(mask.ravel()).cuda()
    b.astar_map(ctx, torch.from_numpy(c.ravel()).cuda(), cells, count, mk, NBAR, S2A, subtract, prec, out, mean)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape(c.shape)
    raw = ocic.astar_map(c, NBAR, S2A, mask)
    want = ocic.astar_map(c, NBAR, S2A, mask, subtract_mean=True) if subtract else raw
    keep = np.ones(n, bool) if mask is None else mask != 0
    assert np.all(got[:, ~keep] == 0.0)
    scale = np.maximum(1.0, np.abs(want))
    assert np.max(np.abs(got - want) / scale) <= TOL_ASTAR[prec]
    wmean = raw[:, keep].mean(axis=1)
    assert np.allclose(mean.cpu().numpy(), wmean, rtol=1e-13, atol=1e-15)


def test_astar_spectrum_matches_oracle(ce):
    """The spectrum of the mean-subtracted A* map of masked counts, through ce_estimate_pk as a
    plain map, against the oracle's A* map and spectrum estimator."""
    b, ctx = ce
    n, nb, count = (96, 96), 24, 4
    mask = workloads.survey_mask(n, seed=5)
    c = seeded_counts(count, n, 9, mask=mask)
    cells = int(np.prod(n))
    a = torch.empty(count * cells, dtype=torch.float64, device="cuda")
    b.astar_map(ctx, torch.from_numpy(c.ravel()).cuda(), cells, count, torch.from_numpy(mask.ravel()).cuda(),
                NBAR, S2A, True, b.F64, a)
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    b.estimate_pk(ctx, n, (1.0, 1.0), b.F64, b.MAP_FIELD, a, count, None, None, nb, p)
    torch.cuda.synchronize()
    want = opk.estimate_pk(ocic.astar_map(c, NBAR, S2A, mask, subtract_mean=True), 1.0, nb)
    assert np.max(np.abs(p.cpu().numpy().reshape(count, nb) / want - 1)) <= 1e-10


def test_histogram_of_simulated_maps_matches_mixture(ce):
    """Lognormal-Poisson maps from the fused pipeline (the paper's 128^2 geometry, sigma_A^2 =
    0.131, N_bar = 9.68, masked): the mean histogram over 64 maps agrees with the
    Poisson-lognormal mixture prediction within 5 of its realization-to-realization standard
    errors (the one-point law does not depend on the correlations)."""
    b, ctx = ce
    w = workloads.WORKLOADS["paper_128"]
    n, nh, R = w["n"], 42, 64
    mask = workloads.survey_mask(n, seed=1)
    plan = b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    s2 = plan.info["sigma2"]
    cells = plan.cells
    mk = torch.from_numpy(mask.ravel()).cuda()
    c = torch.empty(R * cells, dtype=torch.int32, device="cuda")
    p = torch.empty(R * 8, dtype=torch.float64, device="cuda")
    b.pipeline_run_masked(ctx, plan, mk, 12, 3, 0, R, w["nbar"], 8, p, out_counts=c)
    hist = torch.empty(R * nh, dtype=torch.int64, device="cuda")
    b.cic_histogram(ctx, c, cells, R, mk, nh, hist)
    torch.cuda.synchronize()
    plan.release()
    h = hist.cpu().numpy().reshape(R, nh).astype(np.float64)
    pred = ocic.predicted_histogram(w["nbar"], s2, mask, nhist=nh)
    se = h.std(axis=0, ddof=1) / math.sqrt(R)
    big = pred > 50
    assert big.sum() >= 10
    z = (h.mean(axis=0)[big] - pred[big]) / se[big]
    assert np.all(np.abs(z) < 5), z


@pytest.mark.parametrize("n,masked,nbar,s2,nhist", [((16, 16), False, 9.68, 0.131, 42), ((64, 64), True, 9.68, 0.131, 42),
                                                    ((40, 30), True, 1.0, 1.0, 20), ((24, 24), True, 30.0, 0.5, 120)])
def test_prediction_matches_oracle(ce, n, masked, nbar, s2, nhist):
    """The Poisson-lognormal mixture on the GPU (fixed Gauss-Legendre rule in A) against the
    oracle's adaptive quadrature."""
    b, ctx = ce
    cells = int(np.prod(n))
    mask = workloads.survey_mask(n, seed=6) if masked else None
    if masked:
        mask.reshape(-1)[cells // 2] = 1e-3
    out = torch.empty(nhist, dtype=torch.float64, device="cuda")
    b.cic_predict(ctx, None if mask is None else torch.from_numpy(mask.ravel()).cuda(), cells, nbar, s2, nhist, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = ocic.predicted_histogram(nbar, s2, mask, n=n, nhist=nhist)
    big = want > 1e-6 * want.max()
    assert np.max(np.abs(got[big] / want[big] - 1)) <= 1e-9
    assert np.max(np.abs(got - want)) <= 1e-9 * want.max()


def test_argument_errors(ce):
    b, ctx = ce
    c = torch.zeros(64, dtype=torch.int32, device="cuda")
    h = torch.empty(4096 * 2, dtype=torch.int64, device="cuda")
    a = torch.empty(64, dtype=torch.float64, device="cuda")
    assert status_of(b, b.cic_histogram, ctx, c, 64, 1, None, 0, h) == b.E_INVALID
    assert status_of(b, b.cic_histogram, ctx, c, 32, 1, None, 4097, h) == b.E_INVALID
    assert status_of(b, b.cic_histogram, ctx, c, 0, 1, None, 4, h) == b.E_INVALID
    assert status_of(b, b.astar_map, ctx, c, 64, 1, None, 0.0, S2A, False, b.F64, a) == b.E_INVALID
    assert status_of(b, b.astar_map, ctx, c, 64, 1, None, NBAR, -1.0, False, b.F64, a) == b.E_INVALID
    assert status_of(b, b.astar_map, ctx, c, 64, 1, None, NBAR, float("nan"), False, b.F64, a) == b.E_INVALID
    assert status_of(b, b.astar_map, ctx, c, 64, 1, None, float("inf"), S2A, False, b.F64, a) == b.E_INVALID
    assert status_of(b, b.cic_predict, ctx, None, 64, 0.0, S2A, 8, a) == b.E_INVALID
    assert status_of(b, b.cic_predict, ctx, None, 64, NBAR, 0.0, 8, a) == b.E_INVALID
    assert status_of(b, b.cic_predict, ctx, None, 64, NBAR, S2A, 0, a) == b.E_INVALID
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == b.OK


def test_fully_masked_map(ce):
    """Every cell masked: an all-zero histogram, an all-zero A* map and a zero mean."""
    b, ctx = ce
    n = (16, 16)
    mk = torch.zeros(256, dtype=torch.float32, device="cuda")
    c = torch.from_numpy(seeded_counts(2, n, 3).ravel()).cuda()
    h = torch.full((2 * 8,), 9, dtype=torch.int64, device="cuda")
    b.cic_histogram(ctx, c, 256, 2, mk, 8, h)
    a = torch.full((512,), 3.0, dtype=torch.float32, device="cuda")
    m = torch.full((2,), 3.0, dtype=torch.float64, device="cuda")
    b.astar_map(ctx, c, 256, 2, mk, NBAR, S2A, True, b.F32, a, m)
    torch.cuda.synchronize()
    assert int(h.abs().sum()) == 0 and float(a.abs().sum()) == 0.0 and float(m.abs().sum()) == 0.0


def test_full_size_sampled(ce):
    """The 1024^2 FP32 batched geometry: histogram of 8 maps exactly, A* on sampled cells one
    by one against the oracle's root."""
    b, ctx = ce
    n = (1024, 1024)
    count = 8
    cells = n[0] * n[1]
    mask = workloads.survey_mask(n, seed=4)
    c = seeded_counts(count, n, 21, nbar=NBAR, mask=mask)
    ct = torch.from_numpy(c.ravel()).cuda()
    mk = torch.from_numpy(mask.ravel()).cuda()
    h = torch.empty(count * 42, dtype=torch.int64, device="cuda")
    b.cic_histogram(ctx, ct, cells, count, mk, 42, h)
    a = torch.empty(count * cells, dtype=torch.float32, device="cuda")
    b.astar_map(ctx, ct, cells, count, mk, NBAR, S2A, False, b.F32, a)
    torch.cuda.synchronize()
    assert np.array_equal(h.cpu().numpy().reshape(count, 42), ocic.histogram(c, mask, nhist=42))
    rng = np.random.default_rng(0)
    idx = rng.integers(0, count * cells, size=2000)
    ah = a.cpu().numpy()
    fl = c.reshape(-1)
    mf = mask.reshape(-1)
    for i in idx:
        f = float(mf[i % cells])
        want = 0.0 if f == 0 else ocic.astar_root(int(fl[i]), NBAR * f, S2A)
        assert abs(float(ah[i]) - want) <= TOL_ASTAR[0] * max(1.0, abs(want))
