"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical Philox streams.

Tolerances (relative L2 per realization unless stated; fields and delta are also bounded
element by element: max |dg| <= tol sqrt(xi(0)), |d delta| <= tol (1 + |delta|)):
  Philox words          bit-exact
  normals               FP32 1e-6,  FP64 1e-14
  eigenvalues           1e-12 * lambda_max (absolute)
  fields                FP32 1e-5,  FP64 1e-12
  delta (from GPU g)    FP32 1e-5,  FP64 1e-12
  counts, N_tot         bit-exact (oracle fed the GPU's delta)
  P(k) per shell        FP32 1e-5,  FP64 1e-12 (oracle fed the GPU's maps)
  covariance            1e-12 (oracle fed the GPU's spectra)
"""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import embedding, fields as ofields, lognormal_poisson as olp, philox, pk as opk  # noqa: E402
from parity_check import check_delta, check_maps  # noqa: E402

TOL_FIELD = {0: 1e-5, 1: 1e-12}
TOL_PK = {0: 1e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dt(prec):
    return torch.float64 if prec == 1 else torch.float32


def gpu_fields(b, ctx, plan, seed, rid, first, count):
    out = torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda")
    b.generate_fields(ctx, plan, seed, rid, first, count, out)
    torch.cuda.synchronize()
    return out


def test_philox_words_bit_exact(ce):
    b, _ = ce
    for seed, ctr in [(0, (0, 0, 0, 0)), (0x0123456789ABCDEF, (5, 7, 9, 11)),
                      (2 ** 64 - 1, (2 ** 32 - 1000, 1, 2, 3))]:
        n = 4096
        out = torch.empty(4 * n, dtype=torch.int32, device="cuda")
        b.debug_philox(seed, ctr, n, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32).reshape(n, 4)
        ref = philox.philox4x32_10(np.uint64(ctr[0]) + np.arange(n, dtype=np.uint64), ctr[1], ctr[2], ctr[3],
                                   philox.key_from_seed(seed))
        assert np.array_equal(got, np.stack(ref, axis=1))


@pytest.mark.parametrize("prec,tol", [(1, 1e-14), (0, 1e-6)])
@pytest.mark.parametrize("n", [(12, 10), (6, 8, 4)])
def test_noise_normals(ce, prec, tol, n):
    b, ctx = ce
    xi = dict(kind="exp", sigma2=1.0, a=1.0)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    out = torch.empty(2 * plan.embedding_cells, dtype=plan.dtype, device="cuda")
    b.debug_noise(plan, 3, 5, 7, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    got = (got[0::2] + 1j * got[1::2]).reshape(tuple(2 * x for x in n))
    ref = ofields.pair_noise(tuple(2 * x for x in n), 3, 5, 7)
    assert rel(got.view(np.float64), ref.view(np.float64)) <= tol
    plan.release()


PLAN_CASES = [
    ((64, 64), (1.0, 1.0), dict(kind="exp", sigma2=0.5, a=8.0)),
    ((24, 20), (1.0, 0.5), dict(kind="powexp", sigma2=1.0, r0=2.0, gamma=1.8, rc=30.0)),
    ((8, 6, 10), (1.0, 1.0, 1.0), dict(kind="exp", sigma2=0.8, a=1.0)),
    ((48, 40), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=3.0)),
    ((62, 34), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=2.0)),
]


@pytest.mark.parametrize("n,h,xi", PLAN_CASES)
def test_plan_eigenvalues(ce, n, h, xi):
    b, ctx = ce
    ref = embedding.plan(n, h, xi)
    plan = b.plan_embedding(ctx, n, h, xi, 1)
    oct_shape = tuple(x + 1 for x in n)
    out = torch.empty(int(np.prod(oct_shape)), dtype=torch.float64, device="cuda")
    b.plan_eigenvalues(plan, out)
    torch.cuda.synchronize()
    lam = out.cpu().numpy().reshape(oct_shape)
    ref_oct = ref["lam"][tuple(slice(0, x + 1) for x in n)]
    lmax = ref["lambda_max"]
    # the oracle clamps; compare against its unclamped spectrum
    raw = embedding.eigenvalues(embedding.lag_table(n, h, xi))[tuple(slice(0, x + 1) for x in n)]
    assert np.max(np.abs(lam - raw)) <= 1e-12 * lmax
    assert np.max(np.abs(np.maximum(lam, 0) - ref_oct)) <= 1e-12 * lmax
    info = plan.info
    assert abs(info["lambda_max"] - lmax) <= 1e-12 * lmax
    assert abs(info["lambda_min"] - ref["lambda_min"]) <= 1e-12 * lmax
    assert info["n_negative"] == ref["n_negative"]
    assert info["sigma2"] == ref["sigma2"]
    plan.release()


def test_not_psd_rejected(ce):
    b, ctx = ce
    n = (32, 32, 32)
    xi = dict(kind="powexp", sigma2=1.0, r0=10.0, gamma=1.8, rc=0.0)
    with pytest.raises(embedding.NotPSD) as ref:
        embedding.plan(n, (1.0,) * 3, xi)
    with pytest.raises(b.NotPSDError) as err:
        b.plan_embedding(ctx, n, (1.0,) * 3, xi, 0)
    lmax = ref.value.info["lambda_max"]
    assert abs(err.value.info["lambda_min"] - ref.value.info["lambda_min"]) <= 1e-12 * lmax
    assert err.value.info["n_negative"] == ref.value.info["n_negative"]


FIELD_CASES = [
    # name, n, h, xi, prec, first, count
    ("small_2d_f64", (64, 64), (1.0, 1.0), dict(kind="exp", sigma2=0.5, a=8.0), 1, 0, 100),
    ("pow2_2d_f32_odd_count", (256, 256), (1.0, 1.0), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0),
     0, 6, 5),
    ("rect_2d_f32_mixed", (96, 80), (1.0, 0.5), dict(kind="exp", sigma2=1.0, a=3.0), 0, 0, 4),
    ("primes_2d_f64", (62, 34), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=2.0), 1, 2, 3),
    ("primes_2d_f32", (46, 26), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=2.0), 0, 0, 3),
    ("primes_3d_f32", (22, 22, 22), (1.0, 1.0, 1.0), dict(kind="exp", sigma2=0.8, a=1.5), 0, 0, 2),
    ("vol_3d_f64", (16, 12, 20), (1.0, 1.0, 1.0), dict(kind="exp", sigma2=0.8, a=1.5), 1, 0, 3),
    ("vol_3d_f32", (32, 32, 32), (1.0, 1.0, 1.0), dict(kind="powexp", sigma2=2.0, r0=1.5, gamma=1.8, rc=100.0),
     0, 0, 4),
    # primes above 31 (the generic radix): 37 (592 = 16 x 37, 1184 = 32 x 37), 127 (2032, 4064)
    ("prime37_2d_f32", (592, 74), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=4.0), 0, 2, 3),
    ("prime37_2d_f64", (74, 54), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=3.0), 1, 0, 2),
    ("prime127_2d_f32", (2032, 16), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=4.0), 0, 0, 2),
    ("prime41_3d_f32", (82, 20, 24), (1.0, 1.0, 1.0), dict(kind="exp", sigma2=0.8, a=1.5), 0, 0, 2),
    # in-place mixed radix: every radix up to 8 (2N = 3000 = 3.5^3.8, 1260 = 3^2.5.7.4), FP64 beyond
    # the two-buffer limit
    ("mixed_large_2d_f64", (1500, 12), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=4.0), 1, 0, 2),
    ("mixed_357_2d_f32", (630, 40), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=4.0), 0, 2, 3),
    ("mixed_3d_f32", (30, 42, 36), (1.0, 1.0, 1.0), dict(kind="exp", sigma2=0.8, a=1.5), 0, 0, 2),
]


@pytest.mark.parametrize("name,n,h,xi,prec,first,count", FIELD_CASES, ids=[c[0] for c in FIELD_CASES])
def test_fields_match_oracle(ce, name, n, h, xi, prec, first, count):
    b, ctx = ce
    print("case", name, flush=True)
    ref_plan = embedding.plan(n, h, xi)
    ref = ofields.generate_fields(ref_plan, 9, 4, first, count)
    plan = b.plan_embedding(ctx, n, h, xi, prec)
    got = gpu_fields(b, ctx, plan, 9, 4, first, count).cpu().numpy().reshape((count,) + n)
    check_maps(got, ref, TOL_FIELD[prec], math.sqrt(ref_plan["sigma2"]), name)
    plan.release()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("first", [4, 3])
@pytest.mark.parametrize("masked", [False, True])
def test_lognormal_poisson_parity(ce, prec, first, masked):
    b, ctx = ce
    n, xi, nbar = (64, 64), dict(kind="exp", sigma2=0.5, a=8.0), 5.0
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), xi, prec)
    count = 5
    g = gpu_fields(b, ctx, plan, 1, 2, 0, count)
    mask = None
    mask_np = None
    if masked:
        rng = np.random.default_rng(0)
        mask_np = rng.random(n).astype(np.float32)
        mask_np[mask_np < 0.3] = 0.0
        mask = torch.from_numpy(mask_np.ravel()).cuda()
    delta = torch.empty_like(g)
    counts = torch.empty(count * plan.cells, dtype=torch.int32, device="cuda")
    ntot = torch.empty(count, dtype=torch.int64, device="cuda")
    b.lognormal_poisson(ctx, plan, g, count, nbar, mask, 11, 2, first, delta, counts, ntot)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    gh = g.cpu().numpy().astype(np.float64).reshape((count,) + n)
    dh = delta.cpu().numpy().reshape((count,) + n)
    ref_delta = olp.lognormal_delta(gh, plan.info["sigma2"])
    check_delta(dh, ref_delta, TOL_FIELD[prec])
    _, ref_counts, ref_ntot = olp.lognormal_poisson(gh, plan.info["sigma2"], nbar, 11, 2, first,
                                                    mask=mask_np, delta=dh)
    assert np.array_equal(counts.cpu().numpy().reshape((count,) + n), ref_counts)
    assert np.array_equal(ntot.cpu().numpy(), ref_ntot)
    plan.release()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("n,nb", [((64, 64), 32), ((16, 16, 16), 8), ((48, 48), 12), ((58, 58), 14),
                                  ((26, 26, 26), 6), ((48, 80), 12), ((40, 24, 32), 6), ((64, 26), 10),
                                  ((74, 118), 12), ((254, 82), 16)])
def test_pk_field_parity(ce, prec, n, nb):
    b, ctx = ce
    xi = dict(kind="exp", sigma2=1.0, a=2.0)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    count = 5
    g = gpu_fields(b, ctx, plan, 3, 0, 0, count)
    out = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    nm = torch.empty(nb, dtype=torch.int64, device="cuda")
    km = torch.empty(nb, dtype=torch.float64, device="cuda")
    b.estimate_pk(ctx, n, (1.0,) * len(n), prec, b.MAP_FIELD, g, count, None, None, nb, out, nm, km)
    torch.cuda.synchronize()
    gh = g.cpu().numpy().astype(np.float64).reshape((count,) + n)
    ref = opk.estimate_pk(gh, 1.0, nb)
    got = out.cpu().numpy().reshape(count, nb)
    assert np.max(np.abs(got / ref - 1)) <= TOL_PK[prec]
    onm, okm = opk.shell_stats(n, 1.0, nb)
    assert np.array_equal(nm.cpu().numpy(), onm)
    assert np.allclose(km.cpu().numpy(), okm, rtol=1e-13)
    plan.release()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("masked,given_ntot", [(False, True), (False, False), (True, True)])
def test_pk_counts_parity(ce, prec, masked, given_ntot):
    b, ctx = ce
    n, nb, nbar = (64, 64), 32, 5.0
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), dict(kind="exp", sigma2=0.5, a=8.0), prec)
    count = 4
    g = gpu_fields(b, ctx, plan, 5, 1, 0, count)
    mask = mask_np = None
    if masked:
        mask_np = np.ones(n, dtype=np.float32)
        mask_np[10:20, 30:50] = 0.0
        mask_np[40:, :8] = 0.75
        mask = torch.from_numpy(mask_np.ravel()).cuda()
    counts = torch.empty(count * plan.cells, dtype=torch.int32, device="cuda")
    ntot = torch.empty(count, dtype=torch.int64, device="cuda")
    b.lognormal_poisson(ctx, plan, g, count, nbar, mask, 6, 1, 0, None, counts, ntot)
    out = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    b.estimate_pk(ctx, n, (1.0, 1.0), prec, b.MAP_COUNTS_DELTAG, counts, count, ntot if given_ntot else None, mask,
                  nb, out)
    torch.cuda.synchronize()
    ch = counts.cpu().numpy().reshape((count,) + n)
    ref = opk.estimate_pk(ch, 1.0, nb, kind="counts", ntot=ntot.cpu().numpy(), mask=mask_np)
    got = out.cpu().numpy().reshape(count, nb)
    assert np.max(np.abs(got / ref - 1)) <= TOL_PK[prec]
    plan.release()


def test_covariance_parity(ce):
    b, ctx = ce
    rng = np.random.default_rng(1)
    R, nb = 40, 9
    P = rng.gamma(4.0, 1.0, (R, nb))
    pk = torch.from_numpy(P.ravel()).cuda()
    cov = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    cn = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    b.pk_covariance(ctx, pk, R, nb, cov, cn)
    torch.cuda.synchronize()
    rc, rn = opk.covariance(P)
    assert rel(cov.cpu().numpy(), rc.ravel()) <= 1e-12
    assert rel(cn.cpu().numpy(), rn.ravel()) <= 1e-12


PIPE_CASES = [((64, 64), dict(kind="exp", sigma2=0.5, a=8.0), 1, 32, 7),
              ((128, 128), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0), 0, 32, 6),
              ((16, 16, 16), dict(kind="exp", sigma2=0.8, a=1.5), 0, 8, 3),
              ((48, 48), dict(kind="exp", sigma2=1.0, a=3.0), 1, 12, 4),
              ((38, 38), dict(kind="exp", sigma2=1.0, a=3.0), 0, 10, 4),
              ((74, 94), dict(kind="exp", sigma2=1.0, a=3.0), 0, 12, 4),     # primes 37, 47
              ((106, 74), dict(kind="exp", sigma2=1.0, a=3.0), 1, 12, 3),    # primes 53, 37
              ((22, 22, 22), dict(kind="exp", sigma2=0.8, a=1.5), 1, 6, 2),
              # hyperrectangular surveys (square / cubic cells)
              ((64, 96), dict(kind="exp", sigma2=0.8, a=3.0), 0, 16, 5),
              ((48, 32), dict(kind="exp", sigma2=0.8, a=3.0), 1, 10, 4),
              ((16, 24, 12), dict(kind="exp", sigma2=0.8, a=1.5), 0, 5, 3)]


@pytest.mark.parametrize("n,xi,prec,nb,count", PIPE_CASES)
def test_pipeline_matches_unfused_and_oracle(ce, n, xi, prec, nb, count):
    b, ctx = ce
    print("pipeline case", n, prec, flush=True)
    nbar, seed, rid, first = 5.0, 21, 3, 2
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    cells = plan.cells
    f = torch.empty(count * cells, dtype=plan.dtype, device="cuda")
    d = torch.empty_like(f)
    c = torch.empty(count * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(count, dtype=torch.int64, device="cuda")
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    cov = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    cn = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run(ctx, plan, seed, rid, first, count, nbar, nb, p, f, d, c, nt, cov, cn)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    # unfused calls on the same streams
    f2 = gpu_fields(b, ctx, plan, seed, rid, first, count)
    assert torch.equal(f, f2)
    d2 = torch.empty_like(f)
    c2 = torch.empty_like(c)
    nt2 = torch.empty_like(nt)
    b.lognormal_poisson(ctx, plan, f2, count, nbar, None, seed, rid, first, d2, c2, nt2)
    p2 = torch.empty_like(p)
    b.estimate_pk(ctx, n, (1.0,) * len(n), prec, b.MAP_COUNTS_DELTAG, c2, count, nt2, None, nb, p2)
    torch.cuda.synchronize()
    assert torch.equal(d, d2)
    assert torch.equal(c, c2)
    assert torch.equal(nt, nt2)
    assert np.max(np.abs(p.cpu().numpy() / p2.cpu().numpy() - 1)) <= TOL_PK[prec]
    # oracle: fields, counts from the GPU delta, spectra from the GPU counts, covariance from GPU spectra
    ref_plan = embedding.plan(n, (1.0,) * len(n), xi)
    ref_f = ofields.generate_fields(ref_plan, seed, rid, first, count)
    fh = f.cpu().numpy().reshape((count,) + n)
    check_maps(fh, ref_f, TOL_FIELD[prec], math.sqrt(ref_plan["sigma2"]))
    dh = d.cpu().numpy().reshape((count,) + n)
    check_delta(dh, olp.lognormal_delta(fh.astype(np.float64), plan.info["sigma2"]), TOL_FIELD[prec])
    _, rc, rn = olp.lognormal_poisson(fh.astype(np.float64), plan.info["sigma2"], nbar, seed, rid, first, delta=dh)
    assert np.array_equal(c.cpu().numpy().reshape((count,) + n), rc)
    assert np.array_equal(nt.cpu().numpy(), rn)
    rp = opk.estimate_pk(rc, 1.0, nb, kind="counts", ntot=rn)
    assert np.max(np.abs(p.cpu().numpy().reshape(count, nb) / rp - 1)) <= TOL_PK[prec]
    rcov, rcn = opk.covariance(p.cpu().numpy().reshape(count, nb))
    assert rel(cov.cpu().numpy(), rcov.ravel()) <= 1e-12
    assert rel(cn.cpu().numpy(), rcn.ravel()) <= 1e-12
    plan.release()


def test_pipeline_is_bitwise_deterministic(ce):
    b, ctx = ce
    n, nb, count = (128, 128), 32, 6
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=5.0), 0)
    outs = []
    for _ in range(2):
        p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
        c = torch.empty(count * plan.cells, dtype=torch.int32, device="cuda")
        b.pipeline_run(ctx, plan, 1, 0, 0, count, 0.3, nb, p, out_counts=c)
        torch.cuda.synchronize()
        outs.append((p.cpu(), c.cpu()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    plan.release()


@pytest.mark.parametrize("n,prec", [((64, 48), 1), ((16, 12, 20), 0), ((96, 80), 0)])
def test_unpruned_comparator_matches(ce, n, prec):
    b, ctx = ce
    xi = dict(kind="exp", sigma2=1.0, a=3.0) if len(n) == 2 else dict(kind="exp", sigma2=0.8, a=1.5)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    a = gpu_fields(b, ctx, plan, 2, 1, 0, 3)
    b.ctx_set_option(ctx, b.OPT_UNPRUNED, 1)
    try:
        c = gpu_fields(b, ctx, plan, 2, 1, 0, 3)
    finally:
        b.ctx_set_option(ctx, b.OPT_UNPRUNED, 0)
    ah, ch = a.cpu().numpy().reshape(3, -1), c.cpu().numpy().reshape(3, -1)
    check_maps(ch, ah, TOL_FIELD[prec], math.sqrt(plan.info["sigma2"]), "unpruned vs pruned")
    plan.release()


def test_batched_2d_full_size_sampled(ce):
    """The 1024^2-in-2048^2 FP32 workload in the benchmark's launch configuration (256
    realizations in one call); sampled realizations checked against the oracle."""
    b, ctx = ce
    from synth import workloads
    w = workloads.WORKLOADS["batched_2d"]
    n, nb, R, nbar = w["n"], w["nbins"], w["realizations"], w["nbar"]
    plan = b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    cells = plan.cells
    f = torch.empty(R * cells, dtype=torch.float32, device="cuda")
    d = torch.empty_like(f)
    c = torch.empty(R * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(R, dtype=torch.int64, device="cuda")
    p = torch.empty(R * nb, dtype=torch.float64, device="cuda")
    cov = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run(ctx, plan, w["seed"], w["request_id"], 0, R, nbar, nb, p, f, d, c, nt, cov)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    ref_plan = embedding.plan(n, w["h"], w["xi"])
    pk_all = p.cpu().numpy().reshape(R, nb)
    for first in (0, R - 2):
        print("sampled pair", first // 2, flush=True)
        ref = ofields.generate_fields(ref_plan, w["seed"], w["request_id"], first, 2)
        got = f[first * cells:(first + 2) * cells].cpu().numpy().reshape((2,) + n)
        check_maps(got, ref, TOL_FIELD[0], math.sqrt(ref_plan["sigma2"]))
        dh = d[first * cells:(first + 2) * cells].cpu().numpy().reshape((2,) + n)
        check_delta(dh, olp.lognormal_delta(got.astype(np.float64), plan.info["sigma2"]), TOL_FIELD[0])
        _, rc, rn = olp.lognormal_poisson(got.astype(np.float64), plan.info["sigma2"], nbar, w["seed"],
                                          w["request_id"], first, delta=dh)
        assert np.array_equal(c[first * cells:(first + 2) * cells].cpu().numpy().reshape((2,) + n), rc)
        assert np.array_equal(nt[first:first + 2].cpu().numpy(), rn)
        rp = opk.estimate_pk(rc, 1.0, nb, kind="counts", ntot=rn)
        assert np.max(np.abs(pk_all[first:first + 2] / rp - 1)) <= TOL_PK[0]
    rcov, _ = opk.covariance(pk_all)
    assert rel(cov.cpu().numpy(), rcov.ravel()) <= 1e-12
    plan.release()


def test_masked_full_size_log_shells_sampled(ce):
    """The masked 1024^2 survey of the benchmark (256 realizations in one call, FP32) with 20
    shells equally spaced in ln k: sampled realizations against the oracle (counts and N_tot
    bitwise, P(k) to the spectrum tolerance), every realization against ce_estimate_pk_edges
    on the stored counts."""
    import math
    b, ctx = ce
    from synth import workloads
    w = workloads.WORKLOADS["batched_2d"]
    n, R, nbar, nb = w["n"], w["realizations"], w["nbar"], 20
    mask_np = workloads.survey_mask(n, seed=3)
    mask = torch.from_numpy(mask_np.ravel()).cuda()
    edges = np.exp(np.linspace(math.log(math.pi / 256.0), math.log(math.pi), nb + 1))
    plan = b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    cells = plan.cells
    d = torch.empty(R * cells, dtype=torch.float32, device="cuda")
    c = torch.empty(R * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(R, dtype=torch.int64, device="cuda")
    p = torch.empty(R * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run_edges(ctx, plan, w["seed"], w["request_id"], 0, R, nbar, nb, edges, p, out_delta=d,
                         out_counts=c, out_ntot=nt, mask=mask)
    p2 = torch.empty_like(p)
    b.estimate_pk(ctx, n, w["h"], b.F32, b.MAP_COUNTS_DELTAG, c, R, nt, mask, nb, p2, edges=edges)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    got, un = p.cpu().numpy().reshape(R, nb), p2.cpu().numpy().reshape(R, nb)
    assert np.all(np.isfinite(got)) and np.max(np.abs(got / un - 1)) <= TOL_PK[0]
    ref_plan = embedding.plan(n, w["h"], w["xi"])
    for first in (0, R - 2):
        print("sampled masked pair", first // 2, flush=True)
        f = ofields.generate_fields(ref_plan, w["seed"], w["request_id"], first, 2)
        dh = d[first * cells:(first + 2) * cells].cpu().numpy().reshape((2,) + n)
        _, rc, rn = olp.lognormal_poisson(f, plan.info["sigma2"], nbar, w["seed"], w["request_id"], first,
                                          mask=mask_np, delta=dh)
        assert np.array_equal(c[first * cells:(first + 2) * cells].cpu().numpy().reshape((2,) + n), rc)
        assert np.array_equal(nt[first:first + 2].cpu().numpy(), rn)
        rp = opk.estimate_pk(rc, 1.0, nb, kind="counts", ntot=rn, mask=mask_np, edges=edges)
        assert np.max(np.abs(got[first:first + 2] / rp - 1)) <= TOL_PK[0]
    plan.release()


def test_volume_3d_parity_and_full_size_properties(ce):
    b, ctx = ce
    from synth import workloads
    w = workloads.WORKLOADS["volume_3d"]
    # parity at 64^3 in 128^3; the 256^3 two-point function (r0 = 5) is not positive at this
    # side (Sec. 2: positivity is only guaranteed for large embeddings), so use r0 = 2
    n = (64, 64, 64)
    xi_small = dict(w["xi"], r0=2.0, rc=100.0)
    with pytest.raises(b.NotPSDError):
        b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    plan = b.plan_embedding(ctx, n, w["h"], xi_small, b.F32)
    ref_plan = embedding.plan(n, w["h"], xi_small)
    got = gpu_fields(b, ctx, plan, 0, 0, 0, 2).cpu().numpy().reshape((2,) + n)
    ref = ofields.generate_fields(ref_plan, 0, 0, 0, 2)
    check_maps(got, ref, TOL_FIELD[0], math.sqrt(ref_plan["sigma2"]))
    plan.release()
    # full size: 256^3 in 512^3, 8 realizations in one call
    n, nb, R, nbar = w["n"], w["nbins"], w["realizations"], w["nbar"]
    plan = b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    assert plan.info["lambda_min"] > 0
    cells = plan.cells
    f = torch.empty(R * cells, dtype=torch.float32, device="cuda")
    c = torch.empty(R * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(R, dtype=torch.int64, device="cuda")
    p = torch.empty(R * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run(ctx, plan, 0, 0, 0, R, nbar, nb, p, out_fields=f, out_counts=c, out_ntot=nt)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    fv = f.view(R, cells)
    var = fv.double().var(dim=1).cpu().numpy()
    assert np.all(np.abs(var / w["xi"]["sigma2"] - 1) < 0.25)      # super-survey modes make this noisy
    ntot = nt.cpu().numpy()
    assert np.array_equal(ntot, c.view(R, cells).sum(dim=1).cpu().numpy())
    assert np.all(np.abs(ntot / (nbar * cells) - 1) < 0.2)
    pk = p.cpu().numpy()
    assert np.all(np.isfinite(pk)) and np.all(pk > 0)
    # Gaussian-field check at full size: the spectrum of the field follows the closed form of the
    # window-convolved model only statistically; check white-noise floor of counts instead:
    # P_counts >= h^3 / nbar (Poisson) at every shell on average
    assert pk.reshape(R, nb).mean(axis=0).min() > 0.5 / nbar
    plan.release()


@pytest.mark.parametrize("n", [(96, 96), (24, 16, 20)])
def test_masked_pipeline_without_counts(ce, n):
    """The fused masked path stores counts only on request; P(k) and N_tot do not depend on
    it (odd count, FP32)."""
    from synth import workloads
    b, ctx = ce
    nb, count = 12, 7
    mask = torch.from_numpy(workloads.survey_mask(n, seed=5).ravel()).cuda()
    xi = dict(kind="exp", sigma2=0.5, a=2.0 if len(n) == 2 else 1.0)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, b.F32)
    p1 = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    p2 = torch.empty_like(p1)
    t1 = torch.empty(count, dtype=torch.int64, device="cuda")
    t2 = torch.empty_like(t1)
    c = torch.empty(count * plan.cells, dtype=torch.int32, device="cuda")
    b.pipeline_run_masked(ctx, plan, mask, 3, 1, 0, count, 2.0, nb, p1, out_counts=c, out_ntot=t1)
    b.pipeline_run_masked(ctx, plan, mask, 3, 1, 0, count, 2.0, nb, p2, out_ntot=t2)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(t1, t2)
    assert int(c.view(count, -1).sum(dim=1).sub(t1).abs().sum()) == 0
    plan.release()


@pytest.mark.parametrize("n,prec,nb", [((64, 64), 1, 16), ((96, 96), 0, 24), ((128, 128), 0, 20),
                                       ((96, 64), 0, 12), ((16, 16, 16), 0, 6), ((16, 24, 20), 1, 8),
                                       ((32, 32, 32), 0, 10),
                                       # prime radices in every pass: 2N = 124 = 4.31, 88 = 8.11 and
                                       # N = 62, 44; 2N = 148 = 4.37 (ping-pong), 76 = 4.19
                                       ((62, 44), 0, 10), ((74, 38), 1, 8)])
def test_masked_pipeline_matches_unfused_and_oracle(ce, n, prec, nb):
    """Masked survey (Sec. 3.1 rate nbar f rho; Sec. 3.2 contrast on f != 0): the masked
    pipeline equals the unfused calls with the same mask (fields, delta, counts, N_tot bitwise;
    P(k) to the spectrum tolerance: the fused pass transforms N / (f nbar) - 1 and the binning
    pass adds the window term), and the oracle fed the GPU's delta and counts."""
    from synth import workloads
    b, ctx = ce
    print("masked case", n, prec, flush=True)
    xi = dict(kind="exp", sigma2=0.8, a=3.0) if len(n) == 2 else dict(kind="exp", sigma2=0.8, a=1.5)
    mask_np = workloads.survey_mask(n, seed=3)
    mask = torch.from_numpy(mask_np.ravel()).cuda()
    nbar, seed, rid, first, count = 4.0, 8, 6, 2, 5
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    cells = plan.cells
    f = torch.empty(count * cells, dtype=plan.dtype, device="cuda")
    d = torch.empty_like(f)
    c = torch.empty(count * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(count, dtype=torch.int64, device="cuda")
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    cov = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run_masked(ctx, plan, mask, seed, rid, first, count, nbar, nb, p, f, d, c, nt, cov)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    ch = c.cpu().numpy().reshape((count,) + n)
    assert np.all(ch[:, mask_np == 0] == 0)
    # unfused calls
    f2 = gpu_fields(b, ctx, plan, seed, rid, first, count)
    assert torch.equal(f, f2)
    d2, c2, nt2 = torch.empty_like(d), torch.empty_like(c), torch.empty_like(nt)
    b.lognormal_poisson(ctx, plan, f2, count, nbar, mask, seed, rid, first, d2, c2, nt2)
    p2 = torch.empty_like(p)
    b.estimate_pk(ctx, n, (1.0,) * len(n), prec, b.MAP_COUNTS_DELTAG, c2, count, nt2, mask, nb, p2)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(c, c2) and torch.equal(nt, nt2)
    assert torch.max(torch.abs(p / p2 - 1)).item() <= TOL_PK[prec]
    # oracle
    dh = d.cpu().numpy().reshape((count,) + n)
    fh = f.cpu().numpy().astype(np.float64).reshape((count,) + n)
    _, rc, rn = olp.lognormal_poisson(fh, plan.info["sigma2"], nbar, seed, rid, first, mask=mask_np, delta=dh)
    assert np.array_equal(ch, rc) and np.array_equal(nt.cpu().numpy(), rn)
    rp = opk.estimate_pk(rc, 1.0, nb, kind="counts", ntot=rn, mask=mask_np)
    assert np.max(np.abs(p.cpu().numpy().reshape(count, nb) / rp - 1)) <= TOL_PK[prec]
    rcov, _ = opk.covariance(p.cpu().numpy().reshape(count, nb))
    assert rel(cov.cpu().numpy().reshape(nb, nb), rcov) <= 1e-12
    plan.release()


@pytest.mark.parametrize("n,prec", [((64, 64), 1), ((48, 80), 0), ((16, 24, 12), 1)])
def test_linear_edges_equal_default_shells(ce, n, prec):
    """Linear shell edges on (0, pi/h] through ce_estimate_pk_edges give ce_estimate_pk bitwise."""
    import math
    b, ctx = ce
    nb, count = 9, 3
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), dict(kind="exp", sigma2=1.0, a=2.0), prec)
    g = gpu_fields(b, ctx, plan, 5, 0, 0, count)
    p1 = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    p2 = torch.empty_like(p1)
    m1 = torch.empty(nb, dtype=torch.int64, device="cuda")
    m2 = torch.empty_like(m1)
    b.estimate_pk(ctx, n, (1.0,) * len(n), prec, b.MAP_FIELD, g, count, None, None, nb, p1, m1)
    b.estimate_pk(ctx, n, (1.0,) * len(n), prec, b.MAP_FIELD, g, count, None, None, nb, p2, m2,
                  edges=np.linspace(0.0, math.pi, nb + 1))
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(m1, m2)
    plan.release()


@pytest.mark.parametrize("n,prec,masked", [((128, 128), 1, False), ((96, 64), 0, True), ((20, 16, 24), 0, False),
                                           ((62, 44), 0, True)])
def test_log_edges_match_oracle(ce, n, prec, masked):
    """The paper's binning, 20 shells equally spaced in ln k up to the pixel scale, against the
    oracle (field maps; counts with a mask)."""
    import math
    from synth import workloads
    b, ctx = ce
    nb, count = 20, 4
    h = 0.5
    edges = np.exp(np.linspace(math.log(math.pi / h / 30.0), math.log(math.pi / h), nb + 1))
    # a shorter range in 3-D keeps the small embedding positive definite
    plan = b.plan_embedding(ctx, n, (h,) * len(n), dict(kind="exp", sigma2=1.0, a=2.0 if len(n) == 2 else 0.6), prec)
    cells = plan.cells
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    nm = torch.empty(nb, dtype=torch.int64, device="cuda")
    km = torch.empty(nb, dtype=torch.float64, device="cuda")
    if masked:
        mask_np = workloads.survey_mask(n, seed=2)
        mask = torch.from_numpy(mask_np.ravel()).cuda()
        c = torch.empty(count * cells, dtype=torch.int32, device="cuda")
        nt = torch.empty(count, dtype=torch.int64, device="cuda")
        pk0 = torch.empty(count * 8, dtype=torch.float64, device="cuda")
        b.pipeline_run_masked(ctx, plan, mask, 4, 2, 0, count, 3.0, 8, pk0, out_counts=c, out_ntot=nt)
        b.estimate_pk(ctx, n, (h,) * len(n), prec, b.MAP_COUNTS_DELTAG, c, count, nt, mask, nb, p, nm, km,
                      edges=edges)
        torch.cuda.synchronize()
        ref = opk.estimate_pk(c.cpu().numpy().reshape((count,) + n), h, nb, kind="counts",
                              ntot=nt.cpu().numpy(), mask=mask_np, edges=edges)
    else:
        g = gpu_fields(b, ctx, plan, 6, 0, 0, count)
        b.estimate_pk(ctx, n, (h,) * len(n), prec, b.MAP_FIELD, g, count, None, None, nb, p, nm, km, edges=edges)
        torch.cuda.synchronize()
        ref = opk.estimate_pk(g.cpu().numpy().astype(np.float64).reshape((count,) + n), h, nb, edges=edges)
    got = p.cpu().numpy().reshape(count, nb)
    onm, okm = opk.shell_stats(n, h, nb, edges)
    assert np.array_equal(nm.cpu().numpy(), onm)
    ok = onm > 0
    assert np.allclose(km.cpu().numpy()[ok], okm[ok], rtol=1e-13)
    assert np.max(np.abs(got[:, ok] / ref[:, ok] - 1)) <= TOL_PK[prec]
    plan.release()


def test_shell_edge_errors_and_corners(ce):
    import math
    b, ctx = ce
    n, nb = (32, 32), 10
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=2.0), b.F32)
    g = gpu_fields(b, ctx, plan, 5, 0, 0, 2)
    p = torch.empty(2 * nb, dtype=torch.float64, device="cuda")
    nm = torch.empty(nb, dtype=torch.int64, device="cuda")
    # edges up to pi sqrt(2) / h take the corners: every mode but DC is binned
    b.estimate_pk(ctx, n, (1.0, 1.0), b.F32, b.MAP_FIELD, g, 2, None, None, nb, p, nm,
                  edges=np.linspace(0.0, math.pi * math.sqrt(2.0), nb + 1))
    torch.cuda.synchronize()
    assert int(nm.sum()) == 32 * 32 - 1
    for bad in (np.linspace(1.0, 0.0, nb + 1), np.full(nb + 1, 1.0), np.r_[-1.0, np.linspace(0, 3, nb)]):
        with pytest.raises(b.CeError) as e:
            b.estimate_pk(ctx, n, (1.0, 1.0), b.F32, b.MAP_FIELD, g, 2, None, None, nb, p, edges=bad)
        assert e.value.status == b.E_INVALID
    plan.release()


@pytest.mark.parametrize("n,prec", [((128, 128), 0), ((48, 32), 1), ((16, 16, 16), 0)])
def test_pipeline_with_edges(ce, n, prec):
    """The fused path with the paper's log-spaced shells against the oracle fed the GPU's counts,
    and with linear edges equal to ce_pipeline_run bitwise."""
    import math
    b, ctx = ce
    nb, count, nbar = 12, 4, 5.0
    xi = dict(kind="exp", sigma2=0.8, a=3.0 if len(n) == 2 else 1.5)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    c = torch.empty(count * plan.cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(count, dtype=torch.int64, device="cuda")
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    edges = np.exp(np.linspace(math.log(math.pi / 20.0), math.log(math.pi), nb + 1))
    b.pipeline_run_edges(ctx, plan, 9, 2, 0, count, nbar, nb, edges, p, out_counts=c, out_ntot=nt)
    p1 = torch.empty_like(p)
    p2 = torch.empty_like(p)
    b.pipeline_run(ctx, plan, 9, 2, 0, count, nbar, nb, p1)
    b.pipeline_run_edges(ctx, plan, 9, 2, 0, count, nbar, nb, np.linspace(0.0, math.pi, nb + 1), p2)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    # (an empty shell is 0/0 = NaN on both sides)
    assert np.array_equal(p1.cpu().numpy(), p2.cpu().numpy(), equal_nan=True)
    ref = opk.estimate_pk(c.cpu().numpy().reshape((count,) + n), 1.0, nb, kind="counts", ntot=nt.cpu().numpy(),
                          edges=edges)
    got = p.cpu().numpy().reshape(count, nb)
    ok = np.isfinite(ref[0])  # the lowest log shells of a small grid hold no mode
    assert ok.sum() >= nb // 2
    assert np.array_equal(np.isfinite(got[0]), ok)
    assert np.max(np.abs(got[:, ok] / ref[:, ok] - 1)) <= TOL_PK[prec]
    plan.release()


@pytest.mark.parametrize("n,prec", [((128, 128), 0), ((96, 64), 1), ((16, 20, 16), 0)])
def test_masked_pipeline_with_edges(ce, n, prec):
    """The paper's setting end to end: a masked survey binned in ln k.  The fused path with a
    mask and log shells against ce_estimate_pk_edges on its own counts (to the spectrum
    tolerance: the binning pass adds the window term) and against the oracle; linear edges with
    a mask give ce_pipeline_run_masked bitwise."""
    import math
    from synth import workloads
    b, ctx = ce
    print("masked edges case", n, prec, flush=True)
    nb, count, nbar = 14, 5, 4.0
    xi = dict(kind="exp", sigma2=0.8, a=3.0 if len(n) == 2 else 1.5)
    mask_np = workloads.survey_mask(n, seed=7)
    mask = torch.from_numpy(mask_np.ravel()).cuda()
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    cells = plan.cells
    edges = np.exp(np.linspace(math.log(math.pi / 24.0), math.log(math.pi), nb + 1))
    c = torch.empty(count * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(count, dtype=torch.int64, device="cuda")
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run_edges(ctx, plan, 11, 3, 0, count, nbar, nb, edges, p, out_counts=c, out_ntot=nt, mask=mask)
    p2 = torch.empty_like(p)
    b.estimate_pk(ctx, n, (1.0,) * len(n), prec, b.MAP_COUNTS_DELTAG, c, count, nt, mask, nb, p2, edges=edges)
    p3, p4 = torch.empty_like(p), torch.empty_like(p)
    lin = np.linspace(0.0, math.pi, nb + 1)
    b.pipeline_run_masked(ctx, plan, mask, 11, 3, 0, count, nbar, nb, p3)
    b.pipeline_run_edges(ctx, plan, 11, 3, 0, count, nbar, nb, lin, p4, mask=mask)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    assert np.array_equal(p3.cpu().numpy(), p4.cpu().numpy(), equal_nan=True)
    ch = c.cpu().numpy().reshape((count,) + n)
    assert np.all(ch[:, mask_np == 0] == 0)
    ref = opk.estimate_pk(ch, 1.0, nb, kind="counts", ntot=nt.cpu().numpy(), mask=mask_np, edges=edges)
    got, un = p.cpu().numpy().reshape(count, nb), p2.cpu().numpy().reshape(count, nb)
    ok = np.isfinite(ref[0])  # the lowest log shells of a small grid hold no mode
    assert ok.sum() >= nb // 2
    assert np.array_equal(np.isfinite(got[0]), ok) and np.array_equal(np.isfinite(un[0]), ok)
    assert np.max(np.abs(got[:, ok] / un[:, ok] - 1)) <= TOL_PK[prec]
    assert np.max(np.abs(got[:, ok] / ref[:, ok] - 1)) <= TOL_PK[prec]
    plan.release()


@pytest.mark.parametrize("n,h,prec,nb", [((64, 48), (1.0, 0.5), 1, 12), ((96, 80), (0.5, 0.75), 0, 16),
                                         ((16, 24, 20), (1.0, 0.5, 1.0), 0, 8)])
def test_rectangular_cells_match_oracle(ce, n, h, prec, nb):
    """Rectangular cells (h_i differ): field spectra (default and log shells), N_b and mean |k|,
    and the fused pipeline (plain and masked, against ce_estimate_pk on its own counts and the
    oracle, to the P(k) tolerance) on the same shells as the oracle's."""
    import math
    from synth import workloads
    b, ctx = ce
    print("rect cells", n, h, prec, flush=True)
    count, nbar = 4, 3.0
    plan = b.plan_embedding(ctx, n, h, dict(kind="exp", sigma2=0.8, a=2.0 if len(n) == 2 else 0.8), prec)
    cells = plan.cells
    g = gpu_fields(b, ctx, plan, 5, 1, 0, count)
    gh = g.cpu().numpy().astype(np.float64).reshape((count,) + n)
    p = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    nm = torch.empty(nb, dtype=torch.int64, device="cuda")
    km = torch.empty(nb, dtype=torch.float64, device="cuda")
    edges = np.exp(np.linspace(math.log(math.pi / max(h) / 8.0), math.log(math.pi / max(h)), nb + 1))
    for e in (None, edges):
        b.estimate_pk(ctx, n, h, prec, b.MAP_FIELD, g, count, None, None, nb, p, nm, km, edges=e)
        torch.cuda.synchronize()
        onm, okm = opk.shell_stats(n, h, nb, e)
        assert np.array_equal(nm.cpu().numpy(), onm)
        ok = onm > 0
        assert np.allclose(km.cpu().numpy()[ok], okm[ok], rtol=1e-13)
        ref = opk.estimate_pk(gh, h, nb, edges=e)
        assert np.max(np.abs(p.cpu().numpy().reshape(count, nb)[:, ok] / ref[:, ok] - 1)) <= TOL_PK[prec]
    # fused pipeline, plain and masked
    mask_np = workloads.survey_mask(n, seed=4)
    for mask in (None, torch.from_numpy(mask_np.ravel()).cuda()):
        c = torch.empty(count * cells, dtype=torch.int32, device="cuda")
        nt = torch.empty(count, dtype=torch.int64, device="cuda")
        if mask is None:
            b.pipeline_run(ctx, plan, 5, 1, 0, count, nbar, nb, p, out_counts=c, out_ntot=nt)
        else:
            b.pipeline_run_masked(ctx, plan, mask, 5, 1, 0, count, nbar, nb, p, out_counts=c, out_ntot=nt)
        p2 = torch.empty_like(p)
        b.estimate_pk(ctx, n, h, prec, b.MAP_COUNTS_DELTAG, c, count, nt, mask, nb, p2)
        torch.cuda.synchronize()
        assert b.ctx_check(ctx) == 0
        got, un = p.cpu().numpy().reshape(count, nb), p2.cpu().numpy().reshape(count, nb)
        ref = opk.estimate_pk(c.cpu().numpy().reshape((count,) + n), h, nb, kind="counts", ntot=nt.cpu().numpy(),
                              mask=None if mask is None else mask_np)
        ok = np.isfinite(ref[0])
        assert np.array_equal(np.isfinite(got[0]), ok)
        assert np.max(np.abs(got[:, ok] / un[:, ok] - 1)) <= TOL_PK[prec]
        assert np.max(np.abs(got[:, ok] / ref[:, ok] - 1)) <= TOL_PK[prec]
    # the fused path with the log shells on these cells
    c = torch.empty(count * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(count, dtype=torch.int64, device="cuda")
    b.pipeline_run_edges(ctx, plan, 6, 2, 0, count, nbar, nb, edges, p, out_counts=c, out_ntot=nt)
    torch.cuda.synchronize()
    ref = opk.estimate_pk(c.cpu().numpy().reshape((count,) + n), h, nb, kind="counts", ntot=nt.cpu().numpy(),
                          edges=edges)
    got = p.cpu().numpy().reshape(count, nb)
    ok = np.isfinite(ref[0])
    assert ok.sum() >= nb // 2 and np.array_equal(np.isfinite(got[0]), ok)
    assert np.max(np.abs(got[:, ok] / ref[:, ok] - 1)) <= TOL_PK[prec]
    plan.release()


@pytest.mark.parametrize("n,prec,log", [((96, 64), 0, True), ((64, 64), 1, False), ((16, 20, 16), 0, True)])
def test_prepared_mask_equals_per_call_window(ce, n, prec, log):
    """A mask prepared once (sum f and window transform held by a handle) gives the masked
    pipeline's results bit for bit, over two calls with different realizations; a handle
    prepared for another grid or precision is rejected."""
    import math
    from synth import workloads
    b, ctx = ce
    nb, count, nbar = 12, 4, 2.5
    mask = torch.from_numpy(workloads.survey_mask(n, seed=9).ravel()).cuda()
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), dict(kind="exp", sigma2=0.7, a=2.5 if len(n) == 2 else 1.2),
                            prec)
    edges = np.exp(np.linspace(math.log(math.pi / 16.0), math.log(math.pi), nb + 1)) if log else None
    prep = b.mask_prepare(ctx, plan, mask)
    try:
        for first in (0, 2 * count):
            ref = dict(out_pk=torch.empty(count * nb, dtype=torch.float64, device="cuda"),
                       out_counts=torch.empty(count * plan.cells, dtype=torch.int32, device="cuda"),
                       out_ntot=torch.empty(count, dtype=torch.int64, device="cuda"))
            got = {k: torch.empty_like(v) for k, v in ref.items()}
            if log:
                b.pipeline_run_edges(ctx, plan, 7, 5, first, count, nbar, nb, edges, mask=mask, **ref)
            else:
                b.pipeline_run_masked(ctx, plan, mask, 7, 5, first, count, nbar, nb, **ref)
            b.pipeline_run_prepared(ctx, plan, mask, prep, 7, 5, first, count, nbar, nb, edges=edges, **got)
            torch.cuda.synchronize()
            assert b.ctx_check(ctx) == 0
            for k in ref:
                assert np.array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy(), equal_nan=True), (first, k)
        other = b.plan_embedding(ctx, n, (1.0,) * len(n), dict(kind="exp", sigma2=0.7, a=1.2), 1 - prec)
        pk = torch.empty(count * nb, dtype=torch.float64, device="cuda")
        with pytest.raises(b.CeError) as e:
            b.pipeline_run_prepared(ctx, other, mask, prep, 7, 5, 0, count, nbar, nb, pk)
        assert e.value.status == b.E_INVALID
        other.release()
    finally:
        b.mask_release(prep)
    plan.release()


def test_prepared_mask_used_on_another_stream_and_ctx(ce):
    """A handle prepared on one stream (behind other queued work) and used at once on another
    stream through another ctx: the run waits for the handle's event, so its results equal the
    per-call masked pipeline's bit for bit."""
    from synth import workloads
    b, ctx = ce
    n, nb, count, nbar = (128, 96), 12, 4, 2.0
    mask = torch.from_numpy(workloads.survey_mask(n, seed=4).ravel()).cuda()
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), dict(kind="exp", sigma2=0.7, a=2.5), b.F32)
    ref = dict(out_pk=torch.empty(count * nb, dtype=torch.float64, device="cuda"),
               out_counts=torch.empty(count * plan.cells, dtype=torch.int32, device="cuda"),
               out_ntot=torch.empty(count, dtype=torch.int64, device="cuda"))
    b.pipeline_run_masked(ctx, plan, mask, 3, 1, 0, count, nbar, nb, **ref)
    torch.cuda.synchronize()
    got = {k: torch.empty_like(v) for k, v in ref.items()}
    ctx2 = b.ctx_create(0)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    x = torch.randn(4096, 4096, device="cuda")
    try:
        with torch.cuda.stream(sa):
            for _ in range(8):      # queued work ahead of the preparation on stream a
                x = torch.tanh(x @ x * 1e-3)
        prep = b.mask_prepare(ctx, plan, mask, sa)
        try:
            b.pipeline_run_prepared(ctx2, plan, mask, prep, 3, 1, 0, count, nbar, nb, stream=sb, **got)
            torch.cuda.synchronize()
        finally:
            b.mask_release(prep)
        assert b.ctx_check(ctx2) == 0
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
    finally:
        b.ctx_destroy(ctx2)
    plan.release()


SCHEDULES = [dict(), dict(lines=(4, 4, 1, 4)), dict(lines=(32, 32, 8, 32), bin_lds=163840),
             dict(noise_block=4), dict(noise_order=1, bin_lds=16384), dict(lines=(2, 1, 2, 1), noise_block=3),
             dict(noise_pairs=4), dict(noise_pairs=5, noise_block=2), dict(noise_pairs=64, noise_order=1)]


@pytest.mark.parametrize("n,prec,nb", [((128, 96), 0, 24), ((64, 64), 1, 16), ((16, 24, 20), 0, 6),
                                       ((1024, 1024), 0, 128), ((44, 52), 0, 10), ((74, 38), 1, 10),
                                       ((62, 34), 0, 12)])
def test_schedules_give_bitwise_identical_results(ce, n, prec, nb):
    """Every schedule option (lines per workgroup of each pass, noise-pass tile order, blocks and
    pairs per workgroup, binning LDS) changes only the launch shape: fields, delta, counts, N_tot, P(k) and the
    covariance are bitwise identical to the default schedule's."""
    b, _ = ce
    xi = dict(kind="exp", sigma2=0.9, a=3.0 if len(n) == 2 else 1.5)
    count, nbar = 6 if n[0] < 1024 else 4, 0.7
    results = []
    for sch in SCHEDULES:
        ctx = b.ctx_create(0)
        try:
            for opt, v in zip((b.OPT_LINES_NOISE, b.OPT_LINES_INNER, b.OPT_LINES_LAST, b.OPT_LINES_BINS),
                              sch.get("lines", (0, 0, 0, 0))):
                b.ctx_set_option(ctx, opt, v)
            if "bin_lds" in sch:
                b.ctx_set_option(ctx, b.OPT_BIN_LDS, sch["bin_lds"])
            if "noise_block" in sch:
                b.ctx_set_option(ctx, b.OPT_NOISE_BLOCK, sch["noise_block"])
            if "noise_order" in sch:
                b.ctx_set_option(ctx, b.OPT_NOISE_ORDER, sch["noise_order"])
            if "noise_pairs" in sch:
                b.ctx_set_option(ctx, b.OPT_NOISE_PAIRS, sch["noise_pairs"])
            plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
            o = dict(out_pk=torch.empty(count * nb, dtype=torch.float64, device="cuda"),
                     out_fields=torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda"),
                     out_delta=torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda"),
                     out_counts=torch.empty(count * plan.cells, dtype=torch.int32, device="cuda"),
                     out_ntot=torch.empty(count, dtype=torch.int64, device="cuda"),
                     out_cov=torch.empty(nb * nb, dtype=torch.float64, device="cuda"))
            b.pipeline_run(ctx, plan, 5, 2, 4, count, nbar, nb, **o)
            torch.cuda.synchronize()
            assert b.ctx_check(ctx) == 0
            results.append({k: v.cpu() for k, v in o.items()})
            plan.release()
        finally:
            b.ctx_destroy(ctx)
    for sch, r in zip(SCHEDULES[1:], results[1:]):
        for k in r:
            assert torch.equal(r[k], results[0][k]), (sch, k)
