"""GPU edge cases through the C ABI: argument and geometry errors, the degenerate
nbar = 0 map, the smallest and the largest supported sides."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import embedding, fields as ofields  # noqa: E402
from parity_check import check_maps  # noqa: E402

XI = dict(kind="exp", sigma2=1.0, a=3.0)


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


def status_of(b, fn, *args, **kw):
    try:
        fn(*args, **kw)
    except b.CeError as e:
        return e.status
    return b.OK


@pytest.mark.parametrize("n,h,want", [
    ((31, 32), (1.0, 1.0), "E_UNSUPPORTED"),        # odd side
    ((2, 8), (1.0, 1.0), "E_UNSUPPORTED"),          # below the smallest side
    ((8, 2050), (1.0, 1.0), "E_UNSUPPORTED"),       # 2N above 4096 on the last axis
    ((4096, 8), (1.0, 1.0), "E_UNSUPPORTED"),       # 2N above 4096
    ((1024, 1024, 1024), (1.0,) * 3, "E_UNSUPPORTED"),  # embedding cells beyond 2^32
    ((16, 16), (1.0, 0.0), "E_INVALID"),            # cell side not positive
    ((16, 16), (1.0, float("nan")), "E_INVALID"),
])
def test_plan_rejects_unsupported_geometry(ce, n, h, want):
    b, ctx = ce
    assert status_of(b, b.plan_embedding, ctx, n, h, XI, b.F32) == getattr(b, want)


def test_pipeline_argument_errors(ce):
    b, ctx = ce
    plan = b.plan_embedding(ctx, (32, 32), (1.0, 1.0), XI, b.F32)
    pk = torch.empty(8 * 16, dtype=torch.float64, device="cuda")
    assert status_of(b, b.pipeline_run, ctx, plan, 1, 0, 0, 0, 1.0, 16, pk) == b.E_INVALID      # no realizations
    assert status_of(b, b.pipeline_run, ctx, plan, 1, 0, 1, 2, 1.0, 16, pk) == b.E_INVALID      # odd first
    assert status_of(b, b.pipeline_run, ctx, plan, 1, 0, 0, 2, 1.0, 0, pk) == b.E_INVALID       # no shells
    assert status_of(b, b.pipeline_run, ctx, plan, 1, 0, 0, 2, -1.0, 16, pk) == b.E_INVALID     # negative nbar
    assert status_of(b, b.pipeline_run, ctx, plan, 1, 0, 0, 2, float("inf"), 16, pk) == b.E_INVALID
    # first realization so large that the pair index leaves the 32-bit counter word
    assert status_of(b, b.pipeline_run, ctx, plan, 1, 0, 2 ** 33, 2, 1.0, 16, pk) == b.E_INVALID
    with pytest.raises(ValueError):  # the binding refuses an undersized output
        b.pipeline_run(ctx, plan, 1, 0, 0, 9, 1.0, 16, pk)
    plan.release()
    rect = b.plan_embedding(ctx, (32, 16), (1.0, 0.5 ** 0.5), XI, b.F32)
    # the integer shells need cell sides in a ratio of small integers (1 : 0.5 is fine)
    assert status_of(b, b.pipeline_run, ctx, rect, 1, 0, 0, 2, 1.0, 8, pk) == b.E_UNSUPPORTED
    rect.release()
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == b.OK


def test_nbar_zero_gives_empty_maps_and_a_flag(ce):
    """nbar = 0: every count is 0 and N_tot = 0, so the contrast is undefined; the library
    flags it (CE_E_SAMPLER at the next check) instead of failing silently, and the flag is
    cleared by the check."""
    b, ctx = ce
    plan = b.plan_embedding(ctx, (32, 32), (1.0, 1.0), XI, b.F32)
    count, nb = 4, 8
    pk = torch.empty(count * nb, dtype=torch.float64, device="cuda")
    c = torch.full((count * plan.cells,), 7, dtype=torch.int32, device="cuda")
    nt = torch.full((count,), 7, dtype=torch.int64, device="cuda")
    b.pipeline_run(ctx, plan, 1, 0, 0, count, 0.0, nb, pk, out_counts=c, out_ntot=nt)
    torch.cuda.synchronize()
    assert int(c.abs().sum()) == 0 and int(nt.abs().sum()) == 0
    assert b.ctx_check(ctx) == b.E_SAMPLER
    assert b.ctx_check(ctx) == b.OK
    plan.release()


@pytest.mark.parametrize("n,prec", [((4, 4), 1), ((4, 4, 4), 0), ((4, 6), 1),
                                    # short mixed lines (one lane per line): 2N = 12, 44 = 4.11,
                                    # 124 = 4.31, 148 = 4.37, 20 = 4.5, 28 = 4.7
                                    ((6, 22), 0), ((62, 4), 0), ((4, 74), 1), ((6, 10, 14), 0), ((22, 6), 1)])
def test_smallest_sides_match_oracle(ce, n, prec):
    b, ctx = ce
    xi = dict(kind="exp", sigma2=1.0, a=1.0)
    ref_plan = embedding.plan(n, (1.0,) * len(n), xi)
    ref = ofields.generate_fields(ref_plan, 5, 2, 0, 3)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    out = torch.empty(3 * plan.cells, dtype=plan.dtype, device="cuda")
    b.generate_fields(ctx, plan, 5, 2, 0, 3, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape((3,) + n)
    tol = 1e-12 if prec == 1 else 1e-5
    check_maps(got, ref, tol, math.sqrt(ref_plan["sigma2"]), str(n))
    plan.release()


def test_largest_2d_side_matches_oracle(ce):
    """N = 2048 (a 4096^2 embedding, the largest supported side), FP32, one pair."""
    b, ctx = ce
    n, xi = (2048, 2048), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0)
    print("largest side", n, flush=True)
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), xi, b.F32)
    out = torch.empty(2 * plan.cells, dtype=torch.float32, device="cuda")
    b.generate_fields(ctx, plan, 3, 1, 0, 2, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape((2,) + n)
    plan.release()
    ref_plan = embedding.plan(n, (1.0, 1.0), xi)
    ref = ofields.generate_fields(ref_plan, 3, 1, 0, 2)
    check_maps(got, ref, 1e-5, math.sqrt(ref_plan["sigma2"]), "2048^2 survey")


@pytest.mark.parametrize("n,prec", [((2040, 2040), 0), ((1530, 12), 1)])
def test_largest_mixed_sides_match_oracle(ce, n, prec):
    """The largest sides whose embedding has odd factors: 2N = 4080 = 16.3.5.17 (FP32, one pair,
    in-place prime stage on a 4080-point line) and a 3060-point first line in FP64
    (3060 = 4.3.3.5.17, two lines of it in one workgroup's LDS)."""
    b, ctx = ce
    xi = dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0)
    print("largest mixed side", n, prec, b.fft_factors(2 * n[0]), flush=True)
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), xi, prec)
    out = torch.empty(2 * plan.cells, dtype=plan.dtype, device="cuda")
    b.generate_fields(ctx, plan, 6, 3, 0, 2, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape((2,) + n)
    plan.release()
    ref_plan = embedding.plan(n, (1.0, 1.0), xi)
    ref = ofields.generate_fields(ref_plan, 6, 3, 0, 2)
    check_maps(got, ref, 1e-12 if prec == 1 else 1e-5, math.sqrt(ref_plan["sigma2"]), "mixed %s" % (n,))
