"""The allocation-free entry point (ce_pipeline_run_noalloc) through the C ABI against
ce_pipeline_run: every output bit for bit, on two calls in a row (the second with a smaller
input, so stale contents of the shared static scratch would show), 2-D and 3-D, both
precisions, odd counts; a geometry one pair of which exceeds the static scratch is rejected
before anything runs."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


def outputs(plan, count, nb):
    return dict(out_pk=torch.empty(count * nb, dtype=torch.float64, device="cuda"),
                out_fields=torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda"),
                out_delta=torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda"),
                out_counts=torch.empty(count * plan.cells, dtype=torch.int32, device="cuda"),
                out_ntot=torch.empty(count, dtype=torch.int64, device="cuda"),
                out_cov=torch.empty(nb * nb, dtype=torch.float64, device="cuda"),
                out_cnorm=torch.empty(nb * nb, dtype=torch.float64, device="cuda"))


CALLS = [  # (n, xi, precision, count, nbins): the second call of each case is smaller
    [((1024, 1024), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0), 0, 96, 64),
     ((256, 192), dict(kind="exp", sigma2=0.8, a=5.0), 0, 7, 24)],
    [((96, 80), dict(kind="exp", sigma2=1.0, a=3.0), 1, 9, 16),
     ((32, 32), dict(kind="exp", sigma2=0.5, a=4.0), 1, 3, 8)],
    [((128, 128, 128), dict(kind="exp", sigma2=0.8, a=1.5), 0, 6, 12),
     ((16, 24, 20), dict(kind="exp", sigma2=0.8, a=1.5), 0, 3, 6)],
    # prime radices: 2N = 148 = 4.37 (ping-pong), then 124 = 4.31 and 68 = 4.17 (in place)
    [((74, 38), dict(kind="exp", sigma2=0.9, a=3.0), 0, 5, 10),
     ((62, 34), dict(kind="exp", sigma2=0.9, a=3.0), 0, 3, 10)],
]


@pytest.mark.parametrize("calls", CALLS, ids=["2d_f32", "2d_f64", "3d_f32", "primes_f32"])
def test_noalloc_equals_pipeline_run(ce, calls):
    b, ctx = ce
    for k, (n, xi, prec, count, nb) in enumerate(calls):
        print("no-alloc call", k, n, prec, count, flush=True)
        plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
        seed, rid, first, nbar = 13 + k, 2, 6, 0.9
        got, ref = outputs(plan, count, nb), outputs(plan, count, nb)
        b.pipeline_run_noalloc(ctx, plan, seed, rid, first, count, nbar, nb, **got)
        b.pipeline_run(ctx, plan, seed, rid, first, count, nbar, nb, **ref)
        torch.cuda.synchronize()
        assert b.ctx_check(ctx) == 0
        for key in ref:
            assert torch.equal(got[key], ref[key]), (k, key)
        plan.release()


def test_noalloc_rejects_what_does_not_fit(ce):
    b, ctx = ce
    n = (320, 320, 320)   # one pair's intermediates alone exceed the static scratch
    plan = b.plan_embedding(ctx, n, (1.0,) * 3, dict(kind="exp", sigma2=0.5, a=1.0), b.F32)
    pk = torch.empty(2 * 8, dtype=torch.float64, device="cuda")
    with pytest.raises(b.CeError) as e:
        b.pipeline_run_noalloc(ctx, plan, 1, 0, 0, 2, 1.0, 8, pk)
    assert e.value.status == b.E_UNSUPPORTED
    plan.release()
