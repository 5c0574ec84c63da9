"""The autotuner through the C ABI: a tuned schedule gives bitwise the default schedule's results
(fields, delta, counts, N_tot, P(k), covariance), persists as JSON that another context loads,
applies to the batched pipeline's groups, and malformed files or values are rejected."""

import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def b():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    return binding


def run(b, ctx, plan, count, nb, nbar=0.8):
    o = dict(out_pk=torch.empty(count * nb, dtype=torch.float64, device="cuda"),
             out_fields=torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda"),
             out_delta=torch.empty(count * plan.cells, dtype=plan.dtype, device="cuda"),
             out_counts=torch.empty(count * plan.cells, dtype=torch.int32, device="cuda"),
             out_ntot=torch.empty(count, dtype=torch.int64, device="cuda"),
             out_cov=torch.empty(nb * nb, dtype=torch.float64, device="cuda"))
    b.pipeline_run(ctx, plan, 3, 1, 0, count, nbar, nb, **o)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    return {k: v.cpu() for k, v in o.items()}


@pytest.mark.parametrize("n,prec", [((256, 256), 0), ((32, 24, 40), 0), ((96, 80), 1)])
def test_tuned_schedule_is_bitwise_default(b, tmp_path, n, prec):
    h = (1.0,) * len(n)
    xi = dict(kind="exp", sigma2=0.8, a=3.0 if len(n) == 2 else 1.5)
    count, nb = 8, 16
    ctx = b.ctx_create(0)
    try:
        plan = b.plan_embedding(ctx, n, h, xi, prec)
        ref = run(b, ctx, plan, count, nb)
        sch = b.autotune(ctx, plan, count, 0.8, nb, reps=2)
        print("tuned", n, prec, sch, flush=True)
        assert sch["ms"] > 0 and sch["default_ms"] > 0 and sch["ms"] <= sch["default_ms"]
        assert b.schedule_get(ctx, n, h, prec) is not None
        got = run(b, ctx, plan, count, nb)
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
        # persisted and loaded by another context: the same schedule, the same results
        path = tmp_path / "schedules.json"
        b.schedule_save(ctx, path)
        rec = json.loads(path.read_text())
        assert rec["format"] == "cefield-schedules" and len(rec["entries"]) == 1
        ctx2 = b.ctx_create(0)
        try:
            assert b.schedule_get(ctx2, n, h, prec) is None
            b.schedule_load(ctx2, path)
            got2 = b.schedule_get(ctx2, n, h, prec)
            for k in ("lines_noise", "lines_inner", "lines_last", "lines_bins", "noise_order", "noise_block",
                      "noise_pairs", "bin_lds"):
                assert got2[k] == sch[k], k
            plan2 = b.plan_embedding(ctx2, n, h, xi, prec)
            got3 = run(b, ctx2, plan2, count, nb)
            for k in ref:
                assert torch.equal(got3[k], ref[k]), k
            plan2.release()
        finally:
            b.ctx_destroy(ctx2)
        plan.release()
    finally:
        b.ctx_destroy(ctx)


def test_schedule_applies_to_batch_groups(b):
    """A schedule installed for one shape changes only the launch shape of that group in a batch."""
    ctx = b.ctx_create(0)
    try:
        shapes = [((64, 64), 0), ((96, 96), 0), ((64, 64), 1)]
        plans = [b.plan_embedding(ctx, n, (1.0, 1.0), dict(kind="exp", sigma2=0.7, a=3.0), p) for n, p in shapes]
        nb = 12

        def batch():
            items = []
            for k, p in enumerate(plans):
                items.append(dict(plan=p, seed=2, request_id=k, count=3, nbar=1.5, nbins=nb,
                                  out_pk=torch.empty(3 * nb, dtype=torch.float64, device="cuda"),
                                  out_counts=torch.empty(3 * p.cells, dtype=torch.int32, device="cuda"),
                                  out_fields=torch.empty(3 * p.cells, dtype=p.dtype, device="cuda")))
            b.pipeline_run_batch(ctx, items)
            torch.cuda.synchronize()
            return [{k: v.cpu() for k, v in it.items() if isinstance(v, torch.Tensor)} for it in items]

        ref = batch()
        b.schedule_set(ctx, (96, 96), (1.0, 1.0), 0, dict(lines_noise=4, lines_last=1, lines_bins=16,
                                                          noise_block=2, noise_pairs=3, bin_lds=163840))
        b.schedule_set(ctx, (64, 64), (1.0, 1.0), 1, dict(lines_noise=2, lines_bins=1, noise_order=1,
                                                          noise_pairs=8))
        got = batch()
        for r, g in zip(ref, got):
            for k in r:
                assert torch.equal(r[k], g[k]), k
        for p in plans:
            p.release()
    finally:
        b.ctx_destroy(ctx)


def test_schedule_errors(b, tmp_path):
    ctx = b.ctx_create(0)
    try:
        with pytest.raises(b.CeError):
            b.schedule_set(ctx, (64, 64), (1.0, 1.0), 0, dict(lines_noise=3))
        with pytest.raises(b.CeError):
            b.schedule_set(ctx, (64, 64), (1.0, 1.0), 0, dict(bin_lds=1 << 20))
        bad = tmp_path / "bad.json"
        bad.write_text('{"format": "cefield-schedules", "entries": [{"ndim": 2, "n": [64, 64, 1], '
                       '"precision": "f32", "lines": [3, 0, 0, 0]}]}')
        with pytest.raises(b.CeError):
            b.schedule_load(ctx, bad)
        bad.write_text('{"entries": []}')
        with pytest.raises(b.CeError):
            b.schedule_load(ctx, bad)
        with pytest.raises(b.CeError):
            b.schedule_load(ctx, tmp_path / "missing.json")
        assert b.schedule_get(ctx, (64, 64), (1.0, 1.0), 0) is None
        plan = b.plan_embedding(ctx, (32, 32), (1.0, 1.0), dict(kind="exp", sigma2=0.7, a=3.0), 0)
        with pytest.raises(b.CeError):
            b.autotune(ctx, plan, 4, 1.0, 8, reps=0)
        plan.release()
    finally:
        b.ctx_destroy(ctx)


def test_shipped_schedules_load_and_keep_results(b):
    """The package's schedule file loads; the headline shape's entry changes no output bit."""
    ctx = b.ctx_create(0)
    try:
        n, h = (1024, 1024), (1.0, 1.0)
        xi = dict(kind="exp", sigma2=0.8, a=3.0)
        plan = b.plan_embedding(ctx, n, h, xi, 0)
        ref = run(b, ctx, plan, 4, 32)
        b.schedule_load(ctx, b.DEFAULT_SCHEDULES)
        assert b.schedule_get(ctx, n, h, 0) is not None
        assert b.schedule_get(ctx, (256, 256, 256), (1.0,) * 3, 0) is not None
        got = run(b, ctx, plan, 4, 32)
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
        plan.release()
    finally:
        b.ctx_destroy(ctx)
