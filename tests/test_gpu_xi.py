"""Transformed two-point functions on the GPU through the C ABI: the cell-averaged (square
top-hat filtered) omega of App. A and the lognormal target ln(1 + omega) of eq. Lncov, against
the oracle; plans and fields built from them; and the covariance of the lognormal density of
the paper's model against the cell-averaged omega it is built to reproduce."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import embedding, fields as ofields, filtered  # noqa: E402
from parity_check import check_maps  # noqa: E402
from synth import workloads  # noqa: E402

POWEXP = dict(kind="powexp", sigma2=0.185, r0=1.0, gamma=0.7, rc=300.0)
EXP = dict(kind="exp", sigma2=0.5, a=2.5)


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


def gpu_octant(b, ctx, n, h, xi):
    out = torch.empty(int(np.prod([x + 1 for x in n])), dtype=torch.float64, device="cuda")
    b.xi_lag_octant(ctx, n, h, xi, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(tuple(x + 1 for x in n))


@pytest.mark.parametrize("n,h,base,flags", [
    ((32, 32), (1.0, 1.0), POWEXP, dict(cell_average=True)),
    ((40, 24), (1.0, 0.7), POWEXP, dict(cell_average=True, lognormal=True)),
    ((36, 36), (2.0, 2.0), EXP, dict(cell_average=True)),
    ((16, 16, 8), (1.0, 1.0, 1.0), EXP, dict(lognormal=True)),
])
def test_lag_octant_matches_oracle(ce, n, h, base, flags):
    """Direct overlap integral below 15 cells, derivative expansion beyond (2-D), and the
    lognormal map, against the oracle's adaptive quadrature and expansion."""
    b, ctx = ce
    print("lag octant", n, h, base["kind"], flags, flush=True)
    xi = dict(base, **flags)
    got = gpu_octant(b, ctx, n, h, xi)
    want = embedding.lag_octant(n, h, xi)
    assert np.max(np.abs(got - want)) <= 1e-12 * abs(want.flat[0])


def test_table_lognormal(ce):
    b, ctx = ce
    n, h = (8, 10), (1.0, 1.0)
    rng = np.random.default_rng(2)
    tab = rng.uniform(-0.5, 1.0, size=(9, 11))
    got = gpu_octant(b, ctx, n, h, dict(kind="table", table=tab, lognormal=True))
    assert np.max(np.abs(got - np.log1p(tab))) <= 1e-15


@pytest.mark.parametrize("prec", [1, 0])
def test_plan_and_fields_in_omega_mode(ce, prec):
    """A plan from ln(1 + omega^h): eigenvalues, cell variance and fields against the oracle."""
    b, ctx = ce
    n, h = (48, 48), (1.0, 1.0)
    xi = dict(POWEXP, cell_average=True, lognormal=True)
    ref = embedding.plan(n, h, xi)
    plan = b.plan_embedding(ctx, n, h, xi, prec)
    assert abs(plan.info["sigma2"] - ref["sigma2"]) <= 1e-13
    lam = torch.empty((n[0] + 1) * (n[1] + 1), dtype=torch.float64, device="cuda")
    b.plan_eigenvalues(plan, lam)
    torch.cuda.synchronize()
    oct_ref = ref["lam"][: n[0] + 1, : n[1] + 1]
    # the plan keeps the eigenvalues before clamping; the oracle's are clamped at 0
    assert np.max(np.abs(np.maximum(lam.cpu().numpy().reshape(oct_ref.shape), 0) - oct_ref)) <= \
        1e-11 * ref["lambda_max"]
    out = torch.empty(4 * plan.cells, dtype=plan.dtype, device="cuda")
    b.generate_fields(ctx, plan, 7, 3, 2, 4, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape((4,) + n)
    want = ofields.generate_fields(ref, 7, 3, 2, 4)
    tol = 1e-10 if prec == 1 else 1e-5
    check_maps(got, want, tol, math.sqrt(ref["sigma2"]), "omega-mode fields")
    plan.release()


def test_lognormal_density_reproduces_cell_averaged_omega(ce):
    """The paper's model (Sec. 3.1, 128^2 cells, omega averaged over the cells and taken through
    ln(1 + omega)): the density contrast delta = rho - 1 of 512 fused-pipeline realizations has
    covariance omega^h at lags 0, (1,0), (0,1), (1,1), (4,0), (0,9) within 5 standard errors,
    while the unfiltered omega is excluded at lag 0."""
    b, ctx = ce
    w = workloads.WORKLOADS["paper_128_omega"]
    n, R = w["n"], 512
    plan = b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    assert abs(plan.info["sigma2"] - math.log(1.14)) < 2e-3   # sigma_A^2 of the paper
    cells = plan.cells
    delta = torch.empty(R * cells, dtype=torch.float32, device="cuda")
    pk = torch.empty(R * 8, dtype=torch.float64, device="cuda")
    b.pipeline_run(ctx, plan, 21, 4, 0, R, w["nbar"], 8, pk, out_delta=delta)
    torch.cuda.synchronize()
    plan.release()
    d = delta.view(R, *n).double()
    base = {k: v for k, v in w["xi"].items() if k not in ("cell_average", "lognormal")}
    om = lambda r: float(embedding.eval_xi(base, r))  # noqa: E731
    for lag in ((0, 0), (1, 0), (0, 1), (1, 1), (4, 0), (0, 9)):
        a = d[:, : n[0] - lag[0], : n[1] - lag[1]]
        c = d[:, lag[0]:, lag[1]:]
        per = (a * c).mean(dim=(1, 2)).cpu().numpy()   # one estimate per realization
        # the sample mean of delta is not subtracted: <rho> = 1 holds by construction
        se = per.std(ddof=1) / math.sqrt(R)
        want = filtered.cell_average_exact(om, lag, w["h"])
        assert abs(per.mean() - want) < 5 * se, (lag, per.mean(), want, se)
        if lag == (0, 0):
            assert abs(per.mean() - om(0.0)) > 10 * se     # the point variance is not the cell variance


def test_transform_errors(ce):
    b, ctx = ce
    out = torch.empty(20 * 20 * 20, dtype=torch.float64, device="cuda")

    def status(n, xi, bits=None):
        g = b.geometry(n, (1.0,) * len(n))
        x, keep = b.xi_spec(xi)
        if bits is not None:
            x.transform = bits
        import ctypes
        return b._xi_lag_octant(ctx, ctypes.byref(g), ctypes.byref(x), b._ptr(out), None)

    assert status((8, 8, 8), dict(EXP, cell_average=True)) == b.E_UNSUPPORTED
    assert status((8, 8), dict(kind="table", table=np.zeros((9, 9)), cell_average=True)) == b.E_UNSUPPORTED
    assert status((8, 8), EXP, bits=4) == b.E_INVALID
    # a table value <= -1 has no logarithm: the plan is rejected
    tab = np.full((9, 9), 0.1)
    tab[0, 0] = 1.0
    tab[3, 2] = -1.5
    with pytest.raises(b.CeError) as e:
        b.plan_embedding(ctx, (8, 8), (1.0, 1.0), dict(kind="table", table=tab, lognormal=True), b.F64)
    assert e.value.status == b.E_NOT_PSD
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == b.OK
