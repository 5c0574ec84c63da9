"""The k-space sampling comparator (Sec. 3.3, eq. Periodicboxmodes) and the cumulative
information (eq. cuminfo) on the GPU through the C ABI, against the oracle; and the two
statements of Sec. 3.3 that they exist to show: for Gaussian statistics the information is half
the number of modes, and the exact method's information saturates below that of periodic boxes,
which lack the super-survey modes."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import fields as ofields, kspace, pk as opk  # noqa: E402
from parity_check import check_maps  # noqa: E402
from synth import workloads  # noqa: E402


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


CASES = [
    ((16, 16), 32, 1.0, dict(kind="exp", sigma2=0.6, a=2.5)),
    ((12, 20), 24, 0.5, dict(kind="powexp", sigma2=0.185, r0=1.0, gamma=0.7, rc=6.0, lognormal=True)),
    ((32, 32), 32, 1.0, dict(kind="exp", sigma2=1.0, a=4.0)),                      # survey = box
    ((8, 8, 8), 16, 1.0, dict(kind="exp", sigma2=0.8, a=1.5)),
]


@pytest.mark.parametrize("n,box,h,xi", CASES)
def test_box_plan_matches_oracle(ce, n, box, h, xi):
    """Mode variances from the continuous spectrum (DC zeroed) and the cell variance."""
    b, ctx = ce
    print("box plan", n, box, h, xi, flush=True)
    ref = kspace.box_plan(n, box, h, xi)
    plan = b.plan_periodic(ctx, n, (h,) * len(n), box, xi, b.F64)
    lam = torch.empty(int(np.prod(plan.octant)), dtype=torch.float64, device="cuda")
    b.plan_eigenvalues(plan, lam)
    torch.cuda.synchronize()
    got = lam.cpu().numpy().reshape(plan.octant)
    want = ref["lam"][tuple(slice(0, o) for o in plan.octant)]
    assert got.flat[0] == 0.0
    assert np.max(np.abs(got - want)) <= 1e-10 * want.max()
    assert abs(plan.info["sigma2"] / ref["sigma2"] - 1) <= 1e-10
    plan.release()


@pytest.mark.parametrize("prec", [1, 0])
def test_box_fields_match_oracle(ce, prec):
    b, ctx = ce
    n, box, h, xi = CASES[1]
    ref = kspace.box_plan(n, box, h, xi)
    plan = b.plan_periodic(ctx, n, (h, h), box, xi, prec)
    out = torch.empty(6 * plan.cells, dtype=plan.dtype, device="cuda")
    b.generate_fields(ctx, plan, 11, 5, 4, 6, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape((6,) + n)
    want = ofields.generate_fields(ref, 11, 5, 4, 6)
    tol = 1e-10 if prec == 1 else 1e-5
    check_maps(got, want, tol, math.sqrt(ref["sigma2"]), "box fields")
    plan.release()


def test_box_plan_errors(ce):
    b, ctx = ce
    xi = dict(kind="exp", sigma2=1.0, a=2.0)
    for args, want in [(((16, 16), (1.0, 1.0), 8, xi), b.E_INVALID),          # box smaller than the survey
                       (((16, 16), (1.0, 1.0), 33, xi), b.E_INVALID),         # odd box
                       (((16, 16), (1.0, 0.5), 32, xi), b.E_UNSUPPORTED),     # unequal cells
                       (((16, 16), (1.0, 1.0), 4100, xi), b.E_UNSUPPORTED),   # box side above 4096
                       (((16, 16), (1.0, 1.0), 32, dict(xi, cell_average=True)), b.E_UNSUPPORTED),
                       (((16, 16), (1.0, 1.0), 32, dict(kind="powexp", sigma2=1.0, r0=1.0, gamma=0.7, rc=0.0)),
                        b.E_UNSUPPORTED)]:
        with pytest.raises(b.CeError) as e:
            b.plan_periodic(ctx, args[0], args[1], args[2], args[3], b.F32)
        assert e.value.status == want, args


def test_cumulative_information_matches_oracle(ce):
    b, ctx = ce
    rng = np.random.default_rng(3)
    for nb, R in ((1, 5), (7, 40), (64, 400), (300, 2000)):
        X = rng.normal(size=(R, nb)) * rng.uniform(0.5, 2.0, size=nb)
        C = X.T @ X / R + 0.05 * np.eye(nb)
        c = torch.from_numpy(C.ravel()).cuda()
        out = torch.empty(nb, dtype=torch.float64, device="cuda")
        b.cumulative_information(ctx, c, nb, out)
        torch.cuda.synchronize()
        want = opk.cumulative_information(C)
        assert np.max(np.abs(out.cpu().numpy() / want - 1)) <= 1e-10, nb
    # a block that is not positive definite: NaN from that shell on
    C = np.diag([0.5, 0.25, -1.0, 2.0])
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    b.cumulative_information(ctx, torch.from_numpy(C.ravel()).cuda(), 4, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.allclose(o[:2], [2.0, 6.0]) and np.all(np.isnan(o[2:]))


def information_curve(b, ctx, plan, R, nb, seed, field=False):
    """I(<= shell) from R realizations: spectra of delta (lognormal) or of the Gaussian field."""
    cells = plan.cells
    pkv = torch.empty(R * nb, dtype=torch.float64, device="cuda")
    if field:
        f = torch.empty(R * cells, dtype=plan.dtype, device="cuda")
        b.generate_fields(ctx, plan, seed, 1, 0, R, f)
        b.estimate_pk(ctx, plan.n, plan.h, plan.precision, b.MAP_FIELD, f, R, None, None, nb, pkv)
    else:
        d = torch.empty(R * cells, dtype=plan.dtype, device="cuda")
        b.pipeline_run(ctx, plan, seed, 1, 0, R, 1.0, nb, pkv, out_delta=d)
        b.estimate_pk(ctx, plan.n, plan.h, plan.precision, b.MAP_FIELD, d, R, None, None, nb, pkv)
    cn = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
    b.pk_covariance(ctx, pkv, R, nb, None, cn)
    info = torch.empty(nb, dtype=torch.float64, device="cuda")
    b.cumulative_information(ctx, cn, nb, info)
    torch.cuda.synchronize()
    return info.cpu().numpy()


def test_gaussian_information_is_half_the_modes(ce):
    """Gaussian fields on a periodic box that is the survey (no modes beyond it): the spectrum
    shells are independent and I(<= l) is half the number of modes below l (Sec. 3.3), to the
    5% that 8192 realizations and the inverse-covariance bias allow.  The spectrum is flat to 1%
    across the box (an exponential of range 0.02 cells), so every mode of a shell has the same
    power."""
    b, ctx = ce
    n, nb, R = (64, 64), 12, 8192
    plan = b.plan_periodic(ctx, n, (1.0, 1.0), 64, dict(kind="exp", sigma2=1.0, a=0.02), b.F32)
    info = information_curve(b, ctx, plan, R, nb, 5, field=True)
    plan.release()
    nmodes, _ = b.shell_table(n, (1.0, 1.0), nb)
    half = np.cumsum(nmodes) / 2.0
    hartlap = (R - 1) / (R - nb - 2)          # bias of the inverse of a sample covariance
    assert np.all(np.abs(info / (half * hartlap) - 1) < 0.05), (info, half)


def test_exact_information_saturates_below_periodic_boxes(ce):
    """The paper's comparison (Fig. 4, upper panel) on its model: the lognormal density of the
    128^2 map from the exact method carries less spectrum information than the same model
    simulated in 128^2 and 256^2 periodic boxes (k-space sampling, DC zeroed), and the 256^2 box
    is closer to the exact result than the 128^2 one."""
    b, ctx = ce
    w = workloads.WORKLOADS["paper_128_omega"]
    n, nb, R = w["n"], 16, 4096
    exact = b.plan_embedding(ctx, n, w["h"], w["xi"], b.F32)
    kxi = {k: v for k, v in w["xi"].items() if k != "cell_average"}
    curves = {"exact": information_curve(b, ctx, exact, R, nb, 9)}
    exact.release()
    for box in (128, 256):
        p = b.plan_periodic(ctx, n, w["h"], box, kxi, b.F32)
        curves[box] = information_curve(b, ctx, p, R, nb, 9)
        p.release()
    print({k: np.round(v[[0, 3, 7, 15]], 1).tolist() for k, v in curves.items()}, flush=True)
    top = {k: v[-1] for k, v in curves.items()}
    assert top["exact"] < 0.6 * top[256] and top[256] < 0.2 * top[128]
    # the exact curve has reached its plateau: the last half of the shells adds under 10%
    assert curves["exact"][-1] < 1.1 * curves["exact"][nb // 2 - 1]
