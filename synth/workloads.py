"""Seeded synthetic workloads shared by the tests, the benchmark and smoke.

Holds only input descriptions and seeded draws of request parameters; none
of the method's arithmetic lives here.  The shapes follow the paper's setting
(Sec. 3: a 128^2 survey in a 256^2 periodic embedding, lognormal density,
Poisson counts) scaled to the sizes the GPU path is measured on.  The survey
data and the fitted two-point function of the paper are not available; these
analytic two-point functions stand in for them.
"""

import numpy as np

POWEXP_GAMMA = 1.8


def _powexp(sigma2, r0, rc):
    return dict(kind="powexp", sigma2=float(sigma2), r0=float(r0), gamma=POWEXP_GAMMA, rc=float(rc))


WORKLOADS = {
    # 2-D 64^2 survey in a 128^2 embedding, FP64, 100 realizations
    "small_2d": dict(n=(64, 64), h=(1.0, 1.0), xi=dict(kind="exp", sigma2=0.5, a=8.0),
                     precision="f64", realizations=100, nbar=5.0, nbins=32, seed=0, request_id=0),
    # 2-D 1024^2 survey in a 2048^2 embedding, FP32 batched, 256 realizations
    "batched_2d": dict(n=(1024, 1024), h=(1.0, 1.0), xi=_powexp(1.0, 4.0, 300.0),
                       precision="f32", realizations=256, nbar=0.3, nbins=128, seed=0, request_id=0),
    # 3-D 256^3 survey in a 512^3 embedding, FP32 fields, 8 realizations
    "volume_3d": dict(n=(256, 256, 256), h=(1.0, 1.0, 1.0), xi=_powexp(2.0, 5.0, 200.0),
                      precision="f32", realizations=8, nbar=0.1, nbins=64, seed=0, request_id=0),
    # the paper's model input: the unfiltered angular omega (slope -0.7, cell units), averaged
    # over the cells and taken through ln(1 + omega) (cell variance 0.14, sigma_A^2 = 0.131)
    "paper_128_omega": dict(n=(128, 128), h=(1.0, 1.0),
                            xi=dict(kind="powexp", sigma2=0.185, r0=1.0, gamma=0.7, rc=300.0,
                                    cell_average=True, lognormal=True),
                            precision="f32", realizations=64, nbar=9.68, nbins=20, seed=0, request_id=0),
    # the paper's own geometry: 128^2 cells in a 256^2 embedding
    "paper_128": dict(n=(128, 128), h=(1.0, 1.0), xi=_powexp(0.131, 2.0, 300.0),
                      precision="f32", realizations=64, nbar=9.68, nbins=20, seed=0, request_id=0),
}


def uneven_batch(n_requests=4096, seed=4):
    """Mixed 2-D requests: side uniform on {32, 48, ..., 512}, sigma2 in [0.2, 2], r0 in [2, 10]."""
    rng = np.random.default_rng(seed)
    sides = np.arange(32, 513, 16)
    reqs = []
    for i in range(n_requests):
        N = int(rng.choice(sides))
        s2 = float(rng.uniform(0.2, 2.0))
        r0 = float(rng.uniform(2.0, 10.0))
        reqs.append(dict(request_id=i, n=(N, N), h=(1.0, 1.0), xi=_powexp(s2, r0, 300.0),
                         realizations=2, nbar=1.0, nbins=32, seed=0))
    return reqs


def _log_uniform_int(rng, lo, hi):
    """An integer in [lo, hi] drawn log-uniformly."""
    return int(min(hi, max(lo, np.round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))))


def serving_trace(rate=2000.0, duration=20.0, seed=5, max_side_2d=2048, max_side_3d=256, max_realizations=64):
    """Poisson arrivals mixing 2-D and 3-D requests from a menu of 16 two-point functions.
    Sides are every multiple of 16 in range, drawn log-uniformly (16 j, j log-uniform: 2-D
    64..max_side_2d, 3-D 32..max_side_3d); realizations log-uniform in 1 .. max_realizations."""
    rng = np.random.default_rng(seed)
    menu2 = [_powexp(s2, r0, 300.0) for s2, r0 in zip(np.linspace(0.2, 2.0, 8), np.linspace(2.0, 10.0, 8))]
    menu3 = [_powexp(s2, r0, rc) for s2, r0, rc in
             zip(np.linspace(0.2, 2.0, 8), np.linspace(1.0, 2.5, 8), [100.0, 200.0, 300.0] * 3)]
    t = 0.0
    reqs = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            break
        if rng.random() < 0.5:
            N = 16 * _log_uniform_int(rng, 4, max_side_2d // 16)
            n, h, xi = (N, N), (1.0, 1.0), menu2[int(rng.integers(8))]
        else:
            N = 16 * _log_uniform_int(rng, 2, max_side_3d // 16)
            n, h, xi = (N, N, N), (1.0, 1.0, 1.0), menu3[int(rng.integers(8))]
        R = int(np.round(np.exp(rng.uniform(0.0, np.log(max_realizations)))))
        reqs.append(dict(request_id=i, arrival=t, n=n, h=h, xi=xi, realizations=max(R, 1),
                         nbar=float(rng.choice([0.1, 0.3, 1.0, 5.0])), nbins=32, seed=0))
        i += 1
    return reqs


def survey_mask(n, seed=7, holes_per_cell=1.0 / 400.0, edge=0.06):
    """Synthetic surface-fraction map f in [0, 1] shaped like a masked survey: bright-star
    holes (disks of radius 1..4 cells, f = 0), a partially covered border strip (f = 0.85)
    and full coverage elsewhere; cells below 0.7 are fully masked (f = 0)."""
    rng = np.random.default_rng(seed)
    n = tuple(int(x) for x in n)
    f = np.ones(n, dtype=np.float64)
    w = max(1, int(round(edge * min(n))))
    for ax in range(len(n)):
        sl = [slice(None)] * len(n)
        sl[ax] = slice(0, w)
        f[tuple(sl)] = np.minimum(f[tuple(sl)], 0.85)
    for _ in range(max(1, int(np.prod(n) * holes_per_cell))):
        c = [int(rng.integers(0, x)) for x in n]
        r = rng.uniform(1.0, 4.0)
        # the disk lies inside the box of half-side 4 around its centre (no wrap-around)
        box = tuple(slice(max(0, ci - 4), min(x, ci + 5)) for ci, x in zip(c, n))
        grids = np.meshgrid(*[np.arange(b.start, b.stop) for b in box], indexing="ij")
        d2 = sum((g - ci) ** 2 for g, ci in zip(grids, c))
        sub = f[box]
        sub[d2 <= r * r] = 0.0
    f[f < 0.7] = 0.0
    return f.astype(np.float32)
