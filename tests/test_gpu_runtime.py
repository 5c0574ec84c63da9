"""GPU tests of the runtime around the pipeline, through the C ABI: the captured
(HIP graph) pipeline and the request server.  Both must reproduce ce_pipeline_run
bit for bit, so the references here are eager ce_pipeline_run calls (themselves
checked against the oracle in test_gpu_parity.py); the server mix also has one
case checked against the oracle directly.
"""

import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import embedding, fields as ofields, lognormal_poisson as olp, pk as opk  # noqa: E402
from parity_check import check_delta, check_maps  # noqa: E402


@pytest.fixture(scope="module")
def ce():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6072_amd import binding
    ctx = binding.ctx_create(0)
    yield binding, ctx
    binding.ctx_destroy(ctx)


def outputs(cells, count, nb, cov=True):
    return dict(out_pk=torch.empty(count * nb, dtype=torch.float64, device="cuda"),
                out_counts=torch.empty(count * cells, dtype=torch.int32, device="cuda"),
                out_ntot=torch.empty(count, dtype=torch.int64, device="cuda"),
                out_cov=torch.empty(nb * nb, dtype=torch.float64, device="cuda") if cov else None)


def host(o):
    return {k: v.cpu() for k, v in o.items() if v is not None}


GRAPH_CASES = [((128, 128), dict(kind="exp", sigma2=1.0, a=5.0), 0, 8, 32),
               ((24, 24, 24), dict(kind="exp", sigma2=0.8, a=1.5), 1, 4, 12)]


@pytest.mark.parametrize("n,xi,prec,count,nb", GRAPH_CASES)
def test_graph_replays_match_eager(ce, n, xi, prec, count, nb):
    """Four replays with eager pipeline calls between them; replay k must equal the eager
    call for realizations first + k*count .. (the graph advances by itself)."""
    b, ctx = ce
    print("graph case", n, prec, flush=True)
    plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
    seed, rid, first, nbar = 77, 5, 6, 2.0
    g_out = outputs(plan.cells, count, nb)
    g = b.pipeline_graph_create(ctx, plan, seed, rid, first, count, nbar, nb, **g_out)
    try:
        for k in range(4):
            b.pipeline_graph_launch(g)
            torch.cuda.synchronize()
            got = host(g_out)
            ref = outputs(plan.cells, count, nb)
            b.pipeline_run(ctx, plan, seed, rid, first + k * count, count, nbar, nb, **ref)
            torch.cuda.synchronize()
            assert b.ctx_check(ctx) == 0
            ref = host(ref)
            for key in ref:
                assert torch.equal(got[key], ref[key]), (k, key)
    finally:
        b.pipeline_graph_destroy(g)
    plan.release()


def test_graph_rejects_odd_count(ce):
    b, ctx = ce
    plan = b.plan_embedding(ctx, (32, 32), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=3.0), 0)
    o = outputs(plan.cells, 3, 8)
    with pytest.raises(b.CeError):
        b.pipeline_graph_create(ctx, plan, 1, 0, 0, 3, 1.0, 8, **o)
    plan.release()


def wait_all(b, server, tickets, timeout=90.0):
    states = {}
    t0 = time.time()
    while len(states) < len(tickets):
        for t in tickets:
            if t in states:
                continue
            st, status, lat = b.server_poll(server, t)
            if st >= 2:
                states[t] = (st, status, lat)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return states


MIX = [  # n, xi, prec, realizations, nbar, nbins
    ((64, 64), dict(kind="exp", sigma2=0.5, a=8.0), 1, 6, 5.0, 16),
    ((96, 96), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0), 0, 9, 0.3, 24),
    ((32, 32, 32), dict(kind="powexp", sigma2=1.0, r0=10.0, gamma=1.8, rc=0.0), 0, 4, 1.0, 8),  # not PSD
    ((20, 20, 20), dict(kind="exp", sigma2=0.8, a=1.5), 0, 5, 2.0, 10),
    ((64, 64), dict(kind="exp", sigma2=0.5, a=8.0), 1, 4, 1.0, 16),  # same plan as the first
    ((256, 256), dict(kind="exp", sigma2=1.0, a=5.0), 0, 32, 0.3, 64),
    ((40, 40), dict(kind="exp", sigma2=1.0, a=3.0), 1, 1, 5.0, 12),
    ((96, 96), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0), 0, 2, 0.3, 24),
]


@pytest.mark.parametrize("slots", [3, 1])
def test_server_mix_matches_requests_alone(ce, slots):
    b, ctx = ce
    server = b.server_create(0, slots=slots)
    try:
        outs, tickets = [], []
        for i, (n, xi, prec, R, nbar, nb) in enumerate(MIX):
            cells = int(np.prod(n))
            o = outputs(cells, R, nb)
            outs.append(o)
            tickets.append(b.server_submit(server, n, (1.0,) * len(n), xi, prec, 11, 100 + i, R, nbar, nb, **o))
        states = wait_all(b, server, tickets)
        stats = b.server_stats(server)
    finally:
        b.server_destroy(server)
    for i, (n, xi, prec, R, nbar, nb) in enumerate(MIX):
        st, status, lat = states[tickets[i]]
        print("request", i, n, prec, R, "state", st, "status", status, "latency_ms %.2f" % lat, flush=True)
        if i == 2:
            assert st == 3 and status == 2  # CE_E_NOT_PSD, alone
            continue
        assert st == 2 and status == 0 and lat > 0
        plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
        ref = outputs(plan.cells, R, nb)
        if R < 2:
            ref["out_cov"] = None
        b.pipeline_run(ctx, plan, 11, 100 + i, 0, R, nbar, nb, **ref)
        torch.cuda.synchronize()
        assert b.ctx_check(ctx) == 0
        got = host(outs[i])
        for key, v in host(ref).items():
            assert torch.equal(got[key], v), (i, key)
        plan.release()
    assert stats["submitted"] == len(MIX) and stats["completed"] == len(MIX) - 1 and stats["failed"] == 1
    assert stats["cache_hits"] >= 2 and stats["cache_misses"] == 6
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_server_groups_small_requests(ce):
    """A burst of small requests on one slot (ce_server_submit_many): the scheduler admits them
    in groups (one batched call per group), each request still equals its ce_pipeline_run
    alone, and a request that is invalid for the pipeline (negative nbar) fails alone inside
    its group."""
    b, ctx = ce
    shapes = [((32, 32), dict(kind="exp", sigma2=0.5, a=3.0), 0), ((48, 64), dict(kind="exp", sigma2=0.8, a=4.0), 1),
              ((16, 16, 16), dict(kind="exp", sigma2=0.6, a=1.2), 0), ((80, 80), dict(kind="exp", sigma2=1.0, a=5.0), 0)]
    reqs = []
    for i in range(40):
        n, xi, prec = shapes[i % 4]
        reqs.append((n, xi, prec, 1 + i % 5, -1.0 if i == 17 else 0.5 + 0.25 * (i % 3), 8 + (i % 2) * 4))
    # every third request bins in ln k (log-spaced edges up to the pixel scale)
    edges = {i: np.exp(np.linspace(np.log(0.3), np.log(np.pi), reqs[i][5] + 1)) for i in range(0, 40, 3)}
    server = b.server_create(0, slots=1)
    try:
        outs, batch = [], []
        for i, (n, xi, prec, R, nbar, nb) in enumerate(reqs):
            o = outputs(int(np.prod(n)), R, nb)
            outs.append(o)
            batch.append(dict(n=n, h=(1.0,) * len(n), xi=xi, precision=prec, seed=21, request_id=300 + i,
                              realizations=R, nbar=nbar, nbins=nb, edges=edges.get(i), **o))
        # the first ten one by one, the rest queued in one call
        tickets = [b.server_submit_many(server, [q])[0] for q in batch[:10]]
        tickets += b.server_submit_many(server, batch[10:])
        states = wait_all(b, server, tickets)
        stats = b.server_stats(server)
    finally:
        b.server_destroy(server)
    print("launches", stats["launches"], "largest group", stats["largest_group"], flush=True)
    assert stats["largest_group"] >= 2 and stats["launches"] < len(reqs)
    plans = {}
    for i, (n, xi, prec, R, nbar, nb) in enumerate(reqs):
        st, status, _ = states[tickets[i]]
        if i == 17:
            assert st == 3 and status == 1  # CE_E_INVALID, alone
            continue
        assert st == 2 and status == 0, (i, st, status)
        key = (n, prec)
        if key not in plans:
            plans[key] = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
        ref = outputs(plans[key].cells, R, nb)
        if R < 2:
            ref["out_cov"] = None
        if i in edges:
            b.pipeline_run_edges(ctx, plans[key], 21, 300 + i, 0, R, nbar, nb, edges[i], **ref)
        else:
            b.pipeline_run(ctx, plans[key], 21, 300 + i, 0, R, nbar, nb, **ref)
        torch.cuda.synchronize()
        got = host(outs[i])
        for k2, v in host(ref).items():
            assert same(got[k2], v), (i, k2)
    for p in plans.values():
        p.release()
    assert stats["completed"] == len(reqs) - 1 and stats["failed"] == 1


def test_server_submit_many_is_all_or_nothing(ce):
    """A batch submission with one invalid request (bad shell edges) queues nothing."""
    import math
    b, _ = ce
    server = b.server_create(0, slots=1)
    try:
        good = dict(n=(32, 32), h=(1.0, 1.0), xi=dict(kind="exp", sigma2=1.0, a=3.0), precision=0, seed=1,
                    request_id=0, realizations=2, nbar=1.0, nbins=8, **outputs(32 * 32, 2, 8))
        bad = dict(good, request_id=1, edges=np.linspace(math.pi, 0.0, 9))  # descending
        with pytest.raises(b.CeError) as e:
            b.server_submit_many(server, [good, bad, dict(good, request_id=2)])
        assert e.value.status == b.E_INVALID
        stats = b.server_stats(server)
        assert stats["submitted"] == 0 and stats["queued"] == 0
        t = b.server_submit_many(server, [good])
        states = wait_all(b, server, t)
    finally:
        b.server_destroy(server)
    assert states[t[0]][0] == 2


def test_server_request_against_oracle(ce):
    """Served requests checked against the oracle end to end on identical Philox streams: fields
    to the field tolerance (relative L2 and element-wise), delta from the GPU's fields, counts and
    N_tot bit-exact with the oracle fed the GPU's delta, P(k) per shell from the oracle on those
    counts.  Two requests of the same shape are submitted together, so they run as one group of
    the batched pipeline; a third of another shape runs beside them."""
    b, _ = ce
    nb, nbar, seed = 12, 3.0, 3
    cases = [((48, 48), dict(kind="exp", sigma2=0.5, a=6.0), 1, 4, 9),
             ((48, 48), dict(kind="exp", sigma2=0.9, a=3.0), 1, 3, 10),
             ((40, 24), dict(kind="exp", sigma2=0.7, a=4.0), 0, 2, 11)]
    server = b.server_create(0, slots=1)
    outs = []
    try:
        reqs = []
        for n, xi, prec, R, rid in cases:
            cells = n[0] * n[1]
            dt = torch.float64 if prec == 1 else torch.float32
            o = outputs(cells, R, nb, cov=False)
            o["out_fields"] = torch.empty(R * cells, dtype=dt, device="cuda")
            o["out_delta"] = torch.empty(R * cells, dtype=dt, device="cuda")
            outs.append(o)
            reqs.append(dict(n=n, h=(1.0, 1.0), xi=xi, precision=prec, seed=seed, request_id=rid, realizations=R,
                             nbar=nbar, nbins=nb, **o))
        tickets = b.server_submit_many(server, reqs)
        states = wait_all(b, server, tickets)
    finally:
        b.server_destroy(server)
    for (n, xi, prec, R, rid), o, t in zip(cases, outs, tickets):
        st, status, _ = states[t]
        assert st == 2 and status == 0
        ref_plan = embedding.plan(n, (1.0, 1.0), xi)
        tol = 1e-12 if prec == 1 else 1e-5
        g = o["out_fields"].cpu().numpy().reshape((R,) + n)
        check_maps(g, ofields.generate_fields(ref_plan, seed, rid, 0, R), tol, np.sqrt(ref_plan["sigma2"]),
                   "served fields %s" % (n,))
        dh = o["out_delta"].cpu().numpy().reshape((R,) + n)
        check_delta(dh, olp.lognormal_delta(g.astype(np.float64), ref_plan["sigma2"]), tol)
        _, rc, rn = olp.lognormal_poisson(g.astype(np.float64), ref_plan["sigma2"], nbar, seed, rid, 0, delta=dh)
        assert np.array_equal(o["out_counts"].cpu().numpy().reshape((R,) + n), rc)
        assert np.array_equal(o["out_ntot"].cpu().numpy(), rn)
        rp = opk.estimate_pk(rc, 1.0, nb, kind="counts", ntot=rn)
        assert np.max(np.abs(o["out_pk"].cpu().numpy().reshape(R, nb) / rp - 1)) <= tol


def test_batch_fields_and_delta_equal_single_calls(ce):
    """Fields and delta requested from the batched pipeline equal those of ce_pipeline_run
    for each item alone, bit for bit (odd counts, both precisions, one item without them)."""
    b, ctx = ce
    specs = [((32, 32), dict(kind="exp", sigma2=1.0, a=3.0), 0, 3, True),
             ((32, 32), dict(kind="exp", sigma2=0.6, a=2.0), 0, 2, False),
             ((32, 32), dict(kind="exp", sigma2=0.8, a=4.0), 0, 5, True),
             ((20, 24), dict(kind="exp", sigma2=0.8, a=4.0), 1, 4, True)]
    nb, nbar = 10, 2.0
    items, refs, plans = [], [], []
    for k, (n, xi, prec, R, want) in enumerate(specs):
        plan = b.plan_embedding(ctx, n, (1.0, 1.0), xi, prec)
        plans.append(plan)
        o = outputs(plan.cells, R, nb)
        r = outputs(plan.cells, R, nb)
        if want:
            for d in (o, r):
                d["out_fields"] = torch.empty(R * plan.cells, dtype=plan.dtype, device="cuda")
                d["out_delta"] = torch.empty(R * plan.cells, dtype=plan.dtype, device="cuda")
        items.append(dict(plan=plan, seed=4, request_id=30 + k, count=R, nbar=nbar, nbins=nb, **o))
        b.pipeline_run(ctx, plan, 4, 30 + k, 0, R, nbar, nb, **r)
        refs.append(r)
    b.pipeline_run_batch(ctx, items)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    for it, r in zip(items, refs):
        for key in r:
            if r[key] is not None:
                assert torch.equal(it[key].cpu(), r[key].cpu()), key
    for p in plans:
        p.release()


def test_server_rejects_what_never_fits(ce):
    b, _ = ce
    server = b.server_create(0, slots=2, hbm_budget_bytes=1 << 20)
    try:
        o = outputs(128 * 128, 8, 16)
        t = b.server_submit(server, (128, 128), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=5.0), 0, 1, 0, 8,
                            0.3, 16, **o)
        st, status, _ = wait_all(b, server, [t])[t]
    finally:
        b.server_destroy(server)
    assert st == 3 and status == 3  # CE_E_OOM


def test_server_budget_serialises_but_stays_exact(ce):
    """A budget that admits one 256^2 request at a time: later requests wait (admission
    stalls) and still produce what they produce alone."""
    b, ctx = ce
    n, xi, R, nb = (256, 256), dict(kind="exp", sigma2=1.0, a=5.0), 16, 32
    server = b.server_create(0, slots=4, hbm_budget_bytes=40 << 20)
    try:
        outs, tickets = [], []
        for i in range(4):
            o = outputs(256 * 256, R, nb)
            outs.append(o)
            tickets.append(b.server_submit(server, n, (1.0, 1.0), xi, 0, 4, i, R, 0.3, nb, **o))
        states = wait_all(b, server, tickets)
        stats = b.server_stats(server)
    finally:
        b.server_destroy(server)
    assert all(states[t][0] == 2 for t in tickets)
    assert stats["admission_stalls"] > 0 and stats["cache_hits"] == 3
    plan = b.plan_embedding(ctx, n, (1.0, 1.0), xi, 0)
    for i in range(4):
        ref = outputs(plan.cells, R, nb)
        b.pipeline_run(ctx, plan, 4, i, 0, R, 0.3, nb, **ref)
        torch.cuda.synchronize()
        got = host(outs[i])
        for key, v in host(ref).items():
            assert torch.equal(got[key], v), (i, key)
    plan.release()


def test_server_cancel_queued(ce):
    b, _ = ce
    server = b.server_create(0, slots=1)
    try:
        big = outputs(512 * 512, 64, 32)
        t0 = b.server_submit(server, (512, 512), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=5.0), 0, 1, 0, 64,
                             0.3, 32, **big)
        small = outputs(64 * 64, 2, 8)
        t1 = b.server_submit(server, (64, 64), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=5.0), 0, 1, 1, 2,
                             0.3, 8, **small)
        cancelled = b.server_cancel(server, t1) == 0
        states = wait_all(b, server, [t0, t1])
    finally:
        b.server_destroy(server)
    assert states[t0][0] == 2
    # the cancel can lose the race against admission; either outcome must be consistent
    assert states[t1][0] == (4 if cancelled else 2)


def test_batch_matches_items_alone(ce):
    """Ragged batch: several shapes and cell shapes, both precisions, odd counts, odd first realizations of
    pairs, optional outputs; every item equals its own ce_pipeline_run bit for bit."""
    b, ctx = ce
    specs = [  # n, xi, prec, first, count, nbar, nb, with_counts, with_cov
        ((32, 32), dict(kind="exp", sigma2=1.0, a=3.0), 0, 0, 2, 1.0, 8, True, True),
        ((48, 48), dict(kind="exp", sigma2=0.4, a=5.0), 0, 4, 3, 0.5, 12, True, True),
        ((32, 32), dict(kind="exp", sigma2=1.5, a=2.0), 0, 2, 5, 5.0, 8, False, True),
        ((48, 48), dict(kind="exp", sigma2=0.4, a=5.0), 1, 0, 2, 0.5, 12, True, False),
        ((16, 16, 16), dict(kind="exp", sigma2=0.8, a=1.5), 0, 0, 1, 2.0, 6, True, False),
        ((32, 32), dict(kind="exp", sigma2=1.0, a=3.0), 0, 6, 2, 1.0, 16, True, True),  # other nbins
        ((96, 96), dict(kind="powexp", sigma2=1.0, r0=4.0, gamma=1.8, rc=300.0), 0, 0, 4, 0.3, 24, True, True),
        ((16, 16, 16), dict(kind="exp", sigma2=0.8, a=1.5), 0, 2, 4, 2.0, 6, True, True),
        # every FFT variant in one batch: 2N = 60 = 4.3.5 and 84 (in place, radices up to 7),
        # 88 = 8.11 and 104 = 8.13 (in place, primes 11..31), 148 = 4.37 (ping-pong, generic prime)
        ((30, 42), dict(kind="exp", sigma2=0.9, a=3.0), 0, 0, 4, 1.0, 10, True, True),
        ((44, 52), dict(kind="exp", sigma2=0.9, a=3.0), 0, 0, 3, 1.0, 10, True, True),
        ((74, 38), dict(kind="exp", sigma2=0.9, a=3.0), 0, 0, 4, 1.0, 10, True, True),
        ((44, 52), dict(kind="exp", sigma2=0.9, a=3.0), 1, 0, 2, 1.0, 10, True, True),
        ((74, 38), dict(kind="exp", sigma2=0.9, a=3.0), 1, 2, 3, 1.0, 10, True, True),
        ((32, 32), dict(kind="exp", sigma2=1.0, a=3.0), 0, 0, 3, 1.0, 8, True, True),  # 1 x 0.5 cells
    ]
    cells_h = {len(specs) - 1: (1.0, 0.5)}  # same sides as item 0, other cell shape: its own group
    plans, items = [], []
    for k, (n, xi, prec, first, count, nbar, nb, wc, wv) in enumerate(specs):
        plan = b.plan_embedding(ctx, n, cells_h.get(k, (1.0,) * len(n)), xi, prec)
        plans.append(plan)
        o = outputs(plan.cells, count, nb, cov=wv)
        if not wc:
            o["out_counts"] = None
        items.append(dict(plan=plan, seed=3 + k, request_id=40 + k, first_realization=first, count=count,
                          nbar=nbar, nbins=nb, **o))
    for rep in range(2):  # the second call reuses the staging and scratch buffers
        b.pipeline_run_batch(ctx, items)
        torch.cuda.synchronize()
        assert b.ctx_check(ctx) == 0
        for k, it in enumerate(items):
            ref = outputs(it["plan"].cells, it["count"], it["nbins"], cov=it["out_cov"] is not None)
            if it["out_counts"] is None:
                ref["out_counts"] = None
            b.pipeline_run(ctx, it["plan"], it["seed"], it["request_id"], it["first_realization"], it["count"],
                           it["nbar"], it["nbins"], **ref)
            torch.cuda.synchronize()
            got = host({key: it[key] for key in ("out_pk", "out_counts", "out_ntot", "out_cov")})
            for key, v in host(ref).items():
                assert torch.equal(got[key], v), (rep, k, key)
    for p in plans:
        p.release()


def same(a, b):
    """Bitwise equality of two tensors, an empty shell's NaN equal to itself."""
    return np.array_equal(a.numpy(), b.numpy(), equal_nan=True)


def test_batch_with_user_edges(ce):
    """Items with the paper's log-spaced shells (and others with the default shells or other
    edges, same shapes) in one batch: every item equals its own ce_pipeline_run_edges (or
    ce_pipeline_run) bit for bit."""
    import math
    b, ctx = ce
    log8 = np.exp(np.linspace(math.log(0.15), math.log(math.pi), 9))
    log6 = np.exp(np.linspace(math.log(0.3), math.log(math.pi), 7))
    specs = [  # n, xi, prec, count, nbar, nb, edges
        ((32, 32), dict(kind="exp", sigma2=1.0, a=3.0), 0, 4, 1.0, 8, log8),
        ((32, 32), dict(kind="exp", sigma2=1.0, a=3.0), 0, 3, 1.0, 8, None),
        ((32, 32), dict(kind="exp", sigma2=0.5, a=2.0), 0, 2, 2.0, 8, np.linspace(0.0, math.pi, 9)),
        ((48, 64), dict(kind="exp", sigma2=0.4, a=5.0), 1, 5, 0.5, 8, log8),
        ((16, 16, 16), dict(kind="exp", sigma2=0.8, a=1.5), 0, 2, 2.0, 6, log6),
        ((32, 32), dict(kind="exp", sigma2=0.7, a=3.0), 0, 2, 3.0, 8, log8),
    ]
    plans, items = [], []
    for k, (n, xi, prec, count, nbar, nb, edges) in enumerate(specs):
        plan = b.plan_embedding(ctx, n, (1.0,) * len(n), xi, prec)
        plans.append(plan)
        items.append(dict(plan=plan, seed=7 + k, request_id=60 + k, first_realization=0, count=count, nbar=nbar,
                          nbins=nb, edges=edges, **outputs(plan.cells, count, nb)))
    b.pipeline_run_batch(ctx, items)
    torch.cuda.synchronize()
    assert b.ctx_check(ctx) == 0
    for k, it in enumerate(items):
        ref = outputs(it["plan"].cells, it["count"], it["nbins"])
        if it["edges"] is None:
            b.pipeline_run(ctx, it["plan"], it["seed"], it["request_id"], 0, it["count"], it["nbar"], it["nbins"],
                           **ref)
        else:
            b.pipeline_run_edges(ctx, it["plan"], it["seed"], it["request_id"], 0, it["count"], it["nbar"],
                                 it["nbins"], it["edges"], **ref)
        torch.cuda.synchronize()
        got = host({key: it[key] for key in ("out_pk", "out_counts", "out_ntot", "out_cov")})
        for key, v in host(ref).items():
            assert same(got[key], v), (k, key)
    # bad edges reject the whole batch before anything runs
    bad = dict(items[0], edges=log8[::-1].copy())
    with pytest.raises(b.CeError):
        b.pipeline_run_batch(ctx, [items[1], bad])
    for p in plans:
        p.release()


def test_batch_rejects_bad_item_without_launching(ce):
    b, ctx = ce
    plan = b.plan_embedding(ctx, (32, 32), (1.0, 1.0), dict(kind="exp", sigma2=1.0, a=3.0), 0)
    good = dict(plan=plan, count=2, nbar=1.0, nbins=8, **outputs(plan.cells, 2, 8))
    bad = dict(good, first_realization=1)
    sentinel = good["out_pk"].fill_(-7.0).clone()
    with pytest.raises(b.CeError):
        b.pipeline_run_batch(ctx, [good, bad])
    torch.cuda.synchronize()
    assert torch.equal(good["out_pk"], sentinel)
    plan.release()
