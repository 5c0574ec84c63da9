#!/usr/bin/env python3
"""Throughput of the fused circulant-embedding hot path on one MI355X.

One step = one batch of the whole path through the C ABI (ce_pipeline_run):
noise -> scaled inverse FFT pruned to the survey -> crop -> lognormal ->
Poisson counts -> counts P(k) in shells -> spectrum covariance, for the
2-D 1024^2 survey in a 2048^2 embedding (FP32, 256 realizations per step,
nbar = 0.3, 128 shells).  The embedding plan (lag table + FP64 eigenvalue FFT
+ non-negativity check) is built once per (geometry, xi) key before the timed
region, as a serving cache would; its time is reported as plan_ms.

Printed: one JSON line with throughput, per-step latency, the roofline of the
dominant kernel (HIP-event durations measured inside the timed region), the
plain FP64 comparator (FP64, unfused, unpruned, one realization per launch
chain) and the CPU oracle on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cropped realizations/s + % peak HBM GB/s vs plain FP64 path; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per second (FP32/INT32 and,
# on CDNA4, FP64 arithmetic issue at one operation per lane per cycle; packed FP32 is not used).
VALU_PEAK_GOPS = 256 * 64 * 2.4

# Algorithmic VALU lane-operations per unit of work (the op model: transcendentals count 4).
OPS_PHILOX = 60          # 10 rounds x (2 32x32->64 products + 4 XOR)
OPS_BOX_MULLER = 23      # 2 uniforms (2 each), log2/sqrt/sin/cos (4 each, quarter rate), 3 mul
OPS_SCALE = 2            # complex x real sqrt(lambda)
OPS_LOGNORMAL = 7        # sub, mul log2e, exp2 (4), sub 1
OPS_INTENSITY = 3        # FP64 convert, add, mul
OPS_EXP64 = 20           # FP64 exp: range reduction + polynomial
OPS_POIS_STEP = 4        # FP64 mul, mul, add, compare
OPS_SEPARATE = 4         # Hermitian separation per output
OPS_BIN = 5              # |F|^2 in FP64 and the shell sum


def fft_ops(L):
    """4 log2(L) lane-ops per complex element (5 log2 L flops with one FMA per radix-2 butterfly)."""
    import math
    return 4.0 * math.log2(L)


def kernel_ops(name, n, pairs, nb, count, nbar):
    """Algorithmic VALU lane-operations of one launch of a pipeline kernel over `pairs` pairs."""
    d = len(n)
    M = [2 * x for x in n]
    cells = 1
    emb = 1
    for x in n:
        cells *= x
        emb *= 2 * x
    Nl = n[-1]
    W = 2 * (Nl // 2 + 1)
    rows = cells // Nl
    pois = OPS_PHILOX / 2 + 3 + OPS_EXP64 + OPS_POIS_STEP * (nbar + 1)   # per value, one chunk
    if name == "noise_inverse_axis0":
        return pairs * emb * (OPS_PHILOX / 2 + OPS_BOX_MULLER / 2 + OPS_SCALE + fft_ops(M[0]))
    if name == "inverse_axis1":
        return pairs * n[0] * M[1] * M[2] * fft_ops(M[1])
    if name == "inverse_last_fused":
        per_pair = (rows * M[-1] * fft_ops(M[-1]) + 2 * cells * (OPS_LOGNORMAL + OPS_INTENSITY + pois)
                    + cells * fft_ops(Nl) + rows * W * OPS_SEPARATE)
        return pairs * per_pair
    if name == "forward_axis1":
        return pairs * n[0] * n[1] * W * fft_ops(n[1])
    if name == "forward_axis0_bins":
        lines = (n[1] * W) if d == 3 else W
        return pairs * lines * n[0] * (fft_ops(n[0]) + OPS_BIN)
    return 0


SCHEDULE_FILE = os.path.join(ROOT, "paper_1406_6072_amd", "schedules_gfx950.json")


def schedule_file(args):
    """The launch-schedule file the run loads: --schedules, else the schedules shipped with the
    package (none with --schedules none or --retune)."""
    if args.schedules == "none" or (args.retune and not args.schedules):
        return ""
    if args.schedules:
        return args.schedules
    return SCHEDULE_FILE if os.path.exists(SCHEDULE_FILE) else ""


def save_schedules(b, ctx, path):
    """Merge ctx's schedules into the JSON file at path (entries keyed by shape and precision)."""
    import tempfile
    with tempfile.NamedTemporaryFile(suffix=".json", delete=False) as f:
        tmp = f.name
    try:
        b.schedule_save(ctx, tmp)
        new = json.load(open(tmp))
    finally:
        os.unlink(tmp)
    if os.path.exists(path):
        old = json.load(open(path))
        key = lambda e: (e["ndim"], tuple(e["n"]), e["precision"])
        merged = {key(e): e for e in old.get("entries", [])}
        merged.update({key(e): e for e in new["entries"]})
        new["entries"] = sorted(merged.values(), key=lambda e: (e["ndim"], e["n"], e["precision"]))
    with open(path, "w") as f:
        json.dump(new, f, indent=1)
        f.write("\n")


def counters_for(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) and VALU busy of a kernel from the
    committed counter summary, if the kernel sources are unchanged since it was taken; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec.get("kernels", {}).get(kernel)


def cic_leg(b, torch, ctx, plan, mask, counts, R, nb, nbar, n, h, stream, steps):
    """Counts-in-cells statistics of the masked maps (Sec. 3.4): the 42-bin histogram, the
    mean-subtracted A* map (FP32) and its P(k), per step of R maps."""
    cells = plan.cells
    nh = 42
    s2 = plan.info["sigma2"]
    hist = torch.empty(R * nh, dtype=torch.int64, device=counts.device)
    amap = torch.empty(R * cells, dtype=torch.float32, device=counts.device)
    apk = torch.empty(R * nb, dtype=torch.float64, device=counts.device)

    def cstep():
        b.cic_histogram(ctx, counts, cells, R, mask, nh, hist, stream)
        b.astar_map(ctx, counts, cells, R, mask, nbar, s2, True, b.F32, amap, None, stream)
        b.estimate_pk(ctx, n, h, b.F32, b.MAP_FIELD, amap, R, None, None, nb, apk, stream=stream)

    cstep()
    torch.cuda.synchronize()
    b.ctx_profile_read(ctx)
    b.ctx_set_profiling(ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        cstep()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    b.ctx_set_profiling(ctx, False)
    prof = b.ctx_profile_read(ctx)
    kern = {k: round(v[0] / steps, 4) for k, v in prof.items()}
    hist_ms = kern.get("cic_histogram", 0.0)
    # the model's mean histogram for this mask (once per survey, not per step)
    pred = torch.empty(nh, dtype=torch.float64, device=counts.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.cic_predict(ctx, mask, cells, nbar, s2, nh, pred, stream)
    torch.cuda.synchronize()
    predict_ms = (time.perf_counter() - t0) * 1e3
    hist_bytes = 4 * cells * R + 4 * cells  # the counts of every map (int32); the mask (float) once
    return dict(value=round(R / dt, 1), unit="maps/s", ms_per_step=round(1e3 * dt, 3), steps=steps,
                kernels_ms=kern, histogram_GBs=round(hist_bytes / (hist_ms * 1e-3) / 1e9, 1) if hist_ms else None,
                predict_ms=round(predict_ms, 3),
                form="42-bin histogram over f != 0, A* (FP64 solve, mean over f != 0 subtracted, stored FP32), "
                     "P(k) of the A* map through the spectrum estimator")


def information_leg(b, torch, R):
    """The comparison of Sec. 3.3 on the paper's model (128^2 map, cell-averaged omega through
    ln(1 + omega)): cumulative information of the density spectrum from R realizations of the
    exact method and of 128^2, 256^2, 512^2 periodic boxes (k-space sampling, DC zeroed)."""
    from synth import workloads
    w = workloads.WORKLOADS["paper_128_omega"]
    n, h, nb = w["n"], w["h"], 16
    ctx = b.ctx_create(0)
    dev = torch.device("cuda:0")
    cells = n[0] * n[1]
    d = torch.empty(R * cells, dtype=torch.float32, device=dev)
    pkv = torch.empty(R * nb, dtype=torch.float64, device=dev)
    cn = torch.empty(nb * nb, dtype=torch.float64, device=dev)
    info = torch.empty(nb, dtype=torch.float64, device=dev)
    out = dict(map=list(n), shells=nb, realizations=R, model="paper_128_omega")
    # the boxes take the continuous transform of ln(1 + omega) (eq. Periodicboxmodes), omega
    # not cell-averaged; "exact_point" is the exact method on that same omega, so that the
    # spectra differ only by the box (the grid's aliased power near the pixel scale)
    kxi = {k: v for k, v in w["xi"].items() if k != "cell_average"}
    exact_pk = None
    for name in ("exact", "exact_point", 128, 256, 512):
        t0 = time.perf_counter()
        if name == "exact":
            plan = b.plan_embedding(ctx, n, h, w["xi"], b.F32)
        elif name == "exact_point":
            plan = b.plan_embedding(ctx, n, h, kxi, b.F32)
        else:
            plan = b.plan_periodic(ctx, n, h, name, kxi, b.F32)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        b.pipeline_run(ctx, plan, 9, 1, 0, R, w["nbar"], nb, pkv, out_delta=d)
        b.estimate_pk(ctx, n, h, b.F32, b.MAP_FIELD, d, R, None, None, nb, pkv)
        b.pk_covariance(ctx, pkv, R, nb, None, cn)
        b.cumulative_information(ctx, cn, nb, info)
        torch.cuda.synchronize()
        run_s = time.perf_counter() - t0
        curve = info.cpu().numpy()
        # mean spectrum of the density contrast (Sec. 3.3: k-space sampling loses power near the
        # pixel scale); reported for the boxes as a ratio to the exact method's, top three shells
        mpk = pkv.cpu().numpy().reshape(R, nb).mean(axis=0)
        rec = dict(info_last=round(float(curve[-1]), 2), info_mid=round(float(curve[nb // 2 - 1]), 2),
                   plan_s=round(plan_s, 3), run_s=round(run_s, 3),
                   periodic_side=2 * n[0] if isinstance(name, str) else name)
        if name == "exact_point":
            exact_pk = mpk
        elif name != "exact":
            rec["pk_ratio_to_exact_point_top_shells"] = [round(float(x), 4) for x in (mpk / exact_pk)[-3:]]
            rec["pk_ratio_to_exact_point_low_shells"] = [round(float(x), 4) for x in (mpk / exact_pk)[:3]]
        out[name if isinstance(name, str) else "box_%d" % name] = rec
        plan.release()
    nm, _ = b.shell_table(n, h, nb)
    out["gaussian_half_modes"] = float(nm.sum() / 2)
    b.ctx_destroy(ctx)
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched_2d")
    ap.add_argument("--plain-realizations", type=int, default=8)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the oracle comparison of one timed pair")
    ap.add_argument("--no-tune", action="store_true",
                    help="run no ce_autotune: shapes without a loaded schedule keep the default one")
    ap.add_argument("--schedules", default="",
                    help="launch schedules (JSON) loaded before timing; default: the package's "
                         "schedules_gfx950.json; 'none': default schedules (tuned unless --no-tune)")
    ap.add_argument("--batch-lanes", type=int, default=0,
                    help="concurrent lanes of ce_pipeline_run_batch (0: the library's default)")
    ap.add_argument("--retune", action="store_true",
                    help="load no schedule file (unless --schedules names one): tune every shape")
    ap.add_argument("--save-schedules", default="",
                    help="merge the schedules used (loaded or tuned) into this JSON file")
    ap.add_argument("--skip-main", action="store_true",
                    help="skip the headline step and its comparators (profiling of the other legs only)")
    ap.add_argument("--volume-steps", type=int, default=10, help="steps of the 3-D workload leg (0: skip it)")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-step (HIP graph) leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--lines", default="",
                    help="schedule: max lines per workgroup for noise,inner,last,bins (0 = automatic)")
    ap.add_argument("--noise-order", type=int, default=-1, help="schedule: noise-pass tile order (0/1)")
    ap.add_argument("--no-masked", action="store_true", help="skip the masked-survey leg")
    ap.add_argument("--no-cic", action="store_true", help="skip the counts-in-cells leg (histogram, A* and its P(k))")
    ap.add_argument("--info-realizations", type=int, default=4096,
                    help="realizations per method of the information experiment (0: skip it)")
    ap.add_argument("--batch-requests", type=int, default=4096,
                    help="requests of the uneven-batch leg (mixed 2-D sides 32..512); 0 to skip")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--serve-rates", default="250,500,1000,2000",
                    help="offered request rates (1/s) of the open-loop serving leg; empty to skip")
    ap.add_argument("--serve-seconds", type=float, default=4.0, help="arrival window per rate")
    ap.add_argument("--serve-warmup", type=float, default=1.0, help="arrivals before the window (not counted)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-offline", type=int, default=1,
                    help="also run the saturation trace as one batched call (the serving-efficiency reference)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for counter calibration)")
    return ap.parse_args()


def workload_description(w, name):
    n = w["n"]
    d = len(n)
    side = "x".join(str(x) for x in n)
    emb = "x".join(str(2 * x) for x in n)
    return ("%dD survey %s cells in %s periodic embedding, xi=%s, %s, %d realizations per step, "
            "lognormal + Poisson nbar=%g, %d-shell P(k) + covariance (%s)"
            % (d, side, emb, w["xi"], w["precision"].upper(), w["realizations"], w["nbar"], w["nbins"], name))


def kernel_bytes(name, n, prec, pairs, nb, count):
    """Algorithmic HBM bytes of one launch of a pipeline kernel over `pairs` pairs."""
    d = len(n)
    ce = 16 if prec == "f64" else 8   # complex element
    N0, Nl = n[0], n[-1]
    M = [2 * x for x in n]
    cells = 1
    for x in n:
        cells *= x
    W = 2 * (Nl // 2 + 1)
    rows = cells // Nl
    H = rows * W * ce
    octant = 1
    for x in n:
        octant *= x + 1
    octant *= (8 if prec == "f64" else 4)
    if name == "noise_inverse_axis0":
        y1 = N0 * (M[1] * (M[2] if d == 3 else 1)) * ce
        return pairs * y1 + octant
    if name == "inverse_axis1":
        y1 = N0 * M[1] * M[2] * ce
        y2 = N0 * n[1] * M[2] * ce
        return pairs * (y1 + y2)
    if name == "inverse_last_fused":
        yin = rows * M[-1] * ce
        return pairs * (yin + 2 * cells * 4 + H)
    if name == "forward_axis1":
        return pairs * 2 * H
    if name == "forward_axis0_bins":
        return pairs * H
    if name == "bin_reduce":
        return count * nb * 8
    if name == "covariance":
        return count * nb * 8 + 2 * nb * nb * 8
    return 0


def request_alg_bytes(n, realizations, prec="f32"):
    """Algorithmic HBM bytes of the fused path for one request (2-D: 28 N^2 per realization in FP32,
    52 N^2 in FP64; 3-D: 68 N^3 in FP32, 132 N^3 in FP64), plus nothing for the plan."""
    cells = 1
    for x in n:
        cells *= x
    per = {(2, "f32"): 28, (2, "f64"): 52, (3, "f32"): 68, (3, "f64"): 132}[(len(n), prec)]
    return per * cells * realizations


def accuracy_leg(b, torch, ctx, plan, w, pair=0):
    """Error of the fused path against the FP64 oracle on identical Philox streams, for one pair of
    the timed workload (realizations 2 pair, 2 pair + 1 of the same call geometry): fields (relative
    L2, max |dg| / sqrt(xi(0))), delta from the GPU's fields, counts (mismatches with the oracle fed
    the GPU's delta) and N_tot, P(k) per shell (oracle fed the same counts)."""
    import numpy as np
    from oracle import embedding, fields, lognormal_poisson, pk
    n, nb, nbar = w["n"], w["nbins"], w["nbar"]
    cells = plan.cells
    f = torch.empty(2 * cells, dtype=plan.dtype, device="cuda")
    d = torch.empty_like(f)
    c = torch.empty(2 * cells, dtype=torch.int32, device="cuda")
    nt = torch.empty(2, dtype=torch.int64, device="cuda")
    p = torch.empty(2 * nb, dtype=torch.float64, device="cuda")
    b.pipeline_run(ctx, plan, w["seed"], w["request_id"], 2 * pair, 2, nbar, nb, p, f, d, c, nt)
    torch.cuda.synchronize()
    ref_plan = embedding.plan(n, w["h"], w["xi"])
    ref = fields.generate_fields(ref_plan, w["seed"], w["request_id"], 2 * pair, 2)
    g = f.cpu().numpy().astype(np.float64).reshape(ref.shape)
    dg = g - ref
    sig = float(np.sqrt(ref_plan["sigma2"]))
    dh = d.cpu().numpy().reshape(ref.shape)
    rd = lognormal_poisson.lognormal_delta(g, ref_plan["sigma2"])
    _, rc, rn = lognormal_poisson.lognormal_poisson(g, ref_plan["sigma2"], nbar, w["seed"], w["request_id"],
                                                    2 * pair, delta=dh)
    ch = c.cpu().numpy().reshape(ref.shape)
    rp = pk.estimate_pk(rc, 1.0, nb, kind="counts", ntot=rn)
    return dict(pair=pair, fields_rel_l2=float(np.linalg.norm(dg) / np.linalg.norm(ref)),
                fields_max_abs_over_sigma=float(np.max(np.abs(dg)) / sig),
                delta_max_rel=float(np.max(np.abs(dh - rd) / (1 + np.abs(rd)))),
                counts_mismatches=int(np.count_nonzero(ch != rc)), cells=int(ch.size),
                ntot_equal=bool(np.array_equal(nt.cpu().numpy(), rn)),
                pk_max_rel=float(np.max(np.abs(p.cpu().numpy().reshape(2, nb) / rp - 1))),
                tolerances=dict(fields=1e-5 if w["precision"] == "f32" else 1e-12, counts="bit-exact",
                                pk=1e-5 if w["precision"] == "f32" else 1e-12))


def cpu_oracle_sample(w, seconds):
    """The FP64 oracle (as it stands) on whole pairs of the same workload until `seconds` pass."""
    import numpy as np
    from oracle import embedding, fields, lognormal_poisson, pk
    t0 = time.perf_counter()
    plan = embedding.plan(w["n"], w["h"], w["xi"])
    t_plan = time.perf_counter() - t0
    pairs = 0
    spectra = []
    t0 = time.perf_counter()
    while True:
        g = fields.generate_fields(plan, w["seed"], w["request_id"], 2 * pairs, 2)
        _, counts, ntot = lognormal_poisson.lognormal_poisson(g, plan["sigma2"], w["nbar"], w["seed"],
                                                              w["request_id"], 2 * pairs)
        spectra.append(pk.estimate_pk(counts, 1.0, w["nbins"], kind="counts", ntot=ntot))
        pairs += 1
        if time.perf_counter() - t0 >= seconds or pairs >= 64:
            break
    allp = np.concatenate(spectra)
    pk.covariance(allp)
    dt = time.perf_counter() - t0
    return dict(value=2 * pairs / dt, unit="realizations/s", cores=1, kind="oracle",
                sample="%d pairs (%d realizations) of the timed workload, full pipeline incl. covariance; "
                       "plan %.1f s excluded" % (pairs, 2 * pairs, t_plan),
                seconds=dt)


def uneven_batch_leg(b, torch, nreq, reps, sample_every=32, tune=True, schedules="", save="", lanes=0):
    """The uneven batch (4096 requests of 2 realizations, 2-D sides 32..512 step 16, each with its
    own two-point function) through ce_pipeline_run_batch, FP32 and FP64 on identical Philox
    streams; plans are built before the timed region.  Also the same requests as one
    ce_pipeline_run call each (FP32), for the batching gain.  The FP32-vs-FP64 ladder: for every
    request the relative L2 and largest relative shell error of the FP32 P(k) against the FP64
    P(k), the fraction of counts that differ (a Poisson draw flips where the two precisions' delta
    straddle a CDF step), and on every `sample_every`-th request the fields (relative L2 and
    max |dg| / sqrt(xi(0)))."""
    import numpy as np
    from synth import workloads
    reqs = workloads.uneven_batch(nreq)
    ctx = b.ctx_create(0)
    if lanes:
        b.ctx_set_option(ctx, b.OPT_BATCH_LANES, lanes)
    out = dict(requests=len(reqs), realizations=2 * len(reqs),
               distinct_shapes=len({r["n"] for r in reqs}))
    kept = {}
    try:
        for prec, tag in ((b.F32, "f32"), (b.F64, "f64")):
            t0 = time.perf_counter()
            plans = [b.plan_embedding(ctx, r["n"], r["h"], r["xi"], prec) for r in reqs]
            plan_s = time.perf_counter() - t0
            items, alg = [], 0
            for i, (r, p) in enumerate(zip(reqs, plans)):
                R, nb = r["realizations"], r["nbins"]
                it = dict(plan=p, seed=r["seed"], request_id=r["request_id"], count=R, nbar=r["nbar"],
                          nbins=nb, out_pk=torch.empty(R * nb, dtype=torch.float64, device="cuda"),
                          out_counts=torch.empty(R * p.cells, dtype=torch.int32, device="cuda"),
                          out_ntot=torch.empty(R, dtype=torch.int64, device="cuda"),
                          out_cov=torch.empty(nb * nb, dtype=torch.float64, device="cuda"))
                if i % sample_every == 0:
                    it["out_fields"] = torch.empty(R * p.cells, dtype=p.dtype, device="cuda")
                items.append(it)
                alg += request_alg_bytes(r["n"], R, tag) + (4 if tag == "f32" else 8) * (r["n"][0] + 1) ** 2
            # the item table is marshalled once (Python); each timed call is one C call plus the GPU
            t0 = time.perf_counter()
            prepared = b.prepare_batch(items)
            marshal_ms = 1e3 * (time.perf_counter() - t0)
            b.pipeline_run_batch(ctx, prepared)
            torch.cuda.synchronize()
            if b.ctx_check(ctx) != 0:
                raise RuntimeError("device flagged a sampler condition in the uneven batch")
            times = []
            enq = []
            for _ in range(reps):
                t0 = time.perf_counter()
                b.pipeline_run_batch(ctx, prepared)
                enq.append(time.perf_counter() - t0)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            ms = 1e3 * float(np.median(times))
            leg = dict(value=round(2 * len(reqs) / (ms * 1e-3), 1), unit="realizations/s", ms_per_batch=round(ms, 3),
                       alg_GB=round(alg / 1e9, 3), alg_GBs=round(alg / (ms * 1e-3) / 1e9, 1),
                       hbm_frac=round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), plan_s=round(plan_s, 2),
                       python_marshal_ms=round(marshal_ms, 2), host_enqueue_ms=round(1e3 * float(np.median(enq)), 2),
                       form="ce_pipeline_run_batch on a prepared item table (one C call per batch)")
            kept[tag] = [dict(pk=it["out_pk"].cpu().numpy(), counts=it["out_counts"].cpu().numpy(),
                              fields=it["out_fields"].cpu().numpy().astype(np.float64) if "out_fields" in it else None)
                         for it in items]
            if prec == b.F32 and (tune or schedules):
                # the launch schedules of the distinct shapes (from the schedule file; the shapes it
                # lacks tuned on that shape's requests), then the same batch again
                t0 = time.perf_counter()
                if schedules:
                    b.schedule_load(ctx, schedules)
                seen = {}
                for r, p in zip(reqs, plans):
                    seen.setdefault(r["n"], [p, 0, r["h"]])[1] += r["realizations"]
                ntuned = 0
                for nn, (p, R, hh) in seen.items():
                    if tune and b.schedule_get(ctx, nn, hh, b.F32) is None:
                        b.autotune(ctx, p, R, 1.0, 32, reps=2)
                        ntuned += 1
                tune_s = time.perf_counter() - t0
                if save:
                    save_schedules(b, ctx, save)
                b.pipeline_run_batch(ctx, prepared)
                torch.cuda.synchronize()
                tt = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    b.pipeline_run_batch(ctx, prepared)
                    torch.cuda.synchronize()
                    tt.append(time.perf_counter() - t0)
                tms = 1e3 * float(np.median(tt))
                leg["default_schedule"] = dict(ms_per_batch=leg["ms_per_batch"], alg_GBs=leg["alg_GBs"])
                leg.update(value=round(2 * len(reqs) / (tms * 1e-3), 1), ms_per_batch=round(tms, 3),
                           alg_GBs=round(alg / (tms * 1e-3) / 1e9, 1),
                           hbm_frac=round(alg / (tms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           tuned=dict(shapes=len(seen), tuned_here=ntuned, from_file=len(seen) - ntuned,
                                      tune_s=round(tune_s, 2)))
            if prec == b.F32:
                sub = items[:512]
                for it in sub[:8]:
                    b.pipeline_run(ctx, it["plan"], it["seed"], it["request_id"], 0, it["count"], it["nbar"],
                                   it["nbins"], it["out_pk"], out_counts=it["out_counts"], out_ntot=it["out_ntot"],
                                   out_cov=it["out_cov"])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for it in sub:
                    b.pipeline_run(ctx, it["plan"], it["seed"], it["request_id"], 0, it["count"], it["nbar"],
                                   it["nbins"], it["out_pk"], out_counts=it["out_counts"], out_ntot=it["out_ntot"],
                                   out_cov=it["out_cov"])
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                leg["unbatched"] = dict(value=round(2 * len(sub) / dt, 1), unit="realizations/s",
                                        sample="first %d requests, one ce_pipeline_run each" % len(sub))
            out[tag] = leg
            del items
            for p in plans:
                p.release()
    finally:
        b.ctx_destroy(ctx)
    # the ladder: FP32 against FP64 on the same Philox streams
    pk_l2, pk_max, flips, cells, f_l2, f_max = [], [], 0, 0, [], []
    for r, a, d in zip(reqs, kept["f32"], kept["f64"]):
        ok = np.isfinite(d["pk"]) & (d["pk"] != 0)   # shells without modes (small grids) hold NaN
        pa, pd = a["pk"][ok], d["pk"][ok]
        pk_l2.append(float(np.linalg.norm(pa - pd) / np.linalg.norm(pd)))
        pk_max.append(float(np.max(np.abs(pa / pd - 1))))
        flips += int(np.count_nonzero(a["counts"] != d["counts"]))
        cells += a["counts"].size
        if a["fields"] is not None:
            df = a["fields"] - d["fields"]
            f_l2.append(float(np.linalg.norm(df) / np.linalg.norm(d["fields"])))
            f_max.append(float(np.max(np.abs(df)) / np.sqrt(r["xi"]["sigma2"])))
    out["ladder_f32_vs_f64"] = dict(
        pk_rel_l2=dict(median=float(np.median(pk_l2)), max=float(np.max(pk_l2))),
        pk_max_rel_shell=dict(median=float(np.median(pk_max)), max=float(np.max(pk_max))),
        counts_differing_fraction=flips / max(cells, 1),
        fields_rel_l2=dict(requests=len(f_l2), median=float(np.median(f_l2)), max=float(np.max(f_l2))),
        fields_max_abs_over_sigma=float(np.max(f_max)),
        note="identical Philox streams; P(k) differences are dominated by the counts that flip")
    return out


def serving_outputs(torch, trace, nb):
    offs, tot = [], 0
    for r in trace:
        offs.append(tot)
        tot += r["realizations"] * nb + r["realizations"] + (nb * nb if r["realizations"] >= 2 else 0)
    return offs, torch.empty(max(tot, 1), dtype=torch.float64, device="cuda")


def submit_traced(b, torch, server, r, pool, o, nb, request_id):
    R = r["realizations"]
    pk = pool[o:o + R * nb]
    ntot = pool[o + R * nb:o + R * nb + R].view(torch.int64)
    cov = pool[o + R * nb + R:o + R * nb + R + nb * nb] if R >= 2 else None
    return b.server_submit(server, r["n"], r["h"], r["xi"], b.F32, r["seed"], request_id, R, r["nbar"], nb, pk,
                           out_ntot=ntot, out_cov=cov)


def serving_warm(b, torch, server, trace, nb=32):
    """Closed loop: submit every request of the trace at once and wait for all; returns
    (seconds, requests per second).  Builds the plans and grows the slots' scratch as a
    long-running server would have."""
    offs, pool = serving_outputs(torch, trace, nb)
    t0 = time.perf_counter()
    left = {submit_traced(b, torch, server, r, pool, offs[i], nb, r["request_id"]) for i, r in enumerate(trace)}
    while left:
        for t, st, status, ms in b.server_drain(server):
            left.discard(t)
        time.sleep(0.0005)
    dt = time.perf_counter() - t0
    return dt, len(trace) / dt, sum(request_alg_bytes(r["n"], r["realizations"]) for r in trace) / dt / 1e9


def offline_batch(b, torch, trace, nb=32):
    """The requests of a trace run as one ce_pipeline_run_batch call (plans built beforehand, the
    item table prepared once; the same outputs as served: P(k), N_tot, covariance), after one
    untimed call: the throughput the same work reaches without arrival order or admission."""
    offs, pool = serving_outputs(torch, trace, nb)
    ctx = b.ctx_create(0)
    plans = {}
    try:
        items = []
        for i, r in enumerate(trace):
            key = (r["n"], tuple(sorted(r["xi"].items())))
            if key not in plans:
                plans[key] = b.plan_embedding(ctx, r["n"], r["h"], r["xi"], b.F32)
            R, o = r["realizations"], offs[i]
            items.append(dict(plan=plans[key], seed=r["seed"], request_id=r["request_id"], count=R, nbar=r["nbar"],
                              nbins=nb, out_pk=pool[o:o + R * nb],
                              out_ntot=pool[o + R * nb:o + R * nb + R].view(torch.int64),
                              out_cov=pool[o + R * nb + R:o + R * nb + R + nb * nb] if R >= 2 else None))
        prepared = b.prepare_batch(items)
        b.pipeline_run_batch(ctx, prepared)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.pipeline_run_batch(ctx, prepared)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        for p in plans.values():
            p.release()
        b.ctx_destroy(ctx)
    return dict(seconds=round(dt, 4), requests_per_s=round(len(trace) / dt, 1),
                alg_GBs=round(sum(request_alg_bytes(r["n"], r["realizations"]) for r in trace) / dt / 1e9, 1),
                plans=len(plans))


def small_request_leg(b, torch, slots):
    """Closed-loop throughput of a burst of small requests (2-D sides 64..256, 3-D 32..64, 1..4
    realizations) through the server with groups of up to 256 requests per launch and with one
    request per launch."""
    from synth import workloads
    trace = workloads.serving_trace(rate=4000.0, duration=1.0, seed=7, max_side_2d=256, max_side_3d=64,
                                    max_realizations=4)
    out = dict(requests=len(trace), realizations=sum(r["realizations"] for r in trace))
    nb = 32
    offs, pool = serving_outputs(torch, trace, nb)
    reqs = []
    for i, r in enumerate(trace):
        R, o = r["realizations"], offs[i]
        reqs.append(dict(n=r["n"], h=r["h"], xi=r["xi"], precision=b.F32, seed=r["seed"], request_id=r["request_id"],
                         realizations=R, nbar=r["nbar"], nbins=nb, out_pk=pool[o:o + R * nb],
                         out_ntot=pool[o + R * nb:o + R * nb + R].view(torch.int64),
                         out_cov=pool[o + R * nb + R:o + R * nb + R + nb * nb] if R >= 2 else None))

    def burst(server):
        # every request queued in one call, so the scheduler sees them at once
        t0 = time.perf_counter()
        left = set(b.server_submit_many(server, reqs))
        while left:
            for t, st, status, ms in b.server_drain(server):
                left.discard(t)
            time.sleep(0.0002)
        dt = time.perf_counter() - t0
        return dt, len(reqs) / dt

    for tag, mg in (("grouped", 0), ("one_per_launch", 1)):
        server = b.server_create(0, slots=slots, max_group=mg)
        try:
            burst(server)  # plans and scratch
            st0 = b.server_stats(server)
            dt, rps = burst(server)
            st = b.server_stats(server)
        finally:
            b.server_destroy(server)
        out[tag] = dict(seconds=round(dt, 4), requests_per_s=round(rps, 1),
                        realizations_per_s=round(out["realizations"] / dt, 1),
                        launches=int(st["launches"] - st0["launches"]),
                        largest_group=int(st["largest_group"]))
    return out


def serving_leg(b, torch, server, rate, seconds, warmup):
    """Open-loop replay of a Poisson arrival trace of mixed 2-D/3-D requests through the request
    server (continuous batching, plan cache), already warm.  Requests arriving in the first
    `warmup` seconds are not counted.  Latency = completion seen by the server's scheduler minus
    submission; submissions lag the nominal arrival by `max_lateness_ms` at most."""
    import numpy as np
    from synth import workloads
    trace = workloads.serving_trace(rate=rate, duration=warmup + seconds, seed=5)
    nb = 32
    offs, pool = serving_outputs(torch, trace, nb)
    stats0 = b.server_stats(server)
    pending = {}
    lat, real_done, failed, lateness, bytes_done = [], 0, 0, 0.0, 0
    t_start = time.perf_counter()
    i = 0
    backlog_at_end = None
    try:
        while i < len(trace) or pending:
            now = time.perf_counter() - t_start
            while i < len(trace) and trace[i]["arrival"] <= now:
                r = trace[i]
                R = r["realizations"]
                t = submit_traced(b, torch, server, r, pool, offs[i], nb, r["request_id"])
                lateness = max(lateness, now - r["arrival"])
                pending[t] = (r["arrival"] >= warmup, R, request_alg_bytes(r["n"], R))
                i += 1
            if backlog_at_end is None and i == len(trace):
                backlog_at_end = len(pending)
            for t, st, status, ms in b.server_drain(server):
                counted, R, nbytes = pending.pop(t)
                if counted:
                    if st == 2:
                        lat.append(ms)
                        real_done += R
                        bytes_done += nbytes
                    else:
                        failed += 1
            time.sleep(0.0002)
        wall = time.perf_counter() - t_start
        stats = b.server_stats(server)
    finally:
        pass
    counted_reqs = [r for r in trace if r["arrival"] >= warmup]
    span = max(wall - warmup, 1e-9)
    return dict(offered_rate=rate, requests=len(counted_reqs), completed=len(lat), failed=failed,
                realizations_per_s=round(real_done / span, 1), requests_per_s=round(len(lat) / span, 1),
                alg_GBs=round(bytes_done / span / 1e9, 1),
                offered_GBs=round(sum(request_alg_bytes(r["n"], r["realizations"]) for r in counted_reqs)
                                  / seconds / 1e9, 1),
                p50_ms=round(float(np.percentile(lat, 50)), 3) if lat else None,
                p99_ms=round(float(np.percentile(lat, 99)), 3) if lat else None,
                drain_s=round(wall - (warmup + seconds), 3), backlog_at_last_arrival=backlog_at_end,
                max_lateness_ms=round(1e3 * lateness, 3), plan_cache_hits=stats["cache_hits"] - stats0["cache_hits"],
                plan_cache_misses=stats["cache_misses"] - stats0["cache_misses"],
                admission_stalls=stats["admission_stalls"] - stats0["admission_stalls"])


def timed_workload(b, torch, ctx, w, name, steps, warmup, stream, tune=False):
    """Time `steps` fused steps (ce_pipeline_run of the workload's realizations, counts, N_tot,
    P(k), covariance) after `warmup` untimed ones, with per-kernel HIP events recorded by the
    library on the launch stream.  The roofline is that of the kernel with the largest share of
    the step: its algorithmic bytes per launch over its average event duration, against the HBM
    peak (the counter-measured traffic and VALU busy of the committed counter summary beside it,
    when the kernel sources are unchanged; the VALU op model as an extra field).  With `tune`, the
    step is first timed with the default schedule, then ce_autotune picks the launch schedule of
    the workload's shape (installed in ctx) and the timed steps run with it."""
    import numpy as np
    prec = b.F64 if w["precision"] == "f64" else b.F32
    n, h, nb, R, nbar = w["n"], w["h"], w["nbins"], w["realizations"], w["nbar"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    plan = b.plan_embedding(ctx, n, h, w["xi"], prec)
    plan_ms = (time.perf_counter() - t0) * 1e3
    cells = plan.cells
    pk_out = torch.empty(R * nb, dtype=torch.float64, device=dev)
    counts = torch.empty(R * cells, dtype=torch.int32, device=dev)
    ntot = torch.empty(R, dtype=torch.int64, device=dev)
    cov = torch.empty(nb * nb, dtype=torch.float64, device=dev)
    cnorm = torch.empty(nb * nb, dtype=torch.float64, device=dev)

    def step(i):
        b.pipeline_run(ctx, plan, w["seed"], w["request_id"], i * R * 2, R, nbar, nb, pk_out,
                       out_counts=counts, out_ntot=ntot, out_cov=cov, out_cnorm=cnorm, stream=stream)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    if b.ctx_check(ctx) != 0:
        raise RuntimeError("device flagged a sampler condition during warm-up")
    sched = None
    installed = b.schedule_get(ctx, n, h, prec)
    if tune or installed is not None:
        if installed is not None:
            b.schedule_set(ctx, n, h, prec, None)  # the default schedule is timed first
        nd = max(3, steps // 2)
        t0 = time.perf_counter()
        for i in range(nd):
            step(warmup + i)
        torch.cuda.synchronize()
        default_ms = 1e3 * (time.perf_counter() - t0) / nd
        t0 = time.perf_counter()
        if installed is not None:
            b.schedule_set(ctx, n, h, prec, installed)
            sched = dict(chosen={k: v for k, v in installed.items() if k not in ("ms", "default_ms")},
                         source="schedule file", default_ms_per_step=round(default_ms, 4))
        else:
            s = b.autotune(ctx, plan, R, nbar, nb, reps=2)
            sched = dict(chosen={k: v for k, v in s.items() if k not in ("ms", "default_ms")}, source="ce_autotune",
                         tune_s=round(time.perf_counter() - t0, 2), default_ms_per_step=round(default_ms, 4),
                         tuner_ms=dict(chosen=round(s["ms"], 4), default=round(s["default_ms"], 4)))
        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
    b.ctx_profile_read(ctx)
    b.ctx_set_profiling(ctx, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        step(warmup + i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.ctx_set_profiling(ctx, False)
    prof = b.ctx_profile_read(ctx)
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    gpu_ms = float(ev[0].elapsed_time(ev[-1]))

    pairs = (R + 1) // 2
    kernels = {}
    total_bytes = 0
    for kname, (ms, launches) in prof.items():
        per = kernel_bytes(kname, n, w["precision"], pairs, nb, R)
        avg = ms / launches
        total_bytes += per * launches / steps
        kernels[kname] = dict(avg_ms=round(avg, 4), launches=int(launches // steps),
                              alg_bytes=per, alg_GBs=round(per / (avg * 1e-3) / 1e9, 1),
                              share=round(ms / sum(v[0] for v in prof.values()), 3))
        o = kernel_ops(kname, n, pairs, nb, R, nbar)
        if o:
            kernels[kname]["alg_Gops"] = round(o / (avg * 1e-3) / 1e9, 1)
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    dk = kernels[dom]
    achieved = dk["alg_bytes"] / (dk["avg_ms"] * 1e-3) / 1e9
    cnt = counters_for(dom, name)
    ops = kernel_ops(dom, n, pairs, nb, R, nbar)
    roofline = dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if cnt is None else int(cnt["bytes_per_launch"]),
                    alg_bytes=dk["alg_bytes"], avg_ms=dk["avg_ms"],
                    valu_busy=None if cnt is None else cnt.get("valu_busy"),
                    valu_op_model=dict(achieved=round(ops / (dk["avg_ms"] * 1e-3) / 1e9, 1),
                                       peak=round(VALU_PEAK_GOPS, 1), unit="Gop/s",
                                       frac=round(ops / (dk["avg_ms"] * 1e-3) / 1e9 / VALU_PEAK_GOPS, 4)))
    pipe_GBs = total_bytes / (np.median(step_ms) * 1e-3) / 1e9
    return dict(value=round(R * steps / wall, 1), ms_per_step=round(1e3 * wall / steps, 4),
                latency_ms=dict(p50=round(float(np.percentile(step_ms, 50)), 4),
                                p99=round(float(np.percentile(step_ms, 99)), 4), gpu_total=round(gpu_ms, 3)),
                pipeline_hbm=dict(alg_bytes_per_step=int(total_bytes), alg_GBs=round(pipe_GBs, 1),
                                  frac_of_peak=round(pipe_GBs / HBM_PEAK_GBS, 4)),
                roofline=roofline, kernels=kernels, plan_ms=round(plan_ms, 2),
                **({} if sched is None else dict(schedule=sched)),
                _plan=plan, _bufs=(pk_out, counts, ntot, cov, cnorm))


def main_leg(args, b, torch, w, stream):
    """The headline step (ce_pipeline_run of the workload), its oracle accuracy, the captured-graph
    replay, the plain FP64 comparator and the counter calibration copies."""
    import numpy as np
    prec = b.F64 if w["precision"] == "f64" else b.F32
    n, h, nb, R, nbar = w["n"], w["h"], w["nbins"], w["realizations"], w["nbar"]
    dev = torch.device("cuda:0")
    ctx = b.ctx_create(0)

    if args.lines:
        for opt, v in zip((b.OPT_LINES_NOISE, b.OPT_LINES_INNER, b.OPT_LINES_LAST, b.OPT_LINES_BINS),
                          args.lines.split(",")):
            b.ctx_set_option(ctx, opt, int(v))
    if args.noise_order >= 0:
        b.ctx_set_option(ctx, b.OPT_NOISE_ORDER, args.noise_order)
    if schedule_file(args):
        b.schedule_load(ctx, schedule_file(args))
    leg = timed_workload(b, torch, ctx, w, args.workload, args.steps, args.warmup, stream, tune=not args.no_tune)
    if args.save_schedules:
        save_schedules(b, ctx, args.save_schedules)
    plan, bufs = leg.pop("_plan"), leg.pop("_bufs")
    pk_out, counts, ntot, cov, cnorm = bufs
    cells = plan.cells
    value = leg.pop("value")

    out = dict(metric=METRIC, value=value, unit="realizations/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=leg.pop("ms_per_step"), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=w["precision"], data="synthetic",
               config=dict(workload=workload_description(w, args.workload), survey=list(n),
                           embedding=[2 * x for x in n], realizations_per_step=R, nbar=nbar, shells=nb,
                           precision=w["precision"]),
               roofline=leg.pop("roofline"))
    out.update(leg)
    if not args.no_accuracy:
        out["accuracy"] = accuracy_leg(b, torch, ctx, plan, w)
        print("accuracy %s" % json.dumps(out["accuracy"]), file=sys.stderr, flush=True)

    if not args.no_graph:
        # the same step captured once as a HIP graph and replayed (each replay advances the
        # realizations): the host launch work of the passes is gone
        g = b.pipeline_graph_create(ctx, plan, w["seed"], w["request_id"], 0, R, nbar, nb, pk_out, out_counts=counts,
                                    out_ntot=ntot, out_cov=cov, out_cnorm=cnorm)
        try:
            for _ in range(args.warmup):
                b.pipeline_graph_launch(g, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                b.pipeline_graph_launch(g, stream)
            torch.cuda.synchronize()
            gwall = time.perf_counter() - t0
        finally:
            b.pipeline_graph_destroy(g)
        out["graph"] = dict(value=round(R * args.steps / gwall, 1), unit="realizations/s",
                            ms_per_step=round(1e3 * gwall / args.steps, 4),
                            form="ce_pipeline_graph_create once, one ce_pipeline_graph_launch per step")

    if not args.no_plain:
        # plain FP64 comparator: FP64 plan, unpruned inverse FFT, unfused, one realization per chain
        b.ctx_set_option(ctx, b.OPT_UNPRUNED, 1)
        p64 = b.plan_embedding(ctx, n, h, w["xi"], b.F64)
        f1 = torch.empty(cells, dtype=torch.float64, device=dev)
        c1 = torch.empty(cells, dtype=torch.int32, device=dev)
        t1 = torch.empty(1, dtype=torch.int64, device=dev)
        pk1 = torch.empty(args.plain_realizations * nb, dtype=torch.float64, device=dev)

        def plain(r):
            b.generate_fields(ctx, p64, w["seed"], w["request_id"], 2 * r, 1, f1, stream)
            b.lognormal_poisson(ctx, p64, f1, 1, nbar, None, w["seed"], w["request_id"], 2 * r, None, c1, t1, stream)
            b.estimate_pk(ctx, n, h, b.F64, b.MAP_COUNTS_DELTAG, c1, 1, t1, None, nb, pk1[r * nb:(r + 1) * nb],
                          stream=stream)

        plain(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(args.plain_realizations):
            plain(r)
        b.pk_covariance(ctx, pk1, args.plain_realizations, nb, cov, cnorm, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.ctx_set_option(ctx, b.OPT_UNPRUNED, 0)
        pv = args.plain_realizations / dt
        out["plain_fp64"] = dict(value=round(pv, 1), unit="realizations/s",
                                 realizations=args.plain_realizations,
                                 form="FP64, unpruned inverse FFT, unfused calls, one realization (Re) per chain")
        out["speedup_vs_plain_fp64"] = round(value / pv, 1)
        p64.release()

    if args.copy_calibration_mib:
        # known-size kernels for scaling the FETCH_SIZE / WRITE_SIZE counters: a fill (writes
        # nbytes), a reduction (reads nbytes) and a device copy (reads and writes nbytes)
        nbytes = args.copy_calibration_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
        src.fill_(1.0)
        torch.cuda.synchronize()
        total = src.sum()
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_bytes"] = dict(fill_write=nbytes, sum_read=nbytes, copy_each_way=nbytes,
                                        check=float(total.item()))

    plan.release()
    b.ctx_destroy(ctx)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (realizations would shard across "
              "GPUs with no exchange but the final shell sums); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1406_6072_amd import binding as b
    from synth import workloads

    w = workloads.WORKLOADS[args.workload]
    prec = b.F64 if w["precision"] == "f64" else b.F32
    n, h, nb, R, nbar = w["n"], w["h"], w["nbins"], w["realizations"], w["nbar"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = dict(metric=METRIC)
    if not args.skip_main:
        out = main_leg(args, b, torch, w, stream)

    if args.volume_steps and args.workload != "volume_3d":
        # the 3-D workload (256^3 survey in a 512^3 embedding, 8 realizations per step) timed the
        # same way: per-kernel events, algorithmic bytes and the roofline of its largest kernel
        vw = workloads.WORKLOADS["volume_3d"]
        vctx = b.ctx_create(0)
        if schedule_file(args):
            b.schedule_load(vctx, schedule_file(args))
        vleg = timed_workload(b, torch, vctx, vw, "volume_3d", args.volume_steps, 2, stream, tune=not args.no_tune)
        if args.save_schedules:
            save_schedules(b, vctx, args.save_schedules)
        vleg.pop("_plan").release()
        vleg.pop("_bufs")
        vleg["unit"] = "realizations/s"
        vleg["workload"] = workload_description(vw, "volume_3d")
        b.ctx_destroy(vctx)
        out["volume_3d"] = vleg
        print("volume_3d %s" % json.dumps(vleg), file=sys.stderr, flush=True)

    if not args.no_masked:
        # the same workload on a masked survey (star holes and a partial border, 7% of cells out)
        mask = torch.from_numpy(workloads.survey_mask(n, seed=3).ravel()).to(dev)
        ctx = b.ctx_create(0)
        plan = b.plan_embedding(ctx, n, h, w["xi"], prec)
        mc = torch.empty(R * plan.cells, dtype=torch.int32, device=dev)
        pk_out = torch.empty(R * nb, dtype=torch.float64, device=dev)
        ntot = torch.empty(R, dtype=torch.int64, device=dev)
        cov = torch.empty(nb * nb, dtype=torch.float64, device=dev)
        cnorm = torch.empty(nb * nb, dtype=torch.float64, device=dev)

        def mstep(i, counts=None):
            b.pipeline_run_masked(ctx, plan, mask, w["seed"], w["request_id"], i * R * 2, R, nbar, nb, pk_out,
                                  out_counts=counts, out_ntot=ntot, out_cov=cov, out_cnorm=cnorm, stream=stream)

        mstep(0)
        torch.cuda.synchronize()
        b.ctx_profile_read(ctx)
        b.ctx_set_profiling(ctx, True)
        t0 = time.perf_counter()
        msteps = max(3, args.steps // 4)
        for i in range(msteps):
            mstep(1 + i)
        torch.cuda.synchronize()
        mdt = (time.perf_counter() - t0) / msteps
        b.ctx_set_profiling(ctx, False)
        mprof = b.ctx_profile_read(ctx)
        out["masked"] = dict(value=round(R / mdt, 1), unit="realizations/s", ms_per_step=round(1e3 * mdt, 3),
                             kernels_ms={k: round(v[0] / msteps, 4) for k, v in mprof.items()},
                             steps=msteps, masked_fraction=round(float((mask == 0).float().mean()), 4),
                             form="fused pass with the mask's rate, transform of N / (f nbar) - 1, contrast completed in the "
                                  "binning pass with the mask's window transform")
        # the same steps with the mask prepared once (ce_mask_prepare): no per-call window transform
        prep = b.mask_prepare(ctx, plan, mask, stream)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(msteps):
                b.pipeline_run_prepared(ctx, plan, mask, prep, w["seed"], w["request_id"], (1 + i) * R * 2, R, nbar,
                                        nb, pk_out, out_ntot=ntot, out_cov=cov, out_cnorm=cnorm, stream=stream)
            torch.cuda.synchronize()
            pdt = (time.perf_counter() - t0) / msteps
        finally:
            b.mask_release(prep)
        out["masked"]["prepared"] = dict(value=round(R / pdt, 1), ms_per_step=round(1e3 * pdt, 3),
                                         form="ce_mask_prepare once, ce_pipeline_run_prepared per step")
        if not args.no_cic:
            mstep(1 + msteps, counts=mc)  # the counts of one step for the counts-in-cells leg
            out["cic"] = cic_leg(b, torch, ctx, plan, mask, mc, R, nb, nbar, n, h, stream, msteps)
        plan.release()
        b.ctx_destroy(ctx)

    if args.info_realizations:
        out["information"] = information_leg(b, torch, args.info_realizations)
        print("information %s" % json.dumps(out["information"]), file=sys.stderr, flush=True)

    if args.batch_requests:
        out["uneven_batch"] = uneven_batch_leg(b, torch, args.batch_requests, args.batch_reps, tune=not args.no_tune,
                                               schedules=schedule_file(args), save=args.save_schedules,
                                               lanes=args.batch_lanes)
        print("uneven batch %s" % json.dumps(out["uneven_batch"]), file=sys.stderr, flush=True)

    if args.serve_rates:
        from synth import workloads
        rates = [float(x) for x in args.serve_rates.split(",")]
        server = b.server_create(0, slots=args.serve_slots)
        try:
            # a long-running server: every plan of the traces cached, slot scratch grown by one
            # closed-loop pass; a second pass gives the saturation throughput
            warm_trace = workloads.serving_trace(rate=min(max(rates), 1000.0),
                                                 duration=args.serve_warmup + args.serve_seconds, seed=5)
            warm_s, _, _ = serving_warm(b, torch, server, warm_trace)
            sat_trace = workloads.serving_trace(rate=500.0, duration=args.serve_warmup + args.serve_seconds, seed=6)
            sat_s, sat_rps, sat_gbs = serving_warm(b, torch, server, sat_trace)
            legs = []
            for rate in rates:
                leg = serving_leg(b, torch, server, rate, args.serve_seconds, args.serve_warmup)
                legs.append(leg)
                print("serving leg %s" % json.dumps(leg), file=sys.stderr, flush=True)
        finally:
            b.server_destroy(server)
        # the saturation trace's work as one batched call: what the server's closed loop is compared with
        offline = offline_batch(b, torch, sat_trace) if args.serve_offline else None
        # sustainable: the backlog when the last request arrives stays within the slots and the
        # queue drains within 0.5 s of it
        ok = [g["offered_rate"] for g in legs
              if g["backlog_at_last_arrival"] is not None and g["backlog_at_last_arrival"] <= 2 * args.serve_slots
              and g["drain_s"] <= 0.5 and g["failed"] == 0]
        out["serving"] = dict(trace="open-loop Poisson arrivals, 50/50 2-D (sides 64..2048) / 3-D (32..256), "
                                    "sides every multiple of 16 drawn log-uniformly, 1..64 realizations log-uniform, "
                                    "16 two-point functions, nbar in {0.1,0.3,1,5}, 32 shells, FP32; seed 5",
                              window_s=args.serve_seconds, warmup_s=args.serve_warmup, slots=args.serve_slots,
                              warm_pass=dict(requests=len(warm_trace), seconds=round(warm_s, 2)),
                              closed_loop=dict(requests=len(sat_trace), seconds=round(sat_s, 3),
                                               requests_per_s=round(sat_rps, 1), alg_GBs=round(sat_gbs, 1),
                                               realizations_per_s=round(sum(r["realizations"] for r in sat_trace)
                                                                        / sat_s, 1)),
                              offline_batch=offline,
                              served_over_offline=round(sat_gbs / offline["alg_GBs"], 3) if offline else None,
                              legs=legs, max_sustainable_rate_tested=max(ok) if ok else None)
        out["serving"]["small_requests"] = small_request_leg(b, torch, args.serve_slots)
        print("small requests %s" % json.dumps(out["serving"]["small_requests"]), file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_oracle_sample(w, args.cpu_seconds)
        if "value" in out:
            out["speedup_vs_cpu_oracle"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
