#!/usr/bin/env python3
"""Benchmark of the stratified Cox CCD hot path on one MI355X.

Workload: N = 1,000,000 rows, P = 50 AR(1) covariates (corr 0.5^|i-j|),
beta_true iid N(0, 0.25), K = 50,000 equal strata, seed 1 -- one FP64 fit by
cyclic coordinate descent to convergence per step (tolerance 1e-12 on the
largest step of a sweep).  Inputs are resident in HBM before timing starts
(cox_init copies them once).

Prints one JSON line on stdout; progress goes to stderr.
  value          observation-evaluations per second = N x (coordinate
                 evaluations) / wall time, over all timed fits
  roofline       HBM roofline of the persistent CCD kernel: algorithmic bytes
                 per launch (8 B per row per coordinate evaluation for x_j,
                 plus 4 B per row for the row words read once) over the kernel
                 duration measured with HIP events on its stream
  cpu_baseline   the CPU oracle's CCD (plain C, one thread) on a bounded
                 sample of the same workload: its first 20 sweeps (with the
                 host's CPU model and usable thread count)
  mixed_precision  N = 1e6, P = 200 AR(1), K = 5e4: Newton fits with a BF16
                 information matrix and FP64 refinement against the plain FP64
                 Newton path, each checked against the stored oracle optimum
  serving        the 4,096-request stream (n log-uniform in [1e3, 1e5], p in
                 5..100) through the fit server: saturating fits/s with request
                 data in device and in host memory, p50/p99 latency under
                 Poisson arrivals, the plain FP64 path from the same two
                 sources, and the oracle's check of a sample of the fits
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "obs-evals/s and fits/s vs plain FP64 at 1e-10 rel err; p50/p99 fit latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ccd_kernel_ar1_n1e6_p50_K5e4.md")
KERNEL_SOURCES = ["ccd_kernel.hip", "segscan.hpp", "internal.h"]
CONTRACTION_PROFILE = os.path.join(ROOT, "profiles", "newton_counters_n1e6_p200.md")


def recorded_field(profile=TRAFFIC_PROFILE, sources=KERNEL_SOURCES, field="traffic_bytes_per_launch"):
    """A figure from a committed counter summary (HBM bytes per launch by default), or None
    when the kernel sources no longer hash to the value the counters were taken on."""
    import hashlib
    try:
        with open(profile) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    fields = {}
    for line in lines:
        key, sep, val = line.partition(": ")
        if sep and key and " " not in key:
            fields[key] = val.strip()
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2310_16238_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_sources_sha256") != h.hexdigest():
        return None
    try:
        return float(fields[field])
    except (KeyError, ValueError):
        return None


def recorded_traffic():
    return recorded_field()


def cpu_baseline(d, sweeps=20):
    """Oracle CCD (single-threaded C) on the first `sweeps` sweeps of the same data."""
    from oracle import cox_oracle as orc
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    Xc = orc.to_canonical(d.X, L)
    t0 = time.perf_counter()
    r = orc.fit_ccd(d.X, d.time, d.event, layout=L, Xc=Xc, max_sweeps=sweeps)
    dt = time.perf_counter() - t0
    evals = r.iters * d.p
    return {"value": d.n * evals / dt, "unit": "obs-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"first {r.iters} CCD sweeps ({evals} coordinate evaluations) of the same "
                      f"N={d.n} P={d.p} K=50000 data, plain C, one thread, {dt:.1f} s",
            **host_cpu()}


def cpu_baseline_newton(d, steps):
    """Oracle Newton step on all cores: one full FP64 evaluation with the information matrix
    (risk-set sums in plain C on one thread, X' diag(w Lambda) X and xbar'xbar by numpy's BLAS
    on every core) of the same data; fits/s assumes `steps` such steps per fit."""
    import numpy as np
    from oracle import cox_oracle as orc
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    Xc = orc.to_canonical(d.X, L)
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        pass
    t0 = time.perf_counter()
    fe = orc.full_eval(Xc, L, np.zeros(d.p), want_info=True)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(fe.info))
    return {"value": 1.0 / (steps * dt), "unit": "fits/s", "cores": threads or host_cpu()["nproc"],
            "kind": "oracle",
            "sample": f"one full FP64 evaluation with the information matrix of the same N={d.n} P={d.p} data "
                      f"({dt:.1f} s: risk-set sums in plain C on one thread, the P x P products by numpy's "
                      f"BLAS on all cores), times the {steps} Newton steps of the FP64 path",
            "obs_evals_per_s": d.n * d.p / dt, **host_cpu()}


def host_cpu():
    """The host's CPU model and the threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def _rel(a, b):
    import numpy as np
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(float(np.max(np.abs(b))), 1e-300))


def run_serve(args):
    print(json.dumps(serve_leg(args)), flush=True)


def serve_leg(args):
    """Serving stream: independent fits of uneven (n, p) through the fit server, against the
    plain FP64 GPU path (cox_init + cox_fit per request, one after another), both with the
    request data in host memory and with it resident in device memory."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    R = args.requests
    log(f"drawing {R} serving requests (n log-uniform in [1e3, 1e5], p in 5..100, seed 3)")
    with ThreadPoolExecutor(16) as ex:
        reqs = list(ex.map(synth.serving_request, range(R)))
    rows = sum(d.n for d in reqs)
    log(f"  {rows} rows, {sum(d.n * d.p for d in reqs) * 8 / 1e9:.1f} GB of FP64 X")

    # every request's data resident in HBM before the timed regions (X column-major)
    log("placing the requests' data in device memory")
    dev = []
    for d in reqs:
        dev.append((torch.from_numpy(np.ascontiguousarray(d.X.T)).cuda().t(),
                    torch.from_numpy(np.ascontiguousarray(d.time)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(d.event, dtype=np.uint8)).cuda(),
                    None if d.stratum is None else torch.from_numpy(np.ascontiguousarray(d.stratum, dtype=np.int32)).cuda()))
    torch.cuda.synchronize()

    # plain FP64 GPU path on a sample of the stream: one handle and one fit per request, from
    # host inputs and (like for like with the served device-resident run) from device inputs
    sample = list(range(min(args.plain_sample, R)))
    plain = {}
    plain_beta = {}
    for mode, name in [(coxmi.COX_CCD, "ccd"), (coxmi.COX_NEWTON_REFINE, "newton_f64")]:
        for src_kind in ("host", "device"):
            def model(i):
                if src_kind == "device":
                    return coxmi.CoxModel.from_device(*dev[i], mode=mode, tol=1e-12)
                d = reqs[i]
                return coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=mode, tol=1e-12)
            with model(0) as m:
                m.fit()   # warm the code paths
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in sample:
                with model(i) as m:
                    beta, info = m.fit()
                plain_beta[(name, src_kind, i)] = beta
            key = name if src_kind == "host" else f"{name}_device_inputs"
            plain[key] = len(sample) / (time.perf_counter() - t0)
            log(f"plain {key}: {plain[key]:.1f} fits/s over {len(sample)} requests")
    plain_best = max(v for k, v in plain.items() if not k.endswith("_device_inputs"))
    plain_best_dev = max(v for k, v in plain.items() if k.endswith("_device_inputs"))

    def serve(batch, arrivals=None, device=True):
        def submit(srv, i):
            if device:
                return srv.submit_device(*dev[i])
            d = reqs[i]
            return srv.submit(d.X, d.time, d.event, d.stratum)
        with coxmi.CoxServer(hbm_budget=args.hbm_gib << 30, prep_threads=args.prep_threads,
                             fused_rounds=args.fused_rounds) as srv:
            warm = [submit(srv, i) for i in batch[:4]]
            srv.drain()
            for t in warm:
                srv.poll(t)
            st0 = srv.stats()
            tickets = []
            t_start = time.perf_counter()
            for k, i in enumerate(batch):
                if arrivals is not None:
                    delay = arrivals[k] - (time.perf_counter() - t_start)
                    if delay > 0:
                        time.sleep(delay)
                tickets.append(submit(srv, i))
            srv.drain()
            res = [srv.poll(t) for t in tickets]
            st1 = srv.stats()
        sub = np.array([r[2]["submit_s"] for r in res])
        done = np.array([r[2]["done_s"] for r in res])
        lat = done - sub
        span = float(done.max() - sub.min())
        stats = {k: st1[k] - st0[k] for k in ("completed", "iterations", "gpu_busy_s", "launches")}
        if args.fused_rounds:
            stats["phase_s"] = [b - a for a, b in zip(st0["phase_s"], st1["phase_s"])]
        stats.update(resident_peak=st1["resident_peak"], arena_peak=st1["arena_peak"],
                     mean_resident=st1["mean_resident"])
        return res, {"fits_per_s": len(batch) / span, "makespan_s": span,
                     "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                                    "p99": 1e3 * float(np.percentile(lat, 99))},
                     "statuses": sorted(set(int(r[1]["status"]) for r in res)), "server": stats}

    log(f"served, saturating (all {R} requests at once, data in device memory)")
    res_sat, sat = serve(range(R))
    log(f"  {sat['fits_per_s']:.1f} fits/s, p50 {sat['latency_ms']['p50']:.1f} ms, p99 {sat['latency_ms']['p99']:.1f} ms")
    log(f"served, saturating (all {R} requests at once, data in host memory: X crosses PCIe)")
    res_host, sat_host = serve(range(R), device=False)
    log(f"  {sat_host['fits_per_s']:.1f} fits/s, p50 {sat_host['latency_ms']['p50']:.1f} ms, "
        f"p99 {sat_host['latency_ms']['p99']:.1f} ms")
    same = all(np.array_equal(a[0], b[0]) for a, b in zip(res_sat, res_host))
    log(f"  device-resident and host submissions bit-identical: {same}")
    lam = 1.5 * plain_best_dev
    R2 = int(min(R, max(64, args.poisson_seconds * lam)))
    log(f"served, Poisson arrivals at {lam:.1f}/s (1.5 x plain, device inputs), {R2} requests, data in device memory")
    res_poi, poi = serve(range(R2), synth.arrival_times(R2, lam))
    log(f"  {poi['fits_per_s']:.1f} fits/s, p50 {poi['latency_ms']['p50']:.1f} ms, p99 {poi['latency_ms']['p99']:.1f} ms")

    # accuracy on a spread sample: served and plain against the oracle
    from oracle import cox_oracle as orc
    idx = sorted(set(list(range(min(len(sample), 8))) + list(np.linspace(0, R - 1, args.check).astype(int))))
    worst_served, worst_plain = 0.0, 0.0
    verified = 0
    for i in idx:
        d = reqs[i]
        ref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
        e = _rel(res_sat[i][0], ref.beta)
        worst_served = max(worst_served, e)
        verified += int(e <= 1e-10)
        for key, b in plain_beta.items():
            if key[2] == i:
                worst_plain = max(worst_plain, _rel(b, ref.beta))
    log(f"rel err vs oracle on {len(idx)} requests: served {worst_served:.2e} ({verified} within 1e-10), "
        f"plain {worst_plain:.2e}")
    # a wider sample checked more cheaply: the oracle's score (Eq. strat_g) at each served estimate
    from concurrent.futures import ThreadPoolExecutor
    sidx = sorted(set(np.linspace(0, R - 1, min(R, args.score_check)).astype(int)))

    def scaled_score(i):
        d = reqs[i]
        lay = orc.canonical_layout(d.time, d.event, d.stratum)
        g = orc.full_eval(orc.to_canonical(d.X, lay), lay, res_sat[i][0], want_info=False).grad
        E = max(1.0, float(d.event.sum()))
        return float(np.max(np.abs(g) / (E * np.maximum(1.0, np.max(np.abs(d.X), axis=0)))))

    with ThreadPoolExecutor(8) as ex:
        scores = list(ex.map(scaled_score, sidx))
    score_ok = int(sum(v <= 1e-9 for v in scores))
    log(f"oracle score at the served estimate on {len(sidx)} requests: max |g_j| / (E max|x_j|) = {max(scores):.2e} "
        f"({score_ok} within 1e-9)")

    evals = sum(r[1]["coord_evals"] for r in res_sat)
    alg_bytes = sum(r[1]["coord_evals"] * (16.0 * d.n * d.p + 64.0 * d.n) for r, d in zip(res_sat, reqs))
    busy = sat["server"]["gpu_busy_s"]
    achieved = alg_bytes / busy / 1e9
    return {
        "metric": METRIC,
        "value": sat["fits_per_s"],
        "unit": "fits/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * sat["makespan_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 score, f32 contraction", "data": "synthetic",
        "config": {"workload": f"serving stream: {R} independent unpenalised fits, n log-uniform in [1e3, 1e5], "
                               "p uniform in 5..100 with a ones column, K = n/100 strata, seed 3; "
                               "request data resident in device memory",
                   "requests": R, "rows": rows, "fused_rounds": args.fused_rounds},
        "plain_fp64_fits_per_s": plain,
        "speedup_vs_plain": {"device_inputs": sat["fits_per_s"] / plain_best_dev,
                             "host_inputs": sat_host["fits_per_s"] / plain_best},
        "saturating": sat, "poisson": dict(poi, rate_per_s=lam, requests=R2),
        "saturating_host_inputs": sat_host, "host_and_device_inputs_identical": same,
        "rel_err_vs_oracle": {"served_max": worst_served, "plain_max": worst_plain, "requests_checked": len(idx),
                              "requests_within_1e-10": verified,
                              "score_checked": len(sidx), "score_within_1e-9": score_ok,
                              "score_max_scaled": max(scores),
                              "note": "served fits/s counts every fit of the stream; the oracle's Newton fit "
                                      "checks the first listed sample, the oracle's score at the served estimate "
                                      "the second"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "served rounds (all batched kernels), algorithmic bytes 16 n p + 64 n per evaluation",
                     "evaluations": evals},
    }


MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "f64": 78.6}


def contraction_roofline(flops, nbytes, secs, dtype, kernel, traffic=None, mfma_busy=None):
    """Roofline of one information contraction against the floor that binds it: the matrix
    cores (flops / peak of the dtype) or HBM (algorithmic bytes / 8 TB/s), whichever takes
    longer; the other view is reported beside it."""
    mfma = {"achieved": flops / secs / 1e12, "peak": MFMA_PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
            "frac": flops / secs / 1e12 / MFMA_PEAK_TFLOPS[dtype], "algorithmic_flops_per_launch": flops}
    hbm = {"achieved": nbytes / secs / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": nbytes / secs / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": nbytes}
    hbm_bound = nbytes / (HBM_PEAK_GBS * 1e9) >= flops / (MFMA_PEAK_TFLOPS[dtype] * 1e12)
    main, other = (hbm, mfma) if hbm_bound else (mfma, hbm)
    out = {"bound": "hbm" if hbm_bound else "mfma", **main, "traffic": traffic, "kernel": kernel,
           "arithmetic_intensity_flop_per_byte": flops / nbytes,
           "ridge_flop_per_byte": MFMA_PEAK_TFLOPS[dtype] * 1e12 / (HBM_PEAK_GBS * 1e9),
           ("mfma_view" if hbm_bound else "hbm_view"): other}
    if mfma_busy is not None:
        out["mfma_busy"] = mfma_busy
    return out


def run_paper(args):
    """The paper's synthetic setting (Sec. 3.1): binary X with 5% ones, beta ~ N(0,1) x
    Bernoulli(0.2), l1 strength sqrt(2), N=1e6, P=1000, K=5e4 strata -- a CCD fit to convergence.
    Checked against the oracle: its per-column derivatives (Eqs. strat_g, strat_h, plain C) at
    the returned beta must satisfy the l1 optimality conditions on sampled columns."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p, K = args.paper_n, args.paper_p, 50_000
    log(f"drawing the Sec. 3.1 workload N={n} P={p} K={K}, binary X (5% ones), gamma=sqrt(2) (seed 5)")
    d = synth.config_paper(n=n, p=p, K=K)
    t0 = time.perf_counter()
    m = coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=d.gamma, tol=1e-12)
    log(f"cox_init {time.perf_counter() - t0:.1f} s")
    beta, info = m.fit()   # warm
    torch.cuda.synchronize()
    lat, kms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        beta, info = m.fit()
        lat.append(time.perf_counter() - ts)
        kms.append(m.kernel_ms())
    m.close()
    T = float(np.median(lat))
    evals = int(info["coord_evals"])
    log(f"fit: {1e3 * T:.1f} ms, {info['iters']} sweeps, {evals} coordinate evaluations, status {info['status']}, "
        f"{int(np.count_nonzero(beta))} nonzero coefficients")
    newton = {}
    if args.paper_newton:
        # the same penalised fit by proximal Newton with a reduced-precision information matrix
        precs = [(coxmi.COX_BF16, "bf16"), (coxmi.COX_FP8_E4M3, "fp8")]
        for prec, name in precs:
            with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=d.gamma, tol=1e-12,
                                mode=coxmi.COX_NEWTON_REFINE, x_precision=prec, max_iter=200) as mn:
                bn, infn = mn.fit()   # warm
                torch.cuda.synchronize()
                ts = time.perf_counter()
                bn, infn = mn.fit()
                tn = time.perf_counter() - ts
                prof = mn.profile()
            diff = float(np.max(np.abs(bn - beta)) / np.max(np.abs(beta)))
            same_zeros = bool(np.array_equal(bn == 0.0, beta == 0.0))
            newton[name] = {"fit_s": tn, "steps": int(infn["iters"]), "status": int(infn["status"]),
                            "rel_diff_vs_ccd": diff, "zero_pattern_equal": same_zeros, "device_ms": prof}
            log(f"proximal Newton ({name} information): {1e3 * tn:.0f} ms, {infn['iters']} steps, "
                f"rel diff vs CCD {diff:.1e}, zero pattern equal {same_zeros}, profile {prof}")
    # oracle: optimality conditions at the returned beta on sampled columns
    from oracle import cox_oracle as orc
    lay = orc.canonical_layout(d.time, d.event, d.stratum)
    eta = np.ascontiguousarray((d.X @ beta)[lay.perm])
    E = float(d.event.sum())
    nz = np.flatnonzero(beta)
    zero = np.flatnonzero(beta == 0.0)
    cols = sorted(set(list(nz[:4]) + list(zero[:4])))
    worst = 0.0
    for j in cols:
        xj = orc.to_canonical(d.X[:, [j]], lay)
        g = orc.coord_terms(xj, lay, 0, eta)["grad"]
        r = abs(g + d.gamma * np.sign(beta[j])) if beta[j] != 0.0 else max(abs(g) - d.gamma, 0.0)
        worst = max(worst, r / max(1.0, E))
    log(f"oracle l1 optimality residual on columns {cols}: max / E = {worst:.2e}")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle CCD, first sweep")
        Xc = orc.to_canonical(d.X, lay)
        t1 = time.perf_counter()
        r = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=d.gamma, layout=lay, Xc=Xc, max_sweeps=1)
        dt = time.perf_counter() - t1
        cpu = {"value": n * r.iters * p / dt, "unit": "obs-evals/s", "cores": 1, "kind": "oracle",
               "sample": f"first CCD sweep ({p} coordinate evaluations) of the same data, plain C, one thread, "
                         f"{dt:.1f} s"}
    kernel_s = float(np.median(kms)) / 1e3
    bytes_per_launch = 8.0 * n * evals + 4.0 * n
    achieved = bytes_per_launch / kernel_s / 1e9
    out = {
        "metric": METRIC, "value": n * evals / T, "unit": "obs-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * T,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Sec. 3.1 setting: CCD fit to convergence, N={n}, P={p}, binary X with 5% ones, "
                               f"beta ~ N(0,1) x Bernoulli(0.2), gamma=sqrt(2), K={K} strata, FP64, seed 5"},
        "fit_s": T, "sweeps": int(info["iters"]), "us_per_coordinate": 1e6 * kernel_s / max(evals, 1),
        "paper_context": "the paper's GV100 run of this shape (N=1e6, K=5e4, P 1000 or 2000) took 23 s per fit",
        "oracle_l1_residual_over_E": worst, "proximal_newton": newton or None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "ccd_kernel (persistent, one launch per fit)",
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_intervals(args):
    """Sec. 3.3 shape: a treatment coefficient that changes at 10 days (Sec. 2.3), the model
    turned into a Cox model stratified on the two intervals (Sec. 2.2) by cox_split_intervals,
    then an l1 CCD fit to convergence with the two treatment columns unpenalised.  Checked
    against the oracle: the augmented rows from its own split, and the l1 optimality
    conditions at the returned beta on sampled columns (per-column score, plain C)."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p, cut = args.intervals_n, args.intervals_p, 10.0
    log(f"drawing the step-effect workload N={n} P={p}, treatment effect changing at {cut:g} days (seed 6)")
    d = synth.config_step_effect(n=n, p=p, cut=cut)
    tv = np.zeros(p, np.uint8)
    tv[0] = 1
    t0 = time.perf_counter()
    a = coxmi.split_intervals(d.X, d.time, d.event, None, [cut], tv_coef=tv)
    split_s = time.perf_counter() - t0
    na, pa = a["X"].shape
    log(f"cox_split_intervals {split_s:.2f} s: {na} rows x {pa} columns, {int(a['event'].sum())} events")
    pen = np.ones(pa, np.uint8)
    pen[a["col_source"] == 0] = 0
    t0 = time.perf_counter()
    m = coxmi.CoxModel(a["X"], a["time"], a["event"], a["stratum"], gamma=d.gamma, penalize=pen, tol=1e-12)
    init_s = time.perf_counter() - t0
    log(f"cox_init {init_s:.1f} s")
    beta, info = m.fit()   # warm
    torch.cuda.synchronize()
    lat, kms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        beta, info = m.fit()
        lat.append(time.perf_counter() - ts)
        kms.append(m.kernel_ms())
    m.close()
    # the same model built on the device from a handle on the original data (no host copy of X^(aug))
    pen0 = np.ones(p, np.uint8)
    pen0[0] = 0
    t0 = time.perf_counter()
    parent = coxmi.CoxModel(d.X, d.time, d.event, None, gamma=d.gamma, penalize=pen0, tol=1e-12)
    parent_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    child = parent.intervals(d.time, d.event, None, [cut], tv)
    map_s = time.perf_counter() - t0
    beta_map, _ = child.fit()
    child.close()
    parent.close()
    map_diff = float(np.max(np.abs(beta_map - beta)) / np.max(np.abs(beta)))
    log(f"device mapping: parent cox_init {parent_s:.1f} s + cox_init_intervals {map_s:.2f} s "
        f"(host split {split_s:.2f} s + cox_init {init_s:.1f} s); estimates agree to {map_diff:.1e}")
    T = float(np.median(lat))
    evals = int(info["coord_evals"])
    log(f"fit: {1e3 * T:.1f} ms, {info['iters']} sweeps, {evals} coordinate evaluations, status {info['status']}, "
        f"{int(np.count_nonzero(beta))} nonzero; treatment log HR before / after the cut "
        f"{beta[0]:.4f} / {beta[1]:.4f} (simulated {math.log(2.0):.4f} / {math.log(1.1):.4f})")
    # oracle: its own split of the columns it needs, then optimality at the returned beta
    from oracle import cox_oracle as orc
    assert [tuple(c) for c in zip(a["col_source"], a["col_interval"])] == orc.augmented_columns(tv, 2)
    nz_src = sorted(set(int(j) for j in a["col_source"][beta != 0.0]) | {0})
    zero_src = [int(j) for j in a["col_source"][beta == 0.0][:4]]
    src = sorted(set(nz_src) | set(zero_src))
    r = orc.split_intervals(d.X[:, src], d.time, d.event, None, [cut], tv_coef=tv[src])
    same_rows = all(np.array_equal(a[k], r[k]) for k in ("time", "event", "stratum", "row_subject"))
    # augmented column of (source, interval) in the library's numbering
    where = {(int(j), int(k)): c for c, (j, k) in enumerate(zip(a["col_source"], a["col_interval"]))}
    sub_cols = [where[(src[j], int(k))] for j, k in zip(r["col_source"], r["col_interval"])]
    b_sub = beta[sub_cols]
    lay = orc.canonical_layout(r["time"], r["event"], r["stratum"])
    eta = np.ascontiguousarray((r["X"] @ b_sub)[lay.perm])
    E = float(r["event"].sum())
    check = sorted(set(list(np.flatnonzero(b_sub != 0.0)[:6]) + list(np.flatnonzero(b_sub == 0.0)[:4])) | {0, 1})
    worst = 0.0
    for c in check:
        xj = orc.to_canonical(r["X"][:, [c]], lay)
        g = orc.coord_terms(xj, lay, 0, eta)["grad"]
        bj, penalised = b_sub[c], pen[sub_cols[c]] == 1
        if not penalised:
            res = abs(g)
        elif bj != 0.0:
            res = abs(g + d.gamma * np.sign(bj))
        else:
            res = max(abs(g) - d.gamma, 0.0)
        worst = max(worst, res / max(1.0, E))
    log(f"oracle: augmented rows identical {same_rows}; l1 optimality residual on {len(check)} columns: "
        f"max / E = {worst:.2e}")
    kernel_s = float(np.median(kms)) / 1e3
    bytes_per_launch = 8.0 * na * evals + 4.0 * na
    achieved = bytes_per_launch / kernel_s / 1e9
    out = {
        "metric": METRIC, "value": na * evals / T, "unit": "obs-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * T,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Sec. 3.3 shape: N={n} subjects, P={p} (a binary treatment whose coefficient "
                               f"steps at {cut:g} days + {p - 1} binary covariates with 5% ones), split into 2 "
                               f"interval strata ({na} rows x {pa} columns), l1 gamma=sqrt(2) on all but the "
                               f"treatment columns, CCD fit to convergence, FP64, seed 6"},
        "fit_s": T, "split_s": split_s, "init_s": init_s, "sweeps": int(info["iters"]),
        "device_mapping": {"parent_init_s": parent_s, "cox_init_intervals_s": map_s, "rel_diff_vs_split": map_diff},
        "treatment_log_hr": [float(beta[0]), float(beta[1])],
        "us_per_coordinate": 1e6 * kernel_s / max(evals, 1),
        "oracle_rows_identical": bool(same_rows), "oracle_l1_residual_over_E": worst,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "ccd_kernel (persistent, one launch per fit)",
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_cv(args):
    """Sec. 3.2 analysis shape: 10-fold cross-validation of the l1 weight along a path, a refit
    at the chosen weight and bootstrap refits for percentile intervals -- all on handles
    resampled on the device from one upload of X.  Checked against the oracle: the
    cross-validated log likelihood at the chosen weight recomputed from the returned fold
    estimates (scan form, Eq. strat_l), and the l1 optimality conditions of one fold's fit on
    sampled columns."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p, K, F, B = args.cv_n, args.cv_p, 10, args.cv_folds, args.bootstrap
    log(f"drawing the Sec. 3.2-shaped workload N={n} P={p} K={K} strata, binary X (3% ones) (seed 7)")
    d = synth.config_legend(n=n, p=p, K=K)
    pen = np.ones(p, np.uint8)
    pen[0] = 0
    t0 = time.perf_counter()
    if args.cv_newton:   # proximal Newton fits with a BF16 information matrix
        m = coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=0.0, penalize=pen, tol=1e-12,
                           mode=coxmi.COX_NEWTON_REFINE, x_precision=coxmi.COX_BF16, max_iter=300)
    else:
        m = coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=0.0, penalize=pen, tol=1e-12)
    log(f"cox_init {time.perf_counter() - t0:.1f} s")
    if args.cv_newton:
        _, g0, _, _ = m.evaluate_full(np.zeros(p), want_info=False)
    else:
        _, g0, _ = m.evaluate(np.zeros(p))
    gmax = float(np.max(np.abs(g0[pen == 1])))
    gammas = gmax * np.array([0.5, 0.2, 0.1, 0.05, 0.02, 0.01, 0.003, 0.001])
    rng = np.random.default_rng(8)
    fold = rng.integers(0, F, n).astype(np.int32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cvl, betas, status = m.cross_validate(fold, gammas, pen, nfolds=F)
    cv_s = time.perf_counter() - t0
    gi = int(np.argmax(cvl))
    log(f"cross-validation: {F} folds x {len(gammas)} weights in {cv_s:.2f} s ({F * len(gammas) / cv_s:.1f} fits/s); "
        f"cvl {np.round(cvl, 2)}; chosen gamma {gammas[gi]:.2f} (gamma_max {gmax:.1f})")
    served = None
    if args.cv_served:   # the same path with every fold of one weight batched through a fit server
        with coxmi.CoxServer(prep_threads=args.prep_threads) as srv:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cvl_s, betas_s, status_s = m.cross_validate_served(srv, d.X, d.time, d.event, d.stratum, fold, gammas,
                                                               pen, nfolds=F)
            cvs_s = time.perf_counter() - t0
        num = np.max(np.abs(betas_s - betas), axis=2)
        den = np.maximum(np.max(np.abs(betas), axis=2), 1e-300)
        served = {"cv_s": cvs_s, "fits_per_s": F * len(gammas) / cvs_s, "speedup_vs_handle": cv_s / cvs_s,
                  "max_fold_rel_diff_vs_handle": float(np.max(num / den)),
                  "cvl_max_abs_diff_vs_handle": float(np.max(np.abs(cvl_s - cvl))),
                  "same_zero_patterns": bool(np.array_equal(betas_s == 0.0, betas == 0.0)),
                  "statuses_ok": bool(np.all(status_s == 0))}
        log(f"cross-validation through the fit server: {cvs_s:.2f} s ({served['fits_per_s']:.1f} fits/s, "
            f"{served['speedup_vs_handle']:.1f}x); fold estimates vs the handle path {served['max_fold_rel_diff_vs_handle']:.1e}, "
            f"same zero patterns {served['same_zero_patterns']}, cvl diff {served['cvl_max_abs_diff_vs_handle']:.1e}")
    t0 = time.perf_counter()
    m.set_penalty(gammas[gi], pen)
    beta_star, info = m.fit(beta0=betas[0, gi])
    fit_s = time.perf_counter() - t0
    counts = np.stack([rng.multinomial(n, np.full(n, 1.0 / n)) for _ in range(B)]).astype(np.uint32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bb, bstat = m.bootstrap(counts, beta0=beta_star)
    boot_s = time.perf_counter() - t0
    m.close()
    hr = np.exp(bb[:, 0])
    lo, hi = np.quantile(hr, 0.025), np.quantile(hr, 0.975)
    log(f"refit at the chosen weight {fit_s:.2f} s ({int(np.count_nonzero(beta_star))} nonzero); {B} bootstrap refits "
        f"in {boot_s:.2f} s; treatment HR {math.exp(beta_star[0]):.4f}, 95% BPI [{lo:.4f}, {hi:.4f}]")
    # oracle checks
    from oracle import cox_oracle as orc
    lay_all = orc.canonical_layout(d.time, d.event, d.stratum)

    def nll(eta, lay):
        return orc.full_eval(np.ascontiguousarray(eta[lay.perm])[:, None], lay, [1.0], want_info=False).objective

    ref, scale = 0.0, 0.0
    for k in range(F):
        b = betas[k, gi]
        nz = np.flatnonzero(b)
        eta = d.X[:, nz] @ b[nz]
        tr = fold != k
        lay_tr = orc.canonical_layout(d.time[tr], d.event[tr], d.stratum[tr])
        a, t_ = nll(eta, lay_all), nll(eta[tr], lay_tr)
        ref += t_ - a
        scale += abs(a) + abs(t_)
    cv_err = abs(cvl[gi] - ref) / scale
    tr = fold != 0
    b = betas[0, gi]
    nz = np.flatnonzero(b)
    lay_tr = orc.canonical_layout(d.time[tr], d.event[tr], d.stratum[tr])
    eta = np.ascontiguousarray((d.X[:, nz] @ b[nz])[tr][lay_tr.perm])
    E = float(d.event[tr].sum())
    cols = sorted(set([0] + list(nz[:4]) + list(np.flatnonzero(b == 0.0)[:4])))
    worst = 0.0
    for j in cols:
        xj = orc.to_canonical(d.X[tr, j][:, None], lay_tr)
        g = orc.coord_terms(xj, lay_tr, 0, eta)["grad"]
        gam = gammas[gi] * pen[j]
        r = abs(g) if gam == 0.0 else (abs(g + gam * np.sign(b[j])) if b[j] != 0.0 else max(abs(g) - gam, 0.0))
        worst = max(worst, r / max(1.0, E))
    log(f"oracle: cvl at the chosen weight from the fold estimates, |gpu - oracle| / sum|l| = {cv_err:.2e}; "
        f"fold-0 l1 optimality residual on columns {cols}: max / E = {worst:.2e}")
    fits = F * len(gammas) + 1 + B
    total = cv_s + fit_s + boot_s
    out = {
        "metric": METRIC, "value": fits / total, "unit": "fits/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * total,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Sec. 3.2 analysis shape: N={n} rows, P={p} binary covariates (3% ones), K={K} strata; "
                               f"{F}-fold CV over {len(gammas)} l1 weights (column 0 unpenalised), refit at the chosen "
                               f"weight, {B} bootstrap refits; "
                               + ("proximal Newton with BF16 information" if args.cv_newton else "CCD, FP64")
                               + ", to 1e-12, seed 7"},
        "cv_s": cv_s, "refit_s": fit_s, "bootstrap_s": boot_s, "fits": fits,
        "gammas": [float(g) for g in gammas], "cvl": [float(c) for c in cvl], "chosen": gi,
        "treatment_hr": math.exp(beta_star[0]), "treatment_bpi95": [float(lo), float(hi)],
        "statuses_ok": bool(np.all(status == 0) and np.all(bstat == 0)),
        "oracle_cvl_rel_err": cv_err, "oracle_fold0_l1_residual_over_E": worst, "served": served,
        "paper_context": "the paper's LEGEND-HTN analysis (N=946,911, P=9,977, CV and bootstrap) took 1.41 h on its GPU",
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_sparse(args):
    """Sec. 3.2 at its full width on indicator X: N=946,911 rows, P=9,977 indicator covariates with
    3% ones, K=10 strata, one l1 CCD fit (column 0 unpenalised) at gamma = 0.02 gamma_max, X stored
    one bit per row (1.2 GB where FP64 would take 75 GB).  Checked against the oracle: the l1
    optimality conditions at the returned beta on sampled columns (per-column score, plain C)."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p = args.sparse_n, args.sparse_p
    log(f"drawing the full-width Sec. 3.2 workload: N={n} P={p} indicators (3% ones), K=10 strata (seed 9)")
    d = synth.config_legend_sparse(n=n, p=p)
    nnz = int(d.row_idx.size)
    pen = np.ones(p, np.uint8)
    pen[0] = 0
    vals = None
    if args.sparse_values:   # general sparse X: the same pattern with N(0, 1/4) values (seeded)
        vals = np.random.default_rng(19).normal(0.0, 0.5, nnz)
    t0 = time.perf_counter()
    if vals is None:
        m = coxmi.CoxModel.indicator(n, d.col_ptr, d.row_idx, d.time, d.event, d.stratum, gamma=0.0,
                                     penalize=pen, tol=1e-12)
    else:
        m = coxmi.CoxModel.sparse(n, d.col_ptr, d.row_idx, vals, d.time, d.event, d.stratum, gamma=0.0,
                                  penalize=pen, tol=1e-12)
    init_s = time.perf_counter() - t0
    _, g0, _ = m.evaluate(np.zeros(p))
    gmax = float(np.max(np.abs(g0[pen == 1])))
    gamma = 0.02 * gmax
    m.set_penalty(gamma, pen)
    log(f"cox_init ({'indicator' if vals is None else 'sparse'} X) {init_s:.1f} s ({nnz} nonzeros); gamma = 0.02 gamma_max = {gamma:.2f}")
    beta, info = m.fit()   # warm
    torch.cuda.synchronize()
    lat, kms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        beta, info = m.fit()
        lat.append(time.perf_counter() - ts)
        kms.append(m.kernel_ms())
    m.close()
    T = float(np.median(lat))
    evals = int(info["coord_evals"])
    nzb = np.flatnonzero(beta)
    log(f"fit: {T:.2f} s, {info['iters']} sweeps, {evals} coordinate evaluations, status {info['status']}, "
        f"{nzb.size} nonzero; treatment HR {math.exp(beta[0]):.4f} (simulated 0.8)")
    from oracle import cox_oracle as orc
    lay = orc.canonical_layout(d.time, d.event, d.stratum)
    eta = np.zeros(n)

    def colvals(j):
        seg = slice(d.col_ptr[j], d.col_ptr[j + 1])
        return 1.0 if vals is None else vals[seg]

    for j in nzb:
        eta[d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]]] += beta[j] * colvals(j)
    eta = np.ascontiguousarray(eta[lay.perm])
    E = float(d.event.sum())
    cols = sorted(set([0] + list(nzb[:4]) + list(np.flatnonzero(beta == 0.0)[:4]) + [p - 1]))
    worst = 0.0
    for j in cols:
        xj = np.zeros((n, 1))
        xj[d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]], 0] = colvals(j)
        g = orc.coord_terms(orc.to_canonical(xj, lay), lay, 0, eta)["grad"]
        gj = gamma * pen[j]
        r = abs(g) if gj == 0.0 else (abs(g + gj * np.sign(beta[j])) if beta[j] != 0.0 else max(abs(g) - gj, 0.0))
        worst = max(worst, r / E)
    log(f"oracle l1 optimality residual on columns {cols}: max / E = {worst:.2e}")
    kernel_s = float(np.median(kms)) / 1e3
    # per coordinate: the column's bits, and with values its nonzeros (average nnz / p) and wave offsets
    per_coord = n / 8.0 + (0.0 if vals is None else 8.0 * nnz / p + 4.0 * n / 512.0)
    bytes_per_launch = per_coord * evals + 4.0 * n
    achieved = bytes_per_launch / kernel_s / 1e9
    out = {
        "metric": METRIC, "value": n * evals / T, "unit": "obs-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * T,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (indicator X, 1 bit per row)" if vals is None else "f64 (sparse X: bits + FP64 values)",
        "data": "synthetic",
        "config": {"workload": f"Sec. 3.2 at full width: N={n} rows, P={p} "
                               + ("indicator covariates" if vals is None else "sparse covariates with N(0, 1/4) values")
                               + f" (3% nonzero, {nnz} nonzeros), K=10 strata, l1 CCD fit to 1e-12 at gamma = 0.02 "
                               f"gamma_max, column 0 unpenalised, seed 9"},
        "fit_s": T, "init_s": init_s, "sweeps": int(info["iters"]), "nonzero": int(nzb.size),
        "us_per_coordinate": 1e6 * kernel_s / max(evals, 1), "oracle_l1_residual_over_E": worst,
        "paper_context": "the paper's LEGEND-HTN data have this shape (946,911 x 9,977, 97% sparse)",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "ccd_kernel (persistent, " + ("indicator" if vals is None else "sparse") + " X)",
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_legend(args):
    """The Sec. 3.2 analysis at its full width on indicator X: 10-fold cross-validation of the l1
    weight over a path, a refit at the chosen weight and bootstrap refits, on N=946,911 rows and
    P=9,977 indicators (3% ones), K=10 strata, all folds and replicates resampled on the device
    from one upload of the 1.2 GB bit matrix.  Checked against the oracle: the cross-validated
    log likelihood at the chosen weight recomputed from the returned fold estimates (scan form)."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p, F, B = args.sparse_n, args.sparse_p, args.cv_folds, args.bootstrap
    log(f"drawing the full-width Sec. 3.2 workload: N={n} P={p} indicators (3% ones), K=10 strata (seed 9)")
    d = synth.config_legend_sparse(n=n, p=p)
    pen = np.ones(p, np.uint8)
    pen[0] = 0
    m = coxmi.CoxModel.indicator(n, d.col_ptr, d.row_idx, d.time, d.event, d.stratum, gamma=0.0, penalize=pen,
                                 tol=1e-12)
    _, g0, _ = m.evaluate(np.zeros(p))
    gmax = float(np.max(np.abs(g0[pen == 1])))
    gammas = gmax * np.array([0.1, 0.05, 0.02, 0.01])
    rng = np.random.default_rng(10)
    fold = rng.integers(0, F, n).astype(np.int32)
    # the folds one by one through the public calls (cox_cross_validate runs the same steps in one
    # call), so that every fold reports as it ends
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cvl = np.zeros(len(gammas))
    betas = np.zeros((F, len(gammas), p))
    status = []
    for k in range(F):
        tk = time.perf_counter()
        with m.resample((fold != k).astype(np.uint32)) as c:
            prev = np.zeros(p)
            for g, gam in enumerate(gammas):
                c.set_penalty(gam, pen)
                b, inf = c.fit(beta0=prev)
                status.append(inf["status"])
                obj_train, _, _ = c.evaluate(b)
                obj_all, _, _ = m.evaluate(b)           # m carries no penalty
                cvl[g] += (obj_train - gam * float(np.sum(pen * np.abs(b)))) - obj_all
                betas[k, g] = b
                prev = b
        log(f"fold {k}: {len(gammas)} fits in {time.perf_counter() - tk:.1f} s")
    status = np.array(status)
    cv_s = time.perf_counter() - t0
    gi = int(np.argmax(cvl))
    log(f"cross-validation: {F} folds x {len(gammas)} weights in {cv_s:.1f} s; cvl {np.round(cvl, 1)}; "
        f"chosen {gammas[gi]:.2f}")
    t0 = time.perf_counter()
    m.set_penalty(gammas[gi], pen)
    beta_star, info = m.fit(beta0=betas[0, gi])
    fit_s = time.perf_counter() - t0
    counts = np.stack([rng.multinomial(n, np.full(n, 1.0 / n)) for _ in range(B)]).astype(np.uint32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    parts = []
    for i in range(0, B, 2):
        parts.append(m.bootstrap(counts[i:i + 2], beta0=beta_star))
        log(f"bootstrap refits {i + 1}-{min(i + 2, B)} done ({time.perf_counter() - t0:.1f} s)")
    bb = np.concatenate([q[0] for q in parts])
    bstat = np.concatenate([q[1] for q in parts])
    boot_s = time.perf_counter() - t0
    m.close()
    hr = np.exp(bb[:, 0])
    lo, hi = np.quantile(hr, 0.025), np.quantile(hr, 0.975)
    log(f"refit {fit_s:.1f} s ({int(np.count_nonzero(beta_star))} nonzero); {B} bootstrap refits in {boot_s:.1f} s; "
        f"treatment HR {math.exp(beta_star[0]):.4f} (simulated 0.8), 95% BPI [{lo:.4f}, {hi:.4f}]")
    from oracle import cox_oracle as orc
    lay_all = orc.canonical_layout(d.time, d.event, d.stratum)

    def nll(eta, lay):
        return orc.full_eval(np.ascontiguousarray(eta[lay.perm])[:, None], lay, [1.0], want_info=False).objective

    ref, scale = 0.0, 0.0
    for k in range(F):
        b = betas[k, gi]
        eta = np.zeros(n)
        for j in np.flatnonzero(b):
            eta[d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]]] += b[j]
        tr = fold != k
        lay_tr = orc.canonical_layout(d.time[tr], d.event[tr], d.stratum[tr])
        a, t_ = nll(eta, lay_all), nll(eta[tr], lay_tr)
        ref += t_ - a
        scale += abs(a) + abs(t_)
    cv_err = abs(cvl[gi] - ref) / scale
    log(f"oracle: cvl at the chosen weight from the fold estimates, |gpu - oracle| / sum|l| = {cv_err:.2e}")
    fits = F * len(gammas) + 1 + B
    total = cv_s + fit_s + boot_s
    out = {
        "metric": METRIC, "value": fits / total, "unit": "fits/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * total,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (indicator X, 1 bit per row)", "data": "synthetic",
        "config": {"workload": f"Sec. 3.2 analysis at full width: N={n}, P={p} indicators (3% ones), K=10 strata; "
                               f"{F}-fold CV over {len(gammas)} l1 weights, refit, {B} bootstrap refits; CCD to "
                               f"1e-12, FP64, seed 9"},
        "total_s": total, "cv_s": cv_s, "refit_s": fit_s, "bootstrap_s": boot_s, "fits": fits,
        "gammas": [float(g) for g in gammas], "cvl": [float(c) for c in cvl], "chosen": gi,
        "treatment_hr": math.exp(beta_star[0]), "treatment_bpi95": [float(lo), float(hi)],
        "statuses_ok": bool(np.all(status == 0) and np.all(bstat == 0)), "oracle_cvl_rel_err": cv_err,
        "paper_context": "the paper's LEGEND-HTN analysis of this shape (real data) took 1.41 h on its GPU, "
                         "16.2 h on its CPU",
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_bootstrap(args):
    """Bootstrap refits of an unpenalised model (Sec. 3.2's percentile intervals) as independent
    requests to the fit server (each replicate's rows gathered on the device and submitted in
    place), against the same refits one after another on a Newton handle (cox_bootstrap).
    N=20,000 rows, P=20, K=200 strata; the two agree replicate by replicate."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p, K, B = 20_000, 20, 200, args.bootstrap_reps
    d = synth.make("iid", n, p, K, 43, beta_sd=0.5, tie_round=100.0)
    rng = np.random.default_rng(44)
    counts = np.stack([rng.multinomial(n, np.full(n, 1.0 / n)) for _ in range(B)]).astype(np.uint32)
    Xt = torch.from_numpy(np.ascontiguousarray(d.X.T)).cuda()
    tt = torch.from_numpy(np.ascontiguousarray(d.time)).cuda()
    et = torch.from_numpy(np.ascontiguousarray(d.event, dtype=np.uint8)).cuda()
    st = torch.from_numpy(np.ascontiguousarray(d.stratum, dtype=np.int32)).cuda()
    reps = []
    for b in range(B):
        idx = torch.from_numpy(np.repeat(np.arange(n), counts[b])).cuda()
        reps.append((Xt.index_select(1, idx).t(), tt.index_select(0, idx).contiguous(),
                     et.index_select(0, idx).contiguous(), st.index_select(0, idx).contiguous()))
    torch.cuda.synchronize()
    log(f"{B} bootstrap replicates of N={n} P={p} K={K} gathered on the device")
    with coxmi.CoxServer(prep_threads=args.prep_threads) as srv:
        t0 = time.perf_counter()
        tickets = [srv.submit_device(*r) for r in reps]
        assert srv.drain(timeout=600.0)
        serve_s = time.perf_counter() - t0
        served = [srv.poll(t) for t in tickets]
    seq = min(B, 32)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, tol=1e-13) as m:
        m.bootstrap(counts[:1])   # warm
        t0 = time.perf_counter()
        betas, status = m.bootstrap(counts[:seq])
        seq_s = time.perf_counter() - t0
    diff = max(float(np.max(np.abs(served[b][0] - betas[b])) / np.max(np.abs(betas[b]))) for b in range(seq))
    ok = all(r[1]["status"] == 0 for r in served) and bool(np.all(status == 0))
    hr = np.exp(np.array([r[0][1] for r in served]))
    log(f"server: {B} refits in {serve_s:.2f} s ({B / serve_s:.0f} fits/s); one after another: {seq} refits in "
        f"{seq_s:.2f} s ({seq / seq_s:.0f} fits/s); max rel diff {diff:.1e}; statuses ok {ok}; "
        f"95% BPI of exp(beta_1) [{np.quantile(hr, 0.025):.4f}, {np.quantile(hr, 0.975):.4f}]")
    out = {
        "metric": METRIC, "value": B / serve_s, "unit": "fits/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * serve_s,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 contraction, f64 score and solve", "data": "synthetic",
        "config": {"workload": f"{B} bootstrap refits (unpenalised) of N={n} P={p} K={K} through the fit server, "
                               f"replicates gathered on the device, seed 43"},
        "sequential_fits_per_s": seq / seq_s, "speedup": (B / serve_s) / (seq / seq_s),
        "max_rel_diff_vs_sequential": diff, "statuses_ok": ok, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_strata_sweep(args):
    """Sec. 2.7 / Sec. 3.1: with the segmented scan the work per coordinate does not depend on how
    the rows are cut into strata.  N=1e6 rows, P=10 AR(1) columns, the same data cut into K = 1 ..
    N/2 strata; time per coordinate of the persistent kernel (a fixed 20-sweep evaluation run, so
    every K does the same number of coordinates)."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    paper = args.sweep_design == "paper"
    n, p, sweeps = (1_000_000, 1000, 2) if paper else (1_000_000, 10, 20)
    res = {}
    for K in ((1, 10, 1_000, 50_000, 500_000) if paper else (1, 10, 1_000, 50_000, 250_000, 500_000)):
        if paper:   # the Sec. 3.1 design: binary X with 5% ones, beta ~ N(0,1) x Bernoulli(0.2)
            d = synth.config_paper(n=n, p=p, K=K)
        else:
            d = synth.make("ar1", n, p, K, 50, beta_sd=0.3)
        with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=1.0, tol=0.0, max_iter=sweeps) as m:
            m.fit()   # warm
            kms = []
            for _ in range(3):
                _, info = m.fit()
                kms.append(m.kernel_ms())
        del d
        us = 1e3 * float(np.median(kms)) / (sweeps * p)
        res[K] = us
        log(f"K={K}: {us:.2f} us per coordinate ({info['iters']} sweeps)")
    vals = list(res.values())
    out = {
        "metric": "us per coordinate evaluation across strata counts", "value": max(vals) / min(vals),
        "unit": "max/min ratio", "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"N={n}, P={p} binary (5% ones, the Sec. 3.1 design), K strata, {sweeps} CCD sweeps, "
                                f"seed 5") if paper else
                               f"N={n}, P={p} AR(1), the same rows cut into K strata, {sweeps} CCD sweeps, seed 50"},
        "us_per_coordinate": {str(k): v for k, v in res.items()}, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_peaks(args):
    """Measured reference points for the roofline, beside the published peaks: HBM bandwidth of a
    plain device copy (1 GiB each way) and the matrix-core rate of large contiguous BF16 and FP32
    products through the vendor library (torch.matmul), timed with HIP events."""
    import torch

    torch.cuda.set_device(0)
    out = {}
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)   # 1 GiB
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * x.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9
    out["copy_GBps"] = gbs
    log(f"device copy: {gbs:.0f} GB/s (read + write) of {HBM_PEAK_GBS:.0f} published")
    del x, y
    for dt, name, peak in [(torch.bfloat16, "bf16", MFMA_PEAK_TFLOPS["bf16"]), (torch.float32, "fp32", 157.3)]:
        n = 8192
        a = torch.randn(n, n, device="cuda").to(dt).contiguous()
        b = torch.randn(n, n, device="cuda").to(dt).contiguous()
        for _ in range(3):
            torch.matmul(a, b)
        e0.record()
        for _ in range(10):
            torch.matmul(a, b)
        e1.record()
        torch.cuda.synchronize()
        tf = 10 * 2 * n ** 3 / (e0.elapsed_time(e1) / 1e3) / 1e12
        out[f"matmul_{name}_TFLOPs"] = tf
        log(f"matmul {name} {n}^3: {tf:.0f} TFLOP/s of {peak:.0f} published")
    rec = {"metric": "measured reference peaks", "value": out["copy_GBps"], "unit": "GB/s", "n_gpus": 1,
           "steps": 10, "warmup": 3, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 copy; bf16 and fp32 products", "data": "synthetic",
           "config": {"workload": "1 GiB device copy; 8192^3 matrix products"}, "measured": out,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(rec), flush=True)


def run_cough(args):
    """Sec. 3.3 at its full width on indicator X: a treatment whose coefficient steps at 10 days,
    407,828 subjects x 9,666 indicators (3% ones); the interval-stratified model built on the
    device from the indicator handle (cox_init_intervals: ~812k augmented rows, bits gathered),
    one l1 CCD fit at 0.02 gamma_max with the two treatment columns unpenalised.  Checked against
    the oracle: the l1 optimality conditions at the returned beta on sampled augmented columns
    (the oracle's own split of those columns; per-column score, plain C)."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    cut = 10.0
    log(f"drawing the full-width Sec. 3.3 workload: N={args.cough_n} P={args.cough_p} indicators (seed 11)")
    d = synth.config_cough_sparse(n=args.cough_n, p=args.cough_p, cut=cut)
    n, p = d.n, d.col_ptr.shape[0] - 1
    tv = np.zeros(p, np.uint8)
    tv[0] = 1
    t0 = time.perf_counter()
    parent = coxmi.CoxModel.indicator(n, d.col_ptr, d.row_idx, d.time, d.event, None, tol=1e-12)
    init_s = time.perf_counter() - t0
    pen_aug = np.ones(p + 1, np.uint8)
    pen_aug[:2] = 0                       # the treatment's two interval columns come first
    t0 = time.perf_counter()
    m = parent.intervals(d.time, d.event, None, [cut], tv, gamma=0.0, penalize=pen_aug, tol=1e-12)
    map_s = time.perf_counter() - t0
    na, pa, _ = coxmi.cox_shape(m.h)
    _, g0, _ = m.evaluate(np.zeros(pa))
    gamma = 0.02 * float(np.max(np.abs(g0[pen_aug == 1])))
    m.set_penalty(gamma, pen_aug)
    log(f"indicator handle {init_s:.1f} s; cox_init_intervals {map_s:.2f} s: {na} rows x {pa} columns; "
        f"gamma = {gamma:.2f}")
    beta, info = m.fit()   # warm
    torch.cuda.synchronize()
    ts = time.perf_counter()
    beta, info = m.fit()
    T = time.perf_counter() - ts
    kms = m.kernel_ms()
    cv = None
    if args.cough_cv:
        # 10-fold CV as in Sec. 3.3, folds drawn per subject (both interval rows of a subject are
        # held out together); augmented rows are interval-major: all subjects, then those at risk
        # after the cut
        F = args.cough_cv
        fold_subj = np.random.default_rng(12).integers(0, F, n).astype(np.int32)
        row_subj = np.concatenate([np.arange(n), np.flatnonzero(d.time >= cut)])
        assert row_subj.shape[0] == na
        fold = fold_subj[row_subj]
        gammas = gamma / 0.02 * np.array([0.1, 0.05, 0.02, 0.01])
        m.set_penalty(0.0, pen_aug)
        cvl = np.zeros(len(gammas))
        fold_betas = np.zeros((F, len(gammas), pa))
        tc = time.perf_counter()
        for k in range(F):
            tk = time.perf_counter()
            with m.resample((fold != k).astype(np.uint32)) as c:
                prev = np.zeros(pa)
                for g, gam in enumerate(gammas):
                    c.set_penalty(gam, pen_aug)
                    b, _ = c.fit(beta0=prev)
                    obj_train, _, _ = c.evaluate(b)
                    obj_all, _, _ = m.evaluate(b)
                    cvl[g] += (obj_train - gam * float(np.sum(pen_aug * np.abs(b)))) - obj_all
                    fold_betas[k, g] = b
                    prev = b
            log(f"fold {k}: {len(gammas)} fits in {time.perf_counter() - tk:.1f} s")
        cv_s = time.perf_counter() - tc
        gi = int(np.argmax(cvl))
        log(f"cross-validation: {F} folds x {len(gammas)} weights in {cv_s:.1f} s; cvl {np.round(cvl, 1)}; "
            f"chosen {gammas[gi]:.2f}")
        cv = {"folds": F, "gammas": [float(g) for g in gammas], "cvl": [float(c) for c in cvl], "chosen": gi,
              "cv_s": cv_s, "fold_betas_chosen": fold_betas[:, gi], "fold_subj": fold_subj}
    m.close()
    parent.close()
    evals = int(info["coord_evals"])
    log(f"fit: {T:.2f} s, {info['iters']} sweeps, {evals} coordinate evaluations, status {info['status']}, "
        f"{int(np.count_nonzero(beta))} nonzero; treatment log HR before / after the cut {beta[0]:.4f} / "
        f"{beta[1]:.4f} (simulated {math.log(2.0):.4f} / {math.log(1.1):.4f})")
    # oracle: its own split of the sampled columns; the augmented linear predictor per interval
    from oracle import cox_oracle as orc
    cols_aug = orc.augmented_columns(tv, 2)                 # (source, interval) of each augmented column
    b0 = np.array([beta[c] for c, (j, k) in enumerate(cols_aug) if k <= 0 and j >= 0])   # beta on interval 0
    b1 = np.array([beta[c] for c, (j, k) in enumerate(cols_aug) if k < 0 or k == 1])     # beta on interval 1
    eta_k = []
    for bk in (b0, b1):
        e = np.zeros(n)
        for j in np.flatnonzero(bk):
            e[d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]]] += bk[j]
        eta_k.append(e)
    nz = [c for c in np.flatnonzero(beta) if c >= 2][:4]
    zero = list(np.flatnonzero(beta == 0.0)[:4])
    sample = sorted(set([0, 1] + nz + zero))
    srcs = sorted(set(cols_aug[c][0] for c in sample))
    Xs = np.zeros((n, len(srcs)))
    for q, j in enumerate(srcs):
        Xs[d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]], q] = 1.0
    r = orc.split_intervals(Xs, d.time, d.event, None, [cut], tv_coef=tv[srcs])
    eta_aug = np.where(r["row_interval"] == 0, eta_k[0][r["row_subject"]], eta_k[1][r["row_subject"]])
    lay = orc.canonical_layout(r["time"], r["event"], r["stratum"])
    eta_c = np.ascontiguousarray(eta_aug[lay.perm])
    sub_cols = orc.augmented_columns(tv[srcs], 2)
    E = float(r["event"].sum())
    worst = 0.0
    for c in sample:
        j, k = cols_aug[c]
        q = sub_cols.index((srcs.index(j), k))
        g = orc.coord_terms(orc.to_canonical(r["X"][:, [q]], lay), lay, 0, eta_c)["grad"]
        gj = gamma * pen_aug[c]
        res = abs(g) if gj == 0.0 else (abs(g + gj * np.sign(beta[c])) if beta[c] != 0.0 else max(abs(g) - gj, 0.0))
        worst = max(worst, res / E)
    log(f"oracle: augmented rows {r['X'].shape[0]} (library {na}); l1 optimality residual on {len(sample)} columns: "
        f"max / E = {worst:.2e}")
    cv_err = None
    if cv is not None:
        # the CV criterion at the chosen weight from the returned fold estimates, by the oracle
        lay_all = lay

        def nll(eta_rows, L):
            return orc.full_eval(np.ascontiguousarray(eta_rows[L.perm])[:, None], L, [1.0], want_info=False).objective

        ref, scale = 0.0, 0.0
        for k in range(cv["folds"]):
            bk = cv["fold_betas_chosen"][k]
            b0k = np.array([bk[c] for c, (j, kk) in enumerate(cols_aug) if kk <= 0 and j >= 0])
            b1k = np.array([bk[c] for c, (j, kk) in enumerate(cols_aug) if kk < 0 or kk == 1])
            ek = []
            for bb in (b0k, b1k):
                e = np.zeros(n)
                for j in np.flatnonzero(bb):
                    e[d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]]] += bb[j]
                ek.append(e)
            eta_rows = np.where(r["row_interval"] == 0, ek[0][r["row_subject"]], ek[1][r["row_subject"]])
            tr = cv["fold_subj"][r["row_subject"]] != k
            L_tr = orc.canonical_layout(r["time"][tr], r["event"][tr], r["stratum"][tr])
            a, t_ = nll(eta_rows, lay_all), nll(eta_rows[tr], L_tr)
            ref += t_ - a
            scale += abs(a) + abs(t_)
        cv_err = abs(cv["cvl"][cv["chosen"]] - ref) / scale
        log(f"oracle: cvl at the chosen weight from the fold estimates, |gpu - oracle| / sum|l| = {cv_err:.2e}")
        del cv["fold_betas_chosen"], cv["fold_subj"]
    out = {
        "metric": METRIC, "value": na * evals / T, "unit": "obs-evals/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * T,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (indicator X, 1 bit per row)", "data": "synthetic",
        "config": {"workload": f"Sec. 3.3 at full width: {n} subjects x {p} indicators (3% ones), treatment "
                               f"coefficient stepping at {cut:g} days, {na} augmented rows x {pa} columns built on "
                               f"the device, l1 at 0.02 gamma_max, CCD to 1e-12, seed 11"},
        "fit_s": T, "indicator_init_s": init_s, "cox_init_intervals_s": map_s, "sweeps": int(info["iters"]),
        "us_per_coordinate": 1e3 * kms / max(evals, 1), "treatment_log_hr": [float(beta[0]), float(beta[1])],
        "oracle_rows": int(r["X"].shape[0]), "oracle_l1_residual_over_E": worst,
        "cross_validation": cv, "oracle_cvl_rel_err": cv_err,
        "paper_context": "the paper's cough analysis: 812,432 rows x 9,668 columns (real data)",
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_heavy(args):
    """Large heavy-tailed Newton fit: N=1e7, P=500 Student-t(3), 50 nonzero coefficients,
    K=5e5 -- FP8 e4m3 information matrix + FP64 refinement against the FP64 Newton path.
    Full-size check against the oracle: its per-column score (Eq. strat_g, plain C) at the
    returned beta for sampled columns must vanish; and the FP8 and FP64 paths must agree."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    n, p, K = args.heavy_n, 500, max(1, args.heavy_n // 20)
    log(f"drawing the heavy-tailed workload N={n} P={p} K={K} (seed 4)")
    t0 = time.perf_counter()
    last = [t0]

    def progress(j, tot):
        now = time.perf_counter()
        if now - last[0] > 20 or j == tot:
            log(f"  column {j}/{tot} ({now - t0:.0f} s)")
            last[0] = now

    d = synth.config_heavy(n=n, p=p, K=K, progress=progress)
    runs = {}
    betas = {}
    for prec, name in [(coxmi.COX_FP8_E4M3, "fp8"), (coxmi.COX_F64, "f64")]:
        t1 = time.perf_counter()
        m = coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                           tol=1e-12, max_iter=100)
        log(f"{name}: cox_init {time.perf_counter() - t1:.1f} s")
        t1 = time.perf_counter()
        m.fit()   # the first fit also sets up the Newton path (buffers, low-precision copy of X)
        log(f"{name}: first fit with set-up {1e3 * (time.perf_counter() - t1):.0f} ms")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        beta, info = m.fit()
        T = time.perf_counter() - t1
        prof = m.profile()
        m.close()
        betas[name] = beta
        runs[name] = {"fits_per_s": 1.0 / T, "ms_per_fit": 1e3 * T, "newton_steps": int(info["iters"]),
                      "evaluations": int(info["coord_evals"]), "status": int(info["status"]), "device_ms": prof}
        log(f"{name}: {1e3 * T:.0f} ms, {info['iters']} steps, profile {prof}")
    agree = float(np.max(np.abs(betas["fp8"] - betas["f64"])) / np.max(np.abs(betas["f64"])))
    log(f"fp8 vs f64 rel diff {agree:.2e}")
    # oracle: per-column score at the FP8 estimate for sampled columns
    from oracle import cox_oracle as orc
    lay = orc.canonical_layout(d.time, d.event, d.stratum)
    eta = np.ascontiguousarray((d.X @ betas["fp8"])[lay.perm])
    E = float(d.event.sum())
    cols = sorted(set([0, p - 1] + list(np.flatnonzero(d.beta_true)[:3]) + [p // 2]))
    worst = 0.0
    for j in cols:
        xj = orc.to_canonical(d.X[:, [j]], lay)
        g = orc.coord_terms(xj, lay, 0, eta)["grad"]
        worst = max(worst, abs(g) / (E * max(1.0, float(np.max(np.abs(d.X[:, j]))))))
    log(f"oracle score at the FP8 estimate, columns {cols}: max |g_j| / (E max|x_j|) = {worst:.2e}")
    G = int(np.count_nonzero(d.event))
    f8 = runs["fp8"]["device_ms"]
    flops = (n + G) * p * (p + 1.0)
    contr_s = f8["contraction_ms"] / max(f8["contractions"], 1) / 1e3
    out = {
        "metric": METRIC, "value": runs["fp8"]["fits_per_s"], "unit": "fits/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": runs["fp8"]["ms_per_fit"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp8 contraction, f64 score and solve", "data": "synthetic",
        "config": {"workload": f"Newton fit with FP8 information matrix and FP64 refinement: N={n} rows, P=500 "
                               f"Student-t(3) covariates, 50 nonzero coefficients, K={K} strata, seed 4",
                   "n": n, "p": p, "strata": K},
        "plain_fp64_fits_per_s": runs["f64"]["fits_per_s"],
        "speedup_vs_plain": runs["fp8"]["fits_per_s"] / runs["f64"]["fits_per_s"],
        "runs": runs, "fp8_vs_f64_rel_diff": agree, "oracle_score_check": {"columns": [int(c) for c in cols],
                                                                           "max_scaled_score": worst},
        "roofline": contraction_roofline(flops, 1.0 * (n + G) * p + 4.0 * n + 8.0 * p * p, contr_s, "fp8",
                                         "FP8 information contraction (X' diag(b) X and Z'Z)"),
    }
    print(json.dumps(out), flush=True)


def run_mixed(args):
    print(json.dumps(mixed_leg(args, args.steps, args.warmup)), flush=True)


def mixed_leg(args, steps, warmup):
    """Mixed precision Newton: N=1e6, P=200 AR(1), K=5e4 -- BF16 information matrix on the
    matrix cores + FP64 Cholesky and refinement, against the FP64 Newton path."""
    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    log("drawing the N=1e6 P=200 K=5e4 AR(1) workload (seed 2)")
    d = synth.config_mixed()
    gold = {}
    with open(os.path.join(ROOT, "tests", "golden", "newton_mixed_n1e6_p200.txt")) as fh:
        for line in fh:
            if line.startswith("beta "):
                gold["beta"] = np.array([float(v) for v in line.split()[1:]])
    runs = {}
    for prec, name in [(coxmi.COX_BF16, "bf16"), (coxmi.COX_F64, "f64")]:
        m = coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                           tol=1e-13, max_iter=200)
        for _ in range(warmup):
            m.fit()
        torch.cuda.synchronize()
        profs, lat = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            beta, info = m.fit()
            lat.append(time.perf_counter() - ts)
            profs.append(m.profile())
        T = time.perf_counter() - t0
        m.close()
        err = float(np.max(np.abs(beta - gold["beta"])) / np.max(np.abs(gold["beta"])))
        agg = {k: float(np.mean([q[k] for q in profs])) for k in profs[0]}
        runs[name] = {"fits_per_s": steps / T, "ms_per_fit": 1e3 * T / steps,
                      "newton_steps": int(info["iters"]), "evaluations": int(info["coord_evals"]),
                      "rel_err_vs_oracle": err, "status": int(info["status"]), "device_ms": agg}
        log(f"{name}: {runs[name]['ms_per_fit']:.1f} ms/fit, {info['iters']} steps, rel err {err:.2e}, "
            f"eval {agg['evaluation_ms']:.1f} ms / {agg['evaluations']:.0f}, contraction {agg['contraction_ms']:.1f} ms "
            f"/ {agg['contractions']:.0f}, solve {agg['solve_ms']:.1f} ms / {agg['solves']:.0f}")
    n, p = d.n, d.p
    G = int(np.count_nonzero(d.event))   # continuous times: one event per group
    bf = runs["bf16"]["device_ms"]
    flops = (n + G) * p * (p + 1.0)        # symmetric X'WX and Z'Z: p(p+1)/2 entries x 2 flops per term
    contr_bytes = 2.0 * (n + G) * p + 4.0 * n + 8.0 * p * p   # BF16 X and Z, FP32 weights, the FP64 result
    contr_s = bf["contraction_ms"] / max(bf["contractions"], 1.0) / 1e3
    eval_s = bf["evaluation_ms"] / max(bf["evaluations"], 1.0) / 1e3
    eval_bytes = 8.0 * n * p * 2 + 8.0 * n * 12   # X twice (X beta; column pass) + the row vectors
    out = {
        "metric": METRIC,
        "value": runs["bf16"]["fits_per_s"], "unit": "fits/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": runs["bf16"]["ms_per_fit"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 contraction, f64 score and solve", "data": "synthetic",
        "config": {"workload": "Newton fit with BF16 information matrix and FP64 refinement: N=1e6 rows, "
                               "P=200 AR(1) covariates, K=5e4 strata, seed 2", "n": n, "p": p, "strata": 50000},
        "plain_fp64_fits_per_s": runs["f64"]["fits_per_s"],
        "speedup_vs_plain": runs["bf16"]["fits_per_s"] / runs["f64"]["fits_per_s"],
        "runs": runs,
        "roofline": contraction_roofline(flops, contr_bytes, contr_s, "bf16",
                                         "BF16 information contraction (X' diag(b) X and Z'Z)",
                                         traffic=recorded_field(CONTRACTION_PROFILE, ["contraction.hip"]),
                                         mfma_busy=recorded_field(CONTRACTION_PROFILE, ["contraction.hip"],
                                                                  "mfma_busy")),
        "evaluation_roofline": {"bound": "hbm", "achieved": eval_bytes / eval_s / 1e9, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": eval_bytes / eval_s / 1e9 / HBM_PEAK_GBS,
                                "algorithmic_bytes_per_evaluation": eval_bytes},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle Newton step (C risk-set sums, BLAS on all cores)")
        out["cpu_baseline"] = cpu_baseline_newton(d, runs["f64"]["newton_steps"])
        log(f"  {out['cpu_baseline']['sample']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--heavy-n", type=int, default=10_000_000, help="heavy: rows")
    ap.add_argument("--paper-n", type=int, default=1_000_000, help="paper: rows")
    ap.add_argument("--paper-p", type=int, default=1000, help="paper: columns")
    ap.add_argument("--paper-newton", action="store_true",
                    help="paper: also fit by proximal Newton with BF16 and FP8 information matrices")
    ap.add_argument("--bootstrap-reps", type=int, default=512, help="bootstrap: replicates")
    ap.add_argument("--sweep-design", choices=["ar1", "paper"], default="ar1",
                    help="strata-sweep: AR(1) P=10, or the Sec. 3.1 binary design at P=1000")
    ap.add_argument("--cough-n", type=int, default=407_828, help="cough: subjects")
    ap.add_argument("--cough-p", type=int, default=9666, help="cough: indicator columns")
    ap.add_argument("--cough-cv", type=int, default=0, help="cough: folds of a cross-validation (0: none)")
    ap.add_argument("--sparse-n", type=int, default=946_911, help="sparse: rows")
    ap.add_argument("--sparse-p", type=int, default=9977, help="sparse: indicator columns")
    ap.add_argument("--sparse-values", action="store_true",
                    help="sparse: general sparse X (the same pattern with N(0, 1/4) values, cox_init_sparse)")
    ap.add_argument("--cv-n", type=int, default=946_911, help="cv: rows")
    ap.add_argument("--cv-p", type=int, default=1000, help="cv: columns")
    ap.add_argument("--cv-folds", type=int, default=10, help="cv: folds")
    ap.add_argument("--cv-newton", action="store_true", help="cv: proximal Newton fits (BF16 information)")
    ap.add_argument("--bootstrap", type=int, default=20, help="cv: bootstrap refits")
    ap.add_argument("--cv-served", action="store_true",
                    help="cv: also run the path with the fold fits batched through a fit server (P <= 128)")
    ap.add_argument("--intervals-n", type=int, default=407_828, help="intervals: subjects")
    ap.add_argument("--intervals-p", type=int, default=1000, help="intervals: columns before the split")
    ap.add_argument("--workload", choices=["ccd", "serve", "mixed", "heavy", "paper", "intervals", "cv", "sparse", "legend", "bootstrap",
                             "strata-sweep", "peaks", "cough"], default="ccd",
                    help="ccd: the CCD fit of the N=1e6 P=50 workload (default); serve: the serving stream; "
                         "mixed: BF16 + FP64-refinement Newton fits at N=1e6 P=200; heavy: FP8 Newton at N=1e7 P=500; "
                         "paper: the Sec. 3.1 l1 CCD fit; intervals: a step-effect model split into interval strata; "
                         "cv: cross-validation over an l1 path plus bootstrap refits; sparse: the full-width "
                         "Sec. 3.2 fit on indicator X; legend: the full-width Sec. 3.2 analysis (CV, refit, bootstrap); "
                         "bootstrap: unpenalised bootstrap refits through the fit server; strata-sweep: time per "
                         "coordinate across strata counts; peaks: measured copy bandwidth and matrix-core rates; cough: the "
                         "full-width Sec. 3.3 model on indicator X")
    ap.add_argument("--requests", type=int, default=4096, help="serve: requests in the stream")
    ap.add_argument("--plain-sample", type=int, default=32, help="serve: requests timed on the plain FP64 path")
    ap.add_argument("--poisson-seconds", type=float, default=15.0, help="serve: length of the Poisson run")
    ap.add_argument("--fused-rounds", type=int, default=0,
                    help="serve: rounds per persistent launch of the fit server (0: separate launches per round)")
    ap.add_argument("--legs", default="mixed,serve",
                    help="default workload: secondary legs to run after the headline fit (comma-separated: "
                         "mixed = BF16 + refinement Newton at N=1e6 P=200; serve = the serving stream; empty: none)")
    ap.add_argument("--check", type=int, default=16, help="serve: requests checked against the oracle")
    ap.add_argument("--score-check", type=int, default=256,
                    help="serve: requests whose served estimate is checked by the oracle's score")
    ap.add_argument("--hbm-gib", type=int, default=32, help="serve: device budget of the server")
    ap.add_argument("--prep-threads", type=int, default=12, help="serve: host prep threads")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed fits, run a copy kernel (y = 1 * x) over a buffer of this many "
                         "MiB three times: known bytes against which hardware byte counters are scaled")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "mixed":
        run_mixed(args)
        return
    if args.workload == "heavy":
        run_heavy(args)
        return
    if args.workload == "cough":
        run_cough(args)
        return
    if args.workload == "peaks":
        run_peaks(args)
        return
    if args.workload == "strata-sweep":
        run_strata_sweep(args)
        return
    if args.workload == "bootstrap":
        run_bootstrap(args)
        return
    if args.workload == "legend":
        run_legend(args)
        return
    if args.workload == "sparse":
        run_sparse(args)
        return
    if args.workload == "cv":
        run_cv(args)
        return
    if args.workload == "intervals":
        run_intervals(args)
        return
    if args.workload == "paper":
        run_paper(args)
        return

    import numpy as np
    import torch
    from paper_2310_16238_amd import coxmi, synth

    torch.cuda.set_device(0)
    log("drawing the N=1e6 P=50 K=5e4 AR(1) workload (seed 1)")
    d = synth.config_ar1()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    model = coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-12, stream=stream.cuda_stream)
    log(f"cox_init {time.perf_counter() - t0:.2f} s; shape {coxmi.cox_shape(model.h)}")

    for i in range(args.warmup):
        beta, info = model.fit()
        log(f"warmup {i}: sweeps={info['iters']} status={info['status']} kernel={model.kernel_ms():.2f} ms")

    torch.cuda.synchronize()
    lat, kms, evals, statuses = [], [], 0, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        beta, info = model.fit()
        lat.append(time.perf_counter() - ts)
        kms.append(model.kernel_ms())
        evals += info["coord_evals"]
        statuses.append(info["status"])
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    log(f"timed {args.steps} fits in {T:.3f} s; sweeps/fit={info['iters']} statuses={set(statuses)}")

    n = d.n
    evals_per_fit = evals / max(args.steps, 1)
    kernel_s = float(np.mean(kms)) / 1e3
    bytes_per_launch = 8.0 * n * evals_per_fit + 4.0 * n
    achieved = bytes_per_launch / kernel_s / 1e9
    out = {
        "metric": METRIC,
        "value": n * evals / T,
        "unit": "obs-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / max(args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "stratified Cox CCD fit to convergence: N=1e6 rows, P=50 AR(1) covariates, "
                               "K=5e4 strata, FP64, seed 1",
                   "n": n, "p": d.p, "strata": 50000, "tol": 1e-12},
        "fits_per_s": args.steps / T,
        "fit_latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                           "p99": 1e3 * float(np.percentile(lat, 99))},
        "sweeps_per_fit": int(info["iters"]),
        "coord_evals_per_fit": evals_per_fit,
        "kernel_ms_per_fit": 1e3 * kernel_s,
        "us_per_coordinate": 1e6 * kernel_s / evals_per_fit,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(),
                     "kernel": "ccd_kernel (persistent, one launch per fit)",
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    model.close()
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # an elementwise kernel: reads and writes nbytes (a copy engine would not show)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {nbytes} bytes (read {nbytes} + write {nbytes} each)")
        out["copy_probe_bytes"] = nbytes
        del src, dst
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle CCD, first 20 sweeps")
        out["cpu_baseline"] = cpu_baseline(d)
    del d
    legs = [s for s in args.legs.split(",") if s]
    if "mixed" in legs:
        log("leg: BF16 information + FP64 refinement against plain FP64 Newton (N=1e6, P=200)")
        out["mixed_precision"] = _leg(lambda: mixed_leg(args, steps=5, warmup=1))
    if "serve" in legs:
        log(f"leg: serving stream of {args.requests} requests")
        out["serving"] = _leg(lambda: serve_leg(args))
    print(json.dumps(out), flush=True)


def _leg(fn):
    """A secondary workload's result without the headline keys (its error, if it failed)."""
    try:
        r = fn()
    except Exception as e:   # reported in the line rather than hiding the headline
        log(f"  leg failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}
    for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
        r.pop(k, None)
    return r


if __name__ == "__main__":
    main()
