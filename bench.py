"""Benchmark: TSQBX pair-terms/s in FP64 on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-batched] [--no-serve]
                    [--no-high-order] [--no-cpu] [--requests R] [--min-warm S]
                    [--no-sprime] [--no-helmholtz] [--no-lists] [--no-conventional] [--no-shared]
                    [--only headline|batched|high_order|serve|sprime|helmholtz|lists|conventional|
                            shared|helm_batched]
                    [--calibration-copy]

The headline `value` is the plain single- plus double-layer evaluation at
p = 16 on the perturbed-sphere workload (262144 sources, 65536 targets,
ball lists of radius 0.15 about centers 0.02 inside the surface), inputs
resident in device memory, K timed steps.  One step = staging of q = w sigma
plus the evaluation kernel.  The roofline object prices the evaluation
kernel alone: K more launches of it on strengths staged once, timed with HIP
events on the launch stream.  Extra objects report the batched workload (64
geometries, mixed p, one persistent launch vs plain per-geometry launches),
S' (the target normal derivative of the single layer) and the Helmholtz
single + double layer (k = 20) on the headline workload, the device build of
the headline workload's near-field lists, conventional QBX (coefficients
formed per center, then evaluated) against the target-specific single layer,
the row kernel against one wave per target where four targets share each
center, and the served Poisson stream (p50/p99 latency).  The oracle timed on the
host cores is reported as `cpu_baseline`.  Progress goes to stderr; one JSON
line goes to stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TSQBX pair-terms/s FP64 at p=16 (batched vs plain) + p50/p99 request latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk/CU


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def separate_recurrence_flops_per_pair(p: int, layers: int) -> int:
    """Per-pair FP64 work of evaluating each layer with a recurrence of its
    own: 6p + 20 for the single layer and 11p + 36 for the double layer
    (the per-pair estimate of the work the method does, fma = 2).  The kernel
    shares one recurrence among the layers (flops_per_pair), so this figure
    exceeds what it executes.  It is reported as a count only: divided by the
    kernel's time it would exceed the chip's peak, which makes it no rate of
    the ALUs."""
    return (6 * p + 20 if layers & 1 else 0) + (11 * p + 36 if layers & 2 else 0)


def flops_per_pair(p: int, layers: int) -> int:
    """FP64 operations per (target, source) pair executed by the evaluation
    kernel (add/mul = 1, fma = 2, the reciprocal-square-root estimate = 1):
    25 for the pair setup; the single layer alone 5 per order (Clenshaw);
    otherwise 6 per order of the derivative recurrence and the closing sums of
    each layer (single layer 10, double layer 17, S' 13, or 12 when it shares
    1/|d|^3 with the double layer, plus one multiply for each of E_p, E_{p+1}
    used).  S' alone never uses E_{p+1}, so the last recurrence step (4) is
    not executed."""
    if layers == 1:
        # Clenshaw: the first two steps need no arithmetic when unrolled (one
        # target per wave), 5 per further order, 5 to close
        return 28 if p == 0 else (31 if p == 1 else 5 * p + 25)
    f = 6 * max(p, 1) + 19
    if not layers & 3:
        f -= 4                           # no E_{p+1}
    f += 1 if layers & 3 else 0          # E_{p+1}
    f += 1 if layers & 5 else 0          # E_p
    f += 10 if layers & 1 else 0
    f += 17 if layers & 2 else 0
    f += (12 if layers & 2 else 13) if layers & 4 else 0
    return f


def rows_flops_per_pair(p: int, layers: int, per_walk: int = 4) -> float:
    """FP64 operations per pair of the row kernel, which walks a list once for
    per_walk targets: the source's offset from the center, |d|^2, 1/|d| and
    1/|d|^2 (18), and the products that depend on the source and center
    only (nu.d and 1/|d|^3 with the double layer, 6; q/|d| with the single
    layer, 1; q/|d|^3 with S', 1, and 1/|d|^3 when S' comes without the
    double layer, 1) are formed once per source for all of them."""
    shared = 18 + (6 if layers & 2 else 0) + (1 if layers & 1 else 0)
    if layers & 4:
        shared += 1 + (0 if layers & 2 else 1)
    return flops_per_pair(p, layers) - shared * (1.0 - 1.0 / per_walk)


MIN_WARM_S = 0.3
# FP64 operations of one double-precision sincos as executed by the device
# library, measured with FP64 VALU counters on the Helmholtz kernel
HELM_SINCOS_FLOPS = 60


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_eval_p16_slp_dlp_sphere262144_traffic.json")
COUNTER_RECORD = os.path.join(ROOT, "profiles", "k_eval_p16_slp_dlp_sphere262144_counters.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1811_01110_amd", "csrc", f)
                  for f in ("tsqbx_device.h", "tsqbx_eval.hip")]


def kernel_source_sha256() -> str:
    """Hash of the sources the evaluation kernel is compiled from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the evaluation kernel from the committed
    rocprofv3 counter summary, or None when the kernel source has changed
    since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        cur = kernel_source_sha256()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != cur:
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_counters():
    """Per-pair instruction counts and unit utilisations of the evaluation
    kernel from the committed rocprofv3 counter record (same kernel sources),
    with the bound derived from them: the unit whose utilisation is highest
    among the FP64 vector ALU issue slots ("alu") and HBM bandwidth ("hbm"),
    and the busiest unit of all those measured named as the limiter (the
    vector memory pipeline's units count there too).  None when the kernel
    source has changed since the counters were taken."""
    try:
        rec = json.load(open(COUNTER_RECORD))
        cur = kernel_source_sha256()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != cur:
        return None
    util = rec["utilisation"]
    bound = "alu" if util["valu_issue"] >= util["hbm"] else "hbm"
    names = {"valu_issue": "FP64 vector ALU issue", "ta_busy": "vector memory address unit (TA)",
             "td_busy": "vector memory data path (TD)", "hbm": "HBM bandwidth"}
    busiest = max(names, key=lambda k: util[k])
    return {"bound": bound, "limiter": f"{names[busiest]}, {util[busiest]:.0%} busy",
            "utilisation": util, "per_pair": rec["per_pair"],
            "clock_ghz": rec["clock_ghz"], "valu_full_issue_frac": rec["ceiling"]["valu_full_issue"],
            "source": os.path.relpath(COUNTER_RECORD, ROOT)}


def per_launch_ms(fn, n, torch):
    """n further calls, each between its own pair of events on the current
    stream; the durations in ms."""
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def timed_steps(fn, steps, warmup, torch, min_warm_s=None):
    """W warm-up calls (continued until min_warm_s of device work so that the
    clocks settle), then `steps` timed calls between synchronisations."""
    if min_warm_s is None:
        min_warm_s = MIN_WARM_S
    t0 = time.perf_counter()
    n = 0
    while n < warmup or time.perf_counter() - t0 < min_warm_s:
        fn()
        n += 1
        if n % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1e3


def cpu_model():
    """The host CPU's model name, with its family, model and stepping numbers
    when the name alone is only a brand (such as "AMD EPYC")."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = (x.strip() for x in line.split(":", 1))
                    if k in ("model name", "cpu family", "model", "stepping") and k not in fields:
                        fields[k] = v
                if not line.strip() and fields:
                    break
    except OSError:
        return None
    name = fields.get("model name")
    if name is None:
        return None
    if len(name.split()) <= 2 and "cpu family" in fields:
        name += (f" (family {fields['cpu family']}, model {fields.get('model', '?')}, "
                 f"stepping {fields.get('stepping', '?')})")
    return name


def cpu_baseline(g, p, layers):
    import oracle

    t0 = time.perf_counter()
    oracle.evaluate_geometry(g, p=p, layers=layers)
    t1 = time.perf_counter() - t0
    reps = int(max(1, min(math.ceil(10.0 / max(t1, 1e-3)), 30.0 / max(t1, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.evaluate_geometry(g, p=p, layers=layers)
    dt = (time.perf_counter() - t0) / reps
    # one core on a slice of the targets, for a per-core rate
    sel = np.arange(0, g.n_targets, 32)
    t0 = time.perf_counter()
    oracle.evaluate_geometry(g, p=p, layers=layers, select=sel, n_threads=1)
    dt1 = time.perf_counter() - t0
    off = np.asarray(g.list_offsets)
    tc = (np.asarray(g.target_center) if g.target_center is not None
          else np.arange(g.n_targets))[sel]
    slice_terms = int((off[tc + 1] - off[tc]).sum()) * (p + 1) * bin(layers).count("1")
    return {"value": g.pair_terms(p, layers) / dt, "unit": "pair-terms/s",
            "cores": oracle.max_threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"the whole timed workload (all {g.n_targets} targets, p={p}, "
                      f"layers={layers}) evaluated {reps}x by the FP64 C oracle, OpenMP over targets",
            "seconds_per_pass": dt,
            "one_core": {"pair_terms_per_s": slice_terms / dt1, "sample":
                         f"every 32nd target ({len(sel)}), one thread"}}


def roofline_obj(flops, kernel_ms, kernel, **extra):
    """The roofline object of one kernel: executed FP64 operations per launch
    divided by the kernel's average launch duration (HIP events on its
    stream), against the FP64 vector peak."""
    achieved = flops / (kernel_ms / 1e3) / 1e12
    d = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
         "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
         "kernel": kernel, "kernel_ms_per_launch": kernel_ms, "flops_per_launch": flops}
    d.update(extra)
    return d


def plan_flops(items, helm=False):
    """Executed FP64 operations of one run of a plan's persistent kernel."""
    if helm:
        return sum(it["geom"].pairs * helm_flops_per_pair(it["p"], it["layers"]) for it in items)
    return sum(it["geom"].pairs * flops_per_pair(it["p"], it["layers"]) for it in items)


# --plan-tuning: one fixed plan tuning instead of the autotuner (for counter
# runs, whose passes must all time the same launch shape)
FIXED_PLAN_TUNING = None


def tune_and_profile(plan, steps, label):
    """Per-kernel times of the plan with its default tuning, then the plan
    autotuner's choice (or the fixed --plan-tuning) and the per-kernel times
    with it."""
    reps = max(steps // 2, 5)
    default = plan.get_tuning()
    log(f"{label}: profiling the default tuning {default}")
    prof0 = plan.profile(reps)
    t0 = time.perf_counter()
    if FIXED_PLAN_TUNING is not None:
        log(f"{label}: fixed tuning {FIXED_PLAN_TUNING}")
        plan.set_tuning(**FIXED_PLAN_TUNING)
        tuned = plan.get_tuning()
    else:
        log(f"{label}: autotuning the plan")
        tuned, _ = plan.autotune()
    tune_s = time.perf_counter() - t0
    log(f"{label}: tuned {tuned}; profiling it")
    prof1 = plan.profile(reps)
    return {"default": default, "default_stage_ms": prof0["stage_ms"],
            "default_eval_ms": prof0["eval_ms"], "tuned": tuned,
            "tuned_stage_ms": prof1["stage_ms"], "tuned_eval_ms": prof1["eval_ms"],
            "autotune_s": tune_s, "profile_reps": reps}


def max_rel_diff(a_list, b_list):
    num = max((float((a - b).abs().max()) for a, b in zip(a_list, b_list)), default=0.0)
    den = max((float(a.abs().max()) for a in a_list), default=0.0)
    return num / den if den > 0 else num


def bench_batched(ctx, api, torch, W, steps, warmup, geoms=None):
    if geoms is None:
        log("generating 64 batched geometries (mixed p, single layer)")
        geoms = W.config_c()
    items = []
    for g in geoms:
        geom = ctx.geometry(g)
        items.append(dict(geom=geom, p=g.p, layers=g.layers,
                          sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64),
                          out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)))
    pair_terms = sum(it["geom"].pair_terms(it["p"], it["layers"]) for it in items)
    plain_out = [torch.zeros_like(it["out_slp"]) for it in items]

    def plain():
        for it, o in zip(items, plain_out):
            ctx.eval_async(it["geom"], it["sigma"], it["p"], it["layers"], o)
            torch.cuda.synchronize()

    log("timing plain per-geometry launches")
    n_plain = max(steps // 4, 3)
    wall_plain, _ = timed_steps(plain, n_plain, 2, torch)
    plan = ctx.plan(items)
    tuning = tune_and_profile(plan, steps, "batched")
    log("timing the batched plan (graph replay)")
    wall_plan, ev_plan = timed_steps(lambda: plan.execute(), steps, warmup, torch)
    res = {
        "workload": "64 geometries (ellipsoids / perturbed spheres), N log-uniform 2048..65536, "
                    "T=N/4, p in {4,8,12,16}, single layer, ball lists r=8h",
        "pair_terms": pair_terms,
        "plain_pair_terms_per_s": pair_terms * n_plain / wall_plain,
        "batched_pair_terms_per_s": pair_terms * steps / wall_plan,
        "plain_ms": wall_plain / n_plain * 1e3,
        "batched_ms": wall_plan / steps * 1e3,
        "max_rel_diff_batched_vs_plain": max_rel_diff([it["out_slp"] for it in items], plain_out),
        "plan": plan.info(),
        "tuning": tuning,
        "roofline": roofline_obj(plan_flops(items), tuning["tuned_eval_ms"],
                                 "k_persistent<1, -1, G, U> (the plan's evaluation kernel alone)",
                                 stage_kernel_ms=tuning["tuned_stage_ms"]),
    }
    res["speedup"] = res["batched_pair_terms_per_s"] / res["plain_pair_terms_per_s"]
    plan.close()
    for it in items:
        it["geom"].close()
    return res


def bench_helm_batched(ctx, api, torch, W, steps, warmup, geoms=None, k=10.0):
    """The geometries of the batched workload with the Helmholtz single and
    double layer (k = 10, each geometry's own order): one Helmholtz plan
    against plain launches, one per geometry, each followed by a
    synchronisation."""
    if geoms is None:
        log("generating 64 batched geometries (mixed p)")
        geoms = W.config_c()
    rng = np.random.default_rng(20181102)
    items = []
    for g in geoms:
        geom = ctx.geometry(g)
        sig = rng.standard_normal(g.n_sources) + 1j * rng.standard_normal(g.n_sources)
        items.append(dict(geom=geom, p=g.p, layers=3, k=k,
                          sigma=torch.tensor(sig, device="cuda", dtype=torch.complex128),
                          out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128),
                          out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128)))
    pair_terms = sum(it["geom"].pair_terms(it["p"], 3) for it in items)
    plain_out = [(torch.zeros_like(it["out_slp"]), torch.zeros_like(it["out_dlp"])) for it in items]

    def plain():
        for it, (a, b) in zip(items, plain_out):
            ctx.eval_helmholtz_async(it["geom"], it["sigma"], it["p"], 3, k, a, b)
            torch.cuda.synchronize()

    n_plain = max(steps // 4, 3)
    log("timing plain per-geometry Helmholtz launches")
    wall_plain, _ = timed_steps(plain, n_plain, 2, torch)
    plan = ctx.plan_helmholtz(items)
    tuning = tune_and_profile(plan, steps, "Helmholtz batched")
    log("timing the batched Helmholtz plan (graph replay)")
    wall_plan, _ = timed_steps(lambda: plan.execute(), steps, warmup, torch)
    got = [it[key] for it in items for key in ("out_slp", "out_dlp")]
    ref = [x for ab in plain_out for x in ab]
    res = {
        "workload": f"the 64 batched geometries, Helmholtz k={k:g} single + double layer, "
                    "p in {4,8,12,16}, complex density",
        "pair_terms": pair_terms,
        "plain_pair_terms_per_s": pair_terms * n_plain / wall_plain,
        "batched_pair_terms_per_s": pair_terms * steps / wall_plan,
        "plain_ms": wall_plain / n_plain * 1e3,
        "batched_ms": wall_plan / steps * 1e3,
        "max_rel_diff_batched_vs_plain": max_rel_diff(got, ref),
        "plan": plan.info(),
        "tuning": tuning,
        "roofline": roofline_obj(plan_flops(items, helm=True), tuning["tuned_eval_ms"],
                                 "k_helm_persistent<3, G, U> (the plan's evaluation kernel alone)",
                                 stage_kernel_ms=tuning["tuned_stage_ms"]),
    }
    res["speedup"] = res["batched_pair_terms_per_s"] / res["plain_pair_terms_per_s"]
    plan.close()
    for it in items:
        it["geom"].close()
    return res


def bench_d(ctx, api, torch, W, steps, warmup):
    log("generating 16 high-order geometries (k-NN lists 100..8000, p=24, double layer)")
    geoms = W.config_d()
    items = []
    for g in geoms:
        geom = ctx.geometry(g)
        items.append(dict(geom=geom, p=24, layers=2,
                          sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64),
                          out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)))
    pair_terms = sum(it["geom"].pair_terms(24, 2) for it in items)
    plain_out = [torch.zeros_like(it["out_dlp"]) for it in items]

    def plain():
        for it, o in zip(items, plain_out):
            ctx.eval_async(it["geom"], it["sigma"], 24, 2, None, o)
            torch.cuda.synchronize()

    log("timing plain per-geometry launches (high order)")
    wall_plain, _ = timed_steps(plain, 3, 1, torch)
    # the plain kernel alone, for its roofline fraction
    ms_plain_kernel = 0.0
    for it, o in zip(items, plain_out):
        ctx.stage_async(it["geom"], it["sigma"], 2)
        ms = per_launch_ms(lambda: ctx.eval_staged_async(it["geom"], 24, 2, None, o), 3, torch)
        ms_plain_kernel += float(np.mean(ms))
    plan = ctx.plan(items)
    tuning = tune_and_profile(plan, steps, "high order")
    n = max(steps // 2, 3)
    log("timing the high-order plan (graph replay)")
    wall_plan, _ = timed_steps(lambda: plan.execute(), n, 1, torch)
    flops = plan_flops(items)
    res = {
        "workload": "16 perturbed spheres, N=131072, T=32768, p=24, double layer, k-NN lists "
                    "log-uniform 100..8000",
        "pair_terms": pair_terms,
        "plain_pair_terms_per_s": pair_terms * 3 / wall_plain,
        "batched_pair_terms_per_s": pair_terms * n / wall_plan,
        "plain_ms": wall_plain / 3 * 1e3,
        "batched_ms": wall_plan / n * 1e3,
        "plain_kernels_ms": ms_plain_kernel,
        "plain_kernels_frac": flops / (ms_plain_kernel / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
        "max_rel_diff_batched_vs_plain": max_rel_diff([it["out_dlp"] for it in items], plain_out),
        "plan": plan.info(),
        "tuning": tuning,
        "roofline": roofline_obj(flops, tuning["tuned_eval_ms"],
                                 "k_persistent<2, 24, G, U> (the plan's evaluation kernel alone)",
                                 stage_kernel_ms=tuning["tuned_stage_ms"]),
    }
    res["speedup"] = res["batched_pair_terms_per_s"] / res["plain_pair_terms_per_s"]
    plan.close()
    for it in items:
        it["geom"].close()
    return res


SERVE_SLOTS = 256  # requests in flight; a step takes at most 32 of them


def bench_serve(ctx, api, torch, W, n_requests):
    log("generating 32 resident geometries for serving")
    geoms = W.config_e_geometries()
    gs = [ctx.geometry(g) for g in geoms]
    reqs = W.config_e_requests(n_requests, rate_hz=1.0)
    log("staging request densities and outputs in pinned host memory")
    sig = []
    outs = []
    for r in reqs:
        g = gs[r.geometry]
        t = torch.empty(g.n_sources, dtype=torch.float64, pin_memory=True)
        t.numpy()[:] = W.request_sigma(r, g.n_sources)
        sig.append(t)
        outs.append(torch.empty(g.n_targets, dtype=torch.float64, pin_memory=True))
    per_req = [gs[r.geometry].pair_terms(r.p, r.layers) for r in reqs]
    budget = 2 << 30

    def out_args(r, o):
        return (o, None) if r.layers == 1 else (None, o)

    # baseline: one plain synchronous evaluation per request, in arrival order,
    # from and into the same pinned buffers, over the same requests
    log("serving baseline: one plain synchronous evaluation per request")
    k0 = len(reqs)
    t0 = time.perf_counter()
    for r, s_, o in zip(reqs[:k0], sig[:k0], outs[:k0]):  # untimed warm-up
        a, b = out_args(r, o.numpy())
        ctx.eval(gs[r.geometry], s_.numpy(), r.p, r.layers, out_slp=a, out_dlp=b)
        if time.perf_counter() - t0 > MIN_WARM_S:
            break
    t0 = time.perf_counter()
    for r, s_, o in zip(reqs[:k0], sig[:k0], outs[:k0]):
        a, b = out_args(r, o.numpy())
        ctx.eval(gs[r.geometry], s_.numpy(), r.p, r.layers, out_slp=a, out_dlp=b)
    dt = time.perf_counter() - t0
    plain_rate, plain_rps = sum(per_req[:k0]) / dt, k0 / dt
    # saturation: everything submitted at once, after one untimed pass (the
    # first launches of the step kernels load their code)
    def saturation_pass(tuning=None):
        srv = ctx.server(budget, SERVE_SLOTS)
        if tuning:
            srv.set_tuning(**tuning)
        t0 = time.perf_counter()
        for r, s_, o in zip(reqs, sig, outs):
            a, b = out_args(r, o)
            srv.submit_pinned(gs[r.geometry], s_, r.p, r.layers, out_slp=a, out_dlp=b)
        srv.drain(600)
        dt = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return dt, st

    # the server autotuner on bursts of the same request mix and densities
    srv = ctx.server(budget, SERVE_SLOTS)
    default_tuning = srv.get_tuning()
    log("serving: autotuning the server")
    t0 = time.perf_counter()
    tuned, burst_ms = srv.autotune([(gs[r.geometry], r.p, r.layers) for r in reqs],
                                   n_requests=len(reqs), sigmas=sig)
    tune_s = time.perf_counter() - t0
    srv.close()
    log(f"serving: tuned {tuned}")
    serve_tuning = {"default": default_tuning, "tuned": tuned, "autotune_s": tune_s,
                    "tuned_burst_ms": burst_ms}
    log("serving: untimed warm-up pass")
    saturation_pass(tuned)
    log("serving: three timed saturation passes (pinned submissions)")
    passes = [saturation_pass(tuned) for _ in range(3)]
    sat_s, st_sat = sorted(passes, key=lambda x: x[0])[1]  # the median pass
    sat_rps = len(reqs) / sat_s
    # the copying submission path at saturation, for reference
    srv = ctx.server(budget, SERVE_SLOTS)
    srv.set_tuning(**tuned)
    k1 = min(len(reqs), 600)
    t0 = time.perf_counter()
    for r, s_ in zip(reqs[:k1], sig[:k1]):
        srv.submit(gs[r.geometry], s_.numpy(), r.p, r.layers)
    srv.drain(600)
    copy_rps = k1 / (time.perf_counter() - t0)
    srv.close()
    def open_loop(factor):
        """Poisson arrivals at factor x the saturation rate; returns (rate, wall, stats)."""
        rate = factor * sat_rps
        arrivals = np.array([r.arrival_s for r in reqs]) / rate  # unit-rate schedule scaled
        srv = ctx.server(budget, SERVE_SLOTS)
        srv.set_tuning(**tuned)
        log(f"serving: Poisson stream at {rate:.0f} requests/s ({factor}x saturation)")
        t0 = time.perf_counter()
        for r, s_, o, ta in zip(reqs, sig, outs, arrivals):
            while time.perf_counter() - t0 < ta:
                pass
            a, b = out_args(r, o)
            srv.submit_pinned(gs[r.geometry], s_, r.p, r.layers, out_slp=a, out_dlp=b)
        srv.drain(600)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return rate, wall, st

    rate, wall, st = open_loop(0.7)
    sweep = []
    for factor in (0.5, 0.9):
        rate_f, wall_f, st_f = open_loop(factor)
        sweep.append({"factor": factor, "offered_rps": rate_f,
                      "served_pair_terms_per_s": st_f["pair_terms_completed"] / wall_f,
                      "latency_p50_ms": st_f["latency_p50_ms"],
                      "latency_p99_ms": st_f["latency_p99_ms"],
                      "queue_p99_ms": st_f["queue_p99_ms"]})
    helm = bench_serve_helmholtz(ctx, torch, gs, reqs[:300])
    for g in gs:
        g.close()
    sat_stats = st_sat
    return {
        "helmholtz": helm,
        "tuning": serve_tuning,
        "workload": f"{n_requests} requests, Poisson arrivals at 0.7x saturation, 32 resident "
                    "geometries N log-uniform 4096..262144, p in {8,16}, single or double layer, "
                    "densities and outputs in pinned host memory",
        "offered_rps": rate,
        "saturation_rps": sat_rps,
        "saturation_rps_passes": [len(reqs) / p_[0] for p_ in passes],
        "served_pair_terms_per_s": st["pair_terms_completed"] / wall,
        "saturation_pair_terms_per_s": sum(per_req) / sat_s,
        "plain_sequential_pair_terms_per_s": plain_rate,
        "plain_sequential_rps": plain_rps,
        "speedup_saturation_vs_plain": (sum(per_req) / sat_s) / plain_rate,
        "copying_submit_saturation_rps": copy_rps,
        "latency_p50_ms": st["latency_p50_ms"],
        "latency_p90_ms": st["latency_p90_ms"],
        "latency_p99_ms": st["latency_p99_ms"],
        "latency_max_ms": st["latency_max_ms"],
        "queue_p50_ms": st["queue_p50_ms"],
        "queue_p99_ms": st["queue_p99_ms"],
        "other_loads": sweep,
        "steps": st["steps"],
        "peak_bytes_in_flight": st["peak_bytes_in_flight"],
        "budget_bytes": st["budget_bytes"],
        "saturation_steps": sat_stats["steps"],
        "saturation_host_launch_s": sat_stats["host_launch_s"],
        "saturation_busy_s": sat_stats["busy_s"],
        "saturation_wall_s": sat_s,
    }


def bench_serve_helmholtz(ctx, torch, gs, reqs, k=10.0):
    """Helmholtz requests (single + double layer, k = 10, each request's
    geometry and order) on the serving geometries, densities and outputs in
    pinned host memory: one plain synchronous tsqbx_eval_helmholtz per request
    against the server at saturation (pinned submissions)."""
    rng = np.random.default_rng(20181103)
    sig, outs = [], []
    for r in reqs:
        g = gs[r.geometry]
        t = torch.empty(g.n_sources, dtype=torch.complex128, pin_memory=True)
        t.numpy()[:] = rng.standard_normal(g.n_sources) + 1j * rng.standard_normal(g.n_sources)
        sig.append(t)
        outs.append([torch.empty(g.n_targets, dtype=torch.complex128, pin_memory=True)
                     for _ in range(2)])
    per_req = [gs[r.geometry].pair_terms(r.p, 3) for r in reqs]
    log(f"serving Helmholtz: {len(reqs)} plain synchronous calls")
    for r, s_, o in list(zip(reqs, sig, outs))[:20]:  # warm-up
        ctx.eval_helmholtz(gs[r.geometry], s_.numpy(), r.p, 3, k, o[0].numpy(), o[1].numpy())
    t0 = time.perf_counter()
    for r, s_, o in zip(reqs, sig, outs):
        ctx.eval_helmholtz(gs[r.geometry], s_.numpy(), r.p, 3, k, o[0].numpy(), o[1].numpy())
    plain_s = time.perf_counter() - t0
    srv = ctx.server(2 << 30, SERVE_SLOTS)
    for r, s_, o in list(zip(reqs, sig, outs))[:64]:  # untimed: first launches load code
        srv.submit_helmholtz_pinned(gs[r.geometry], s_, r.p, 3, k, out_slp=o[0], out_dlp=o[1])
    srv.drain(600)
    log("serving Helmholtz: saturation run")
    t0 = time.perf_counter()
    for r, s_, o in zip(reqs, sig, outs):
        srv.submit_helmholtz_pinned(gs[r.geometry], s_, r.p, 3, k, out_slp=o[0], out_dlp=o[1])
    srv.drain(600)
    sat_s = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return {"workload": f"{len(reqs)} Helmholtz requests (k={k:g}, single + double layer, p in "
                        "{8,16}) on the serving geometries, densities and outputs in pinned "
                        "host memory",
            "plain_sequential_rps": len(reqs) / plain_s,
            "saturation_rps": len(reqs) / sat_s,
            "saturation_pair_terms_per_s": sum(per_req) / sat_s,
            "speedup_saturation_vs_plain": plain_s / sat_s,
            "failed": st["failed"]}


def bench_host_call(ctx, g, geom, steps, p=16, layers=3):
    """The headline workload through the synchronous host-array call
    (tsqbx_eval): the density upload, the evaluation and the output downloads
    over PCIe, from and into pageable numpy arrays.  Reported beside the
    device-resident rate, never as the headline value."""
    sig = np.ascontiguousarray(g.sigma, dtype=np.float64)
    outs = [np.zeros(g.n_targets) for _ in range(2)]
    for _ in range(3):
        ctx.eval(geom, sig, p, layers, *outs)
    n = max(steps // 2, 5)
    log(f"timing the host-array call, {n} calls")
    t0 = time.perf_counter()
    for _ in range(n):
        ctx.eval(geom, sig, p, layers, *outs)
    dt = (time.perf_counter() - t0) / n
    return {"workload": "the headline workload through tsqbx_eval with host arrays (density "
                        "upload and output downloads over PCIe included)",
            "ms_per_call": dt * 1e3, "pair_terms_per_s": geom.pair_terms(p, layers) / dt,
            "host_bytes_per_call": 8 * g.n_sources + 8 * g.n_targets * 2}


def bench_sprime(ctx, api, torch, g, geom, steps, warmup):
    """S' (the target normal derivative of the single layer) on the headline
    workload: alone, and with the single and double layer in the same pass."""
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    outs = [torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) for _ in range(3)]
    res = {"workload": "perturbed sphere r=1+0.1f, 262144 sources, 65536 targets, ball lists "
                       "r=0.15, p=16, target normals of the surface"}
    p = 16
    for name, layers in (("sprime", 4), ("all_three", 7)):
        step = lambda: ctx.eval_async(geom, sig, p, layers, *outs)
        log(f"timing S' ({name}) {steps} steps")
        wall, ev = timed_steps(step, steps, warmup, torch)
        fpp = flops_per_pair(p, layers)
        ctx.stage_async(geom, sig, layers)
        kern = lambda: ctx.eval_staged_async(geom, p, layers, *outs)
        _, ev_k = timed_steps(kern, steps, warmup, torch)
        res[name] = {
            "layers": layers, "pair_terms_per_s": geom.pair_terms(p, layers) / (wall / steps),
            "ms_per_step": wall / steps * 1e3, "event_ms_per_step": ev / steps * 1e3,
            "tuning": ctx.get_tuning(p, layers, geom.pairs // g.n_targets),
            "roofline": roofline_obj(geom.pairs * fpp, ev_k / steps * 1e3,
                                     f"k_eval<16, {layers}, G, U>", flops_per_pair=fpp),
        }
    return res


def _cpow_flops(m: int) -> int:
    """FP64 operations of (w)^m by the kernel's squaring chain."""
    if m <= 1:
        return 0
    return _cpow_flops(m // 2) + 5 if m % 2 == 0 else _cpow_flops(m - 1) + 6


def conventional_flops_per_pair(p: int) -> int:
    """FP64 operations (fma = 2) per (source, center) pair of the conventional
    kernel's formation: for each order m, the source geometry and 1/|y-c|
    (21), (d_x - i d_y)^m / |y-c|^(2m+1) (4 + the squaring chain), the first
    two degrees and then 9 per further degree (5 for m = 0, which is real).
    The per-center lane sums and the per-target evaluation, O((p+1)^2) each,
    are left out (under 0.1 % on the workloads here)."""
    tot = 0
    for m in range(p + 1):
        f = 21 + (4 + _cpow_flops(m) if m else 0) + (2 if m else 1)
        if m < p:
            f += 4 if m else 2
        f += max(p - m - 1, 0) * (9 if m else 5)
        tot += f
    return tot


def bench_conventional(ctx, api, torch, W, g, geom, steps, warmup):
    """Target-specific single layer against conventional QBX (local coefficients
    formed per center from its list, then evaluated; the first approach of
    Sec. 2.4) on the same geometry, order and outputs.  The paper's claim is
    the cost ratio: O(p+1) per source-target pair against O((p+1)^2) per
    source-center pair."""
    res = {}
    cases = [("sphere262144", g, geom, (5, 8, 16))]
    ga = W.config_a()
    geom_a = ctx.geometry(ga)
    cases.append(("dense4096", ga, geom_a, (8,)))
    for name, gg, gm, orders in cases:
        sig = torch.tensor(gg.sigma, device="cuda", dtype=torch.float64)
        o1 = torch.zeros(gg.n_targets, device="cuda", dtype=torch.float64)
        o2 = torch.zeros(gg.n_targets, device="cuda", dtype=torch.float64)
        for p in orders:
            ts = lambda: ctx.eval_async(gm, sig, p, 1, o1)
            cv = lambda: ctx.eval_conventional_async(gm, sig, p, o2)
            log(f"timing target-specific vs conventional, {name} p={p}")
            w_ts, ev_ts = timed_steps(ts, steps, warmup, torch)
            w_cv, ev_cv = timed_steps(cv, max(steps // 4, 3), 2, torch)
            n_cv = max(steps // 4, 3)
            torch.cuda.synchronize()
            d = (o1 - o2).abs().max().item()
            scale = o1.abs().max().item()
            res[f"{name}_p{p}"] = {
                "pairs": gm.pairs, "n_targets": gg.n_targets, "p": p,
                "target_specific_ms": ev_ts / steps * 1e3,
                "conventional_ms": ev_cv / n_cv * 1e3,
                "speedup_target_specific": (ev_cv / n_cv) / (ev_ts / steps),
                "target_specific_pair_terms_per_s": gm.pair_terms(p, 1) / (ev_ts / steps),
                "target_specific_flops_per_pair": flops_per_pair(p, 1),
                "target_specific_tflops": gm.pairs * flops_per_pair(p, 1) / (ev_ts / steps) / 1e12,
                "conventional_flops_per_pair": conventional_flops_per_pair(p),
                "conventional_tflops": gm.pairs * conventional_flops_per_pair(p)
                / (ev_cv / n_cv) / 1e12,
                "max_abs_diff_over_max_abs": d / scale if scale > 0 else 0.0,
            }
        del sig, o1, o2
    geom_a.close()
    res["workload"] = ("single layer through tsqbx_eval_async (target-specific) and "
                       "tsqbx_eval_conventional_async (coefficients formed per center and "
                       "evaluated in one launch) on the p=16 perturbed sphere (262144 sources, "
                       "65536 targets) and the dense 4096-source sphere; times from HIP events, "
                       "staging included in both")
    return res


def helm_flops_per_pair(p: int, layers: int, sincos_flops: int = HELM_SINCOS_FLOPS) -> int:
    """FP64 operations per pair of the Helmholtz kernel (add/mul = 1,
    fma = 2, reciprocal-square-root estimate = 1), by the operations each
    layer adds.  Always: pair setup 27, sincos (as measured with FP64
    counters), h_0 and h_1 8, and per further order the Legendre (3) and
    Hankel (5) recurrences.  The single or double layer: the terms
    m_n = (2n+1) j_n P_n (table multiply and product, 2 per further order,
    1 at n = 1).  Single layer: the complex sum (2 at n = 0, 4 at n = 1 and
    per further order) and the product with the complex density (8).  P_n'
    (double layer or S'): 3 per further order.  Double layer: nu . d 5, the
    n = 0 and n = 1 terms 8 and 13, three complex sums (14 per further order)
    and the closing bracket with the density 30.  S': nu_t . d 5, the n = 0
    and n = 1 terms 2 and 9, two complex sums with their table multiply (11
    per further order) and the closing bracket with the density 17."""
    f = 27 + sincos_flops + 8
    orders = max(p - 1, 0)
    f += orders * 8
    if layers & 3:
        f += orders * 2 + (1 if p >= 1 else 0)
    if layers & 1:
        f += 2 + (4 if p >= 1 else 0) + orders * 4 + 8
    if layers & 6:
        f += orders * 3
    if layers & 2:
        f += 5 + 8 + (13 if p >= 1 else 0) + orders * 14 + 30
    if layers & 4:
        f += 5 + 2 + (9 if p >= 1 else 0) + orders * 11 + 17
    return f


def bench_helmholtz(ctx, api, torch, g, geom, steps, warmup, k=20.0, p=16):
    """Helmholtz single + double layer (the Brakhage-Werner pair of the
    paper's large experiment, k = 20) on the headline geometry; then the
    single layer alone, S' alone and all three layers."""
    rng = np.random.default_rng(20181101)
    sig = torch.tensor(rng.standard_normal(g.n_sources) + 1j * rng.standard_normal(g.n_sources),
                       device="cuda", dtype=torch.complex128)
    outs = [torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128) for _ in range(3)]
    res = {"workload": f"perturbed sphere r=1+0.1f, 262144 sources, 65536 targets, ball lists "
                       f"r=0.15, Helmholtz k={k:g}, p={p}, complex density"}
    for name, layers in (("slp_dlp", 3), ("slp", 1), ("sprime", 4), ("all_three", 7)):
        if layers & 4 and not geom.has_target_normals:
            continue
        step = lambda: ctx.eval_helmholtz_async(geom, sig, p, layers, k, *outs)
        log(f"timing Helmholtz ({name}) {steps} steps")
        wall, ev = timed_steps(step, steps, warmup, torch)
        fpp = helm_flops_per_pair(p, layers)
        achieved = geom.pairs * fpp / (ev / steps) / 1e12
        res[name] = {
            "layers": layers, "pair_terms_per_s": geom.pair_terms(p, layers) / (wall / steps),
            "ms_per_step": wall / steps * 1e3, "event_ms_per_step": ev / steps * 1e3,
            "flops_per_pair": fpp, "achieved_tflops": achieved,
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "kernel": f"k_helm_eval<{layers}, G, U> (+ k_helm_stage, k_helm_table)",
            "tuning": ctx.get_tuning(p, layers | api.HELMHOLTZ, geom.pairs // g.n_targets),
        }
    return res


def bench_shared(ctx, api, torch, W, steps, warmup):
    """Geometry B's sources with four near-surface targets per center (16384
    centers, 65536 targets, the same pairs per target): the row kernel (one
    list walk for four targets of a center, the plain path's default here)
    against one wave per target (TSQBX_PER_TARGET), single + double layer,
    p = 16, kernels alone on strengths staged once."""
    log("generating geometry B with four targets per center")
    g = W.config_b_shared(4)
    geom = ctx.geometry(g)
    p, layers = 16, 3
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    outs = {k: [torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) for _ in range(2)]
            for k in ("rows", "per_target")}
    ctx.stage_async(geom, sig, layers)
    flops = {"rows": geom.pairs * rows_flops_per_pair(p, layers),
             "per_target": geom.pairs * flops_per_pair(p, layers)}
    res = {"workload": "perturbed sphere r=1+0.1f, 262144 sources; 16384 centers 0.02 inside, "
                       "4 targets each on the segment to the surface (65536 targets); ball lists "
                       "r=0.15; p=16, single+double layer",
           "pairs": geom.pairs, "pair_terms": geom.pair_terms(p, layers)}
    for name, flags in (("rows", 0), ("per_target", api.PER_TARGET)):
        o = outs[name]
        kern = lambda: ctx.eval_staged_async(geom, p, layers, o[0], o[1], flags=flags)
        log(f"timing the {name} kernel, {steps} launches")
        _, ev = timed_steps(kern, steps, warmup, torch)
        ms = ev / steps * 1e3
        res[name] = {"kernel_ms_per_launch": ms,
                     "pair_terms_per_s": res["pair_terms"] / (ms / 1e3),
                     "roofline": roofline_obj(flops[name], ms, "k_eval_rows<16, 3>"
                                              if name == "rows" else "k_eval<16, 3, 64, 2>")}
    torch.cuda.synchronize()
    res["speedup_rows_vs_per_target"] = (res["per_target"]["kernel_ms_per_launch"] /
                                         res["rows"]["kernel_ms_per_launch"])
    res["identical_results"] = bool(all(torch.equal(a, b) for a, b in zip(outs["rows"],
                                                                          outs["per_target"])))
    geom.close()
    return res


def bench_lists(ctx, api, torch, g, steps, with_host=True):
    """Near-field ball lists of the headline workload (262144 sources, 65536
    centers, r = 0.15) built on the device, against the host grid generator
    that produced the workload's lists; then the k-nearest lists of one
    config D geometry against the host k-d tree."""
    src = torch.tensor(g.sources, device="cuda", dtype=torch.float64)
    ctr = torch.tensor(g.centers, device="cuda", dtype=torch.float64)
    off, idx = ctx.ball_lists(src, ctr, 0.15)  # sizes the output, warms up
    cap = int(idx.numel())
    torch.cuda.synchronize()
    n = max(steps // 4, 3)
    log(f"timing device ball lists, {n} builds")
    t0 = time.perf_counter()
    for _ in range(n):
        off, idx = ctx.ball_lists(src, ctr, 0.15, capacity=cap)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    # compulsory HBM bytes of a build: points read once, offsets and entries written
    ball_bytes = 24 * (g.n_sources + g.n_centers) + 8 * (g.n_centers + 1) + 4 * cap
    res = {"workload": "ball lists r=0.15 of the perturbed sphere: 262144 sources, 65536 centers",
           "entries": cap, "ms_per_build": dt * 1e3, "entries_per_s": cap / dt,
           "roofline": {"bound": "hbm", "achieved": ball_bytes / dt / 1e9, "peak": 8000.0,
                        "unit": "GB/s", "frac": ball_bytes / dt / 8e12, "traffic": None,
                        "algorithmic_bytes": ball_bytes},
           "same_as_host_generator": bool(np.array_equal(off.cpu().numpy(), g.list_offsets)
                                          and np.array_equal(idx.cpu().numpy(), g.list_sources))}
    # the device lists straight into a geometry, built on the device, against
    # the host build (layout on the host, then the upload) from the same lists
    def dev_arr(a, dtype):
        return None if a is None else torch.tensor(np.ascontiguousarray(a), device="cuda",
                                                   dtype=dtype)
    dev = dict(sources=src, weights=dev_arr(g.weights, torch.float64),
               normals=dev_arr(g.normals, torch.float64), centers=ctr, list_offsets=off,
               list_sources=idx.contiguous(), targets=dev_arr(g.targets, torch.float64),
               target_center=dev_arr(g.target_center, torch.int32))
    ctx.geometry_device(**dev).close()  # warm-up
    torch.cuda.synchronize()
    log(f"timing device geometry builds from the device lists, {n} builds")
    t0 = time.perf_counter()
    for _ in range(n):
        gd = ctx.geometry_device(**dev)
        gd.close()
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t0) / n
    gd = ctx.geometry_device(**dev)
    host_arrays = dict(sources=g.sources, weights=g.weights, normals=g.normals, centers=g.centers,
                       list_offsets=off.cpu().numpy(), list_sources=idx.cpu().numpy(),
                       targets=g.targets, target_center=g.target_center)
    log("timing a geometry from the same lists as host arrays, once")
    t0 = time.perf_counter()
    gh = api.Geometry(ctx, **host_arrays)  # uploads, then lays out on the device
    dh = time.perf_counter() - t0
    log("timing the host-only layout of the same lists, once")
    t0 = time.perf_counter()
    preview = api.geometry_layout(**host_arrays)
    dl = time.perf_counter() - t0
    a, b = gd.read_layout(), gh.read_layout()
    keys = ("source_order", "target_order", "target_row", "row_offsets", "rows")
    res["geometry_from_device_lists"] = {
        "device_ms_per_build": dg * 1e3, "host_arrays_ms_per_build": dh * 1e3,
        "host_layout_ms": dl * 1e3, "host_layout_over_device": dl / dg,
        "same_layout_as_host_layout": bool(all(np.array_equal(a[k], preview[k]) and
                                               np.array_equal(b[k], preview[k]) for k in keys))}
    gd.close()
    gh.close()
    from paper_1811_01110_amd import workloads as W

    if with_host:
        log("timing the host grid generator once")
        t0 = time.perf_counter()
        W.csr_ball(g.centers, g.sources, 0.15)
        res["host_generator_s"] = time.perf_counter() - t0
        res["host_generator_threads"] = min(16, os.cpu_count() or 1)
    # k nearest: one geometry of config D
    log("generating one config D geometry for the k-nearest lists")
    d = W.config_d(n_geometries=1)[0]
    counts = np.diff(d.list_offsets)
    src = torch.tensor(d.sources, device="cuda", dtype=torch.float64)
    ctr = torch.tensor(d.centers, device="cuda", dtype=torch.float64)
    cnt = torch.tensor(counts.astype(np.int32), device="cuda")
    off, idx = ctx.knn_lists(src, ctr, cnt)  # warm-up
    torch.cuda.synchronize()
    log(f"timing device k-nearest lists, {n} builds")
    t0 = time.perf_counter()
    for _ in range(n):
        off, idx = ctx.knn_lists(src, ctr, cnt)
    torch.cuda.synchronize()
    dk = (time.perf_counter() - t0) / n
    knn_bytes = 24 * (d.n_sources + d.n_centers) + 4 * d.n_centers + 8 * (d.n_centers + 1) + \
        4 * int(counts.sum())
    knn = {"workload": "k nearest of one config D geometry: 131072 sources on a perturbed "
                       "sphere, 32768 centers, k log-uniform 100..8000",
           "roofline": {"bound": "hbm", "achieved": knn_bytes / dk / 1e9, "peak": 8000.0,
                        "unit": "GB/s", "frac": knn_bytes / dk / 8e12, "traffic": None,
                        "algorithmic_bytes": knn_bytes},
           "entries": int(counts.sum()), "ms_per_build": dk * 1e3,
           "entries_per_s": float(counts.sum()) / dk,
           "same_as_host_kdtree": bool(np.array_equal(off.cpu().numpy(), d.list_offsets)
                                       and np.array_equal(idx.cpu().numpy(), d.list_sources))}
    if with_host:
        log("timing the host k-d tree lists once")
        t0 = time.perf_counter()
        W.csr_knn(d.centers, d.sources, counts)
        knn["host_kdtree_s"] = time.perf_counter() - t0
    res["knn"] = knn
    return res


def calibration_copy(torch):
    """One plain 256 MiB device-to-device copy: the known-size kernel that
    hardware byte counters (FETCH_SIZE, WRITE_SIZE) are scaled against."""
    src = torch.ones(1 << 25, device="cuda", dtype=torch.float64)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    global MIN_WARM_S, FIXED_PLAN_TUNING
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-high-order", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--min-warm", type=float, default=0.3,
                    help="seconds of warm-up work before each timed region")
    ap.add_argument("--no-sprime", action="store_true")
    ap.add_argument("--no-helmholtz", action="store_true")
    ap.add_argument("--no-lists", action="store_true")
    ap.add_argument("--no-conventional", action="store_true")
    ap.add_argument("--plan-tuning", default=None,
                    help="fixed plan tuning instead of the autotuner, e.g. group_lanes=16,unroll=2,"
                         "waves_per_block=2,oversubscription=16,step_cost=1000")
    ap.add_argument("--no-shared", action="store_true")
    ap.add_argument("--only", choices=["headline", "batched", "high_order", "serve", "sprime",
                                       "helmholtz", "helm_batched", "lists", "conventional",
                                       "shared"],
                    help="run one section (for profiling); the JSON line then carries only it")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run a 256 MiB device copy first (for counter calibration)")
    args = ap.parse_args()
    MIN_WARM_S = args.min_warm
    if args.plan_tuning:
        FIXED_PLAN_TUNING = {k: int(v) for k, v in
                             (kv.split("=") for kv in args.plan_tuning.split(","))}
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the evaluation shards by "
              "targets across GPUs, and this benchmark measures one GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1811_01110_amd import api
    from paper_1811_01110_amd import workloads as W

    if args.calibration_copy:
        calibration_copy(torch)
    if args.only and args.only not in ("headline", "sprime", "helmholtz", "lists",
                                       "conventional"):
        ctx = api.Context(0)
        fn = {"batched": bench_batched, "high_order": bench_d,
              "helm_batched": bench_helm_batched, "shared": bench_shared}.get(args.only)
        if fn is not None:
            res = fn(ctx, api, torch, W, args.steps, args.warmup)
        else:
            res = bench_serve(ctx, api, torch, W, args.requests)
        ctx.close()
        print(json.dumps({"section": args.only, args.only: res}), flush=True)
        return

    log("generating the p=16 perturbed-sphere workload")
    g = W.config_b()
    p, layers = 16, 3
    ctx = api.Context(0)
    geom = ctx.geometry(g)
    if args.only in ("sprime", "helmholtz", "lists", "conventional"):
        if args.only == "lists":
            res = bench_lists(ctx, api, torch, g, args.steps, with_host=False)
        elif args.only == "conventional":
            res = bench_conventional(ctx, api, torch, W, g, geom, args.steps, args.warmup)
        else:
            fn = bench_sprime if args.only == "sprime" else bench_helmholtz
            res = fn(ctx, api, torch, g, geom, args.steps, args.warmup)
        geom.close()
        ctx.close()
        print(json.dumps({"section": args.only, args.only: res}), flush=True)
        return
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    os_ = torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)
    od_ = torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)
    step = lambda: ctx.eval_async(geom, sig, p, layers, os_, od_)
    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    wall, ev = timed_steps(step, args.steps, args.warmup, torch)
    pair_terms = geom.pair_terms(p, layers)
    ms = wall / args.steps * 1e3
    flops = geom.pairs * flops_per_pair(p, layers)
    # the evaluation kernel alone: the same launches on the strengths staged once
    log("timing the evaluation kernel alone")
    ctx.stage_async(geom, sig, layers)
    kern = lambda: ctx.eval_staged_async(geom, p, layers, os_, od_)
    _, ev_k = timed_steps(kern, args.steps, args.warmup, torch)
    achieved = flops / (ev_k / args.steps) / 1e12
    per_launch = per_launch_ms(kern, args.steps, torch)
    tuning = ctx.get_tuning(p, layers, geom.pairs // geom.n_targets)

    out = {
        "metric": METRIC,
        "value": pair_terms / (ms / 1e3),
        "unit": "pair-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain single+double layer, p=16: perturbed sphere r=1+0.1f, 262144 "
                        "sources, 65536 targets, centers 0.02 inside, ball lists r=0.15",
            "p": p, "layers": "slp+dlp", "n_sources": g.n_sources, "n_targets": g.n_targets,
            "pairs": geom.pairs, "mean_list": geom.pairs / g.n_targets,
            "parallelism": "single GPU", "tuning": tuning,
        },
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(),
            "kernel": "k_eval<16, 3, G, U>", "kernel_ms_per_launch": ev_k / args.steps * 1e3,
            "kernel_ms_median": float(np.median(per_launch)), "kernel_ms_min": min(per_launch),
            "event_ms_per_step": ev / args.steps * 1e3,
            "flops_per_pair": flops_per_pair(p, layers),
            "separate_recurrences_flops_per_pair": separate_recurrence_flops_per_pair(p, layers),
        },
    }
    counters = measured_counters()
    if counters is not None:
        # the ceiling of this design: the vector-memory data path at full
        # occupancy (frac / td_busy) or every VALU issue slot used
        frac = out["roofline"]["frac"]
        counters["ceiling_frac"] = min(frac / counters["utilisation"]["td_busy"],
                                       counters["valu_full_issue_frac"])
        out["roofline"]["counters"] = counters
        out["roofline"]["bound"] = counters["bound"]
    if args.only == "headline":
        geom.close()
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    out["host_call"] = bench_host_call(ctx, g, geom, args.steps, p, layers)
    if not args.no_cpu:
        log("timing the CPU oracle on the same workload")
        out["cpu_baseline"] = cpu_baseline(g, p, layers)
    if not args.no_sprime:
        out["sprime"] = bench_sprime(ctx, api, torch, g, geom, args.steps, args.warmup)
    if not args.no_helmholtz:
        out["helmholtz"] = bench_helmholtz(ctx, api, torch, g, geom, args.steps, args.warmup)
    if not args.no_lists:
        out["lists"] = bench_lists(ctx, api, torch, g, args.steps, with_host=not args.no_cpu)
    if not args.no_conventional:
        out["conventional"] = bench_conventional(ctx, api, torch, W, g, geom, args.steps,
                                                 args.warmup)
    geom.close()
    del sig, os_, od_
    if not args.no_shared:
        out["shared_centers"] = bench_shared(ctx, api, torch, W, args.steps, args.warmup)
    if not args.no_batched:
        log("generating 64 batched geometries (mixed p)")
        geoms_c = W.config_c()
        out["batched"] = bench_batched(ctx, api, torch, W, args.steps, args.warmup, geoms_c)
        if not args.no_helmholtz:
            out["helmholtz_batched"] = bench_helm_batched(ctx, api, torch, W, args.steps,
                                                          args.warmup, geoms_c)
        del geoms_c
    if not args.no_high_order:
        out["batched_high_order"] = bench_d(ctx, api, torch, W, args.steps, args.warmup)
    if not args.no_serve:
        out["serving"] = bench_serve(ctx, api, torch, W, args.requests)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
