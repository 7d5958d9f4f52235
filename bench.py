#!/usr/bin/env python3
"""Benchmark of the IRE tracing hot path on one MI355X.

One step = one complete IRE run of the benchmark cloud: zero the absorbed-
energy accumulators, trace every package (launch, shell stepping, scattering,
absorption with immediate re-emission, escape), and finalize the per-shell
temperatures into device memory.  The model's tables and shells are resident
on the device before the timed region (they are built once per model).

Prints ONE JSON line (see the fields below).  `roofline` reports the tracing
kernel against the VALU issue peak: algorithmic work = sum over event types of
(events of that type in the launch) x (VALU instructions that event's path
executes per lane), divided by the kernel duration measured with HIP events on
the launch stream.  `cpu_baseline` times the FP64 oracle on the host cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU instructions one lane executes per event on the FP32 tracer's paths:
# a crossing is one sweep step, and a launch, scattering or absorption is its
# own path plus the step that found it (least-squares fit of SQ_INSTS_VALU
# over one-lane runs of six clouds, with the sweeps' steps fitted apart from
# the events so that steps that move nothing after the lane parked are not
# counted as work; profiles/valu_fit_one_lane_clouds.md holds the fit and its
# command).
VALU_PER_EVENT = {"cross": 17.15, "launch": 236.77, "scat": 240.30, "abs": 266.73}

# HBM bytes per tracer launch from FETCH_SIZE and WRITE_SIZE, scaled by a
# plain 1 GiB copy (profiles/ire_trace_f32_ext101_tauV10_1e8.md); valid for
# the tracer as profiled and set to None whenever the kernel changes.
TRAFFIC_BYTES = {"ext101_tauV10_1e8": 6.068e8}

# MI355X VALU lane-instruction issue peak: the published FP32 vector rate of
# 157.3 TFLOP/s is 78.6e12 FMAs per second, i.e. 256 CUs x 4 SIMDs x 32 lanes
# at 2.4 GHz.  Plain (unpacked) FP32 instructions reach it: a stream of
# independent v_fma_f32 / v_add_f32 measures 5.5-5.8e13 lane-operations per
# second on the device (profiles/valu_issue_rate.md), above the 16-lane
# figure of 3.9e13 an older reading of the peak used; the hardware
# transcendentals run at a quarter of the plain rate.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12

WORKLOADS = {
    # name: (factory, packages, description)
    "ext101_tauV10_1e8": ("cfg_external_large", 100_000_000,
                          "external sphere, 101 equal shells, central tau_V=10, 1e8 packages"),
    "central200_tauV100_1e8": ("cfg_central", 100_000_000,
                               "central 5000 K 1 Lsun source, 200 log shells 10 AU-0.1 pc, tau_V=100, 1e8 packages"),
    "ext50_tauV1_1e5": ("cfg_external_small", 100_000,
                        "external sphere, 50 equal shells, central tau_V=1, 1e5 packages"),
    "batch4096": ("batch_parameters", None,
                  "batched study: 4096 models, shells U{20..400}, tau_V logU(0.1,1000), density exponent U(0,2), "
                  "external or central source, packages logU(1e5,1e7), one persistent launch"),
    "surrogate1e6": ("batch_parameters", None,
                     "learned surrogate: MLP 6(+log r) -> 4x256 SiLU -> log10 T, 5-member BF16 ensemble trained on "
                     "batched IRE runs of the study generator; inference on 1e6 models with IRE fallback where "
                     "the ensemble spread exceeds 2 %"),
}


def algorithmic_ops(stats: dict) -> float:
    return (VALU_PER_EVENT["cross"] * stats["n_cross"] + VALU_PER_EVENT["launch"] * stats["n_launch"]
            + VALU_PER_EVENT["scat"] * stats["n_scat"] + VALU_PER_EVENT["abs"] * stats["n_abs"])


def host_cpu() -> dict:
    """The host's processor: model name, logical CPUs, CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(model: dict, key: str, n_one: int, n_all: int, seeds: int, note: str) -> dict:
    """The serial FP64 oracle on the host: one run on one core, and `seeds`
    independent runs on the cores of this GPU's share of the host (at most 16
    threads: the share of one GPU on these hosts).  `value` is the all-core
    aggregate rate."""
    import oracle
    oracle.build(force=False)
    cpu = host_cpu()
    threads = max(1, min(16, cpu["usable_cpus"]))
    t0 = time.perf_counter()
    oracle.run(model, seed=1, **{key: n_one})
    one = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.ensemble(model, seeds=range(1, seeds + 1), threads=threads, **{key: n_all})
    dt = time.perf_counter() - t0
    return {"value": seeds * n_all / dt, "unit": "packages/s", "cores": threads, "kind": "oracle",
            "one_core_packages_per_s": n_one / one,
            "sample": f"{seeds} independent seeds x {n_all:,} packages of the same cloud on {threads} threads "
                      f"({dt:.1f} s wall), and one run of {n_one:,} packages on one core ({one:.1f} s); serial FP64 "
                      f"oracle ({note})",
            **cpu}


def bench_batch(args) -> dict:
    """Models/s of the batched study in one persistent launch (HIP-graph replay),
    against per-model launches of a random sample of the same models."""
    import numpy as np
    import torch

    from paper_2408_13807_amd import ire, workloads

    scale = float(os.environ.get("IRE_BENCH_BATCH_SCALE", "1.0"))
    params = workloads.batch_parameters(4096, seed=3)
    torch.cuda.set_device(0)
    b = ire.batch_from_workloads(params, package_scale=scale)
    # schedule knobs for experiments (defaults otherwise)
    knobs = {k: int(os.environ[e]) for k, e in (("aggregate", "IRE_BENCH_AGG"), ("batch", "IRE_BENCH_BATCH"),
                                                ("item_packages", "IRE_BENCH_ITEM")) if e in os.environ}
    if knobs:
        b.set_options(**knobs)
    n_pkg = int(sum(max(1, round(int(x) * scale)) for x in params["n_pkg"]))
    for w in range(args.warmup):
        b.run()
        b.results(allow_limit=True)
    ms, ev = [], None
    t0 = time.perf_counter()
    for s in range(args.steps):
        b.run()
        st = b.results(allow_limit=True)["stats"]
        ms.append(st["ms_run"])
        ev = st if ev is None else {k: ev[k] + st[k] for k in ("n_cross", "n_launch", "n_scat", "n_abs", "n_pass", "n_step_slots")}
    t1 = time.perf_counter()
    b.close()
    # per-model launches of a sample of the same models (same budgets)
    rng = np.random.default_rng(0)
    sample = rng.choice(4096, 64, replace=False)
    t_single = 0.0
    for m in sample:
        mm = workloads.batch_model(params, int(m))
        key = "n_ps" if params["central"][m] else "n_ext"
        npk = max(1, round(int(params["n_pkg"][m]) * scale))
        ts = time.perf_counter()
        ire.run_model(mm, seed=int(params["seed"][m]) & 0xFFFFFFFF, allow_limit=True, **{key: npk})
        t_single += time.perf_counter() - ts
    single_models_per_s = len(sample) / t_single
    k_ms = sum(ms) / len(ms)
    per_launch = {k: ev[k] / args.steps for k in ("n_cross", "n_launch", "n_scat", "n_abs", "n_pass", "n_step_slots")}
    achieved = algorithmic_ops(per_launch) / (k_ms * 1e-3) / 1e12
    value = 4096 * args.steps / (t1 - t0)
    return {
        "metric": "models/s (IRE, batched parameter study in one persistent launch)",
        "value": value, "unit": "models/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["batch4096"][2], "models": 4096, "packages": n_pkg,
                   "package_scale": scale, "stepping": "fp32", "accumulators": "fp64"},
        "packages_per_s": n_pkg * args.steps / (t1 - t0),
        "device_ms_avg": k_ms,
        "events_per_launch": per_launch,
        "per_model_launch_models_per_s": single_models_per_s,
        "per_model_sample": "64 random models of the study, one ire_run each, same package budgets",
        "speedup_vs_per_model": value / single_models_per_s,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s (VALU lane-instructions)", "frac": achieved / VALU_PEAK_TOPS, "traffic": None},
    }


def bench_surrogate(args) -> dict:
    """Models/s of surrogate inference with IRE fallback on 1e6 study models,
    with the surrogate's T error against IRE on held-out models, next to the
    batched IRE's models/s on a sample of the same models."""
    import numpy as np
    import torch

    from paper_2408_13807_amd import surrogate as S, workloads as wl

    env = os.environ.get
    n_train = int(env("IRE_SUR_TRAIN_MODELS", "200000"))
    train_scale = float(env("IRE_SUR_TRAIN_SCALE", "1.0"))
    fit_steps = int(env("IRE_SUR_STEPS", "60000"))
    n_eval = int(env("IRE_SUR_EVAL_MODELS", "1024"))
    ref_scale = float(env("IRE_SUR_REF_SCALE", "16.0"))
    n_inf = int(env("IRE_SUR_MODELS", "1000000"))
    thr = float(env("IRE_SUR_THRESHOLD", "0.02"))
    torch.cuda.set_device(0)
    note = {}

    def say(msg):
        print(f"[surrogate bench] {msg}", file=sys.stderr, flush=True)

    def chunks(what):
        return lambda done, total, secs: say(f"{what}: {done}/{total} models, {secs:.1f} s of IRE")

    # training set and fit (one-time cost, reported)
    pt = wl.batch_parameters(n_train, seed=101)
    t0 = time.perf_counter()
    r = S.ire_profiles(pt, np.arange(n_train), package_scale=train_scale, progress=chunks("training data"))
    X, y = S.training_set(pt, np.arange(n_train), r["T"])
    t1 = time.perf_counter()
    say(f"fitting the ensemble on {len(y)} rows, {fit_steps} steps")
    net = S.fit(X, y, steps=fit_steps, batch=4096, seed=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say(f"fit done in {t2 - t1:.1f} s")
    note.update(train_models=n_train, train_package_scale=train_scale, train_rows=int(len(y)),
                train_data_s=t1 - t0, fit_steps=fit_steps, fit_s=t2 - t1,
                final_loss=[float(v) for v in net.last_loss])

    # accuracy on held-out models: the surrogate and the tracer at 1x and 4x each
    # model's budget against IRE at ref_scale x the budget (independent seeds)
    pe = wl.batch_parameters(n_eval, seed=202)
    ev = np.arange(n_eval)

    def reseeded(k):
        q = dict(pe)
        q["seed"] = pe["seed"] + np.uint64(k << 20)
        return q

    ref = S.ire_profiles(pe, ev, package_scale=ref_scale, progress=chunks("reference"))
    own = S.ire_profiles(reseeded(1), ev, package_scale=1.0, progress=chunks("IRE at 1x"))
    own4 = S.ire_profiles(reseeded(2), ev, package_scale=4.0, progress=chunks("IRE at 4x"))
    p = S.predict_models(net, pe, ev)
    Ts = 10.0 ** p["logT"].astype(np.float64)
    acc = p["model_spread"] <= thr
    summary = S.error_summary(Ts, ref["T"], ref["row_off"], acc, {"ire_1x": own["T"], "ire_4x": own4["T"]})
    # the fallback gate at other spread thresholds: accepted share and models within 2 % (worst shell)
    gates = {}
    for g in (0.005, 0.01, 0.02, 0.03, 0.05):
        a = p["model_spread"] <= g
        gs = S.error_summary(Ts, ref["T"], ref["row_off"], a, {"ire_1x": own["T"]})
        gates[f"{g:g}"] = {"accepted_fraction": float(a.mean()),
                           "after_fallback_within_2pct_max": gs["max"]["after_fallback"],
                           "after_fallback_within_2pct_p95": gs["p95"]["after_fallback"],
                           "accepted_within_2pct_max": gs["max"]["surrogate_accepted"]}
    note.update(eval_models=n_eval, eval_reference=f"IRE at {ref_scale:g}x each model's package budget",
                error_definitions="per model, over its shells, of |T - T_ref| / T_ref: the worst shell (max), the 95th "
                                  "percentile (p95) and the median; fractions of models within 2 % by each",
                accepted_fraction=float(acc.mean()), errors=summary, gate_thresholds=gates)

    # timed inference on n_inf models: inputs resident in HBM
    pi = wl.batch_parameters(n_inf, seed=303)
    q = wl.study_model_inputs(pi)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    mx, ro, ra, rad = dev(q["model_x"]), dev(q["row_off"]), dev(q["radius_off"]), dev(q["radius"])
    n_rows = int(q["row_off"][-1])
    mean = torch.empty(n_rows, dtype=torch.float32, device="cuda")
    spread = torch.empty_like(mean)
    mspread = torch.empty(n_inf, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        net.predict_models_dev(n_inf, n_rows, mx.data_ptr(), ro.data_ptr(), ra.data_ptr(), rad.data_ptr(),
                               len(q["radius"]), mean.data_ptr(), spread.data_ptr(), mspread.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    t_pred, t_fb, n_flag, fb = [], [], 0, None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        net.predict_models_dev(n_inf, n_rows, mx.data_ptr(), ro.data_ptr(), ra.data_ptr(), rad.data_ptr(),
                               len(q["radius"]), mean.data_ptr(), spread.data_ptr(), mspread.data_ptr(), stream=stream)
        torch.cuda.synchronize()
        t_pred.append(time.perf_counter() - ts)
        flagged = np.nonzero(mspread.cpu().numpy() > thr)[0]
        n_flag = len(flagged)
        say(f"predicted {n_inf} models in {t_pred[-1]:.2f} s; {n_flag} flagged for the IRE fallback")
        tf0 = time.perf_counter()
        if n_flag:
            fb = S.ire_profiles(pi, flagged, package_scale=1.0, progress=chunks("fallback"))
        t_fb.append(time.perf_counter() - tf0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    value = n_inf * args.steps / (t1 - t0)

    # plain batched IRE on a sample of the same models (same budgets)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(n_inf, 4096, replace=False))
    ts = time.perf_counter()
    S.ire_profiles(pi, sample, package_scale=1.0, progress=chunks("batched IRE sample"))
    ire_mps = len(sample) / (time.perf_counter() - ts)
    # the network's dense FLOPs: 7 inputs (6 parameters and log r), depth hidden
    # layers of 256 and the output layer (the MFMA pads the inputs to 32: 3 % more work)
    flop = 2.0 * n_rows * net.members * (7 * 256 + (net.depth - 1) * 256 * 256 + 256)
    pred_s = sum(t_pred) / len(t_pred)
    achieved = flop / pred_s / 1e12
    net.close()
    note.update(inference_models=n_inf, inference_rows=n_rows, predict_s=pred_s,
                fallback_models=n_flag, fallback_s=sum(t_fb) / len(t_fb),
                fallback_device_s=fb["device_s"] if fb else 0.0, fallback_events=fb["events"] if fb else None,
                ire_batched_models_per_s=ire_mps, ire_sample="4096 random models of the same 1e6, one batched launch",
                speedup_vs_batched_ire=value / ire_mps)
    return {
        "metric": "models/s (surrogate inference with IRE fallback at 2 % ensemble spread)",
        "value": value, "unit": "models/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": WORKLOADS["surrogate1e6"][2], "models": n_inf},
        "surrogate": note,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "kernel": "sur_predict_kernel (prediction only, dense BF16 MFMA FLOPs of all members)"},
    }


def bench_single(args, workload: str, variants: bool, cpu: bool) -> dict:
    """Packages/s of one cloud model: each step a complete IRE run into device memory."""
    import torch

    from paper_2408_13807_amd import ire, workloads

    factory, n_pkg, desc = WORKLOADS[workload]
    model = getattr(workloads, factory)()
    key = "n_ps" if model.get("J") is None else "n_ext"
    n = len(model["rho"])
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    A = torch.zeros(n, dtype=torch.float64, device="cuda")
    T = torch.zeros(n, dtype=torch.float64, device="cuda")

    h = ire.IREModel(0)
    h.set_model(model)
    base_opts = dict(batch=int(os.environ.get("IRE_BENCH_BATCH", "0")),
                     aggregate=int(os.environ.get("IRE_BENCH_AGG", "-1")),
                     quorum=int(os.environ.get("IRE_BENCH_QUORUM", "0")), replicas=args.replicas)
    h.set_options(**base_opts)
    if args.tune:
        # event-pass schedule timed on this cloud before the warm-up (a sample of the run)
        q, b = h.tune_schedule(**{key: n_pkg})
        base_opts.update(quorum=q, batch=b)
    schedule = {"tuned": bool(args.tune), "quorum": base_opts["quorum"] or "default",
                "parked_lanes": base_opts["batch"] or "default"}

    def step(seed: int):
        h.run(seed=seed, stream=stream, **{key: n_pkg})
        h.results_dev(A.data_ptr(), T.data_ptr(), stream=stream)

    for w in range(args.warmup):
        step(10_000 + w)
    torch.cuda.synchronize()

    kernel_ms = []
    events = None
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(1 + s)
        st = h.stats()           # synchronises; tracing-kernel time from HIP events on `stream`
        kernel_ms.append(st["ms_trace"])
        events = st if events is None else {k: events[k] + st[k] for k in ("n_cross", "n_launch", "n_scat", "n_abs", "n_pass", "n_step_slots")}
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    # the optional weightings of the same cloud (reported, not the value): centre-weighted
    # background directions (Eq. 5, k_bg = 0.2) and the forced first interaction (Eqs. 9-12);
    # and eight independent accumulator groups instead of one running total per shell
    out_variants = {}
    variant_opts = (("k_bg=0.2", dict(k_bg=0.2)), ("ffi", dict(ffi=1)), ("k_bg=0.2+ffi", dict(k_bg=0.2, ffi=1)),
                    ("replicas=8", dict(replicas=8)))
    for vname, vopt in variant_opts if variants else ():
        h.set_options(**{**base_opts, **vopt})
        ms = []
        for s in range(2):
            step(20_000 + s)
            ms.append(h.stats()["ms_trace"])
        out_variants[vname] = {"kernel_ms": ms[-1], "kernel_packages_per_s": n_pkg / (ms[-1] * 1e-3),
                               "T_center_K": float(T[0].item())}
    h.set_options(**base_opts)

    # PCIe-inclusive rate: host model in, host results out (reported, not the value)
    tp0 = time.perf_counter()
    h.set_model(model)
    h.run(seed=99, **{key: n_pkg})
    host_res = h.results()
    tp1 = time.perf_counter()

    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n_pkg * args.steps / (t1 - t0)
    k_ms = sum(kernel_ms) / len(kernel_ms)
    per_launch = {k: events[k] / args.steps for k in ("n_cross", "n_launch", "n_scat", "n_abs", "n_pass", "n_step_slots")}
    ops = algorithmic_ops(per_launch)
    achieved = ops / (k_ms * 1e-3) / 1e12
    line = {
        "metric": "photon packages/s (IRE tracing, one cloud model)",
        "value": value,
        "unit": "packages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "shells": n, "packages": n_pkg,
                   "stepping": "fp32", "accumulators": "fp64", "accumulator_groups": args.replicas,
                   "event_pass_schedule": schedule, "parallelism": "single GPU"},
        "kernel_ms_avg": k_ms,
        "kernel_packages_per_s": n_pkg / (k_ms * 1e-3),
        "events_per_launch": per_launch,
        "pcie_inclusive_packages_per_s": n_pkg / (tp1 - tp0),
        "T_center_K": float(host_res["T"][0]),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s (VALU lane-instructions)", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": TRAFFIC_BYTES.get(workload) if args.replicas == 1 else None,
                     "limiter": "workgroup-wide event passes (barrier waits, parked lanes) that keep the returning "
                                "FP64 atomics on the shells' accumulators (one address per shell) few"
                     if args.replicas == 1 else "VALU issue"},
    }
    if variants:
        line["variants"] = out_variants
    if cpu:
        line["cpu_baseline"] = cpu_baseline(model, key, 3_000_000, 3_000_000, 16, "same cloud")
    h.close()
    return line


def say(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ext101_tauV10_1e8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--replicas", type=int, default=1,
                    help="accumulator groups of the timed single-model launch (1: one running total per shell)")
    ap.add_argument("--tune", action="store_true",
                    help="time candidate event-pass schedules on the cloud first and use the fastest")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the weighted and replica variants (profiling runs of the default launch)")
    ap.add_argument("--only", action="store_true",
                    help="the chosen workload alone (the default run adds the central-source cloud, the batched "
                         "study and the surrogate to the benchmark cloud's line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2

    if args.workload == "batch4096":
        print(json.dumps(bench_batch(args)), flush=True)
        return 0
    if args.workload == "surrogate1e6":
        print(json.dumps(bench_surrogate(args)), flush=True)
        return 0

    line = bench_single(args, args.workload, variants=not args.no_variants, cpu=not args.no_cpu_baseline)
    say(f"{args.workload}: {line['value']:.4g} packages/s, VALU fraction {line['roofline']['frac']:.3f}")
    if args.only or args.workload != "ext101_tauV10_1e8":
        print(json.dumps(line), flush=True)
        return 0
    # the other configurations of the study, each with its own timing, roofline and one-time costs
    sub = argparse.Namespace(**vars(args))
    # the central source's absorptions crowd into its innermost shells, and the
    # schedule tuner (ire_tune_schedule, timed on a sample of the run before the
    # warm-up) picks smaller event passes for it
    sub.steps, sub.warmup, sub.replicas, sub.tune = 5, 2, 1, True
    c = bench_single(sub, "central200_tauV100_1e8", variants=False, cpu=False)
    line["central_source"] = {k: c[k] for k in ("metric", "value", "unit", "steps", "warmup", "ms_per_step", "config",
                                                "kernel_ms_avg", "kernel_packages_per_s", "events_per_launch",
                                                "roofline")}
    say(f"central source: {c['value']:.4g} packages/s, VALU fraction {c['roofline']['frac']:.3f}")
    sub.steps, sub.warmup = 2, 1
    line["batched_study"] = bench_batch(sub)
    say(f"batched study: {line['batched_study']['value']:.4g} models/s")
    sub.steps, sub.warmup = 1, 1
    line["surrogate"] = bench_surrogate(sub)
    say(f"surrogate: {line['surrogate']['value']:.4g} models/s")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
