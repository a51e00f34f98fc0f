#!/usr/bin/env python
"""Benchmark: fused selected inversion + selected quadratic solve (SI+SQ) on one MI355X.

One step = one fused SI+SQ solve (factor of A, forward B-chain, backward SI and
SQ sweeps) of the workload, with A and B already resident in HBM.  Prints one
JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload bt_n64_b512]
                    [--partitions P] [--compare-partitions Q ...] [--no-cpu-baseline]

Without --partitions every form the workload names is timed (sequential RGF
and the partitioned variant); the value is the fastest of them and the others
are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 MFMA
FP32_PEAK_TFLOPS = 157.3    # MI355X dense FP32 MFMA
HBM_PEAK_GBS = 8000.0
METRIC = "SI+SQ solves/s, % FP64/FP32 MFMA peak, p50/p99 latency vs plain RGF"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def latency_summary(xs):
    """Per-solve times in ms: p50 and p99, the mean, and the half-width of the
    mean's 95% confidence interval (Student t over the timed solves)."""
    n = len(xs)
    mean = sum(xs) / n
    out = {"p50": round(percentile(xs, 50), 3), "p99": round(percentile(xs, 99), 3),
           "mean": round(mean, 3)}
    if n > 1:
        from scipy.stats import t as student_t
        sd = (sum((x - mean) ** 2 for x in xs) / (n - 1)) ** 0.5
        out["ci95"] = round(float(student_t.ppf(0.975, n - 1)) * sd / n ** 0.5, 3)
    return out


def time_solves(torch, sol, dA, dB, XR, XL, steps, warmup):
    for _ in range(warmup):
        sol.solve(dA, dB, XR, XL)
    sol.sync()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        sol.solve(dA, dB, XR, XL)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol.sync()
    lat = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return t1 - t0, lat


def measured_traffic(kernel, workload, partitions):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated
    against a plain copy) as last measured with rocprofv3 counters, or None if
    there is no measurement for this workload or a source it depends on (the
    kernel, and the scheduler that decides what each launch holds) changed
    since."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(root, "profiles", "traffic.json")) as f:
            rec = json.load(f).get(kernel)
        if not rec or rec["workload"] != workload or rec["partitions"] != partitions:
            return None
        for src, digest in rec["sources_sha256"].items():
            with open(os.path.join(root, src), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def oracle_floor(workload, partitions):
    """What the oracle alone says about FP64 rounding on this workload (stored
    by tests/golden/make_fullsize_floors.py, which calls only the oracle):
    the spread of two oracle evaluations of the reported form whose rounding
    differs ("floor") and the oracle's own difference between this form's
    ordering and the sequential sweep ("vs_sequential"), which bounds what a
    correct GPU result can be held to against the sequential oracle."""
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(root, "tests", "golden", f"fullsize_floors_{workload}.json")) as f:
            rec = json.load(f)["forms"].get(f"P{partitions}")
    except (OSError, ValueError, KeyError):
        return None
    if not rec:
        return None
    out = {"floor": rec.get("floor")}
    if "vs_sequential" in rec:
        out["vs_sequential"] = rec["vs_sequential"]
    return out


def cpu_baseline(A, B, seconds, XR_gpu, XL_gpu):
    """The oracle (sequential RGF, NumPy complex128) on the host cores, bounded sample."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 0) for p in threadpool_info()] or [0])
    except Exception:
        threads = 0
    cores = threads or len(os.sched_getaffinity(0))
    n_done, t_total, res = 0, 0.0, None
    while t_total < seconds and n_done < 5:
        t0 = time.perf_counter()
        res = oracle.rgf_bta(A, B) if A.tip.shape[0] else oracle.rgf_bt(A, B)
        t_total += time.perf_counter() - t0
        n_done += 1
        if t_total / n_done * (n_done + 1) > 2.0 * seconds:
            break
    # parity of the timed GPU result against this oracle run (same inputs)
    def blocks(M, f):
        v = getattr(M, f)
        if isinstance(v, (list, tuple)):                    # blocks of different sizes
            return [np.asarray(x) for x in v if np.size(x)]
        v = np.asarray(v)
        if v.size == 0:
            return []
        return [v] if v.ndim == 2 else list(v)

    def rel(X, R):
        worst = 0.0
        fields = ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip")
        big = max((np.linalg.norm(r) for f in fields for r in blocks(R, f)), default=0.0)
        for f in fields:
            for x, r in zip(blocks(X, f), blocks(R, f)):
                den = max(np.linalg.norm(r), 1e-6 * big)
                worst = max(worst, float(np.linalg.norm(x - r) / den))
        return worst
    errR = rel(XR_gpu, res[0])
    errL = rel(XL_gpu, res[1])
    return dict(value=n_done / t_total, unit="solves/s", cores=cores, kind="oracle",
                sample=f"{n_done} full sequential RGF solve(s) of the same workload "
                       f"(NumPy complex128, {t_total:.1f} s)"), (errR, errL)


def bench_batch(args, torch, S):
    """Uneven batched energy sweep: mixed batched vs FP64 batched vs plain per-instance RGF."""
    from paper_2601_04904_amd.synth import batch_specs
    from paper_2601_04904_amd.synth_device import gen_problem_device
    specs_all = batch_specs(512)
    specs = specs_all[: args.batch_count]
    log(f"[bench] batch of {len(specs)} uneven instances (first of the 512-instance sweep)")
    probs = [gen_problem_device(sp["n"], sp["b"], sp["a"], sp["E"], sp["eta"], sp["seed"]) for sp in specs]
    torch.cuda.synchronize()
    flops = sum(S.flops(sp["n"], sp["b"], sp["a"], 1)[0] for sp in specs)

    def run_batched(precision, waves, router=None):
        out = {}
        t_total = 0.0
        errs, fbs = [], []
        for w0 in range(0, len(specs), waves):
            sub = list(range(w0, min(len(specs), w0 + waves)))
            precs = [router.choose(specs[i]["eta"], specs[i]["a"],
                                   S.flops(specs[i]["n"], specs[i]["b"], specs[i]["a"], 1)[0])
                     if router else precision for i in sub]
            wspecs = [dict(n=specs[i]["n"], b=specs[i]["b"], a=specs[i]["a"], precision=pr, flags=args.flags)
                      for i, pr in zip(sub, precs)]
            XR = [S.DeviceBlocks.empty(specs[i]["n"], specs[i]["b"], specs[i]["a"]) for i in sub]
            XL = [S.DeviceBlocks.empty(specs[i]["n"], specs[i]["b"], specs[i]["a"]) for i in sub]
            bs = S.BatchSolver(wspecs)
            A = [probs[i][0] for i in sub]
            B = [probs[i][1] for i in sub]
            bs.solve(A, B, XR, XL)   # warm-up: builds and uploads the schedule
            bs.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, f = bs.solve(A, B, XR, XL)
            bs.sync()
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            errs += e
            fbs += f
            if router:
                for i, pr, fb in zip(sub, precs, f):
                    if pr == S.BT_MIXED:
                        router.record(specs[i]["eta"], specs[i]["a"], fb)
            bs.destroy()
            del XR, XL
        out["solves_per_s"] = round(len(specs) / t_total, 3)
        out["tflops_executed"] = round(flops / t_total / 1e12, 3)
        out["seconds"] = round(t_total, 3)
        if precision == S.BT_MIXED:
            out["max_err_estimate"] = max(errs)
            out["fp64_fallbacks"] = int(sum(fbs))
        if router:
            out["routed_to_fp64"] = router.routed
        return out

    from paper_2601_04904_amd.serving import PrecisionRouter
    mixed_spec = run_batched(S.BT_MIXED, args.batch_wave)
    log(f"[bench] mixed batched, every instance tried in mixed precision: {mixed_spec}")
    mixed = run_batched(S.BT_MIXED, args.batch_wave,
                        router=PrecisionRouter(probe_max_flops=args.probe_max_tflop * 1e12 / 20))
    log(f"[bench] mixed batched with precision routing: {mixed}")
    fp64 = run_batched(S.BT_FP64, args.batch_wave)
    log(f"[bench] fp64 batched: {fp64}")
    # plain RGF: FP64, one instance at a time, one launch per block product, one stream
    nplain = len(specs) if args.plain_count < 0 else min(len(specs), args.plain_count)
    t_plain = 0.0
    for i in range(nplain):
        sp = specs[i]
        sol = S.Solver(sp["n"], sp["b"], sp["a"], flags=S.BT_PLAIN)
        XR, XL = S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]), S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"])
        sol.solve(probs[i][0], probs[i][1], XR, XL)
        sol.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.solve(probs[i][0], probs[i][1], XR, XL)
        sol.sync()
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        sol.destroy()
        if (i + 1) % 64 == 0:
            log(f"[bench] plain RGF: {i + 1} of {nplain} instances, {t_plain:.1f} s timed")
    plain = dict(solves_per_s=round(nplain / t_plain, 3), instances=nplain)
    log(f"[bench] plain RGF: {plain}")
    out = {
        "metric": METRIC, "value": mixed["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * len(specs) / mixed["solves_per_s"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": f"batch_{len(specs)}_uneven", "n": "U{16..96}", "b": "U{64..384}",
                   "a": "U{0,128,256}", "eta": 1e-3, "wave": args.batch_wave, "hip_graph": bool(args.graph),
                   "tile_shapes": "autotuned" if args.tuned else "default rule"},
        "mixed_batched": mixed, "mixed_batched_no_routing": mixed_spec, "fp64_batched": fp64, "plain_rgf": plain,
        "mixed_vs_plain_rgf": round(mixed["solves_per_s"] / plain["solves_per_s"], 3),
        "pct_fp32_peak_mixed_executed": round(100 * mixed["tflops_executed"] / FP32_PEAK_TFLOPS, 2),
        "pct_fp64_peak_fp64_executed": round(100 * fp64["tflops_executed"] / FP64_PEAK_TFLOPS, 2),
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, torch, S):
    """Poisson serving trace through the continuous-batching engine vs plain RGF:
    the configured rate (saturating one GPU), then, with --unsaturated-factor,
    the same requests at that fraction of the capacity the first run measured."""
    from paper_2601_04904_amd import serving
    from paper_2601_04904_amd.synth import serving_trace
    budget = int(args.serve_budget_gb * 1e9)

    def run(rate):
        trace = serving_trace(args.requests, rate=rate, seed=0, n_range=(16, args.serve_max_n),
                              b_choices=tuple(range(128, args.serve_max_b + 1, 64)))
        reqs = serving.requests_from_trace(trace, partitions=serving.auto_partitions)
        eng = serving.ServingEngine(budget_bytes=budget, max_inflight=args.inflight, max_wave=args.max_wave,
                                    router=serving.PrecisionRouter(probe_max_flops=args.probe_max_tflop * 1e12),
                                    log=log)
        stats = eng.replay(reqs)
        stats["waves"] = eng.waves
        stats["errors"] = eng.errors
        stats["routed_to_fp64"] = eng.router.routed
        stats["arena_waits"] = eng.arena_waits
        log(f"[bench] serving at {rate:g}/s: {stats}")
        # plain RGF on the same trace: FP64, sequential sweep, one request at a
        # time, one launch per single-term product, one stream
        plain_reqs = serving.requests_from_trace(trace)
        for r in plain_reqs:
            r.precision = "fp64"
            r.flags = S.BT_PLAIN
        peng = serving.ServingEngine(budget_bytes=budget, max_inflight=1, max_wave=1, log=log)
        pstats = peng.replay(plain_reqs)
        log(f"[bench] plain RGF serving at {rate:g}/s: {pstats}")
        ok = not eng.errors and not stats.get("failed")
        return stats, pstats, ok

    stats, pstats, ok = run(args.rate)
    # a run in which any wave failed has no valid throughput
    value = round(stats["solves_per_s"], 4) if ok else None
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * stats["wall_s"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": f"serve_{args.requests}_poisson_{args.rate:g}", "n": f"U{{16..{args.serve_max_n}}}",
                   "b": f"U{{128..{args.serve_max_b}}} step 64", "a": "U{0,256,512}", "fp64_share": 0.3,
                   "budget_gb": args.serve_budget_gb, "inflight": args.inflight,
                   "partitions": "2 per request (n >= 8), plain RGF sequential"},
        "latency_s": {"p50": stats["p50_s"], "p99": stats["p99_s"]},
        "serving": stats, "plain_rgf": pstats,
        "vs_plain_rgf_solves": round(stats["solves_per_s"] / pstats["solves_per_s"], 3) if pstats["solves_per_s"] else None,
    }
    if args.unsaturated_factor > 0 and ok:
        cap = stats["requests"] / stats["wall_s"]              # requests/s the engine sustained
        rate2 = args.unsaturated_factor * cap
        st2, ps2, ok2 = run(rate2)
        out["unsaturated"] = {
            "rate_per_s": round(rate2, 4), "of_capacity": args.unsaturated_factor,
            "latency_s": {"p50": st2["p50_s"], "p99": st2["p99_s"]},
            "serving": st2 if ok2 else None, "plain_rgf": ps2,
            "vs_plain_rgf_solves": round(st2["solves_per_s"] / ps2["solves_per_s"], 3) if ps2["solves_per_s"] and ok2 else None,
        }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bt_n64_b512",
                    help="bt_n16_b32 | bt_n64_b512 | bta_n128_b384_a512 | sd_n32_b1024 | "
                         "vb_n48_b256to512 | vbta_n48_b256to512_a256 | batch | serve | copy")
    ap.add_argument("--partitions", type=int, default=None,
                    help="time only this partition count (default: every form the workload names)")
    ap.add_argument("--compare-partitions", type=int, nargs="*", default=None,
                    help="also time these partition counts and report them beside the value")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph", type=int, default=1,
                    help="1: run each solve's launch list as a captured HIP graph (BT_GRAPH)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: pick product tile shapes with the autotuner before timing")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-wave", type=int, default=32)
    ap.add_argument("--plain-count", type=int, default=-1,
                    help="instances of the batch timed with plain RGF (-1: all of them)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--unsaturated-factor", type=float, default=0.7,
                    help="serve: also replay the trace at this fraction of the measured capacity (0: skip)")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--serve-max-n", type=int, default=256)
    ap.add_argument("--serve-max-b", type=int, default=1024)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--inflight", type=int, default=2)
    ap.add_argument("--max-wave", type=int, default=8)
    ap.add_argument("--fused", type=int, default=1,
                    help="1: workloads with blocks and tip <= 64 also run the sequential sweep as one "
                         "fused launch (BT_FUSED), a candidate for the value")
    ap.add_argument("--antihermitian", type=int, default=1,
                    help="1: also time the reported form with BT_SIGMA_ANTIHERMITIAN (the synthetic "
                         "Sigma^< is anti-Hermitian) and report it beside the value")
    ap.add_argument("--reduced-parts", type=int, nargs="*", default=[],
                    help="also time each named partitioned form with its reduced system solved by the "
                         "partitioned scheme with this many parts, recursively (reported, not the value)")
    ap.add_argument("--probe-max-tflop", type=float, default=2.0,
                    help="serving: largest request (TFLOP) spent on probing the mixed path")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the partitioned "
              "solve runs its partitions concurrently on one device and does not shard across "
              "GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2601_04904_amd import solver as S
    from paper_2601_04904_amd.synth import CONFIGS, VAR_CONFIGS, config_problem

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.workload == "copy":
        # calibration for HBM traffic counters: a plain device copy of known size
        nbytes = 1 << 30
        x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        print(json.dumps({"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                          "copies": 3, "GB_per_s": round(2 * nbytes / dt / 1e9, 1)}), flush=True)
        return
    tuned = None
    if args.autotune and args.workload != "copy":
        t0 = time.perf_counter()
        tuned = S.autotune()
        log(f"[bench] autotuned {len(tuned)} product launch classes in {time.perf_counter() - t0:.1f} s")
    args.flags = S.BT_GRAPH if args.graph else 0
    args.tuned = tuned
    if args.workload == "batch":
        return bench_batch(args, torch, S)
    if args.workload == "serve":
        return bench_serve(args, torch, S)
    if args.workload in VAR_CONFIGS:
        # diagonal blocks of different sizes (Sec. II-A)
        vc = VAR_CONFIGS[args.workload]
        sizes = list(vc["sizes"])
        n, b, a = len(sizes), max(sizes), vc["a"]
        cfg = argparse.Namespace(name=args.workload, E=vc["E"], eta=vc["eta"], seed=vc["seed"],
                                 partitions=vc["partitions"])
        Blocks = S.VarDeviceBlocks
        new_blocks = lambda: S.VarDeviceBlocks.empty(sizes, a)
    else:
        cfg = CONFIGS[args.workload]
        n, b, a = cfg.n, cfg.b, cfg.a
        sizes = None
        Blocks = S.DeviceBlocks
        new_blocks = lambda: S.DeviceBlocks.empty(n, b, a)
    # the forms the workload names (e.g. sequential and P=8); the value is the
    # fastest of them, the others are reported beside it
    forms = [args.partitions] if args.partitions is not None else list(cfg.partitions)
    # by default the two-partition form is timed beside the named ones where the
    # workload names both the sequential and a many-partition form: on one GPU
    # it is the fastest (no middle partitions, no fill), reported, not the value
    default_extra = [2] if args.partitions is None and 1 in forms and max(forms) > 2 else []
    extra = [q for q in (args.compare_partitions if args.compare_partitions is not None else default_extra)
             if q not in forms]
    log(f"[bench] workload {cfg.name}: n={n} b={b if sizes is None else 'per block'} a={a} "
        f"forms P={forms} extra P={extra} eta={cfg.eta}")
    t0 = time.perf_counter()
    A, B = config_problem(args.workload)
    log(f"[bench] generated inputs in {time.perf_counter() - t0:.1f} s")
    dA, dB = Blocks.from_host(A), Blocks.from_host(B)
    XR, XL = new_blocks(), new_blocks()

    # forms: (key, partitions, extra flags); with blocks and tip of at most
    # 64 the sequential sweep also runs as one fused launch (BT_FUSED)
    fusable = max(sizes or [b]) <= 64 and a <= 64
    # (key, partitions, flags, reduced_parts); 0 = the library's default split
    variants = [(f"P{q}", q, 0, 0) for q in forms + extra]
    if fusable and args.fused:
        variants.append(("P1_fused", 1, S.BT_FUSED, 0))
    named = [k for k, q, _, r in variants if q in forms and r == 0]
    variants += [(f"P{q}_reduced{r}", q, 0, r) for q in forms if q >= 3 for r in args.reduced_parts]
    timed = {}
    for key, q, fl, r in variants:
        sol = S.Solver(n, b, a, partitions=q, flags=args.flags | fl, sizes=sizes, reduced_parts=r)
        el, lt = time_solves(torch, sol, dA, dB, XR, XL, args.steps, args.warmup)
        exP, usP = S.flops(n, b, a, q, sizes=sizes, reduced_parts=r)
        timed[key] = dict(P=q, flags=fl, reduced_parts=r, elapsed=el, lat=lt,
                          launches=sol.last_launch_count(), ex=exP, us=usP)
        sol.destroy()
        log(f"[bench] {key}: {1e3 * el / args.steps:.2f} ms/solve, {timed[key]['launches']} launches/solve")
    best = min(named, key=lambda k: timed[k]["elapsed"])
    P, pflags = timed[best]["P"], timed[best]["flags"]
    elapsed, lat, launches = timed[best]["elapsed"], timed[best]["lat"], timed[best]["launches"]
    ex, us = timed[best]["ex"], timed[best]["us"]
    ms = 1e3 * elapsed / args.steps

    # roofline of the dominant kernel of the reported form, from HIP events
    # recorded around each launch; while profiling the library runs the
    # launches one after another on one stream, so each event pair times the
    # kernel alone (in the timed solves the two streams' launches overlap)
    sol = S.Solver(n, b, a, partitions=P, sizes=sizes, flags=pflags)
    sol.solve(dA, dB, XR, XL)
    sol.profile(True)
    for _ in range(args.profile_steps):
        sol.solve(dA, dB, XR, XL)
    stats = sol.profile_stats()
    sol.profile(False)
    sol.sync()
    dom_name = max(stats, key=lambda k: stats[k]["total_ms"])
    dom = stats[dom_name]
    per_launch_ms = dom["total_ms"] / dom["launches"]
    if dom_name.startswith("product"):
        peak = FP64_PEAK_TFLOPS if dom_name == "product_fp64" else FP32_PEAK_TFLOPS
        achieved = dom["flops"] / (dom["total_ms"] * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4), traffic=None)
    elif dom_name == "fused":
        # one workgroup per instance: FP64 vector multiply-adds on one CU
        # per instance, against the chip's FP64 peak (and one CU's share)
        achieved = dom["flops"] / (dom["total_ms"] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 4), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP64_PEAK_TFLOPS, 5), traffic=None,
                    workgroups=1, frac_of_one_cu=round(achieved / (FP64_PEAK_TFLOPS / 256), 4))
    elif dom_name.startswith("inv_panel"):
        # Gauss-Jordan steps run on the FP64 vector units (pivot search and
        # row updates); bound by FP64 VALU issue and by the per-column latency
        achieved = dom["flops"] / (dom["total_ms"] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=None)
    else:
        achieved = dom["bytes"] / (dom["total_ms"] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None)
    roof["traffic"] = measured_traffic(dom_name, cfg.name, P)
    roof["kernel"] = dom_name
    roof["launches_per_solve"] = dom["launches"] / args.profile_steps
    roof["avg_launch_us"] = round(per_launch_ms * 1e3, 2)
    roof["algorithmic_bytes_per_launch"] = round(dom["bytes"] / dom["launches"])
    roof["algorithmic_flops_per_launch"] = round(dom["flops"] / dom["launches"])
    kernel_share = {k: round(v["total_ms"] / args.profile_steps, 3) for k, v in stats.items()}
    log(f"[bench] P={P} per-solve kernel ms: {kernel_share}")
    sol.destroy()

    def form_entry(k):
        t = timed[k]
        sec = t["elapsed"] / args.steps
        extra_keys = {"reduced_parts": t["reduced_parts"]} if t["reduced_parts"] else {}
        return dict(partitions=t["P"], fused=bool(t["flags"]), solves_per_s=round(args.steps / t["elapsed"], 4),
                    ms_per_step=round(1e3 * sec, 3), launches=t["launches"],
                    pct_fp64_peak_executed=round(100 * t["ex"] / sec / 1e12 / FP64_PEAK_TFLOPS, 2),
                    pct_fp64_peak_useful=round(100 * t["us"] / sec / 1e12 / FP64_PEAK_TFLOPS, 2),
                    latency_ms=latency_summary(t["lat"]), **extra_keys)
    compare = {k: form_entry(k) for k, _, _, _ in variants if k != best}

    # the same form with the anti-Hermitian Sigma^< option (not the value: it
    # assumes the structure of the input), with its difference to the general path
    ah = None
    if args.antihermitian and sizes is None:
        XLg = XL.to_host()
        solh = S.Solver(n, b, a, partitions=P, flags=args.flags | pflags | S.BT_SIGMA_ANTIHERMITIAN)
        el_h, lat_h = time_solves(torch, solh, dA, dB, XR, XL, args.steps, args.warmup)
        ex_h, _ = S.flops(n, b, a, P, flags=S.BT_SIGMA_ANTIHERMITIAN)
        solh.destroy()
        XLh = XL.to_host()
        num = sum(float(np.linalg.norm(getattr(XLh, f) - getattr(XLg, f)) ** 2) for f in S.FIELDS)
        den = sum(float(np.linalg.norm(getattr(XLg, f)) ** 2) for f in S.FIELDS)
        sec = el_h / args.steps
        ah = dict(partitions=P, solves_per_s=round(args.steps / el_h, 4), ms_per_step=round(1e3 * sec, 3),
                  flops_executed=ex_h, pct_fp64_peak_executed=round(100 * ex_h / sec / 1e12 / FP64_PEAK_TFLOPS, 2),
                  pct_fp64_peak_useful=round(100 * us / sec / 1e12 / FP64_PEAK_TFLOPS, 2),
                  latency_ms=latency_summary(lat_h),
                  xl_rel_diff_vs_general=float(np.sqrt(num / max(den, 1e-300))))
        log(f"[bench] P={P} with BT_SIGMA_ANTIHERMITIAN: {1e3 * sec:.2f} ms/solve, "
            f"X^< difference to the general path {ah['xl_rel_diff_vs_general']:.2e}")
        # restore the general path's outputs for the CPU-baseline comparison below
        sol_g = S.Solver(n, b, a, partitions=P, flags=args.flags | pflags)
        sol_g.solve(dA, dB, XR, XL)
        sol_g.sync()
        sol_g.destroy()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        XRh, XLh = XR.to_host(), XL.to_host()
        cpu, (eR, eL) = cpu_baseline(A, B, args.cpu_seconds, XRh, XLh)
        cpu["gpu_max_rel_err_vs_oracle"] = {"XR": eR, "XL": eL}
        fl = oracle_floor(cfg.name, P)
        if fl is not None:
            cpu["oracle_floor"] = fl
        log(f"[bench] cpu {cpu['value']:.4f} solves/s on {cpu['cores']} threads; "
            f"GPU error vs oracle R={eR:.2e} L={eL:.2e}")

    tflops_ex = ex / (elapsed / args.steps) / 1e12
    tflops_us = us / (elapsed / args.steps) / 1e12
    out = {
        "metric": METRIC,
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n": n, "b": b if sizes is None else sizes, "a": a,
                   "partitions": P, "fused": bool(pflags),
                   "E": cfg.E, "eta": cfg.eta, "seed": cfg.seed, "hip_graph": bool(args.graph),
                   "tile_shapes": "autotuned" if args.tuned else "default rule"},
        "tflops_executed": round(tflops_ex, 3),
        "tflops_useful": round(tflops_us, 3),
        "pct_fp64_peak_executed": round(100 * tflops_ex / FP64_PEAK_TFLOPS, 2),
        "pct_fp64_peak_useful": round(100 * tflops_us / FP64_PEAK_TFLOPS, 2),
        "latency_ms": latency_summary(lat),
        "launches_per_solve": launches,
        "kernel_ms_per_solve": kernel_share,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if compare:
        out["other_forms"] = compare
    if ah:
        out["antihermitian_sigma_form"] = ah
    print(json.dumps(out), flush=True)
    sol.destroy()


if __name__ == "__main__":
    main()
