#!/usr/bin/env python3
"""Throughput benchmark of the MI355X Gaussian random field sampler.

One step = one batch of the headline workload through the whole sampling path:
512 x 512 periodic grid on the unit torus, Matern covariance (sigma 1, length
scale 0.1, nu 1.5), float32, one-FFT (Hermitian) algorithm, 1024 independent
fields with seeds 0..1023, output resident in HBM.  value = grid points per
second (2^28 points per step / seconds per step).

Printed alongside on the same JSON line:
  roofline      the dominant kernel of the step (the pass with the largest total
                time): algorithmic work per launch / its mean launch duration,
                from HIP events recorded between the launches of the sampler
                run in sequence on the launch stream; the HBM fraction of that
                kernel and of the whole step next to it; the per-pass table
  cpu_baseline  the float64 oracle on a bounded sample of the same workload, on
                one core and on all cores of the host (one process per core),
                timed before the GPU is initialised
  extra         two-FFT algorithm on the same workload, the 256^3 x 16
                exponential workload, 4096 fields of uneven sizes in one
                batch, forward+adjoint vs forward at 1024^2 x 64, d = 1
                sampling, the convergence study of Section 4, and the
                float32-vs-float64 error of sampled fields
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes per cycle x 2.4 GHz, in tera lane-ops/s
# (a wave64 instruction occupies its SIMD for 4 cycles; an FMA is one op; the
# half-rate transcendentals count as two).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def gen_pass_ops_per_point(n1, stages=None):
    """Algorithmic VALU lane-ops per output point of the column generation pass (one-FFT,
    d = 2, radix-8 column transform of length n1 = 8^s): Philox-4x32-10 (10 rounds x
    (2 32x32->64 products + 2 three-input xors) per 4 normals) = 10; Box-Muller per
    pair (2 conversions, 2 scalings, log, sqrt, sin, cos at two slots each, 3 products)
    = 15 -> 7.5; filter (h/sqrt2 and two products per complex entry) = 1.5; radix-8
    Stockham stages: 7 ops per complex per stage + 3.5 for the twiddles of every stage
    but the first, per real point half of that.  `stages`: the radix-8 stages the pass
    runs (all s by default; s - 1 when the last-axis pass completes the transform)."""
    import math
    s = round(math.log(n1, 8))
    k = s if stages is None else stages
    return 10 + 7.5 + 1.5 + (7 * k + 3.5 * (k - 1)) / 2

# HBM bytes per launch of the headline step's kernels (one launch = one cache-sized
# chunk of 256 fields), from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
# launches in sequence) scaled by the same counters on a 1 GiB device copy (FETCH x2,
# WRITE x1); profiles/grf_sample_512x512x1024_f32.md.  Set an entry to None when its
# kernel changes.
MEASURED_TRAFFIC = {
    "column noise+inverse FFT (axis 1)": (2408 * 2 + 275738) * 1024,
    "last-axis C2R": (131139 * 2 + 262144) * 1024,
    "column noise+inverse FFT (axis 1) but its last stage": (2412 * 2 + 277270) * 1024,
    "last stage of axis 1 + last-axis C2R": (131144 * 2 + 262144) * 1024,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--unchunked-ref", action="store_true",
                    help="also time the sampler with one launch per pass over the whole batch")
    ap.add_argument("--profile-stage", type=int, default=None,
                    help="profiling mode: launch only this stage of the headline step (-1: the whole "
                         "sampler), --steps times")
    ap.add_argument("--profile-alg", type=int, default=2, help="algorithm for --profile-stage")
    ap.add_argument("--profile-dims", type=str, default="512,512", help="grid for --profile-stage")
    ap.add_argument("--profile-batch", type=int, default=1024)
    ap.add_argument("--profile-boundary", type=str, default="periodic",
                    help="boundary for --profile-stage: periodic | neumann | dirichlet")
    ap.add_argument("--profile-draw-order", type=str, default="counter",
                    help="draw order for --profile-stage: counter | recursive")
    ap.add_argument("--profile-adjoint", action="store_true",
                    help="profiling mode: the adjoint of the 1024^2 x 64 training step (dL/dphi = 2 w phi), "
                         "--steps times")
    ap.add_argument("--profile-adjoint-reflect", choices=["neumann", "dirichlet"], default=None,
                    help="profiling mode: forward and adjoint of the reflecting sampler on 512^2 x 256 fields "
                         "(dL/dphi = phi), --steps times each")
    ap.add_argument("--profile-uneven", action="store_true",
                    help="profiling mode: sample the 4096 uneven fields (graph replay), --steps times")
    ap.add_argument("--copy-calib", action="store_true",
                    help="profiling mode: device copy of 1 GiB, --steps times (counter calibration)")
    return ap.parse_args()


def profile_mode(args):
    """Kernel launches only, for rocprofv3 counter runs (prints one line)."""
    import ctypes

    import torch

    import paper_1105_2737_amd as grf
    if args.profile_adjoint:
        import numpy as np
        from synth import loss_weights
        plan = grf.Plan((1024, 1024), alg=2, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
        phi = plan.sample(seed=0, batch=64)
        w = torch.from_numpy(loss_weights((64, 1024, 1024), seed=1).astype(np.float32)).cuda()
        g = 2 * w * phi
        for _ in range(args.warmup + args.steps):
            plan.backward(g, seed=0)
        torch.cuda.synchronize()
        print(f"profiled the adjoint of 1024^2 x 64, {args.steps} times", flush=True)
        return
    if args.profile_adjoint_reflect is not None:
        plan = grf.Plan((512, 512), alg=2, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5,
                        boundary=args.profile_adjoint_reflect)
        phi = plan.sample(seed=0, batch=256)
        for _ in range(args.warmup + args.steps):
            plan.sample(seed=0, batch=256, out=phi)
        g = phi.clone()
        for _ in range(args.warmup + args.steps):
            plan.backward(g, seed=0)
        torch.cuda.synchronize()
        print(f"profiled the {args.profile_adjoint_reflect} sampler and its adjoint on 512^2 x 256, "
              f"{args.steps} times each", flush=True)
        return
    if args.profile_uneven:
        from synth import uneven_fields
        bt = grf.Batch(uneven_fields(4096, seed=0))
        ob = bt.empty()
        bt.tune(out=ob)
        for _ in range(args.warmup + args.steps):
            bt.sample(out=ob)
        torch.cuda.synchronize()
        print(f"profiled the 4096 uneven fields, {args.steps} times", flush=True)
        return
    if args.copy_calib:
        a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy calibration: {args.steps} x {a.numel() * 4} bytes", flush=True)
        return
    dims = tuple(int(x) for x in args.profile_dims.split(","))
    cov = "exponential" if len(dims) == 3 else "matern"
    plan = grf.Plan(dims, alg=args.profile_alg, dtype=torch.float32, cov=cov, sigma=1.0,
                    length_scale=0.05 if len(dims) == 3 else 0.1, nu=1.5, boundary=args.profile_boundary,
                    draw_order=args.profile_draw_order)
    batch = args.profile_batch
    out = torch.empty((batch,) + dims, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(args.warmup + args.steps):
        if args.profile_stage < 0:   # every launch of the sampler, in sequence
            grf.grf_sample(plan.handle, 0, batch, None, ctypes.c_void_p(out.data_ptr()), None, 0, stream)
        else:
            grf.grf_sample_stage(plan.handle, args.profile_stage, 0, batch, None, ctypes.c_void_p(out.data_ptr()),
                                 None, 0, stream)
    torch.cuda.synchronize()
    print(f"profiled stage {args.profile_stage} of alg {args.profile_alg} on {dims} x {batch}, "
          f"{args.profile_boundary} boundary, {args.profile_draw_order} draw order", flush=True)


# Secondary workloads follow host-side work (plan creation, float64 checks) that
# leaves the GPU idle; its clock then takes some 25 ms of load to ramp up again
# (the headline step reads 0.73 ms for its first 20 steps after 2 s idle, 0.633 ms
# from the 40th on).  Their timed regions therefore follow at least this much
# warm-up of the same work; the headline's follows its per-launch measurements.
EXTRA_WARM_S = 0.1


def timed(fn, steps, warmup, torch, warm_s=0.0):
    """Seconds per call of fn over `steps` calls, after `warmup` calls and, if
    warm_s > 0, more calls until warm_s seconds have passed."""
    tw = time.perf_counter()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    while time.perf_counter() - tw < warm_s:
        fn()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_ms(fn, reps, torch):
    """Mean duration of fn's launches on the current stream (HIP events)."""
    s = torch.cuda.current_stream()
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


PASS_NAMES = {0: "column noise+inverse FFT (axis 1)", 1: "inverse FFT (axis 2)", 2: "forward FFT (axis 2)",
              3: "column fwd FFT x h x inv FFT", 4: "column adjoint", 5: "last-axis C2R",
              6: "last-axis noise+R2C", 7: "last-axis R2C",
              9: "reflecting: column coefficients+DCT (axis 1)", 10: "reflecting: DCT (axis 2)",
              11: "reflecting: last-axis DCT", 12: "reflecting: 1D coefficients+DCT",
              13: "column noise (recursive order)+inverse FFT (axis 1)", 14: "filter on the packed spectrum",
              109: "column fwd FFT x h x inv FFT (d = 3)", 110: "filter on the packed plane slots",
              111: "column noise+inverse FFT (axis 1) but its last stage",
              112: "last stage of axis 1 + last-axis C2R",
              113: "column noise (recursive order)+inverse FFT (axis 1) but its last stage"}


def pass_bytes(kind, field_bytes):
    """Algorithmic HBM bytes of one field through pass `kind` (output-sized packed spectrum)."""
    return field_bytes * (1 if kind in (0, 6, 9, 12, 13, 111, 113) else 2)


def launch_table(plan, batch, torch, grf, reps):
    """Each launch of plan.sample, run in sequence as in the sampler with HIP events
    recorded between launches on the launch stream: per launch (kind, fields, mean ms)."""
    import ctypes
    n = grf.grf_sample_stage_count(plan.handle, batch)
    info = [grf.grf_sample_stage_info(plan.handle, batch, st) for st in range(n)]
    out = torch.empty((batch,) + plan.dims, dtype=plan.dtype, device="cuda")
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    op = ctypes.c_void_p(out.data_ptr())

    def one(evs=None):
        for st in range(n):
            if evs is not None:
                evs[st].record(s)
            grf.grf_sample_stage(plan.handle, st, 0, batch, None, op, None, 0, sp)
        if evs is not None:
            evs[n].record(s)
    one()
    tot = [0.0] * n
    for _ in range(reps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        one(evs)
        torch.cuda.synchronize()
        for st in range(n):
            tot[st] += evs[st].elapsed_time(evs[st + 1])
    del out
    return [(k, c, t / reps) for (k, f, c), t in zip(info, tot)]


def stage_ms(plan, batch, stage, torch, grf, reps):
    """Mean duration of launch `stage` of plan.sample run `reps` times back to back
    between two HIP events on the launch stream (after one whole sample, so
    that it transforms the data it transforms in the sampler): the kernel's own
    duration, as a kernel trace reports it."""
    import ctypes
    out = torch.empty((batch,) + plan.dims, dtype=plan.dtype, device="cuda")
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    op = ctypes.c_void_p(out.data_ptr())
    n = grf.grf_sample_stage_count(plan.handle, batch)
    for st in range(n):
        grf.grf_sample_stage(plan.handle, st, 0, batch, None, op, None, 0, sp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        grf.grf_sample_stage(plan.handle, stage, 0, batch, None, op, None, 0, sp)
    e1.record(s)
    torch.cuda.synchronize()
    del out
    return e0.elapsed_time(e1) / reps


def by_kind(table, field_bytes):
    """Aggregate a launch table per pass kind: launches, total ms, algorithmic bytes."""
    agg = {}
    for k, c, t in table:
        a = agg.setdefault(k, {"launches": 0, "ms": 0.0, "bytes": 0, "fields": 0})
        a["launches"] += 1
        a["ms"] += t
        a["fields"] += c
        a["bytes"] += pass_bytes(k, field_bytes) * c
    return agg


def kind_rows(agg):
    return [{"kernel": PASS_NAMES[k], "launches": a["launches"], "ms": round(a["ms"], 4),
             "algorithmic_GB": round(a["bytes"] / 1e9, 4), "GBps": round(a["bytes"] / (a["ms"] * 1e-3) / 1e9, 1)}
            for k, a in agg.items()]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_fields(job):
    """Worker of the all-core leg: oracle fields seeds[0] .. seeds[1]-1."""
    from oracle import grf as ogrf, spectra
    lo, hi = job
    t0 = time.perf_counter()
    for b in range(lo, hi):
        ogrf.sample((512, 512), (1.0, 1.0), spectra.MATERN, 1.0, 0.1, 1.5, seed=b, batch=1, alg=2)
    return time.perf_counter() - t0


def cpu_baseline(seconds, batch=1024, P=512 * 512):
    """The float64 oracle on the headline workload, timed on the host before any
    GPU work: one core (fields in sequence, as many as fit in `seconds`), then
    all cores of the process's CPU set (capped at 16: one worker process per
    core, each sampling its own share of a field subset sized from the
    single-core rate to take about `seconds` / 2)."""
    import multiprocessing as mp
    from oracle import grf as ogrf, spectra
    t0 = time.perf_counter()
    n1 = 0
    while time.perf_counter() - t0 < seconds and n1 < batch:
        ogrf.sample((512, 512), (1.0, 1.0), spectra.MATERN, 1.0, 0.1, 1.5, seed=n1, batch=1, alg=2)
        n1 += 1
    t1 = time.perf_counter() - t0
    one = P * n1 / t1
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    ncores = max(1, min(16, ncores))
    per = max(1, int(round(0.5 * seconds * n1 / t1)))     # fields per worker
    nall = min(batch, per * ncores)
    jobs = [(i * nall // ncores, (i + 1) * nall // ncores) for i in range(ncores)]
    ctx = mp.get_context("fork")                          # no GPU state exists yet in this process
    t0 = time.perf_counter()
    with ctx.Pool(ncores) as pool:
        pool.map(_oracle_fields, jobs, chunksize=1)
    tall = time.perf_counter() - t0
    return {"value": round(P * nall / tall, 1), "unit": "points/s", "cores": ncores, "kind": "oracle",
            "sample": f"{nall} of the 1024 fields (seeds 0..{nall - 1}) split over {ncores} worker processes, "
                      "512x512 one-FFT float64 oracle (numpy Philox + Box-Muller, Hermitian arrangement, numpy "
                      "irfftn), wall clock including the pool start",
            "single_core": {"value": round(one, 1), "cores": 1,
                            "sample": f"{n1} fields (seeds 0..{n1 - 1}) in sequence"},
            "cpu_model": cpu_model()}


def main():
    args = parse()
    if (args.profile_stage is not None or args.copy_calib or args.profile_adjoint or args.profile_uneven
            or args.profile_adjoint_reflect is not None):
        if args.gpus != 1:
            sys.exit(2)
        profile_mode(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(fields are independent; a multi-GPU run would shard the batch without communication).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1105_2737_amd as grf

    cpu = None if args.no_cpu else cpu_baseline(args.cpu_seconds)

    torch.cuda.init()
    dev = torch.cuda.current_device()
    dims, batch = (512, 512), 1024
    P = dims[0] * dims[1]
    plan = grf.Plan(dims, alg=2, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
    out = torch.empty((batch,) + dims, dtype=torch.float32, device="cuda")

    # float32 vs the float64 template on fields {0, 1, B/2, B-1} of the headline workload
    p64 = grf.Plan(dims, alg=2, dtype=torch.float64, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
    plan.sample(seed=0, batch=batch, out=out)
    err_fields = (0, 1, batch // 2, batch - 1)
    head_err = 0.0
    for b in err_fields:
        f64 = p64.sample(seed=b, batch=1)[0]
        head_err = max(head_err, float((out[b].double() - f64).abs().max() / f64.abs().max()))
    del p64, f64

    # per-launch times in sequence; roofline of the dominant kernel (the pass with the
    # largest total time per step), per launch: algorithmic work / mean launch duration
    fbytes = P * 4
    table = launch_table(plan, batch, torch, grf, max(args.steps // 5, 100))
    agg = by_kind(table, fbytes)
    dom = max(agg, key=lambda k: agg[k]["ms"])
    d = agg[dom]
    kname, kms_seq = PASS_NAMES[dom], d["ms"] / d["launches"]
    kbytes = d["bytes"] / d["launches"]
    kpoints = d["fields"] * P / d["launches"]
    # the dominant kernel's own duration: its first launch of the step repeated back to back
    kstage = next(i for i, (k, c, t) in enumerate(table) if k == dom)
    kms = stage_ms(plan, batch, kstage, torch, grf, max(args.steps, 50))
    total_bytes = 12 * P * batch                       # packed spectrum write + read, output write

    # the timed region: W warm-up steps, then K steps
    sec = timed(lambda: plan.sample(seed=0, batch=batch, out=out), args.steps, args.warmup, torch)
    value = P * batch / sec

    # one launch per pass over the whole batch (no cache-sized chunks), for reference
    unchunked_step = None
    if args.unchunked_ref:
        os.environ["GRF_CHUNK_BYTES"] = str(1 << 40)
        unchunked_step = timed(lambda: plan.sample(seed=0, batch=batch, out=out), args.steps, args.warmup, torch)
        del os.environ["GRF_CHUNK_BYTES"]
    traffic = MEASURED_TRAFFIC.get(kname)
    k_hbm = kbytes / (kms * 1e-3) / 1e9
    if dom in (0, 111):
        # VALU-bound (noise generation in registers): algorithmic lane-ops vs the VALU issue peak
        import math
        nst = round(math.log(dims[0], 8)) - (1 if dom == 111 else 0)
        ops = gen_pass_ops_per_point(dims[0], nst) * kpoints
        achieved = ops / (kms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_PEAK_TOPS, 2),
                    "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                    "algorithmic_ops_per_point": gen_pass_ops_per_point(dims[0], nst),
                    "algorithmic_ops_per_launch": int(ops)}
    else:
        roofline = {"bound": "hbm", "achieved": round(k_hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(k_hbm / HBM_PEAK_GBS, 4)}
    roofline.update({
        "traffic": None if traffic is None else round(traffic / 1e9, 4), "traffic_unit": "GB/launch",
        "kernel": kname, "kernel_ms_per_launch": round(kms, 4),
        "kernel_ms_per_launch_in_sequence": round(kms_seq, 4), "launches_per_step": len(table),
        "algorithmic_bytes_per_launch": int(kbytes),
        # the HBM view: the dominant kernel's algorithmic bytes per launch / its launch
        # duration, and the whole step's 12 B/point model / the timed step, vs 8 TB/s
        "hbm_GBps": round(k_hbm, 1), "hbm_frac": round(k_hbm / HBM_PEAK_GBS, 4),
        "whole_step_hbm_GBps": round(total_bytes / sec / 1e9, 1),
        "whole_step_hbm_frac": round(total_bytes / sec / 1e9 / HBM_PEAK_GBS, 4),
        "passes": kind_rows(agg), "pass_sum_ms": round(sum(a["ms"] for a in agg.values()), 4),
        "unchunked_step_ms": None if unchunked_step is None else round(unchunked_step * 1e3, 4)})

    result = {
        "metric": "GRF points/s + HBM-roofline % (512^2, 256^3 FP32); batched & fwd+adjoint vs plain",
        "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512x512 unit torus, Matern(sigma=1, ell=0.1, nu=1.5), one-FFT algorithm, "
                               "1024 fields (seeds 0..1023)", "global_batch": batch, "grid": list(dims),
                   "algorithm": "one-FFT (Hermitian)", "parallelism": "single GPU"},
        "fields_per_s": round(batch / sec, 1),
        "max_rel_err_vs_fp64": head_err, "error_fields": list(err_fields),
        "roofline": roofline,
    }
    del out
    torch.cuda.empty_cache()

    extra = {}
    if not args.no_extra:
        out2 = torch.empty((batch,) + dims, dtype=torch.float32, device="cuda")
        # two-FFT algorithm on the same workload
        p1 = grf.Plan(dims, alg=1, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
        o1 = torch.empty((batch,) + dims, dtype=torch.float32, device="cuda")
        s1 = timed(lambda: p1.sample(seed=0, batch=batch, out=o1), args.steps, args.warmup, torch, EXTRA_WARM_S)
        extra["two_fft_512"] = {"points_per_s": round(P * batch / s1, 1), "ms_per_step": round(s1 * 1e3, 4),
                                "model_frac": round(20 * P * batch / s1 / 1e9 / HBM_PEAK_GBS, 4),
                                "time_ratio_vs_one_fft": round(s1 / sec, 3),
                                "passes": kind_rows(by_kind(launch_table(p1, batch, torch, grf, 10), P * 4))}
        del o1
        # error vs float64 of sampled fields (both algorithms)
        errs = {}
        for alg, pl in ((2, plan), (1, p1)):
            p64 = grf.Plan(dims, alg=alg, dtype=torch.float64, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
            e = []
            for b in (0, 1, batch // 2, batch - 1):
                f32 = pl.sample(seed=b, batch=1).double()
                f64 = p64.sample(seed=b, batch=1)
                e.append(float((f32 - f64).abs().max() / f64.abs().max()))
            errs[f"alg{alg}"] = max(e)
        extra["max_rel_err_vs_fp64_512"] = errs
        torch.cuda.empty_cache()

        # the training-path variant of the headline step: per-field (sigma, ell, nu), so that the
        # generating pass evaluates the spectral density per entry instead of reading the plan's table
        gth = torch.Generator().manual_seed(3)
        th = torch.stack([0.5 + 1.5 * torch.rand(batch, generator=gth), 0.05 + 0.15 * torch.rand(batch, generator=gth),
                          0.5 + 2.0 * torch.rand(batch, generator=gth)], 1).double().cuda()
        st = timed(lambda: plan.sample(seed=0, batch=batch, theta=th, out=out2), args.steps, args.warmup, torch, EXTRA_WARM_S)
        p64t = grf.Plan(dims, alg=2, dtype=torch.float64, cov="matern")
        et = []
        for b in (0, batch - 1):
            f64 = p64t.sample(seed=b, batch=1, theta=th[b])[0]
            et.append(float((out2[b].double() - f64).abs().max() / f64.abs().max()))
        extra["per_field_theta_512"] = {
            "points_per_s": round(P * batch / st, 1), "ms_per_step": round(st * 1e3, 4),
            "time_ratio_vs_shared_theta": round(st / sec, 3),
            "model_frac": round(12 * P * batch / st / 1e9 / HBM_PEAK_GBS, 4),
            "theta": "sigma ~ U[0.5, 2], ell ~ U[0.05, 0.2], nu ~ U[0.5, 2.5] per field (torch generator seed 3)",
            "max_rel_err_vs_fp64": max(et), "error_fields": [0, batch - 1]}
        del p64t, out2
        torch.cuda.empty_cache()

        # 256^3 x 16, exponential l = 0.05, one-FFT
        d3, b3 = (256, 256, 256), 16
        p3 = grf.Plan(d3, alg=2, dtype=torch.float32, cov="exponential", sigma=1.0, length_scale=0.05)
        o3 = torch.empty((b3,) + d3, dtype=torch.float32, device="cuda")
        s3 = timed(lambda: p3.sample(seed=0, batch=b3, out=o3), max(args.steps, 20), max(args.warmup, 10), torch, EXTRA_WARM_S)
        ab3 = 20 * 2 ** 24 * b3
        extra["one_fft_256cubed_x16"] = {
            "points_per_s": round(2 ** 24 * b3 / s3, 1), "ms_per_step": round(s3 * 1e3, 4),
            "model_GBps": round(ab3 / s3 / 1e9, 1), "model_frac": round(ab3 / s3 / 1e9 / HBM_PEAK_GBS, 4),
            "passes": kind_rows(by_kind(launch_table(p3, b3, torch, grf, 5), 2 ** 24 * 4))}
        p3_64 = grf.Plan(d3, alg=2, dtype=torch.float64, cov="exponential", sigma=1.0, length_scale=0.05)
        e3 = []
        for b in (0, 1, b3 // 2, b3 - 1):
            f64 = p3_64.sample(seed=b, batch=1)[0]
            e3.append(float((o3[b].double() - f64).abs().max() / f64.abs().max()))
        extra["one_fft_256cubed_x16"]["max_rel_err_vs_fp64"] = max(e3)
        extra["one_fft_256cubed_x16"]["error_fields"] = [0, 1, b3 // 2, b3 - 1]
        # the two-FFT algorithm on the same workload: five passes over the spectrum, 36 B/point
        p3a = grf.Plan(d3, alg=1, dtype=torch.float32, cov="exponential", sigma=1.0, length_scale=0.05)
        s3a = timed(lambda: p3a.sample(seed=0, batch=b3, out=o3), max(args.steps // 5, 3), 1, torch, EXTRA_WARM_S)
        f64 = grf.Plan(d3, alg=1, dtype=torch.float64, cov="exponential", sigma=1.0,
                       length_scale=0.05).sample(seed=0, batch=1)[0]
        extra["two_fft_256cubed_x16"] = {
            "points_per_s": round(2 ** 24 * b3 / s3a, 1), "ms_per_step": round(s3a * 1e3, 4),
            "time_ratio_vs_one_fft": round(s3a / s3, 3),
            "model_GBps": round(36 * 2 ** 24 * b3 / s3a / 1e9, 1),
            "max_rel_err_vs_fp64_field0": float((o3[0].double() - f64).abs().max() / f64.abs().max())}
        del o3, f64
        torch.cuda.empty_cache()

        # 4096 fields of uneven sizes: persistent launches in a hipGraph vs one field per launch
        from synth import uneven_fields
        fields = uneven_fields(4096, seed=0)
        bt = grf.Batch(fields)
        ob = bt.empty()
        t0 = time.perf_counter()
        bt.tune(out=ob)
        t_tune = time.perf_counter() - t0
        sb_graph = timed(lambda: bt.sample(out=ob), args.steps, args.warmup, torch, EXTRA_WARM_S)
        sb_plain = timed(lambda: bt.sample(out=ob, plain=True), 3, 1, torch, EXTRA_WARM_S)
        npts = bt.offsets[-1]
        bt.sample(out=ob)
        errs = []
        check = sorted(int(f) for f in np.random.default_rng(2).choice(len(fields), 32, replace=False))
        for f in check:
            d = fields[f]
            p64 = grf.Plan(d["dims"], alg=2, dtype=torch.float64, cov="matern", sigma=1.0,
                           length_scale=d["length_scale"], nu=d["nu"])
            f64 = p64.sample(seed=d["seed"], batch=1)[0]
            errs.append(float((bt.field(ob, f).double() - f64).abs().max() / f64.abs().max()))
        launches, wait_errors = bt.info()
        # the same batch as a column launch and a row launch (the route before the one-launch kernel)
        os.environ["GRF_BATCH_LAUNCHES"] = "2"
        bt2 = grf.Batch(fields)
        del os.environ["GRF_BATCH_LAUNCHES"]
        bt2.tune(out=ob)
        sb_two = timed(lambda: bt2.sample(out=ob), args.steps, args.warmup, torch, EXTRA_WARM_S)
        del bt2
        bt.sample(out=ob)
        extra["batched_uneven_4096"] = {
            "launches_per_sample": launches, "wait_errors": wait_errors,
            "two_launch_ms": round(sb_two * 1e3, 4),
            "points": int(npts), "ms_per_step": round(sb_graph * 1e3, 4),
            "points_per_s": round(npts / sb_graph, 1), "fields_per_s": round(4096 / sb_graph, 1),
            "plain_one_field_per_launch_ms": round(sb_plain * 1e3, 4),
            "speedup_vs_plain": round(sb_plain / sb_graph, 3),
            "model_frac": round(12 * npts / sb_graph / 1e9 / HBM_PEAK_GBS, 4),
            "tune_seconds": round(t_tune, 3), "max_rel_err_vs_fp64": max(errs),
            "error_fields": "32 fields drawn by numpy.random.default_rng(2)"}
        del ob, bt
        torch.cuda.empty_cache()

        # forward + adjoint vs forward, 1024^2 x 64
        d5, b5 = (1024, 1024), 64
        p5 = grf.Plan(d5, alg=2, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
        from synth import loss_weights
        w = torch.from_numpy(loss_weights((b5,) + d5, seed=1).astype(np.float32)).cuda()
        o5 = torch.empty((b5,) + d5, dtype=torch.float32, device="cuda")
        sf = timed(lambda: p5.sample(seed=0, batch=b5, out=o5), args.steps, args.warmup, torch, EXTRA_WARM_S)
        g = 2 * w * o5
        w2 = 2 * w                     # dL/dphi = 2 w phi in one elementwise pass

        def fwd_bwd():
            p5.sample(seed=0, batch=b5, out=o5)
            torch.mul(o5, w2, out=g)
            p5.backward(g, seed=0)
        sfb = timed(fwd_bwd, args.steps, args.warmup, torch, EXTRA_WARM_S)
        sb = timed(lambda: p5.backward(g, seed=0), args.steps, args.warmup, torch, EXTRA_WARM_S)
        sbz = timed(lambda: p5.backward(g, seed=0, need_noise_grad=True), args.steps, args.warmup, torch, EXTRA_WARM_S)
        # float32 forward and adjoint vs the float64 template on fields {0, 1, B/2, B-1}
        p5_64 = grf.Plan(d5, alg=2, dtype=torch.float64, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
        p5.sample(seed=0, batch=b5, out=o5)
        gt32, _ = p5.backward(2 * w * o5, seed=0)
        ef, eg = [], []
        for b in (0, 1, b5 // 2, b5 - 1):
            f64 = p5_64.sample(seed=b, batch=1)
            ef.append(float((o5[b].double() - f64[0]).abs().max() / f64.abs().max()))
            gt64, _ = p5_64.backward(2 * w[b:b + 1].double() * f64, seed=b)
            eg.append(float((gt32[b] - gt64[0]).abs().max() / gt64[0].abs().max()))
        extra["adjoint_1024_x64"] = {"fwd_ms": round(sf * 1e3, 4), "fwd_plus_adjoint_ms": round(sfb * 1e3, 4),
                                     "adjoint_ms": round(sb * 1e3, 4),
                                     "adjoint_with_noise_grad_ms": round(sbz * 1e3, 4),
                                     "ratio_adjoint_vs_fwd": round(sb / sf, 3),
                                     "ratio_fwd_bwd_vs_fwd": round(sfb / sf, 3),
                                     "fwd_points_per_s": round(2 ** 20 * b5 / sf, 1),
                                     "max_rel_err_vs_fp64_fwd": max(ef), "max_rel_err_vs_fp64_grad_theta": max(eg),
                                     "loss": "L = sum w phi^2, w ~ U[0,1] from numpy.random.default_rng(1)"}
        del w, w2, o5, g
        torch.cuda.empty_cache()

        # the adjoint in 3D (256^3 x 16, exponential l = 0.05), with and without dL/dz
        p3a = grf.Plan((256, 256, 256), alg=2, dtype=torch.float32, cov="exponential", sigma=1.0, length_scale=0.05)
        o3a = torch.empty((16, 256, 256, 256), dtype=torch.float32, device="cuda")
        s3f = timed(lambda: p3a.sample(seed=0, batch=16, out=o3a), max(args.steps // 10, 5), 2, torch, EXTRA_WARM_S)
        g3 = o3a.clone()
        s3b = timed(lambda: p3a.backward(g3, seed=0), max(args.steps // 10, 5), 2, torch, EXTRA_WARM_S)
        s3z = timed(lambda: p3a.backward(g3, seed=0, need_noise_grad=True), max(args.steps // 10, 5), 2, torch, EXTRA_WARM_S)
        # the adjoint of the other samplers on the headline grid (512^2 x 256 fields)
        av = {}
        oav = torch.empty((256, 512, 512), dtype=torch.float32, device="cuda")
        for nm, kw in (("two_fft", dict(alg=1)), ("neumann", dict(boundary="neumann")),
                       ("dirichlet", dict(boundary="dirichlet")), ("recursive_order", dict(draw_order="recursive"))):
            pv = grf.Plan((512, 512), dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5, **kw)
            sfv = timed(lambda: pv.sample(seed=0, batch=256, out=oav), max(args.steps // 10, 5), 2, torch, EXTRA_WARM_S)
            gv = oav.clone()
            sbv = timed(lambda: pv.backward(gv, seed=0), max(args.steps // 10, 5), 2, torch, EXTRA_WARM_S)
            av[nm] = {"fwd_ms": round(sfv * 1e3, 4), "adjoint_ms": round(sbv * 1e3, 4),
                      "ratio_adjoint_vs_fwd": round(sbv / sfv, 3)}
            del pv, gv
        extra["adjoint_variants_512_x256"] = av
        del oav
        torch.cuda.empty_cache()
        extra["adjoint_256cubed_x16"] = {"fwd_ms": round(s3f * 1e3, 4), "adjoint_ms": round(s3b * 1e3, 4),
                                         "adjoint_with_noise_grad_ms": round(s3z * 1e3, 4),
                                         "ratio_adjoint_vs_fwd": round(s3b / s3f, 3),
                                         "upstream_gradient": "dL/dphi = phi (L = |phi|^2 / 2)"}
        del p3a, o3a, g3
        torch.cuda.empty_cache()

        # the covariance family of Section 4, eq. (5), Figure 3(d)'s anisotropic case
        # (m = 5, k = 3, l = n = 1) on the headline grid and batch (filter from the plan's table)
        pp = grf.Plan(dims, lengths=(4.0, 4.0), alg=2, dtype=torch.float32, cov="paper", m=5.0, k=3, l=1, n=1)
        op = torch.empty((batch,) + dims, dtype=torch.float32, device="cuda")
        sp = timed(lambda: pp.sample(seed=0, batch=batch, out=op), args.steps // 5, args.warmup // 5, torch, EXTRA_WARM_S)
        pp64 = grf.Plan(dims, lengths=(4.0, 4.0), alg=2, dtype=torch.float64, cov="paper", m=5.0, k=3, l=1, n=1)
        ep = []
        for b in (0, 1, batch // 2, batch - 1):
            f64 = pp64.sample(seed=b, batch=1)[0]
            ep.append(float((op[b].double() - f64).abs().max() / f64.abs().max()))
        extra["paper_family_fig3d_512"] = {"points_per_s": round(P * batch / sp, 1), "ms_per_step": round(sp * 1e3, 4),
                                           "max_rel_err_vs_fp64": max(ep)}
        del op
        torch.cuda.empty_cache()

        # reflecting boundaries (cosine / sine transforms) on the headline grid and batch
        # and on 256^3 x 16: Neumann and Dirichlet on every axis
        refl = {}
        for rdims, rb, rfam in (((512, 512), batch, dict(cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)),
                                ((256, 256, 256), 16, dict(cov="exponential", sigma=1.0, length_scale=0.05))):
            orf = torch.empty((rb,) + rdims, dtype=torch.float32, device="cuda")
            npts = orf.numel()
            for bc in ("neumann", "dirichlet"):
                pr = grf.Plan(rdims, alg=2, dtype=torch.float32, boundary=bc, **rfam)
                sr = timed(lambda: pr.sample(seed=0, batch=rb, out=orf), max(args.steps // 5, 5), max(args.warmup // 5, 2), torch, EXTRA_WARM_S)
                pr64 = grf.Plan(rdims, alg=2, dtype=torch.float64, boundary=bc, **rfam)
                er = []
                for b in (0, rb - 1):
                    f64 = pr64.sample(seed=b, batch=1)[0]
                    er.append(float((orf[b].double() - f64).abs().max() / f64.abs().max()))
                key = "x".join(str(v) for v in rdims) + f"_x{rb}_{bc}"
                refl[key] = {"points_per_s": round(npts / sr, 1), "ms_per_step": round(sr * 1e3, 4),
                             "max_rel_err_vs_fp64": max(er), "error_fields": [0, rb - 1],
                             "passes": kind_rows(by_kind(launch_table(pr, rb, torch, grf, 5), (npts // rb) * 4))}
                del pr, pr64, f64
            del orf
            torch.cuda.empty_cache()
        extra["reflecting_boundaries"] = refl

        # the recursive algorithm's draw order (Section 3): each entry's draws sit at a
        # computed index of the field's sequence; headline grid and batch, and 256^3
        rec = {}
        for rdims, rb, rfam in (((512, 512), batch, dict(cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)),
                                ((256, 256, 256), 16, dict(cov="exponential", sigma=1.0, length_scale=0.05))):
            orc = torch.empty((rb,) + rdims, dtype=torch.float32, device="cuda")
            npts = orc.numel()
            pq = grf.Plan(rdims, alg=2, dtype=torch.float32, draw_order="recursive", **rfam)
            sq = timed(lambda: pq.sample(seed=0, batch=rb, out=orc), max(args.steps // 5, 5), max(args.warmup // 5, 2), torch, EXTRA_WARM_S)
            pq64 = grf.Plan(rdims, alg=2, dtype=torch.float64, draw_order="recursive", **rfam)
            eq = []
            for b in (0, rb - 1):
                f64 = pq64.sample(seed=b, batch=1)[0]
                eq.append(float((orc[b].double() - f64).abs().max() / f64.abs().max()))
            key = "x".join(str(v) for v in rdims) + f"_x{rb}"
            rec[key] = {"points_per_s": round(npts / sq, 1), "ms_per_step": round(sq * 1e3, 4),
                        "max_rel_err_vs_fp64": max(eq), "error_fields": [0, rb - 1],
                        "passes": kind_rows(by_kind(launch_table(pq, rb, torch, grf, 5), (npts // rb) * 4))}
            del pq, pq64, f64, orc
            torch.cuda.empty_cache()
        extra["recursive_draw_order"] = rec

        # d = 1: sampling throughput (65536 fields of 4096 points, 1 GiB written) and the
        # convergence study of Section 4 (10^8 samples per grid, n = 2..12, estimator fused
        # into the sampler)
        p1d = grf.Plan((4096,), lengths=(2 * 3.141592653589793,), alg=2, dtype=torch.float32, cov="matern",
                       sigma=1.0, length_scale=0.07 ** 0.5, nu=3.5)
        o1d = torch.empty((65536, 4096), dtype=torch.float32, device="cuda")
        s1d = timed(lambda: p1d.sample(seed=0, batch=65536, out=o1d), args.steps // 5, args.warmup // 5, torch, EXTRA_WARM_S)
        f64 = grf.Plan((4096,), lengths=(2 * 3.141592653589793,), alg=2, dtype=torch.float64, cov="matern",
                       sigma=1.0, length_scale=0.07 ** 0.5, nu=3.5).sample(seed=0, batch=1)[0]
        extra["one_fft_1d_4096_x65536"] = {
            "points_per_s": round(2 ** 28 / s1d, 1), "ms_per_step": round(s1d * 1e3, 4),
            "GBps_written": round(2 ** 30 / s1d / 1e9, 1), "model_frac": round(2 ** 30 / s1d / 1e9 / HBM_PEAK_GBS, 4),
            "max_rel_err_vs_fp64_field0": float((o1d[0].double() - f64).abs().max() / f64.abs().max())}
        p1a = grf.Plan((4096,), lengths=(2 * 3.141592653589793,), alg=1, dtype=torch.float32, cov="matern",
                       sigma=1.0, length_scale=0.07 ** 0.5, nu=3.5)
        s1a = timed(lambda: p1a.sample(seed=0, batch=65536, out=o1d), max(args.steps // 10, 3), 1, torch, EXTRA_WARM_S)
        extra["two_fft_1d_4096_x65536"] = {"points_per_s": round(2 ** 28 / s1a, 1), "ms_per_step": round(s1a * 1e3, 4),
                                          "time_ratio_vs_one_fft": round(s1a / s1d, 3)}
        del o1d
        torch.cuda.empty_cache()
        from paper_1105_2737_amd import study
        rows, summary = study.run(samples=10 ** 8, nmin=2, nmax=12, out=lambda line: None)
        extra["section4_convergence_study"] = {
            "samples_per_grid": 10 ** 8, "e_n": {r["N"]: r["e_n"] for r in rows},
            "slopes_per_doubling": summary["slopes_per_doubling"],
            "monte_carlo_error_scale": summary["monte_carlo_error_scale"],
            "total_seconds": round(sum(r["seconds"] for r in rows), 3),
            "points_per_s_at_N4096": rows[-1]["points_per_s"]}
    result["extra"] = extra

    if cpu is not None:
        result["cpu_baseline"] = cpu
    result["device"] = torch.cuda.get_device_name(dev)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
