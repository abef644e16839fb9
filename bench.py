#!/usr/bin/env python3
"""Benchmark of the Vegas Monte-Carlo collision integral on one MI355X.

Workload: 2<->3 contact process of a single Bose-Einstein scalar (m = 1, |M|^2 = 1), f = 0.8 f_BE(T = 1.5) on a
128-node logarithmic grid in [0.01, 30], sigma_E = 0.005, both pinned sides (multiplicities 2 and 3), separate
gain and loss integrators: 512 work items, 10 Vegas iterations of 2^18 samples each (9-dimensional).

A step is one full collision evaluation C[f] (all 10 iterations of all 512 items, with map adaptation and
integrator reuse across steps) in the batched FP32-integrand form.  The JSON line reports its throughput in
integrand samples/s, the speedup over the plain per-grid-point FP64 launch measured on the same workload
(same estimator, same sigma), the roofline of the dominant sample kernel (timed with HIP events on the
library's stream over the timed region) and the CPU reference timed on a bounded sample of the same items.
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

# Peaks of the VALU in operations per second (one op = one lane's add, mul, fma, compare, logic or integer op):
# 256 CUs x 4 SIMDs x 2.4 GHz x lanes per cycle, 32 for FP32/INT32 (the published 157.3 TFLOP/s vector FP32, counting
# an fma as 2 flops) and 16 for FP64 (78.6 TFLOP/s).
PEAK_FP32_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12  # 78.6
PEAK_FP64_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 39.3
# HBM bytes per launch of the screening kernel on this workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch
# scaled by a 256 MiB device copy (fetch x2.0, write x1.0), measured on the current kernel; None once it changes.
TRAFFIC_BYTES_SCREEN = 37.94e6
TIMING_EVERY = 7


def ops_common(n_int: int) -> int:
    """Arithmetic operations every sample needs (each +, -, *, /, fma, sqrt, exp, log, sin, cos, compare/select and
    each 32x32->64 multiply or 3-way xor of Philox counts one): Philox 40 per block (10 rounds x 2 multiplies + 2
    xors) x D/4 (the D words of a sample are a quarter block each: consecutive samples share blocks); 7 per
    dimension (uniform from the word, bin, offset, map edge and width, x, its bin count); 13 per integrated particle
    (momentum components, energy); conserved momentum 3 (n_int + 1) + 5; energy sum, Gaussian argument and its test
    (n_int + 2) + 5."""
    D = 3 * n_int
    return 10 * D + 7 * D + 13 * n_int + 3 * (n_int + 1) + 5 + (n_int + 2) + 5


def ops_weight(n_int: int) -> int:
    """Further operations of a sample whose W can be nonzero (in or near the energy shell): Jacobian 2 per
    dimension and 2 per integrated particle; f lookups 8 (n_int + 1) + 2; statistical factor 3 (n_int + 2); weight
    2 (n_int + 2) + 4; accumulation of W, W^2 and the W^2 histogram 5 + 2 D.  With ops_common this is the whole
    estimator for one sample (329 operations at n_int = 3)."""
    D = 3 * n_int
    return 2 * D + 2 * n_int + 8 * (n_int + 1) + 2 + 3 * (n_int + 2) + 2 * (n_int + 2) + 4 + 5 + 2 * D


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, threads):
    """The CPU oracle (as it stands) on a bounded sample of the same items, on `threads` threads (OpenMP over items),
    and its single-thread rate on a smaller sample."""
    from oracle import binding as ob
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    p = w.processes[0]

    def run(nodes, nitn, th):
        keep = [items[i] for i in range(n) if items[i].eval_idx in nodes]
        arr = (ob.Item * len(keep))(*keep)
        t0 = time.perf_counter()
        rc, r = ow.run_items(arr, len(keep), p.n_samples, nitn, seed=0, epoch=0, threads=th)
        dt = time.perf_counter() - t0
        assert rc == 0
        return len(keep), len(keep) * p.n_samples * nitn, dt

    stride = 1  # the whole workload: about 30 s of oracle work on 16 threads
    n_items, samples, dt = run(set(range(0, 128, stride)), p.n_iter, threads)
    n1, s1, dt1 = run(set(range(0, 128, 32)), 1, 1)  # 4 nodes x 4 items, one iteration, one thread
    return {"value": samples / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "%d of 512 items (grid nodes 0,%d,...,%d x 2 sides x 2 terms), %d samples x %d iterations "
                      "each = %.3g samples in %.1f s" % (n_items, stride, 128 - stride, p.n_samples, p.n_iter,
                                                         samples, dt) if stride > 1 else
                      "the whole workload: 512 items, %d samples x %d iterations each = %.3g samples in %.1f s" % (
                          p.n_samples, p.n_iter, samples, dt),
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "single_thread_value": s1 / dt1,
            "single_thread_sample": "%d items (grid nodes 0,32,64,96), %d samples x 1 iteration = %.3g samples in "
                                    "%.1f s" % (n1, p.n_samples, s1, dt1)}


def config_line(n, args):
    """One JSON line for one of the other workloads (not the headline): 1 = 2->2 MB, 3 = two species, three
    processes under expansion with Heun steps replayed from a HIP graph, 4 = adjoint of the 2<->3 collision
    integral, 5 = 2->4 FD with a time-dependent mass."""
    import numpy as np
    import torch
    from paper_2603_28848_amd import boltzmc as bm
    from paper_2603_28848_amd import workloads as wl

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(reps):
            fn(k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def samples(ctx, w, opts):
        tot = 0
        for p, pr in enumerate(w.processes):
            ni, _ = ctx.plan_size(p, -1, opts)
            tot += ni * (opts.n_samples or pr.n_samples) * (opts.n_iter or pr.n_iter)
        return tot

    def eval_rate(w, precision, launch, reps, freeze=0):
        ctx = bm.from_workload(w)
        o = bm.default_opts(seed=0, epoch=0, precision=precision, launch=launch, freeze_maps=freeze)
        if launch == bm.LAUNCH_BATCHED:
            ctx.autotune(-1, -1, o)
        ctx.collision(-1, -1, o)

        def run(k):
            o.epoch = 1000 + k
            ctx.collision(-1, -1, o)
        return samples(ctx, w, o) / timed(run, reps)

    def frozen_sigma(w, precision, launch):
        ctx = bm.from_workload(w)
        return ctx.collision(-1, -1, bm.default_opts(seed=0, epoch=0, precision=precision, launch=launch,
                                                      freeze_maps=1))[1]

    line = {"n_gpus": 1, "data": "synthetic", "higher_is_better": True}
    if n in (1, 5):
        w = wl.w22_mb() if n == 1 else wl.w24_fd()
        reps = max(1, args.steps)
        r32 = eval_rate(w, bm.FP32I, bm.LAUNCH_BATCHED, reps)
        r64 = eval_rate(w, bm.FP64, bm.LAUNCH_BATCHED, reps)
        p64 = eval_rate(w, bm.FP64, bm.LAUNCH_PLAIN, max(1, args.plain_steps))
        s32, s64 = frozen_sigma(w, bm.FP32I, bm.LAUNCH_BATCHED), frozen_sigma(w, bm.FP64, bm.LAUNCH_PLAIN)
        ok = (s32 > 0) & (s64 > 0)
        line.update({"metric": "collision-integrand samples/s (batched FP32-integrand)", "value": r32,
                     "unit": "samples/s", "config": {"workload": w.name, "batched_fp64_samples_per_s": r64,
                                                     "plain_fp64_samples_per_s": p64,
                                                     "speedup_vs_plain_fp64": r32 / p64,
                                                     "sigma_ratio_fp32i_over_plain_fp64": float(np.median(
                                                         s32[ok] / s64[ok])),
                                                     "sigma_ratio_max_dev": float(np.max(np.abs(
                                                         s32[ok] / s64[ok] - 1.0)))}})
    elif n == 3:
        w = wl.w_multi()
        side = torch.cuda.Stream()
        ctx = bm.from_workload(w, stream=side)
        o = bm.default_opts(seed=0, epoch=0, precision=bm.FP32I)
        ctx.autotune(-1, -1, o)
        per_step = 2 * samples(ctx, w, o)
        n_cap = 10
        ctx.graph_capture_steps(n_cap, 1, -1.0, 0.3, 1.0, o)
        ctx.graph_replay()  # first replay: warm-up
        reps = max(1, args.steps)
        dt = timed(lambda k: ctx.graph_replay(), reps)
        t, last_dt = ctx.graph_status()
        line.update({"metric": "Heun-step samples/s (HIP-graph replay, FP32 integrand)",
                     "value": per_step * n_cap / dt, "unit": "samples/s",
                     "config": {"workload": w.name, "samples_per_heun_step": per_step, "steps_per_replay": n_cap,
                                "replays_timed": reps, "ms_per_heun_step": dt / n_cap * 1e3, "t_end": t,
                                "last_dt": last_dt}})
    elif n == 4:
        w = wl.w23_adjoint()
        ctx = bm.from_workload(w)
        o = bm.default_opts(seed=0, epoch=0, precision=bm.FP64, freeze_maps=1, n_iter=1, eval_stride=1)
        ni, no = ctx.plan_size(-1, -1, o)
        per_eval = ni * w.processes[0].n_samples
        ctx.collision(-1, -1, o)
        fwd = timed(lambda k: ctx.collision(-1, -1, o), max(1, args.steps))
        v = np.ones(no)
        ctx.vjp(v, -1, -1, o)
        bwd = timed(lambda k: ctx.vjp(v, -1, -1, o), max(1, args.steps))
        line.update({"metric": "adjoint (VJP) samples/s, frozen-map FP64 collision integral",
                     "value": per_eval / bwd, "unit": "samples/s",
                     "config": {"workload": w.name, "items": ni, "samples_per_evaluation": per_eval,
                                "forward_samples_per_s": per_eval / fwd, "vjp_over_forward_time": bwd / fwd}})
    else:
        raise SystemExit("--config takes 1, 3, 4 or 5 (2 is the default headline line)")
    line["steps"] = args.steps
    print(json.dumps(line))
    sys.stdout.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--config", type=int, default=2,
                    help="2 (default): the headline 2<->3 line; 1, 3, 4, 5: the other workloads, one line each")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the collision-integral items shard across GPUs with one small "
              "all-gather per evaluation, which the library does not implement; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.config != 2:
        config_line(args.config, args)
        return

    import numpy as np
    import torch
    from paper_2603_28848_amd import boltzmc as bm
    from paper_2603_28848_amd import workloads as wl

    w = wl.w23_be()
    p = w.processes[0]
    n_int = len(p.ins) + len(p.outs) - 2

    if args.copy_calibration:
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- batched FP32-integrand: the timed path ----
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=0, epoch=0, precision=bm.FP32I, launch=bm.LAUNCH_BATCHED)
    n_items, n_out = ctx.plan_size(-1, -1, opts)
    samples_per_step = n_items * p.n_samples * p.n_iter
    tuned = ctx.autotune(-1, -1, opts)  # launch shape only; results do not depend on it
    for k in range(max(1, args.warmup)):
        opts.epoch = k
        ctx.collision(-1, -1, opts)
    torch.cuda.synchronize()
    # HIP events time every 7th sample phase of the timed steps (7 and the 10 iterations per step are coprime, so
    # the timed phases cover every iteration index; each timed phase adds two event records between kernels)
    ctx.set_timing(True, every=TIMING_EVERY)
    ctx.get_timing(reset=True)
    ctx.get_sample_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        opts.epoch = 1000 + k
        ctx.collision(-1, -1, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    screen_ms, second_ms, n_launch = ctx.get_kernel_timing(reset=True)
    n_listed = ctx.get_sample_stats(reset=True)
    ctx.set_timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = samples_per_step / ((t1 - t0) / args.steps)

    # ---- plain per-grid-point FP64 and batched FP64 on fresh contexts (one warm-up evaluation each) ----
    def rate(precision, launch, steps):
        c2 = bm.from_workload(w)
        o = bm.default_opts(seed=0, epoch=0, precision=precision, launch=launch)
        if launch == bm.LAUNCH_BATCHED:
            c2.autotune(-1, -1, o)
        c2.collision(-1, -1, o)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for k in range(steps):
            o.epoch = 1000 + k
            c2.collision(-1, -1, o)
        torch.cuda.synchronize()
        return samples_per_step * steps / (time.perf_counter() - ta)

    plain64 = rate(bm.FP64, bm.LAUNCH_PLAIN, args.plain_steps)
    batched64 = rate(bm.FP64, bm.LAUNCH_BATCHED, max(1, args.plain_steps))

    # ---- the two estimators at equal sample counts: sigma of batched FP32-integrand vs plain FP64, both on the
    # uniform maps (frozen, so that map adaptation does not enter the comparison) ----
    def frozen_sigma(precision, launch):
        c3 = bm.from_workload(w)
        return c3.collision(-1, -1, bm.default_opts(seed=0, epoch=0, precision=precision, launch=launch,
                                                     freeze_maps=1))[1]

    sig32 = frozen_sigma(bm.FP32I, bm.LAUNCH_BATCHED)
    sig64 = frozen_sigma(bm.FP64, bm.LAUNCH_PLAIN)
    ok = (sig32 > 0) & (sig64 > 0)
    sigma_ratio = float(np.median(sig32[ok] / sig64[ok]))

    # ---- roofline of the dominant kernel (the screening pass) and of the second pass ----
    # a launch = one sample phase (one Vegas iteration of all 512 items): every sample screened once, the listed
    # ones (in or near the energy shell) evaluated again by the second pass
    screen_s = screen_ms / max(1, n_launch) / 1e3
    second_s = second_ms / max(1, n_launch) / 1e3
    samples_per_launch = samples_per_step / p.n_iter
    listed_per_launch = n_listed / (args.steps * p.n_iter)  # the listed samples of every phase of the timed steps
    screen_ops = ops_common(n_int) * samples_per_launch
    second_ops = ops_weight(n_int) * listed_per_launch
    achieved = screen_ops / screen_s / 1e12
    achieved_second = second_ops / second_s / 1e12

    line = {
        "metric": "2<->3 collision-integrand samples/s (batched FP32-integrand) + speedup vs plain per-grid-point "
                  "FP64 at equal MC sigma",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "2<->3 BE scalar m=1 |M|^2=1, f=0.8 f_BE(T=1.5) on 128 log nodes [0.01,30], sigma_E=0.005, "
                        "both sides (mult 2, 3), gain/loss split: 512 items x 10 Vegas iterations x 2^18 samples",
            "items": n_items,
            "samples_per_step": samples_per_step,
            "precision": "FP32 integrand, FP64 kinematics and accumulation",
            "launch": "batched persistent (autotuned: %d blocks/CU, chunk %d)" % (tuned[0], tuned[1]),
            "plain_fp64_samples_per_s": plain64,
            "batched_fp64_samples_per_s": batched64,
            "speedup_vs_plain_fp64": value / plain64,
            "speedup_fp32i_vs_fp64_batched": value / batched64,
            "sigma_ratio_fp32i_over_plain_fp64": sigma_ratio,
            "sigma_ratio_max_dev": float(np.max(np.abs(sig32[ok] / sig64[ok] - 1.0))),
            "sample_phase_avg_ms": (screen_s + second_s) * 1e3,
            "screen_avg_ms": screen_s * 1e3,
            "second_pass_avg_ms": second_s * 1e3,
            "sample_phases_timed": n_launch,
            "timed_every": TIMING_EVERY,
        },
        "roofline": {"bound": "alu", "kernel": "k_screen (FP32/INT32 screening pass, every sample)",
                     "achieved": achieved, "peak": PEAK_FP32_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_FP32_TOPS, "traffic": TRAFFIC_BYTES_SCREEN,
                     "ops_per_sample": ops_common(n_int), "samples_per_launch": samples_per_launch,
                     "ops_per_launch": screen_ops, "avg_launch_ms": screen_s * 1e3,
                     "second_pass": {"kernel": "k_shell (listed samples: FP64 kinematics, FP32 integrand)",
                                     "achieved": achieved_second, "peak": PEAK_FP64_TOPS, "unit": "TOP/s",
                                     "frac": achieved_second / PEAK_FP64_TOPS, "ops_per_sample": ops_weight(n_int),
                                     "samples_per_launch": listed_per_launch,
                                     "listed_fraction": listed_per_launch / samples_per_launch,
                                     "avg_launch_ms": second_s * 1e3}},
    }
    if not args.no_cpu_baseline:
        # the host share of one GPU is 16 threads (OMP_NUM_THREADS on the GPU hosts), whatever nproc reports
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline(w, threads)
    print(json.dumps(line))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
