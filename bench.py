"""Benchmark of the AIDW hot path on one MI355X.

One step = one AIDW evaluation (both full passes over all m data points for
every query: kNN -> alpha -> weighted average) of the paper-scale workload:
m = n = 2^20 points uniform in [0, 1000]^2, k = 15, alpha levels 1..5,
R_min = 0, R_max = 2, FP32-scaled precision, inputs resident in HBM.

Prints ONE JSON line.  `value` is pair-evaluations per second (2*m*n per
step / step time).  `roofline` prices the fused kernel at 9 algorithmic FLOP
per pair evaluation against the FP32 vector peak; `cpu_baseline` times the
FP64 CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-evals/s (n*m*2 passes) and % FP32 VALU peak; p50/p99 latency"
FLOP_PER_PAIR = 9.0          # pass 1: 6 FLOP, pass 2: 12 FLOP, mean 9
PEAK_FP32_TFLOPS = 157.3     # 256 CU x 2.4 GHz x 128 lanes x 2 (FMA)


# The sources that decide what one step launches and what those kernels do:
# the traffic counters in the profile are used only while these are unchanged.
KERNEL_SOURCES = ["paper_1511_02186_amd/csrc/kernels_f32.hip",
                  "paper_1511_02186_amd/csrc/device_math.h",
                  "paper_1511_02186_amd/csrc/common.h",
                  "paper_1511_02186_amd/csrc/kernels_order.hip",
                  "paper_1511_02186_amd/csrc/api.hip"]
TRAFFIC_PROFILE = "profiles/aidw_f32_fused_spec_paper_scale_m1048576_n1048576.md"


def kernel_sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per fused launch from the committed rocprofv3 counters, or
    None when they were taken on other kernel sources (or are missing)."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=1 << 20)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="queries of the workload timed on the CPU oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip timing the plain FP64 kernel at the same size")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-problem batched launch")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-grid", action="store_true",
                    help="skip timing pass 1 through the uniform grid (AIDW_FLAG_GRID_KNN)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the issue-cost probe (SIMD cycles of an FP32 FMA and an exp2)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the 2000 req/s Poisson serving run (5 s of arrivals)")
    ap.add_argument("--serve-sweep-requests", type=int, default=200,
                    help="requests of each lower-rate serving run (250, 500, 1000 req/s)")
    ap.add_argument("--ablation", action="store_true",
                    help="time the data-access designs (scalar / LDS-tiled / naive loads, "
                         "SoA / AoaS) at all of the paper's sizes, end to end like its Table 1 "
                         "(the default run times the 1000K row only)")
    ap.add_argument("--no-ablation", action="store_true", help="skip the 1000K ablation row")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the plain FP64 small workload, the clustered workload and "
                         "standard IDW")
    ap.add_argument("--check", type=int, default=256,
                    help="queries checked against the oracle after timing (0 = none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy, the reference for HBM counters")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(one GPU runs the whole query set; more GPUs would each take a share of the queries)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1511_02186_amd import aidw, workloads

    inst = workloads.paper_scale(m=args.m, n=args.n)
    dev = "cuda:0"
    data_xy, data_z, query_xy = aidw.to_device(inst, dev)
    out = torch.empty(inst.n, dtype=torch.float32, device=dev)
    ctx = aidw.Context(0)
    stream = torch.cuda.current_stream()

    def step():
        ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min, inst.R_max,
                        inst.area, flags=aidw.AIDW_FLAG_ASYNC, out=out)

    # what one step launches, as the library plans it
    kernels = aidw.aidw_describe_launch(ctx.h, ctx.problem(
        data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min, inst.R_max, inst.area))

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("bench: warmup done (%d steps), timing %d steps" % (args.warmup, args.steps),
          file=sys.stderr, flush=True)

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])  # ms, one launch each
    ms = float(per.mean())
    pairs = float(inst.pair_evals())
    value = pairs / (ms * 1e-3)
    achieved = FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper_scale_uniform_square", "m": inst.m, "n": inst.n,
                   "k": inst.k, "alpha_levels": list(inst.levels), "R_min": inst.R_min,
                   "R_max": inst.R_max, "precision": "fp32_scaled",
                   "pair_evals_per_step": pairs},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic() if inst.m == inst.n == 1 << 20 else None,
                     "kernel": kernels, "flop_per_pair_eval": FLOP_PER_PAIR,
                     "duration": "all launches of one step (HIP events around the step)"},
        "step_ms": {"p10": float(np.percentile(per, 10)), "p50": float(np.median(per)),
                    "p90": float(np.percentile(per, 90)), "wall_s": wall},
    }

    if args.check:
        import oracle

        idx = np.sort(np.random.default_rng(0).choice(inst.n, args.check, replace=False))
        got = out.cpu().numpy()[idx]
        want = oracle.run(inst.data_x, inst.data_y, inst.data_z, inst.query_x[idx],
                          inst.query_y[idx], inst.k, inst.levels, inst.R_min, inst.R_max,
                          inst.area)
        scale = oracle.run(inst.data_x, inst.data_y, np.abs(inst.data_z), inst.query_x[idx],
                           inst.query_y[idx], inst.k, inst.levels, inst.R_min, inst.R_max,
                           inst.area)
        result["max_rel_err_vs_oracle"] = float(np.max(np.abs(got - want) / scale))
        result["checked_queries"] = int(args.check)

    if not args.no_fp64:
        inst64 = workloads.paper_scale(m=args.m, n=args.n, dtype=np.float64)
        d64 = aidw.to_device(inst64, dev)
        o64 = torch.empty(inst64.n, dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        print("bench: timing the plain FP64 kernel once", file=sys.stderr, flush=True)
        e0.record(stream)
        ctx.interpolate(*d64, inst64.k, inst64.levels, inst64.R_min, inst64.R_max, inst64.area,
                        flags=aidw.AIDW_FLAG_ASYNC, out=o64)
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1)
        result["fp64_plain"] = {"ms": ms64, "pair_evals_per_s": pairs / (ms64 * 1e-3),
                                "speedup_fp32_scaled_vs_fp64": ms64 / ms}

    if not args.no_probe:
        c = aidw.aidw_probe_issue_costs(ctx.h)
        # A stream of FP32 FMAs alone reaches 2 / fma_cycles of the packed-FMA
        # peak: the ceiling of any kernel built without packed FP32.
        c["fma_only_frac_of_peak"] = 2.0 / c["fma_cycles"]
        result["issue_costs"] = c
    if not args.no_grid:
        result["grid_knn"] = bench_grid(ctx, torch, aidw, step_args=(
            data_xy, data_z, query_xy, inst), full_ms=ms, pairs=pairs)
    if not args.no_legs:
        result["plain_fp64_small"] = bench_c1(ctx, torch, aidw, workloads)
        result["clustered"] = bench_c3(ctx, torch, aidw, workloads)
        result["standard_idw"] = bench_idw(ctx, torch, aidw, step_args=(
            data_xy, data_z, query_xy, inst), aidw_ms=ms)
    if args.ablation:
        result["ablation"] = bench_ablation(ctx, torch, aidw, workloads)
    elif not args.no_ablation:
        # the 1000K row of Table 1 in FP32, the FP64 designs at 100K (an FP64
        # design takes about 7 s at 1000K)
        result["ablation"] = bench_ablation(ctx, torch, aidw, workloads, sizes=(1024000,),
                                            fp64_sizes=(102400,))
    if not args.no_batch:
        result["batched"] = bench_batched(ctx, torch, aidw, workloads)
    if not args.no_serve:
        result["serving"] = bench_serving_all(torch, aidw, workloads, args.serve_requests,
                                              args.serve_sweep_requests)

    if not args.no_cpu:
        import oracle

        cores = oracle.default_threads()
        idx = np.arange(args.cpu_sample)
        print("bench: timing the CPU oracle on %d queries x %d data points with %d threads"
              % (len(idx), inst.m, cores), file=sys.stderr, flush=True)
        t = time.perf_counter()
        oracle.run(inst.data_x, inst.data_y, inst.data_z, inst.query_x[idx], inst.query_y[idx],
                   inst.k, inst.levels, inst.R_min, inst.R_max, inst.area, threads=cores)
        dt = time.perf_counter() - t
        result["cpu_baseline"] = {
            "value": 2.0 * inst.m * len(idx) / dt, "unit": "pair-evals/s", "cores": cores,
            "kind": "oracle",
            "sample": "first %d queries of the workload against all %d data points (%.1f s)"
                      % (len(idx), inst.m, dt),
            # the whole step at the sampled rate (the oracle's cost per query
            # does not depend on the query)
            "full_step_s_extrapolated": 2.0 * inst.m * inst.n / (2.0 * inst.m * len(idx) / dt),
            "gpu_speedup": (2.0 * inst.m * inst.n / (ms * 1e-3)) / (2.0 * inst.m * len(idx) / dt)}

    ctx.close()
    print(json.dumps(result), flush=True)


def bench_ablation(ctx, torch, aidw, workloads, sizes=(10240, 51200, 102400, 512000, 1024000),
                   fp64_sizes=(10240, 51200, 102400, 512000, 1024000), with_fp32=True):
    """The paper's Table 1 axes on this GPU: m = n = N points in a square,
    every data-access design and layout, in FP32-scaled arithmetic (with the
    production launch beside them) and in plain FP64 (the paper's Sec. 4.2
    experiment).  Times are kernel-only (HIP events) and end to end (pinned
    host -> device copy of the inputs, kernel, device -> host copy of the
    output), as in Sec. 4."""
    designs = [("%s_%s" % (a, l), ai, li)
               for ai, a in enumerate(["scalar", "tiled", "naive"])
               for li, l in enumerate(["soa", "aoas"])]
    rows = []
    for N in sorted(set(sizes) | set(fp64_sizes)):
        runs = []
        if with_fp32 and N in sizes:
            runs += [("production", None, None, False)] + [(d, a, l, False) for d, a, l in designs]
        if N in fp64_sizes:
            runs += [("fp64_" + d, a, l, True) for d, a, l in designs]
        inst = workloads.paper_scale(m=N, n=N, seed=7)
        inst64 = workloads.paper_scale(m=N, n=N, seed=7, dtype=np.float64)
        for name, acc, lay, f64 in runs:
            print("bench: ablation N=%d %s" % (N, name), file=sys.stderr, flush=True)
            src = inst64 if f64 else inst
            host = [torch.from_numpy(a).pin_memory() for a in
                    (src.data_xy(), src.data_z.copy(), src.query_xy())]
            out_h = torch.empty(N, dtype=host[0].dtype).pin_memory()
            dev = [h.to("cuda", non_blocking=True) for h in host]
            out = torch.empty(N, dtype=host[0].dtype, device="cuda")
            ctx.bind_current_stream()
            p = ctx.problem(dev[0], dev[1], dev[2], inst.k, out, inst.levels, inst.R_min,
                            inst.R_max, inst.area, flags=aidw.AIDW_FLAG_ASYNC)

            def run():
                if acc is None:
                    aidw.check(aidw.aidw_interpolate_ex(ctx.h, p))
                else:
                    aidw.check(aidw.aidw_interpolate_variant(ctx.h, p, acc, lay))

            run()
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record()
            for d, h in zip(dev, host):
                d.copy_(h, non_blocking=True)
            e[1].record()
            run()
            e[2].record()
            out_h.copy_(out, non_blocking=True)
            e[3].record()
            torch.cuda.synchronize()
            kern = e[1].elapsed_time(e[2])
            rows.append({"N": N, "design": name, "kernel_ms": kern,
                         "end_to_end_ms": e[0].elapsed_time(e[3]),
                         "pair_evals_per_s": 2.0 * N * N / (kern * 1e-3)})
    return {"workload": "m = n = N uniform points in [0, 1000]^2, k = 15 (N as in the paper's "
                        "Table 1, 1K = 1024); designs: scalar / LDS-tiled / naive loads x SoA / "
                        "AoaS, FP32-scaled and plain FP64", "rows": rows}


def _time_ms(torch, run, reps):
    """Median and minimum of `reps` HIP-event timings of run() on the current stream."""
    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), float(np.min(times))


def bench_c1(ctx, torch, aidw, workloads, reps=20):
    """The plain FP64 workload: m = n = 1024 uniform in [0,1]^2, k = 10, FP64
    inputs and the plain FP64 kernel, checked against the oracle on every
    query (relative error, and the fraction of queries whose k-nearest index
    set equals the oracle's)."""
    import oracle

    print("bench: plain FP64, m = n = 1024", file=sys.stderr, flush=True)
    inst = workloads.uniform_small(m=1024, n=1024, seed=0, dtype=np.float64)
    d = aidw.to_device(inst)
    out = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    knn = torch.empty((inst.n, inst.k), dtype=torch.int32, device="cuda")
    ctx.bind_current_stream()
    p = ctx.problem(*d, inst.k, out, inst.levels, inst.R_min, inst.R_max, inst.area, knn_idx=knn,
                    flags=aidw.AIDW_FLAG_ASYNC)
    kernels = aidw.aidw_describe_launch(ctx.h, p)
    ms, ms_min = _time_ms(torch, lambda: aidw.check(aidw.aidw_interpolate_ex(ctx.h, p)), reps)
    got, got_knn = out.cpu().numpy(), knn.cpu().numpy()
    want, _, _, want_knn = oracle.run(inst.data_x, inst.data_y, inst.data_z, inst.query_x,
                                      inst.query_y, inst.k, inst.levels, inst.R_min, inst.R_max,
                                      inst.area, diag=True)
    return {"workload": "m = n = 1024 U[0,1]^2, z = sin 4x cos 3y + N(0, 0.01^2), k = 10, FP64, "
                        "seed 0", "kernel": kernels, "ms": ms, "ms_min": ms_min,
            "pair_evals_per_s": inst.pair_evals() / (ms * 1e-3),
            "max_rel_err_vs_oracle": float(np.max(np.abs(got - want) / np.abs(want))),
            "knn_exact_frac": float(np.mean(np.all(np.sort(got_knn, 1) == np.sort(want_knn, 1), 1))),
            "checked_queries": inst.n}


def bench_c3(ctx, torch, aidw, workloads, reps=10, check=512):
    """The clustered precision workload: m = n = 2^18, 64 Gaussian clusters
    plus background, 1 % of the queries on data points, k = 10, FP32-scaled;
    error against the oracle on sampled queries and on every on-point one."""
    import oracle

    print("bench: clustered, m = n = 2^18", file=sys.stderr, flush=True)
    inst = workloads.clustered()
    d = aidw.to_device(inst)
    out = torch.empty(inst.n, dtype=torch.float32, device="cuda")
    ctx.bind_current_stream()
    p = ctx.problem(*d, inst.k, out, inst.levels, inst.R_min, inst.R_max, inst.area,
                    flags=aidw.AIDW_FLAG_ASYNC)
    kernels = aidw.aidw_describe_launch(ctx.h, p)
    ms, ms_min = _time_ms(torch, lambda: aidw.check(aidw.aidw_interpolate_ex(ctx.h, p)), reps)
    got = out.cpu().numpy()
    on = np.asarray(inst.meta.get("on_point_queries", []), dtype=np.int64)
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.choice(inst.n, check, replace=False), on[:256]]))
    args = (inst.data_x, inst.data_y)
    want = oracle.run(*args, inst.data_z, inst.query_x[idx], inst.query_y[idx], inst.k,
                      inst.levels, inst.R_min, inst.R_max, inst.area)
    scale = oracle.run(*args, np.abs(inst.data_z), inst.query_x[idx], inst.query_y[idx], inst.k,
                       inst.levels, inst.R_min, inst.R_max, inst.area)
    pairs = float(inst.pair_evals())
    return {"workload": "m = n = 2^18, 90 % from 64 Gaussians (sigma 1e-4..1e-1) + 10 % "
                        "uniform, 1 % of queries on data points, k = 10, FP32-scaled, seed 2",
            "kernel": kernels, "ms": ms, "ms_min": ms_min, "pair_evals_per_s": pairs / (ms * 1e-3),
            "frac_fp32_peak": FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "max_rel_err_vs_oracle": float(np.max(np.abs(got[idx] - want) / scale)),
            "checked_queries": int(idx.size)}


def bench_idw(ctx, torch, aidw, step_args, aidw_ms, reps=5):
    """Standard IDW (Eq. 1, constant power) on the benchmark workload, beside
    AIDW: the paper's comparison of the two (AIDW adds the kNN pass)."""
    data_xy, data_z, query_xy, inst = step_args
    out = torch.empty(inst.n, dtype=torch.float32, device=data_xy.device)
    res = {}
    for power in (2.0, 5.0):
        print("bench: standard IDW, power %g" % power, file=sys.stderr, flush=True)
        ctx.bind_current_stream()
        p = ctx.problem(data_xy, data_z, query_xy, 1, out, area=1.0, flags=aidw.AIDW_FLAG_ASYNC)
        q = ctx.problem(data_xy, data_z, query_xy, 1, out, (power,) * 5, 0.0, 1.0, 1.0)
        kernels = aidw.aidw_describe_launch(ctx.h, q)
        ms, ms_min = _time_ms(torch, lambda: aidw.check(aidw.aidw_idw(ctx.h, p, power)), reps)
        res["power_%g" % power] = {"kernel": kernels, "ms": ms, "ms_min": ms_min,
                                   "aidw_over_idw_time": aidw_ms / ms}
    return res


def bench_grid(ctx, torch, aidw, step_args, full_ms, pairs, steps=3):
    """The same workload with pass 1 through the uniform grid: identical
    r_obs and alpha, pass 2 still over all m points.  The pair count stays
    the method's 2 m n, so the rate is an effective one."""
    data_xy, data_z, query_xy, inst = step_args
    out = torch.empty(inst.n, dtype=torch.float32, device=data_xy.device)
    flags = aidw.AIDW_FLAG_ASYNC | aidw.AIDW_FLAG_GRID_KNN
    print("bench: timing pass 1 through the grid", file=sys.stderr, flush=True)

    def run():
        ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min, inst.R_max,
                        inst.area, flags=flags, out=out)

    run()
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record(stream)
    for _ in range(steps):
        run()
    e[1].record(stream)
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1]) / steps
    return {"ms_per_step": ms, "effective_pair_evals_per_s": pairs / (ms * 1e-3),
            "speedup_vs_full_scan": full_ms / ms, "steps": steps}


def bench_batched(ctx, torch, aidw, workloads):
    """512 independent problems of uneven size in one graph-replayed launch."""
    print("bench: batched launch (512 problems)", file=sys.stderr, flush=True)
    insts = workloads.batched()
    dev = []
    for i in insts:
        d = aidw.to_device(i)
        dev.append((i, d, torch.empty(i.n, device="cuda")))
    probs = [ctx.problem(d[0], d[1], d[2], i.k, o, i.levels, i.R_min, i.R_max, i.area)
             for i, d, o in dev]
    ctx.bind_current_stream()
    b = aidw.aidw_batch_create(ctx.h, probs)
    try:
        aidw.check(aidw.aidw_batch_launch(b))
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            aidw.check(aidw.aidw_batch_launch(b, aidw.AIDW_FLAG_ASYNC))
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
    finally:
        aidw.aidw_batch_destroy(b)
    pairs = float(sum(i.pair_evals() for i in insts))
    ms = float(np.median(times))
    return {"workload": "512 problems, m log-uniform [1024, 65536], n log-uniform "
                        "[1024, 32768], uniform or clustered, k in {8, 10, 15}",
            "pair_evals": pairs, "ms": ms, "pair_evals_per_s": pairs / (ms * 1e-3),
            "frac_fp32_peak": FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "launch": "hipGraph replay, median of 5"}


def _serving_data(torch, spec, gen):
    """A serving data set on the device: (data_xy, data_z), area 1.  Uniform
    points in the unit square, or 90 % from 64 isotropic Gaussians (centres
    uniform, sigma log-uniform in [1e-4, 1e-1], clamped to the square) plus
    10 % uniform background; z = sum over the centres of exp(-10 |p - c|^2)."""
    m, kind, _ = spec
    xy = torch.rand((2, m), device="cuda", generator=gen)
    if kind == 0:
        return xy, (torch.sin(4 * xy[0]) * torch.cos(3 * xy[1])).contiguous()
    centres = torch.rand((64, 2), device="cuda", generator=gen)
    sig = torch.exp(torch.empty(64, device="cuda").uniform_(np.log(1e-4), np.log(1e-1),
                                                            generator=gen))
    n_mix = int(round(0.9 * m))
    pick = torch.randint(0, 64, (n_mix,), device="cuda", generator=gen)
    pts = centres[pick] + sig[pick, None] * torch.randn((n_mix, 2), device="cuda", generator=gen)
    xy[:, :n_mix] = pts.clamp(0.0, 1.0).t()
    d2 = ((xy.t()[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    return xy.contiguous(), torch.exp(-10.0 * d2).sum(-1).contiguous()


def bench_serving(ctx, torch, aidw, workloads, count, rate=2000.0, seed=4, check_jobs=0):
    """Poisson arrivals of jobs with m log-uniform in [4096, 2^20] and n
    log-uniform in [256, 2^18], uniform or clustered points; data sets used
    by more than one request are registered once (library-owned, resident),
    the others are passed by pointer.  The handle's HBM budget is 64 GB."""
    print("bench: serving run (%d requests at %g/s)" % (count, rate), file=sys.stderr, flush=True)
    reqs, specs = workloads.serving_stream(count=count, rate=rate, seed=seed)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    uses = {}
    for r in reqs:
        uses[r.dataset] = uses.get(r.dataset, 0) + 1
    data = {i: _serving_data(torch, sp, gen) for i, sp in enumerate(specs)}
    torch.cuda.synchronize()
    ids = {}
    for i, n_use in uses.items():
        if n_use > 1:
            xy, z = data[i]
            ids[i] = aidw.aidw_dataset_register(ctx.h, xy.data_ptr(), z.data_ptr(), z.numel(), 1.0)
    jobs = []
    for r in reqs:
        q = torch.rand((2, r.n), device="cuda", generator=gen)
        out = torch.empty(r.n, device="cuda")
        if r.dataset in ids:
            spec = aidw.make_job(q, r.k, out, dataset=ids[r.dataset])
        else:
            xy, z = data[r.dataset]
            spec = aidw.make_job(q, r.k, out, data_xy=xy, data_z=z, area=1.0)
        jobs.append((q, out, spec))
    torch.cuda.synchronize()
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=16 << 30)
    try:
        t0 = time.perf_counter()
        tickets = []
        for r, (_, _, spec) in zip(reqs, jobs):
            delay = r.t_arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(aidw.aidw_server_submit(srv, spec))
        res = [aidw.aidw_server_wait(srv, t, 600.0) for t in tickets]
        wall = time.perf_counter() - t0
        _, stats = aidw.aidw_server_stats(srv)
    finally:
        aidw.aidw_server_destroy(srv)
        for d in ids.values():
            aidw.aidw_dataset_release(ctx.h, d)
    ok = sum(1 for st, js, _ in res if st == aidw.AIDW_OK and js == aidw.AIDW_OK)
    err, checked = serving_error(torch, reqs, jobs, data, check_jobs)
    lat = np.array([l for _, _, l in res]) * 1e3
    pairs = float(sum(2.0 * specs[r.dataset][0] * r.n for r in reqs))
    span = reqs[-1].t_arrival
    return {"workload": "Poisson %g req/s, m log-uniform [4096, 2^20], n log-uniform "
                        "[256, 2^18], k in {8, 10, 15}, uniform or clustered points, "
                        "20 %% data-set reuse (registered)" % rate,
            "requests": count, "completed": ok, "registered_datasets": len(ids),
            "wall_s": wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "pair_evals_per_s": pairs / wall, "offered_pair_evals_per_s": pairs / span,
            "ticks": stats["ticks"], "max_rel_err_vs_oracle": err,
            "checked": "%d queries of %d jobs spread over the run" % checked}


def serving_error(torch, reqs, jobs, data, check_jobs, per_job=2):
    """Max relative error against the FP64 oracle over `per_job` queries of
    `check_jobs` jobs spread evenly over the run."""
    import oracle

    if check_jobs <= 0:
        return None, (0, 0)
    worst, nq = 0.0, 0
    picks = np.unique(np.linspace(0, len(reqs) - 1, min(check_jobs, len(reqs))).astype(int))
    for i in picks:
        r = reqs[i]
        q, out, _ = jobs[i]
        xy, z = (t.cpu().numpy() for t in data[r.dataset])
        idx = np.unique(np.linspace(0, r.n - 1, per_job).astype(int))
        Q = q.cpu().numpy()[:, idx]
        want = oracle.run(xy[0], xy[1], z, Q[0], Q[1], r.k, area=1.0)
        scale = oracle.run(xy[0], xy[1], np.abs(z), Q[0], Q[1], r.k, area=1.0)
        got = out.cpu().numpy()[idx].astype(np.float64)
        worst = max(worst, float(np.max(np.abs(got - want) / scale)))
        nq += len(idx)
    return worst, (nq, len(picks))


def bench_serving_all(torch, aidw, workloads, count, sweep_count):
    """The 2000 req/s run, then lower rates toward the knee of the latency
    curve, on a handle with a 64 GB HBM budget."""
    ctx = aidw.Context(0, hbm_budget_bytes=64 << 30)
    try:
        res = bench_serving(ctx, torch, aidw, workloads, count, check_jobs=50)
        sweep = []
        for rate in (250.0, 500.0, 1000.0):
            r = bench_serving(ctx, torch, aidw, workloads, sweep_count, rate=rate, seed=40)
            sweep.append({k: r[k] for k in ("requests", "completed", "p50_ms", "p99_ms",
                                             "pair_evals_per_s", "offered_pair_evals_per_s")})
            sweep[-1]["rate"] = rate
        res["rate_sweep"] = sweep
        return res
    finally:
        ctx.close()


if __name__ == "__main__":
    main()
