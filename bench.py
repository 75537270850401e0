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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=1 << 20)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="queries of the workload timed on the CPU oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64", action="store_true", help="also time the plain FP64 kernel once")
    ap.add_argument("--check", type=int, default=64,
                    help="queries checked against the oracle after timing (0 = none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy, the reference for HBM counters")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the path shards by queries, see DESIGN.md)" % args.gpus, file=sys.stderr)
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
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "aidw_f32_fused", "flop_per_pair_eval": FLOP_PER_PAIR},
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

    if args.fp64:
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
                      % (len(idx), inst.m, dt)}

    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
