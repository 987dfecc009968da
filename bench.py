"""Benchmark: 2-D Jacobi through annotated launches on one MI355X.

Workload (one step): 100 ping-pong sweeps of the five-point Jacobi stencil on
a 16384 x 16384 float32 field (~U[0,1), seed 1), as 100 annotated launches
    global [r, c] => read x[r-1:r+1, c-1:c+1], write y[r, c]
with 512-row chunks and 512-row superblocks (32 tasks per launch, 3200 per
step), followed by lt_sync.  Planning, DAG edges and issue are inside the
timed region.  Inputs are resident in HBM before timing starts.

Metric: effective GB/s = algorithmic bytes / wall time, where a sweep moves
8 bytes per point (read x once, write y once): 100 * 16384^2 * 8 B per step.
The grouped executor (ready tasks of a launch share one dispatch) gives the
reported value; the plain executor (one dispatch per task) is reported
beside it.  p50/p99 are per-step wall times.

roofline: dominant kernel k_jacobi2d, achieved = algorithmic bytes per
dispatch / mean dispatch duration measured with HIP events on the runtime's
compute stream during the timed steps; peak = 8 TB/s HBM.
cpu_baseline: the CPU oracle timed on a bounded number of sweeps of the same
field on this host's cores.

python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 16384
SWEEPS = 100
CHUNK_ROWS = 512
BYTES_PER_POINT = 8
HBM_PEAK_GBS = 8000.0


def run_gpu(mode: int, steps: int, warmup: int, x0: np.ndarray, torch):
    import paper_2202_05549_amd as L

    field_bytes = N * N * 4
    budget = 2 * field_bytes + (64 << 20)
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    ctx = L.Context(device=0, device_budget_bytes=budget, device_arena=arena.data_ptr(),
                    arena_bytes=budget, exec_mode=mode)
    try:
        a = ctx.array([N, N], chunk=[CHUNK_ROWS, 0])
        b = ctx.array([N, N], chunk=[CHUNK_ROWS, 0])
        a.write(x0)
        b.fill(0.0)
        ctx.sync()

        def step():
            inp, out = a, b
            for _ in range(SWEEPS):
                ctx.launch("jacobi2d_f32", [N, N], [1, 256], [CHUNK_ROWS, 0], args=[N, N, out, inp])
                inp, out = out, inp
            ctx.sync()

        for _ in range(warmup):
            step()
        ctx.profile(True)
        ctx.profile_reset()
        ctx.reset_stats()
        torch.cuda.synchronize()
        times = []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            step()
            times.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        prof = ctx.profile_get()
        stats = ctx.stats()
        ctx.profile(False)
    finally:
        ctx.close()
        del arena
    return total, times, prof, stats


def cpu_baseline(x0: np.ndarray, budget_s: float = 12.0):
    import oracle

    a = np.array(x0, copy=True)
    b = np.empty_like(a)
    t0 = time.perf_counter()
    oracle.lib().or_jacobi2d_sweep_f32(N, N, a.ctypes.data, b.ctypes.data)
    one = time.perf_counter() - t0
    sweeps = int(max(1, min(SWEEPS, budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.jacobi2d(a, sweeps, inplace=True)
    dt = time.perf_counter() - t0
    gbs = sweeps * N * N * BYTES_PER_POINT / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d sweeps of the 16384x16384 float32 field (of %d per step), %.2f s" % (sweeps, SWEEPS, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", choices=["both", "grouped", "plain"], default="both")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not part of this build "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    print("[bench] generating 16384^2 field", file=sys.stderr, flush=True)
    x0 = synthetic.jacobi2d_input(N, seed=1)
    step_bytes = SWEEPS * N * N * BYTES_PER_POINT

    res = {}
    modes = {"grouped": 1, "plain": 0}
    for name, mode in modes.items():
        if args.mode != "both" and args.mode != name:
            continue
        print("[bench] %s executor: %d warmup + %d timed steps" % (name, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        total, times, prof, stats = run_gpu(mode, args.steps, args.warmup, x0, torch)
        k = prof.get("jacobi2d_f32", {"dispatches": 0, "total_ms": float("nan")})
        per_dispatch_points = (N * N) if mode == 1 else (CHUNK_ROWS * N)
        avg_ms = k["total_ms"] / max(1, k["dispatches"])
        res[name] = {
            "ms_per_step": total / args.steps * 1e3,
            "gbs": step_bytes / (total / args.steps) / 1e9,
            "p50_ms": float(np.percentile(times, 50)) * 1e3,
            "p99_ms": float(np.percentile(times, 99)) * 1e3,
            "dispatches_per_step": k["dispatches"] / args.steps,
            "kernel_avg_ms": avg_ms,
            "kernel_gbs": per_dispatch_points * BYTES_PER_POINT / (avg_ms * 1e-3) / 1e9,
            "plan_ms_per_step": stats["plan_seconds"] / args.steps * 1e3,
        }
        print("[bench] %s: %s" % (name, json.dumps(res[name])), file=sys.stderr, flush=True)

    main_name = "grouped" if "grouped" in res else "plain"
    m = res[main_name]
    line = {
        "metric": "effective GB/s (% HBM or host-link roofline), plain vs batched; p50/p99 latency",
        "value": round(m["gbs"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "jacobi2d 16384x16384 f32 ~U[0,1) seed 1, 100 ping-pong sweeps, "
                               "512-row chunks and superblocks, in HBM",
                   "executor": main_name, "sweeps_per_step": SWEEPS, "tasks_per_step": SWEEPS * N // CHUNK_ROWS},
        "hbm_frac": round(m["gbs"] / HBM_PEAK_GBS, 4),
        "p50_ms": round(m["p50_ms"], 3),
        "p99_ms": round(m["p99_ms"], 3),
        "roofline": {"bound": "hbm", "achieved": round(m["kernel_gbs"], 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(m["kernel_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_jacobi2d", "kernel_avg_ms": round(m["kernel_avg_ms"], 4)},
    }
    if "plain" in res and main_name != "plain":
        p = res["plain"]
        line["plain"] = {"value": round(p["gbs"], 2), "ms_per_step": round(p["ms_per_step"], 4),
                         "p50_ms": round(p["p50_ms"], 3), "p99_ms": round(p["p99_ms"], 3),
                         "kernel_gbs": round(p["kernel_gbs"], 2),
                         "dispatches_per_step": p["dispatches_per_step"]}
        line["batched_over_plain"] = round(m["gbs"] / p["gbs"], 3)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(x0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
