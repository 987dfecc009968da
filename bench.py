"""Benchmarks of the annotated-launch runtime on one MI355X.

Default workload (``--workload jacobi``): 100 ping-pong sweeps of the
five-point Jacobi stencil on a 16384 x 16384 float32 field (~U[0,1), seed 1)
as 100 annotated launches
    global [r, c] => read x[r-1:r+1, c-1:c+1], write y[r, c]
with 512-row chunks and 512-row superblocks (32 tasks per launch, 3200 per
step), then lt_sync.  Planning, DAG edges and issue are inside the timed
region; inputs are resident in HBM before timing starts.  Three executors:
plain (one dispatch per task), grouped (the edge-free tasks of a launch
share one dispatch) and drain (the whole step as one batch: one persistent
dispatch, task edges resolved on the device).  ``value`` is the fastest of
grouped and drain; plain is reported beside it.

Other workloads (one JSON line each):
  stencil1d  1-D 3-point stencil, 2^20 float32, 8 chunks of 2^17, one
             launch per step, plain per-chunk dispatches (also grouped/drain)
  gemm_ooc   C = A B, 65536^2 float32 operands in pinned host memory, device
             budget 16 GiB, 4096^2 superblocks in serpentine order
  batch      8192 independent launches, stencil1d and hist256 mixed, sizes
             log-uniform 2^10..2^24: plain vs batched (drain) vs graph replay
  serve      Poisson request stream of Jacobi, k-means and GEMM requests
             through the serving loop (see paper_2202_05549_amd/serve.py)

roofline: the dominant kernel's algorithmic bytes (or FLOP) per dispatch /
its mean dispatch duration, timed with HIP events on the runtime's own
stream during the timed steps.  cpu_baseline: the CPU oracle timed on a
bounded sample of the same workload on this host's cores (jacobi only).

python bench.py [--workload W] [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
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

METRIC = "effective GB/s (% HBM or host-link roofline), plain vs batched; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK = 157.3
FP32_VECTOR_PEAK = 157.3  # 256 CU x 128 lanes x 2 FLOP x 2.4 GHz, no packed instructions needed
PCIE_NOMINAL_GBS = 63.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(times, q):
    return float(np.percentile(np.asarray(times) * 1e3, q))


def median_runs(fn, runs=5):
    """Times ``runs`` calls of ``fn`` (after the caller's warm-up); returns
    the median duration and all of them, in seconds."""
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), ts


def cpu_model():
    """Model name of this host's CPU (from /proc/cpuinfo), for the CPU
    baselines."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def base_line(workload_cfg, steps, warmup):
    return {"metric": METRIC, "n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "data": "synthetic", "config": workload_cfg}


def torch_arena(torch, nbytes):
    t = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    return t


def calibration_copy(torch, nbytes=1 << 30):
    """One elementwise copy kernel of known size: it reads and writes
    ``nbytes`` each, so its FETCH_SIZE / WRITE_SIZE counters give the scale
    between counter readings and HBM bytes on this device."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log("calibration copy: %d bytes read, %d bytes written" % (nbytes, nbytes))
    del src, dst


# HBM traffic per dispatch of the dominant kernels, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE passes scaled by the calibration copy, with the
# digest of the kernel sources they were taken on: once the sources change,
# the figure no longer describes the kernel and ``traffic`` is null.
# the code of k_jacobi2d_stack<4>: its body (with the window it falls back
# to), the kernel and its launcher
JACOBI_SOURCES = [
    ("bodies.h", "// ---------------------------------------------------------------- jacobi2d",
     "// Rows [tr0, tr0 + 8 NG)"),
    ("kernels.hip", "// ================================================================= jacobi2d",
     "// Marching tiles of 8 NG rows"),
    ("kernels.hip", "// Stacked tiles of 4 RB rows", "// ================================================================ hist256"),
]

# the code of k_gemm: the whole file (kernel, block order and launcher)
GEMM_SOURCES = [("gemm.hip", "#include <hip/hip_runtime.h>", "}  // namespace lt")]

# the code of k_kmeans (assignment): its section of kernels.hip
KMEANS_SOURCES = [("kernels.hip", "// ========================================================== kmeans assign",
                   "// ============================================================== copy boxes")]
# the code of the k-means update kernels: their section of reduce.hip and the slot rule
KMU_SOURCES = [("reduce.hip", "// ======================================================== k-means update",
                "// ========================================================= k-means centres"),
               ("kernels.h", "// k-means update: points per workgroup tile", "// Runtime helpers.")]

# the code of k_drain on the 1-D mix: the drain loop and its launcher, the
# 1-D stencil and histogram bodies it runs, and the task record
# the drain tile size the k_drain counters were taken at (0: the per-body defaults)
DRAIN_TRAFFIC_TILE = 0
DRAIN_SOURCES = [("drain.hip", "#include <hip/hip_runtime.h>", "// Device scratch of the no-allocation batch issue"),
                 ("bodies.h", "// -------------------------------------------------------------- stencil1d",
                  "// ---------------------------------------------------------------- jacobi2d"),
                 ("bodies.h", "// ---------------------------------------------------------------- hist256",
                  "}  // namespace body"),
                 ("kernels.h", "// ------------------------------------------------------------ batched path",
                  "hipError_t launch_drain(")]

TRAFFIC = {
    # k_jacobi2d_stack<4>, one 16384 x 16384 sweep per dispatch: FETCH_SIZE
    # 524,789 KiB x 2.000 (the 1 GiB copy reads 524,309 KiB) + WRITE_SIZE
    # 1,048,588 KiB x 1.000 (the copy writes 1,048,576 KiB)
    "k_jacobi2d_stack": {"sources": JACOBI_SOURCES, "digest": "2c942b8000dd6944",
                         "bytes_per_dispatch": 524789 * 1024 * 2.000 + 1048588 * 1024},
    # k_gemm, one 4096^2 C tile with K = 65536 per dispatch (out-of-core GEMM
    # 65536^3, 256 dispatches): FETCH_SIZE 4,046,964 KiB x 2.000 (the 1 GiB
    # copy reads 524,309 KiB) + WRITE_SIZE 68,518 KiB x 1.000
    "k_gemm": {"sources": GEMM_SOURCES, "digest": "09089ee7a4180e74",
               "bytes_per_dispatch": 4046964 * 1024 * 2.000 + 68518 * 1024},
    # k_kmeans_s<16, 1, 2>, one dispatch per assignment launch of 2^26 points
    # (d = 16, K = 64): FETCH_SIZE 2,097,203 KiB x 2.000 + WRITE_SIZE 262,144
    # KiB x 1.000, the 64 B of each point and its 4 B label
    "k_kmeans": {"sources": KMEANS_SOURCES, "digest": "bf09ff7bc641c700",
                 "bytes_per_dispatch": 2097203 * 1024 * 2.000 + 262144 * 1024},
    # k_kmeans_update_c<16, 8>, one dispatch per 2^22-point superblock:
    # FETCH_SIZE 139,326 KiB x 2.000 + WRITE_SIZE 4,224 KiB x 1.000 (512
    # partial slots of 64 x 16 float64 sums and 64 counts)
    "k_kmeans_update": {"sources": KMU_SOURCES, "digest": "7435618759144446",
                        "bytes_per_dispatch": 139326 * 1024 * 2.000 + 4224 * 1024},
    # k_drain<27, 4>, one dispatch per step of the 8192-launch mix at
    # superblock 2^24, 1024 workgroups, per-body drain tiles (graph replay):
    # FETCH_SIZE 27,213,872 KiB x 2.000 + WRITE_SIZE 27,245,512 KiB x 1.000 =
    # 83.63 GB, against 83.02 GB of algorithmic bytes
    "k_drain": {"sources": DRAIN_SOURCES, "digest": "8c90a005240dfe0c",
                "bytes_per_dispatch": 27213872 * 1024 * 2.000 + 27245512 * 1024},
}


def _union(iv):
    """Merged, sorted intervals of an (k, 2) array."""
    if len(iv) == 0:
        return np.zeros((0, 2))
    iv = iv[np.argsort(iv[:, 0])]
    out = [list(iv[0])]
    for a, b in iv[1:]:
        if a <= out[-1][1]:
            out[-1][1] = max(out[-1][1], b)
        else:
            out.append([a, b])
    return np.array(out)


def _meet(u, v):
    """Total length of the intersection of two merged interval lists."""
    i = j = 0
    tot = 0.0
    while i < len(u) and j < len(v):
        lo, hi = max(u[i][0], v[j][0]), min(u[i][1], v[j][1])
        if hi > lo:
            tot += hi - lo
        if u[i][1] < v[j][1]:
            i += 1
        else:
            j += 1
    return tot


def copy_overlap(spans):
    """Copy/compute overlap from the library's device-clock spans: per
    direction, the time some copy of that direction is in flight (union of
    its spans), and the share of it during which some kernel also runs,
    (copy time AND kernel time) / copy time; and the share of kernel time
    during which some copy runs (for a link-bound pass, the compute hidden
    under the copies)."""
    names = spans["name"]
    iv = np.stack([spans["start_ms"], spans["end_ms"]], axis=1) if len(spans) else np.zeros((0, 2))
    is_copy = (names == b"copy_h2d") | (names == b"copy_d2h")
    kern = _union(iv[~is_copy])
    kbusy = float((kern[:, 1] - kern[:, 0]).sum()) if len(kern) else 0.0
    out = {"kernel_busy_ms": round(kbusy, 3),
           "kernel_under_copy_frac": round(_meet(kern, _union(iv[is_copy])) / kbusy, 4) if kbusy > 0 else None}
    for d in ("h2d", "d2h"):
        u = _union(iv[names == ("copy_" + d).encode()])
        busy = float((u[:, 1] - u[:, 0]).sum()) if len(u) else 0.0
        out[d] = {"copies": int((names == ("copy_" + d).encode()).sum()), "busy_ms": round(busy, 3),
                  "overlap_frac": round(_meet(u, kern) / busy, 4) if busy > 0 else None}
    return out


def jacobi_kernel_name(variant):
    if variant in (8, 16, 32):
        return "k_jacobi2d"
    if variant in (132, 164, 228):
        return "k_jacobi2d_march"
    return "k_jacobi2d_stack"


def kernel_digest(sources):
    """sha256 over the source sections that make up a kernel: each entry is
    (file, first line marker, marker of the line after the section)."""
    import hashlib

    h = hashlib.sha256()
    for f, start, end in sources:
        with open(os.path.join(ROOT, "paper_2202_05549_amd", "csrc", f)) as fh:
            text = fh.read()
        i = text.index(start)
        j = text.index(end, i + len(start))
        h.update(text[i:j].encode())
    return h.hexdigest()[:16]


def traffic_for(kernel, per_dispatch_scale=1.0):
    t = TRAFFIC.get(kernel)
    if not t or kernel_digest(t["sources"]) != t["digest"]:
        return None
    return int(round(t["bytes_per_dispatch"] * per_dispatch_scale))


# =================================================================== jacobi
N = 16384
SWEEPS = 100
CHUNK_ROWS = 512


def jacobi_run(L, torch, x0, executor, steps, warmup, rows=None):
    field_bytes = N * N * 4
    budget = 2 * field_bytes + (256 << 20)
    arena = torch_arena(torch, budget)
    ctx = L.Context(device=0, device_budget_bytes=budget, device_arena=arena.data_ptr(), arena_bytes=budget,
                    exec_mode=0 if executor == "plain" else 1)
    try:
        if rows:
            ctx.tune("jacobi2d_f32", rows)
        a = ctx.array([N, N], chunk=[CHUNK_ROWS, 0])
        b = ctx.array([N, N], chunk=[CHUNK_ROWS, 0])
        a.write(x0)
        b.fill(0.0)
        ctx.sync()

        def step():
            if executor == "drain":
                ctx.batch_begin()
            inp, out = a, b
            for _ in range(SWEEPS):
                ctx.launch("jacobi2d_f32", [N, N], [1, 256], [CHUNK_ROWS, 0], args=[N, N, out, inp])
                inp, out = out, inp
            if executor == "drain":
                ctx.batch_end()
            ctx.sync()

        for _ in range(warmup):
            step()
        # HIP events around each step's dispatches on their stream during
        # the timed steps (grouped: the 100 sweeps between two events), so
        # the kernel time per dispatch includes the gaps between dispatches
        # and can never exceed the wall, and no event sits between two
        # sweeps; plain: per-task events would slow its host path, so its
        # kernel time comes from a separate profiled step
        ctx.profile(executor != "plain", steps=executor == "grouped")
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
        stats = ctx.stats()
        prof = ctx.profile_get()
        if executor == "plain":  # kernel time from a separate profiled step
            ctx.profile(True)
            ctx.profile_reset()
            step()
            prof = ctx.profile_get()
        ctx.profile(False)
    finally:
        ctx.close()
        del arena
    return total, times, prof, stats


def jacobi_cpu_baseline(x0, budget_s=24.0):
    import oracle

    a = np.array(x0, copy=True)
    b = np.empty_like(a)
    # warm-up: the first sweep also pays the first touch of b; the sample is
    # sized on the second
    oracle.lib().or_jacobi2d_sweep_f32(N, N, a.ctypes.data, b.ctypes.data)
    t0 = time.perf_counter()
    oracle.lib().or_jacobi2d_sweep_f32(N, N, a.ctypes.data, b.ctypes.data)
    one = time.perf_counter() - t0
    # about budget_s of CPU work (the estimate from one sweep runs high, so 10-25 s
    # in practice), as five runs of equal length: whole steps of SWEEPS sweeps
    # per run where they fit (up to 4), else the sweeps that fit
    per = int(max(1, min(4 * SWEEPS, budget_s / 5 / max(one, 1e-3))))
    if per > SWEEPS:
        per -= per % SWEEPS
    med, ts = median_runs(lambda: oracle.jacobi2d(a, per, inplace=True))
    return {"value": round(per * N * N * 8 / med / 1e9, 3), "unit": "GB/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "median of 5 runs of %d sweeps of the 16384x16384 float32 field (%d per step) after a "
                      "warm-up sweep; runs %.2f-%.2f s" % (per, SWEEPS, min(ts), max(ts))}


def bench_jacobi(args, L, torch):
    import synthetic

    log("generating the 16384^2 field")
    x0 = synthetic.jacobi2d_input(N, seed=1)
    step_bytes = SWEEPS * N * N * 8
    res = {}
    execs = ("grouped", "drain", "plain") if args.executor == "all" else (args.executor,)
    for ex in execs:
        log("%s executor: %d warm-up + %d timed steps" % (ex, args.warmup, args.steps))
        total, times, prof, stats = jacobi_run(L, torch, x0, ex, args.steps, args.warmup, args.rows)
        kname = "drain" if ex == "drain" else "jacobi2d_f32"
        k = prof.get(kname, {"dispatches": 0, "total_ms": float("nan")})
        per_dispatch_bytes = {"grouped": N * N * 8, "plain": CHUNK_ROWS * N * 8, "drain": step_bytes}[ex]
        avg_ms = k["total_ms"] / max(1, k["dispatches"])
        res[ex] = {"ms_per_step": total / args.steps * 1e3, "gbs": step_bytes / (total / args.steps) / 1e9,
                   "p50_ms": pct(times, 50), "p99_ms": pct(times, 99), "kernel_avg_ms": avg_ms,
                   "kernel_gbs": per_dispatch_bytes / (avg_ms * 1e-3) / 1e9,
                   "dispatches_per_step": stats["dispatches"] / args.steps,
                   "plan_ms_per_step": stats["plan_seconds"] / args.steps * 1e3}
        log("%s: %s" % (ex, json.dumps(res[ex])))
    best = max([e for e in ("grouped", "drain") if e in res] or list(res), key=lambda e: res[e]["gbs"])
    m = res[best]
    jk = jacobi_kernel_name(args.rows)
    line = base_line({"workload": "jacobi2d 16384x16384 f32 ~U[0,1) seed 1, 100 ping-pong sweeps, 512-row chunks "
                                  "and superblocks, in HBM", "executor": best, "sweeps_per_step": SWEEPS,
                      "tasks_per_step": SWEEPS * N // CHUNK_ROWS}, args.steps, args.warmup)
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["ms_per_step"], 4),
                 "dtype": "f32", "hbm_frac": round(m["gbs"] / HBM_PEAK_GBS, 4), "p50_ms": round(m["p50_ms"], 3),
                 "p99_ms": round(m["p99_ms"], 3),
                 "roofline": {"bound": "hbm", "achieved": round(m["kernel_gbs"], 2), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(m["kernel_gbs"] / HBM_PEAK_GBS, 4),
                              # measured on the default variant (k_jacobi2d_stack<4>) only
                              "traffic": traffic_for(jk) if best == "grouped" and args.rows in (0, 304) else None,
                              "kernel": "k_drain" if best == "drain" else jk,
                              "kernel_avg_ms": round(m["kernel_avg_ms"], 4)}})
    for ex in execs:
        if ex == best:
            continue
        r = res[ex]
        line[ex] = {"value": round(r["gbs"], 2), "ms_per_step": round(r["ms_per_step"], 4),
                    "p50_ms": round(r["p50_ms"], 3), "p99_ms": round(r["p99_ms"], 3),
                    "kernel_gbs": round(r["kernel_gbs"], 2), "dispatches_per_step": r["dispatches_per_step"]}
    if "plain" in res and best != "plain":
        line["batched_over_plain"] = round(m["gbs"] / res["plain"]["gbs"], 3)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = jacobi_cpu_baseline(x0)
    return line


# ================================================================ stencil1d
def bench_stencil1d(args, L, torch):
    import synthetic

    n, chunk = 1 << 20, 1 << 17
    x0 = synthetic.stencil1d_input(n, 0)
    res = {}
    for ex in ("plain", "grouped", "drain", "graph"):
        arena = torch_arena(torch, 64 << 20)
        ctx = L.Context(device_budget_bytes=64 << 20, device_arena=arena.data_ptr(), arena_bytes=64 << 20,
                        exec_mode=0 if ex == "plain" else 1)
        x = ctx.array([n], chunk=[chunk])
        y = ctx.array([n], chunk=[chunk])
        x.write(x0)
        ctx.sync()
        graph = None
        if ex == "graph":
            # the launch recorded once as a HIP graph (a persistent drain
            # over its 8 tasks) and replayed: no planning per step
            ctx.graph_begin()
            ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
            graph = ctx.graph_end()

        def step():
            if ex == "graph":
                ctx.graph_launch(graph)
                ctx.sync()
                return
            if ex == "drain":
                ctx.batch_begin()
            ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
            if ex == "drain":
                ctx.batch_end()
            ctx.sync()

        steps = max(args.steps, 200)
        for _ in range(max(args.warmup, 10)):
            step()
        # HIP events on one dispatch per step (plain: every 8th of the 8
        # per-task dispatches) during the timed steps
        ctx.profile(True, every=8 if ex == "plain" else 1)
        ctx.profile_reset()
        times = []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            step()
            times.append(time.perf_counter() - s0)
        total = time.perf_counter() - t0
        prof = ctx.profile_get()
        out = y.read()
        if graph is not None:
            ctx.graph_destroy(graph)
        ctx.close()
        del arena
        # every executor's output is the plain path's, bit for bit
        if ex == "plain":
            ref_out = out
        elif not np.array_equal(out, ref_out):
            raise RuntimeError("stencil1d %s output differs from the plain path's" % ex)
        # a graph replay is timed as a whole (queue upload, counter clear,
        # drain, status copy)
        kname = {"plain": "stencil1d_f32", "grouped": "stencil1d_f32", "drain": "drain", "graph": "graph"}[ex]
        k = prof[kname]
        per_dispatch = {"plain": chunk * 8, "grouped": n * 8, "drain": n * 8, "graph": n * 8}[ex]
        avg_ms = k["total_ms"] / k["dispatches"]
        res[ex] = {"gbs": n * 8 / (total / steps) / 1e9, "us_per_launch": total / steps * 1e6,
                   "p50_us": pct(times, 50) * 1e3, "p99_us": pct(times, 99) * 1e3,
                   "kernel_gbs": per_dispatch / (avg_ms * 1e-3) / 1e9, "kernel_avg_us": avg_ms * 1e3,
                   "dispatches_per_launch": {"plain": 8, "grouped": 1, "drain": 1, "graph": 1}[ex], "steps": steps}
        log("%s: %s" % (ex, json.dumps(res[ex])))
    m = res["plain"]
    line = base_line({"workload": "stencil1d 2^20 f32 ~U(-1,1) seed 0, 8 chunks of 2^17, one launch per step, "
                                  "plain per-chunk dispatches, data warm in the 256 MB Infinity Cache",
                      "executor": "plain"}, m["steps"], max(args.warmup, 10))
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["us_per_launch"] / 1e3, 5),
                 "dtype": "f32", "p50_us": round(m["p50_us"], 2), "p99_us": round(m["p99_us"], 2),
                 "roofline": {"bound": "hbm", "achieved": round(m["kernel_gbs"], 2), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(m["kernel_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                              "kernel": "k_stencil1d", "kernel_avg_us": round(m["kernel_avg_us"], 3),
                              "note": "launch-latency bound: 1 MiB per dispatch, data cache-resident"}})
    for ex in ("grouped", "drain", "graph"):
        r = res[ex]
        line[ex] = {"value": round(r["gbs"], 2), "p50_us": round(r["p50_us"], 2), "p99_us": round(r["p99_us"], 2),
                    "kernel_gbs": round(r["kernel_gbs"], 2)}
    line["graph"]["note"] = "kernel_gbs times the whole replay (queue upload, counter clear, drain, status copy)"
    return line


# ====================================================== runtime-compiled body
# The paper's example stencil as a user __device__ function (Sec. 3.5), with
# the 1-D stencil workload's weights; compiled at run time by the library.
USER_STENCIL = r"""
__device__ void stencil(dim3 virtBlockIdx, int n, lt::Vector<float> output, const lt::Vector<float> input) {
    int i = blockDim.x * virtBlockIdx.x + threadIdx.x;
    if (i >= n) return;
    float left = i - 1 >= 0 ? input[i - 1] : 0.0f;
    float mid = input[i];
    float right = i + 1 < n ? input[i + 1] : 0.0f;
    output[i] = 0.25f * (left + right) + 0.5f * mid;
}
"""
# The same arithmetic written for bandwidth: four elements per thread with
# 16-byte accesses through the views (the rows are 16-byte aligned in the
# chunks this benchmark uses), scalar halo reads at the ends.
USER_STENCIL4 = r"""
__device__ void stencil4(dim3 virtBlockIdx, long long n, lt::Vector<float> output, const lt::Vector<float> input) {
    const long long i0 = ((long long)virtBlockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    if (i0 + 4 <= n) {
        const float4 c = *reinterpret_cast<const float4 *>(&input[i0]);
        const float l = i0 > 0 ? input[i0 - 1] : 0.0f;
        const float r = i0 + 4 < n ? input[i0 + 4] : 0.0f;
        float4 o;
        o.x = 0.25f * (l + c.y) + 0.5f * c.x;
        o.y = 0.25f * (c.x + c.z) + 0.5f * c.y;
        o.z = 0.25f * (c.y + c.w) + 0.5f * c.z;
        o.w = 0.25f * (c.z + r) + 0.5f * c.w;
        typedef float v4 __attribute__((ext_vector_type(4)));
        const v4 ov = {o.x, o.y, o.z, o.w};
        __builtin_nontemporal_store(ov, reinterpret_cast<v4 *>(&output[i0]));
    } else {
        for (long long i = i0; i < n; ++i) {
            const float l = i > 0 ? input[i - 1] : 0.0f;
            const float r = i + 1 < n ? input[i + 1] : 0.0f;
            output[i] = 0.25f * (l + r) + 0.5f * input[i];
        }
    }
}
"""


def bench_rtc(args, L, torch):
    """Runtime-compiled user bodies beside the built-in body on the same
    launches: the 1-D stencil workload (2^20, 8 chunks, plain and grouped:
    launch-bound) and a 2^28-element field in 8 chunks (grouped, HBM-bound).
    Two user bodies: the paper's example (one element per thread) and the
    same arithmetic with four elements per thread and 16-byte accesses.
    Reports wall time per launch, device time per dispatch (HIP events) and
    the compile time of the user bodies' versions."""
    import synthetic

    cases = [("c1_plain", 1 << 20, 1 << 17, 0, 200), ("c1_grouped", 1 << 20, 1 << 17, 1, 200),
             ("large_grouped", 1 << 28, 1 << 25, 1, 20)]
    res = {}
    for tag, n, chunk, mode, steps in cases:
        x0 = synthetic.stencil1d_input(n, 0)
        ref = None
        for body in ("builtin", "user", "user4"):
            nbytes = 2 * n * 4 + (64 << 20)
            arena = torch_arena(torch, nbytes)
            ctx = L.Context(device_budget_bytes=nbytes, device_arena=arena.data_ptr(), arena_bytes=nbytes,
                            exec_mode=mode)
            name, grid, sbk = "stencil1d_f32", n, chunk
            before = L.Context.rtc_stats()
            if body == "user":
                ctx.define_source("user_stencil", USER_STENCIL, "stencil",
                                  [("n", "int"), ("output", np.float32, 1), ("input", np.float32, 1)],
                                  "global i => read input[i-1:i+1], write output[i]")
                name = "user_stencil"
            elif body == "user4":
                ctx.define_source("user_stencil4", USER_STENCIL4, "stencil4",
                                  [("n", "int"), ("output", np.float32, 1), ("input", np.float32, 1)],
                                  "global i => read input[4*i-1:4*i+4], write output[4*i:4*i+3]")
                name, grid, sbk = "user_stencil4", (n + 3) // 4, chunk // 4
            x = ctx.array([n], chunk=[chunk])
            y = ctx.array([n], chunk=[chunk])
            x.write(x0)
            ctx.sync()

            def step():
                ctx.launch(name, [grid], [256], [sbk], args=[n, y, x])
                ctx.sync()

            for _ in range(max(args.warmup, 5)):
                step()
            out = y.read()
            if ref is None:
                ref = out
            ctx.profile(True)
            ctx.profile_reset()
            times = []
            t0 = time.perf_counter()
            for _ in range(steps):
                s0 = time.perf_counter()
                step()
                times.append(time.perf_counter() - s0)
            total = time.perf_counter() - t0
            prof = ctx.profile_get()
            ctx.close()
            del arena
            k = prof[{"builtin": "stencil1d_f32", "user": "stencil", "user4": "stencil4"}[body]]
            avg_ms = k["total_ms"] / k["dispatches"]
            per_dispatch = n * 8 / k["dispatches"] * steps
            r = {"us_per_launch": total / steps * 1e6, "gbs": n * 8 / (total / steps) / 1e9,
                 "p50_us": pct(times, 50) * 1e3, "p99_us": pct(times, 99) * 1e3,
                 "kernel_avg_us": avg_ms * 1e3, "kernel_gbs": per_dispatch / (avg_ms * 1e-3) / 1e9,
                 "dispatches_per_launch": k["dispatches"] / steps, "same_result": bool(np.array_equal(out, ref))}
            if body != "builtin":
                after = L.Context.rtc_stats()
                r["versions_compiled"] = after["compiles"] - before["compiles"]
                r["compile_s"] = after["compile_seconds"] - before["compile_seconds"]
            res.setdefault(tag, {})[body] = r
            log("%s %s: %s" % (tag, body, json.dumps(r)))
        for body in ("user", "user4"):
            res[tag][body + "_over_builtin_wall"] = (res[tag][body]["us_per_launch"] /
                                                     res[tag]["builtin"]["us_per_launch"])
    m = res["large_grouped"]["user4"]
    line = base_line({"workload": "runtime-compiled user stencil body (the paper's example kernel with "
                                  "0.25/0.5/0.25 weights, four elements per thread) on a 2^28 f32 field "
                                  "~U(-1,1) seed 0, 8 chunks of 2^25, grouped dispatch, beside the built-in body",
                      "executor": "grouped"}, cases[-1][4], max(args.warmup, 5))
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["us_per_launch"] / 1e3, 4),
                 "dtype": "f32", "p50_ms": round(m["p50_us"] / 1e3, 4), "p99_ms": round(m["p99_us"] / 1e3, 4),
                 "roofline": {"bound": "hbm", "achieved": round(m["kernel_gbs"], 2), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(m["kernel_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                              "kernel": "lt_rtc_* (user stencil4)", "kernel_avg_us": round(m["kernel_avg_us"], 2)},
                 "cases": {t: {b: ({k: (round(v, 4) if isinstance(v, float) else v) for k, v in res[t][b].items()}
                                   if isinstance(res[t][b], dict) else round(res[t][b], 4)) for b in res[t]}
                           for t in res}})
    return line


# ================================================================= gemm_ooc
def bench_gemm_ooc(args, L, torch):
    import synthetic

    n, T = 65536, 4096
    steps = args.steps if args.steps_given else 3
    warmup = args.warmup if args.warmup_given else 1
    streams = args.compute_streams or 1
    band = args.sb_band
    if band > 0:
        order, order_name = L.LT_ORDER_BANDS, "bands of %d superblock rows, column by column" % band
    else:
        order, order_name = L.LT_ORDER_SERPENTINE, "serpentine order"
    ctx = L.Context(device_budget_bytes=16 << 30, stage_threshold_bytes=8 << 30, sb_order=order, sb_band=max(band, 0),
                    n_compute_streams=streams)
    try:
        log("allocating 48 GiB of pinned host memory")
        A = ctx.pinned((n, n))
        B = ctx.pinned((n, n))
        Cm = ctx.pinned((n, n))
        log("generating operands")
        synthetic.gemm_operand(0, n, T, out=A, workers=16)
        synthetic.gemm_operand(1, n, T, out=B, workers=16)
        a = ctx.array_host(A, chunk=[T, 0])
        b = ctx.array_host(B, chunk=[0, T])
        c = ctx.array_host(Cm, chunk=[T, T])

        def step():
            ctx.launch("gemm_f32", [n, n], [1, 1], [T, T], args=[n, n, n, c, a, b])
            ctx.sync()

        for _ in range(warmup):
            step()
        ctx.profile(True)
        ctx.profile_reset()
        ctx.reset_stats()
        times = []
        for i in range(steps):
            log("timed step %d" % i)
            s0 = time.perf_counter()
            step()
            times.append(time.perf_counter() - s0)
        total = sum(times)
        prof = ctx.profile_get()["gemm_f32"]
        overlap = copy_overlap(ctx.profile_spans())
        log("copy/compute overlap over the timed steps: %s" % json.dumps(overlap))
        st = ctx.stats()
        cpu = None
        if not args.no_cpu:
            cpu = gemm_cpu_baseline(A, B, n)
    finally:
        ctx.close()
    flops = 2.0 * n ** 3
    wall = total / steps
    kernel_tflops = flops / (prof["total_ms"] / steps * 1e-3) / 1e12
    compulsory = 3 * n * n * 4
    h2d = st["bytes_h2d"] / steps
    d2h = st["bytes_d2h"] / steps
    line = base_line({"workload": "out-of-core GEMM 65536^3 f32 ~N(0,1) seed 2, A/B/C in pinned host memory "
                                  "(48 GiB), device budget 16 GiB, 4096^2 superblocks in " + order_name,
                      "executor": "plain", "stage_threshold_bytes": 8 << 30, "compute_streams": streams},
                     steps, warmup)
    line.update({"value": round(compulsory / wall / 1e9, 2), "unit": "GB/s", "ms_per_step": round(wall * 1e3, 2),
                 "dtype": "f32", "tflops_wall": round(flops / wall / 1e12, 2),
                 "mfma_frac_wall": round(flops / wall / 1e12 / MFMA_FP32_PEAK, 4),
                 "link": {"h2d_gib": round(h2d / 2**30, 2), "d2h_gib": round(d2h / 2**30, 2),
                          "compulsory_gib": 48.0, "h2d_gbs_avg": round(h2d / wall / 1e9, 2),
                          "link_busy_frac_at_57gbs": round((h2d + d2h) / 57e9 / wall, 3)},
                 "kernel_busy_frac": round(prof["total_ms"] / steps * 1e-3 / wall, 4),
                 "overlap": overlap,
                 "p50_ms": round(pct(times, 50), 2), "p99_ms": round(pct(times, 99), 2),
                 "roofline": {"bound": "mfma", "achieved": round(kernel_tflops, 2), "peak": MFMA_FP32_PEAK,
                              "unit": "TFLOP/s", "frac": round(kernel_tflops / MFMA_FP32_PEAK, 4), "traffic": traffic_for("k_gemm"),
                              "kernel": "k_gemm", "kernel_avg_ms": round(prof["total_ms"] / prof["dispatches"], 3)}})
    if cpu:
        line["cpu_baseline"] = cpu
    return line


def gemm_cpu_baseline(A, B, n, rows=16):
    """The oracle's float64-accumulated product timed on ``rows`` rows of C
    (a panel of A times all of B): one warm-up panel, then the median of
    five, extrapolated to the whole product by FLOP count."""
    import oracle

    oracle.gemm(A[:rows], B)
    med, ts = median_runs(lambda: oracle.gemm(A[rows:2 * rows], B))
    rate = 2.0 * rows * n * n / med
    return {"value": round(rate / 1e12, 4), "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "median of 5 runs of %d rows of C (A panel %d x %d times B %d x %d) after a warm-up "
                      "panel; runs %.2f-%.2f s; extrapolated to the whole 65536^3 product: %.0f s"
                      % (rows, rows, n, n, n, min(ts), max(ts), 2.0 * n ** 3 / rate)}


# ==================================================================== batch
def bench_batch(args, L, torch):
    import synthetic
    from paper_2202_05549_amd import autotune

    plan = synthetic.batch_plan(8192)
    ns = np.array([n for _, n in plan], dtype=np.int64)
    kinds = np.array([k for k, _ in plan])
    names = ["stencil1d_f32" if k == 0 else "hist256_i32" for k in kinds]
    elems = int(ns.sum())
    algo_bytes = int((ns[kinds == 0] * 8).sum() + (ns[kinds == 1] * 4).sum() + 1024 * (kinds == 1).sum())
    budget = int(algo_bytes * 1.05) + (8 << 30)
    arena = torch_arena(torch, budget)
    ctx = L.Context(device_budget_bytes=budget, device_arena=arena.data_ptr(), arena_bytes=budget)
    log("creating %d arrays (%.1f GB of inputs and outputs), inputs from the seeded recipe" %
        (len(plan), algo_bytes / 1e9))
    from concurrent.futures import ThreadPoolExecutor

    # launch l's input is synthetic.batch_data(kind, n, l, seed 3), as in the
    # tests; drawn by a pool of threads, written in launch order
    arrs = []
    with ThreadPoolExecutor(16) as ex:
        futs = [ex.submit(synthetic.batch_data, k, n, l, 3) for l, (k, n) in enumerate(plan[:64])]
        for l, (k, n) in enumerate(plan):
            v = futs[l].result()
            futs[l] = None
            if l + 64 < len(plan):
                kk, nn = plan[l + 64]
                futs.append(ex.submit(synthetic.batch_data, kk, nn, l + 64, 3))
            if k == 0:
                x = ctx.array([n])
                y = ctx.array([n])
            else:
                x = ctx.array([n], np.int32)
                y = ctx.array([256], np.int32)
            x.write(v)
            arrs.append((y, x))
    torch.cuda.synchronize()
    grids = ns[:, None]
    res = {}
    # outputs of a fixed sample of launches (the largest, the smallest and a
    # seeded draw) after each executor: every executor must give the plain
    # path's results bit for bit
    order = np.argsort(ns)
    sample = sorted(set(np.random.default_rng(17).choice(len(plan), 48, replace=False).tolist())
                    | set(order[-6:].tolist()) | set(order[:2].tolist()))
    sample_out = {}

    def run(mode, sb, wg=1024, flush=0, steps=None, times=None, graph=None, vec=0, tile=0):
        ctx.configure(drain_workgroups=wg, batch_flush_tasks=flush, drain_vectors=vec, drain_tile=tile)
        sbs = np.full((len(plan), 1), sb, dtype=np.int64)
        args_t = L.Context.arg_table(len(plan), [ns, [a[0] for a in arrs], [a[1] for a in arrs]])
        s0 = time.perf_counter()
        if mode == "graph":
            ctx.graph_launch(graph)
        else:
            if mode == "batched":
                ctx.batch_begin()
            ctx.launch_many(names, grids, [1], sbs, args_t)
            if mode == "batched":
                ctx.batch_end()
        ctx.sync()
        dt = time.perf_counter() - s0
        if times is not None:
            times.append(dt)
        return dt

    if args.tuned:
        # fixed parameters instead of the sweep (counter runs of one configuration)
        sb, wg, flush, vec, tile = (int(v) for v in args.tuned.split(":"))
        best = {"sb": sb, "wg": wg, "flush": flush, "vec": vec, "tile": tile}
        best_plain = {"sb": sb}
        log("fixed parameters: %s" % best)
    else:
        log("autotuning superblock size, drain width, flush size, vector groups and tile size on the full mix")
        # coordinate descent from the library defaults, two timings per
        # point, and the three fastest points timed twice more
        best = autotune.tune("batch8192", {"sb": [1 << 20, 1 << 22, 1 << 24], "wg": [1024, 2048],
                                           "flush": [0, 4096], "vec": [2, 4], "tile": [0, 16384, 32768]},
                             lambda sb, wg, flush, vec, tile: run("batched", sb, wg, flush, vec=vec, tile=tile),
                             reps=2, cache=None, log=log, strategy="descent", confirm=2,
                             start={"sb": 1 << 24, "wg": 1024, "flush": 0, "vec": 4, "tile": 0})
        log("tuned: %s" % best)
        best_plain = autotune.tune("batch8192_plain", {"sb": [1 << 18, 1 << 20, 1 << 22, 1 << 24]},
                                   lambda sb: run("plain", sb), reps=2, cache=None, log=log)
        log("tuned plain: %s" % best_plain)
    modes = ("batched", "graph") if args.executor == "drain" else ("plain", "batched", "graph")
    for mode in modes:
        graph = None
        if mode == "graph":
            ctx.configure(drain_workgroups=best["wg"], batch_flush_tasks=0, drain_vectors=best["vec"],
                          drain_tile=best["tile"])
            ctx.graph_begin()
            ctx.launch_many(names, grids, [1], np.full((len(plan), 1), best["sb"], dtype=np.int64),
                            L.Context.arg_table(len(plan), [ns, [a[0] for a in arrs], [a[1] for a in arrs]]))
            graph = ctx.graph_end()
        sb = best_plain["sb"] if mode == "plain" else best["sb"]
        for _ in range(args.warmup):
            run(mode, sb, best["wg"], best["flush"] if mode == "batched" else 0, graph=graph, vec=best["vec"],
                tile=best["tile"])
        ctx.profile(mode != "plain")
        ctx.profile_reset()
        ctx.reset_stats()
        times = []
        for _ in range(args.steps):
            run(mode, sb, best["wg"], best["flush"] if mode == "batched" else 0, times=times, graph=graph,
                vec=best["vec"], tile=best["tile"])
        prof = ctx.profile_get()
        stats = ctx.stats()
        ctx.profile(False)
        if graph is not None:
            ctx.graph_destroy(graph)
        outs = [arrs[i][0].read() for i in sample]
        if mode == "plain":
            sample_out["plain"] = outs
        elif "plain" not in sample_out:
            sample_out[mode] = None
        else:
            same = all(np.array_equal(a, b) for a, b in zip(outs, sample_out["plain"]))
            sample_out[mode] = same
            log("%s: %d sampled launches identical to plain: %s" % (mode, len(sample), same))
        wall = float(np.mean(times))
        r = {"gbs": algo_bytes / wall / 1e9, "ms_per_step": wall * 1e3, "p50_ms": pct(times, 50),
             "p99_ms": pct(times, 99), "dispatches_per_step": stats["dispatches"] / args.steps,
             "tasks_per_step": stats["tasks"] / args.steps, "plan_ms_per_step": stats["plan_seconds"] / args.steps * 1e3}
        # device time of the drain dispatches; a graph replay is timed as a
        # whole (queue upload, counter clear, drain, flag copy)
        kname = "graph" if mode == "graph" else "drain"
        if kname in prof:
            k = prof[kname]
            r["drain_ms"] = k["total_ms"] / args.steps
            r["kernel_gbs"] = algo_bytes / (r["drain_ms"] * 1e-3) / 1e9
        res[mode] = r
        log("%s: %s" % (mode, json.dumps(r)))
    # the batching pattern's two executors: a batch drained per step, or the
    # same batch recorded once as a HIP graph and replayed
    ex = "graph" if res["graph"]["gbs"] > res["batched"]["gbs"] else "batched"
    m = res[ex]
    line = base_line({"workload": "batching: 8192 independent launches, stencil1d f32 ~U(-1,1) and hist256 int32 "
                                  "bounded Zipf(1.1), sizes floor(2^U(10,24)) seed 3 (%d elements)" % elems,
                      "executor": {"graph": "batch recorded as a HIP graph (persistent drain), replayed",
                                   "batched": "batched (persistent drain)"}[ex],
                      "superblock": best["sb"], "drain_workgroups": best["wg"], "batch_flush_tasks": best["flush"],
                      "drain_vectors": best["vec"], "drain_tile": best["tile"], "plain_superblock": best_plain["sb"]},
                     args.steps, args.warmup)
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["ms_per_step"], 3),
                 "dtype": "f32+i32", "p50_ms": round(m["p50_ms"], 3), "p99_ms": round(m["p99_ms"], 3),
                 "hbm_frac": round(m["gbs"] / HBM_PEAK_GBS, 4),
                 "roofline": {"bound": "hbm", "achieved": round(m.get("kernel_gbs", float("nan")), 2),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(m.get("kernel_gbs", float("nan")) / HBM_PEAK_GBS, 4),
                              # counters were taken on one drain per step at superblock 2^24
                              # with 4-vector groups
                              "traffic": (traffic_for("k_drain") if ex == "graph" and best["sb"] == 1 << 24
                                          and best["tile"] == DRAIN_TRAFFIC_TILE and best["vec"] == 4 else None),
                              "kernel": "k_drain", "kernel_ms_per_step": round(m.get("drain_ms", float("nan")), 3)},
                 "plain": {k: round(v, 3) for k, v in res["plain"].items()} if "plain" in res else None,
                 "batched": {k: round(v, 3) for k, v in res["batched"].items()},
                 "graph": {k: round(v, 3) for k, v in res["graph"].items()},
                 "batched_over_plain": round(res["batched"]["gbs"] / res["plain"]["gbs"], 3) if "plain" in res else None,
                 "graph_over_plain": round(res["graph"]["gbs"] / res["plain"]["gbs"], 3) if "plain" in res else None,
                 "sample_check": {"launches": len(sample),
                                  "elements": int(ns[sample].sum()),
                                  "batched_equals_plain": sample_out["batched"],
                                  "graph_equals_plain": sample_out["graph"]}})
    if not args.no_cpu:
        line["cpu_baseline"] = batch_cpu_baseline(plan, sample)
    ctx.close()
    del arena
    return line


def batch_cpu_baseline(plan, sample, budget_s=12.0):
    """The oracle's stencil and histogram over the inputs of a sample of the
    mix's launches (the same seeded recipe): one warm-up pass, then five runs
    of repeated passes, about budget_s of CPU work in all; GB/s of
    algorithmic bytes at the median run."""
    import oracle
    import synthetic

    data = [(plan[i][0], synthetic.batch_data(plan[i][0], plan[i][1], i, 3)) for i in sample]
    nbytes = sum(v.size * (8 if k == 0 else 4) + (0 if k == 0 else 1024) for k, v in data)

    def one_pass():
        for k, v in data:
            oracle.stencil1d(v) if k == 0 else oracle.hist256(v)
    t0 = time.perf_counter()
    one_pass()
    one = time.perf_counter() - t0
    reps = int(max(1, min(40, budget_s / 5 / max(one, 1e-3))))

    def run():
        for _ in range(reps):
            one_pass()
    med, ts = median_runs(run)
    return {"value": round(reps * nbytes / med / 1e9, 3), "unit": "GB/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "%d launches of the mix (%d elements): median of 5 runs of %d passes after a warm-up "
                      "pass; runs %.2f-%.2f s" % (len(data), sum(v.size for _, v in data), reps, min(ts), max(ts))}


# ==================================================================== serve
# ============================================================ jacobi_tiled
def bench_jacobi_tiled(args, L, torch):
    """The same Jacobi sweeps over a tiled distribution (2048 x 2048 tiles,
    superblock = tile): plain tiles, whose halo reads must be assembled from
    up to 9 chunks, against halo tiles (STENCIL, halo 1), whose reads are
    served by one chunk after its replicas are refreshed from their owners;
    row slabs (512 rows, contiguous in HBM) for reference."""
    import synthetic

    n, sweeps, T = 16384, 20, 2048
    x0 = synthetic.jacobi2d_input(n, seed=1)
    step_bytes = sweeps * n * n * 8
    budget = 4 * n * n * 4 + (1 << 30)
    res = {}
    for name, chunk, halo, sb in (("halo_tiles", [T, T], [1, 1], [T, T]), ("plain_tiles", [T, T], None, [T, T]),
                                  ("row_slabs", [512, 0], None, [512, 0])):
        arena = torch_arena(torch, budget)
        ctx = L.Context(device_budget_bytes=budget, device_arena=arena.data_ptr(), arena_bytes=budget,
                        exec_mode=L.LT_EXEC_GROUPED)
        try:
            a = ctx.array([n, n], chunk=chunk, halo=halo)
            b = ctx.array([n, n], chunk=chunk, halo=halo)
            a.write(x0)
            b.fill(0.0)
            ctx.sync()

            def step():
                inp, out = a, b
                for _ in range(sweeps):
                    ctx.launch("jacobi2d_f32", [n, n], [1, 256], sb, args=[n, n, out, inp])
                    inp, out = out, inp
                ctx.sync()

            for _ in range(args.warmup):
                step()
            ctx.reset_stats()
            times = []
            for _ in range(args.steps):
                s0 = time.perf_counter()
                step()
                times.append(time.perf_counter() - s0)
            st = ctx.stats()
        finally:
            ctx.close()
            del arena
        wall = float(np.mean(times))
        res[name] = {"gbs": step_bytes / wall / 1e9, "ms_per_step": wall * 1e3,
                     "d2d_gb_per_step": st["bytes_d2d"] / args.steps / 1e9,
                     "assembled_per_step": st["assembled_regions"] / args.steps,
                     "halo_copies_per_step": st["halo_copies"] / args.steps,
                     "dispatches_per_step": st["dispatches"] / args.steps}
        log("%s: %s" % (name, json.dumps(res[name])))
    m = res["halo_tiles"]
    line = base_line({"workload": "jacobi2d 16384x16384 f32, 20 sweeps, 2048x2048 tiles with a one-element halo "
                                  "(STENCIL distribution), superblock = tile, in HBM",
                      "executor": "grouped"}, args.steps, args.warmup)
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["ms_per_step"], 3),
                 "dtype": "f32", "hbm_frac": round(m["gbs"] / HBM_PEAK_GBS, 4),
                 "plain_tiles": {k: round(v, 3) for k, v in res["plain_tiles"].items()},
                 "row_slabs": {k: round(v, 3) for k, v in res["row_slabs"].items()},
                 "halo_over_plain_tiles": round(m["gbs"] / res["plain_tiles"]["gbs"], 3),
                 "halo_tiles": {k: round(v, 3) for k, v in m.items()}})
    return line


# ===================================================================== disk
def bench_disk(args, L, torch):
    """Out-of-core Jacobi through the memory hierarchy: 8192 x 8192 float32
    ping-pong fields (512 MiB) with a 128 MiB device budget.  Spilled chunks
    live in pinned host memory (no host budget), or, with a 128 MiB host
    budget, the rest move to the spill file (the disk tier)."""
    import tempfile

    import synthetic

    n, sweeps, rows = 8192, 10, 512
    x0 = synthetic.jacobi2d_input(n, seed=1)
    step_bytes = sweeps * n * n * 8
    res = {}
    spill_dir = tempfile.mkdtemp(prefix="lt_bench_")
    for name, hb in (("host_tier", 0), ("disk_tier", 128 << 20)):
        ctx = L.Context(device_budget_bytes=128 << 20, host_budget_bytes=hb, spill_dir=spill_dir,
                        stage_threshold_bytes=64 << 20)
        try:
            a = ctx.array([n, n], chunk=[rows, 0])
            b = ctx.array([n, n], chunk=[rows, 0])
            a.write(x0)
            b.fill(0.0)
            ctx.sync()
            inp, out = a, b
            # one untimed pass pins the spill buffers (first touch), then a
            # timed pass of the same sweeps
            for timed in (False, True):
                ctx.reset_stats()
                s0 = time.perf_counter()
                for _ in range(sweeps):
                    ctx.launch("jacobi2d_f32", [n, n], [1, 256], [rows, 0], args=[n, n, out, inp])
                    inp, out = out, inp
                ctx.sync()
                wall = time.perf_counter() - s0
            st = ctx.stats()
        finally:
            ctx.close()
        res[name] = {"gbs": step_bytes / wall / 1e9, "ms_per_step": wall * 1e3,
                     "h2d_gb": st["bytes_h2d"] / 1e9, "d2h_gb": st["bytes_d2h"] / 1e9,
                     "disk_write_gb": st["bytes_disk_write"] / 1e9, "disk_read_gb": st["bytes_disk_read"] / 1e9,
                     "disk_gbs": (st["bytes_disk_write"] + st["bytes_disk_read"]) / wall / 1e9}
        log("%s: %s" % (name, json.dumps(res[name])))
    m = res["disk_tier"]
    line = base_line({"workload": "jacobi2d 8192x8192 f32, 10 sweeps, 512-row chunks, device budget 128 MiB, "
                                  "host spill budget 128 MiB, the rest in a spill file (disk tier)",
                      "executor": "plain"}, 1, 1)
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["ms_per_step"], 2),
                 "dtype": "f32", "disk_tier": {k: round(v, 3) for k, v in m.items()},
                 "host_tier": {k: round(v, 3) for k, v in res["host_tier"].items()},
                 "disk_over_host": round(m["gbs"] / res["host_tier"]["gbs"], 3)})
    return line


# =================================================================== kmeans
def bench_kmeans(args, L, torch):
    """The K-Means loop: assignment, centre update (reduce(+) of per-cluster
    sums and counts) and new centres, 5 rounds over points resident in HBM."""
    import synthetic

    N, d, K, iters, sb = 1 << 26, 16, 64, 5, 1 << 22
    log("generating %d points (d=%d, K=%d)" % (N, d, K))
    X, mu, _ = synthetic.kmeans_blobs(N, d, K, seed=4)
    cen0 = (mu + np.random.default_rng(5).normal(0, 1.5, mu.shape)).astype(np.float32)
    step_bytes = iters * N * 2 * (d * 4 + 4)
    budget = N * (d * 4 + 4) + (1 << 30)
    arena = torch_arena(torch, budget)
    ctx = L.Context(device_budget_bytes=budget, device_arena=arena.data_ptr(), arena_bytes=budget,
                    exec_mode=L.LT_EXEC_GROUPED)
    try:
        x = ctx.array([N, d], chunk=[sb, 0])
        lb = ctx.array([N], np.int32, chunk=[sb])
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        cen = ctx.array([K, d])
        x.write(X)
        del X
        ctx.sync()
        if args.kmu_variant:
            ctx.tune("kmeans_update_f32", args.kmu_variant)
        if args.kma_variant:
            ctx.tune("kmeans_assign_f32", args.kma_variant)

        def step():
            cen.write(cen0)
            for _ in range(iters):
                ctx.launch("kmeans_assign_f32", [N], [256], [sb], args=[N, d, K, lb, x, cen])
                ctx.launch("kmeans_update_f32", [N], [1], [sb], args=[N, d, K, sums, counts, x, lb])
                ctx.launch("kmeans_centres_f32", [K, d], [1, 16], [K, d], args=[K, d, cen, sums, counts])
            ctx.sync()

        for _ in range(args.warmup):
            step()
        ctx.profile(True)
        ctx.profile_reset()
        times = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            step()
            times.append(time.perf_counter() - s0)
        total = time.perf_counter() - t0
        prof = ctx.profile_get()
        ctx.profile(False)
    finally:
        ctx.close()
        del arena
    ka, ku = prof.get("kmeans_assign_f32"), prof.get("kmeans_update_f32")
    log("profile: %s" % json.dumps(prof))
    ms = total / args.steps * 1e3
    gbs = step_bytes / (total / args.steps) / 1e9
    # per dispatch: a launch's 16 superblocks share one dispatch for the
    # assignment; the update runs one dispatch per superblock
    a_avg = ka["total_ms"] / ka["dispatches"]
    u_avg = ku["total_ms"] / ku["dispatches"]
    a_pts = N * iters * args.steps / ka["dispatches"]
    u_pts = N * iters * args.steps / ku["dispatches"]
    a_tflops = a_pts * 3 * K * d / (a_avg * 1e-3) / 1e12
    u_gbs = u_pts * (d * 4 + 4) / (u_avg * 1e-3) / 1e9
    a_share = ka["total_ms"] / (ka["total_ms"] + ku["total_ms"])
    line = base_line({"workload": "k-means loop: %d points d=%d (Gaussian blobs, seed 4), K=%d, 5 rounds of "
                                  "assignment + centre update (float64 reduce(+) of sums and counts) + new centres, "
                                  "%d-point superblocks, in HBM" % (N, d, K, sb),
                      "executor": "grouped"}, args.steps, args.warmup)
    line.update({"value": round(gbs, 2), "unit": "GB/s", "ms_per_step": round(ms, 3), "dtype": "f32+f64",
                 "p50_ms": round(pct(times, 50), 3), "p99_ms": round(pct(times, 99), 3),
                 # peak: the FP32 vector rate (128 lanes per CU per clock, 2 FLOP
                 # per FMA); the sub + FMA per (cluster, feature) issues two
                 # instructions for 3 FLOP, so this body can reach 3/4 of it
                 "roofline": {"bound": "alu", "achieved": round(a_tflops, 2), "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                              "frac": round(a_tflops / FP32_VECTOR_PEAK, 4), "mix_ceiling": round(0.75 * FP32_VECTOR_PEAK, 1),
                              "traffic": traffic_for("k_kmeans"), "kernel": "k_kmeans",
                              "kernel_avg_ms": round(a_avg, 4), "time_share": round(a_share, 3)},
                 "update": {"kernel": "k_kmeans_update", "bound": "hbm", "achieved_gbs": round(u_gbs, 1),
                            "frac": round(u_gbs / HBM_PEAK_GBS, 4), "kernel_avg_ms": round(u_avg, 4),
                            "traffic": traffic_for("k_kmeans_update")}})
    if not args.no_cpu:
        import oracle

        # one round over 2^24 points takes about 1.3 s on the GPU machine's 16 cores
        ns = 1 << 24
        Xs, mus, _ = synthetic.kmeans_blobs(ns, d, K, seed=4)
        c0 = (mus + np.random.default_rng(5).normal(0, 1.5, mus.shape)).astype(np.float32)
        oracle.kmeans_lloyd(Xs, c0, 1)
        med, ts = median_runs(lambda: oracle.kmeans_lloyd(Xs, c0, 1))
        line["cpu_baseline"] = {"value": round(ns * 2 * (d * 4 + 4) / med / 1e9, 3), "unit": "GB/s",
                                "cores": oracle.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
                                "sample": "median of 5 runs of one round over %d points (of %d x 5 per step) "
                                          "after a warm-up round; runs %.2f-%.2f s" % (ns, N, min(ts), max(ts))}
    return line


def link_peak(torch, nbytes=1 << 30, reps=5):
    """Pinned host <-> device copy rates (GB/s) of 1 GiB copies through the
    HIP runtime (torch's copy_, i.e. hipMemcpyAsync), measured here: the
    host-link roofline of the out-of-core legs."""
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    out = {}
    for name, dst, src in (("h2d", d, h), ("d2h", h, d)):
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        out[name] = reps * nbytes / (time.perf_counter() - t0) / 1e9
    del h, d
    return out


def bench_kmeans_ooc(args, L, torch):
    """Out-of-core k-means assignment (the paper's single-GPU K-Means study,
    Sec. 4.3): 10^9 points of d = 16 (64 GB) and their labels in pinned host
    memory, device budget 64 GiB, K = 64.  A step is one assignment pass from
    a cold device (the arrays are created over the host buffers before the
    step and destroyed after it): every chunk of points crosses the host
    link once, every chunk of labels comes back.  Chunk sizes are swept as in
    the paper (64 MiB to 4 GiB of points per chunk); the best one is
    ``value``.  Bound: the host link."""
    import synthetic

    N, d, K = args.kmeans_points, 16, 64
    budget = 64 << 30
    steps = args.steps if args.steps_given else 3
    warmup = args.warmup if args.warmup_given else 1
    link = link_peak(torch)
    log("host link (pinned 1 GiB copies): H2D %.1f GB/s, D2H %.1f GB/s" % (link["h2d"], link["d2h"]))
    arena = torch_arena(torch, budget)
    ctx = L.Context(device_budget_bytes=budget, device_arena=arena.data_ptr(), arena_bytes=budget,
                    stage_threshold_bytes=16 << 30, exec_mode=L.LT_EXEC_GROUPED)
    sweep = [1 << 20, 1 << 22, 1 << 24, 1 << 26]
    res = {}
    try:
        log("allocating %.1f GB of pinned host memory" % (N * (d * 4 + 4) / 1e9))
        X = ctx.pinned((N, d))
        lab = ctx.pinned((N,), np.int32)
        log("generating %d points (d=%d, K=%d) in bands" % (N, d, K))
        _, mu = synthetic.kmeans_blobs_banded(N, d, K, seed=4, out=X)
        cen0 = (mu + np.random.default_rng(5).normal(0, 1.5, mu.shape)).astype(np.float32)
        cen = ctx.array([K, d])
        cen.write(cen0)
        ctx.sync()
        for c in sweep:
            times, h2d, d2h, kms, ovl = [], [], [], [], []
            for it in range(warmup + steps):
                x = ctx.array_host(X, chunk=[c, 0])
                lb = ctx.array_host(lab, chunk=[c])
                ctx.sync()
                ctx.reset_stats()
                ctx.profile(True)
                ctx.profile_reset()
                s0 = time.perf_counter()
                ctx.launch("kmeans_assign_f32", [N], [256], [c], args=[N, d, K, lb, x, cen])
                ctx.sync()
                dt = time.perf_counter() - s0
                st = ctx.stats()
                prof = ctx.profile_get().get("kmeans_assign_f32", {"total_ms": float("nan")})
                spans = ctx.profile_spans()
                ctx.profile(False)
                x.destroy()
                lb.destroy()
                ctx.sync()
                if it >= warmup:
                    times.append(dt)
                    h2d.append(st["bytes_h2d"])
                    d2h.append(st["bytes_d2h"])
                    kms.append(prof["total_ms"])
                    ovl.append(copy_overlap(spans))
            wall = float(np.median(times))
            r = {"chunk_points": c, "chunk_mib": c * d * 4 / 2**20, "wall_ms": wall * 1e3,
                 "p50_ms": pct(times, 50), "p99_ms": pct(times, 99),
                 "gbs": N * (d * 4 + 4) / wall / 1e9,
                 "h2d_gb": float(np.median(h2d)) / 1e9, "d2h_gb": float(np.median(d2h)) / 1e9,
                 "h2d_gbs": float(np.median(h2d)) / wall / 1e9,
                 "kernel_busy_frac": float(np.median(kms)) * 1e-3 / wall,
                 "overlap": ovl[len(ovl) // 2]}
            r["link_frac"] = r["h2d_gbs"] / link["h2d"]
            res[c] = r
            log("chunk %d points (%.0f MiB): %s" % (c, r["chunk_mib"], json.dumps(r)))
    finally:
        ctx.close()
        del arena
    best = max(res, key=lambda c: res[c]["gbs"])
    m = res[best]
    line = base_line({"workload": "out-of-core k-means assignment: %d points d=%d (Gaussian blobs, banded seed 4) "
                                  "and labels in pinned host memory (%.1f GB), K=%d, device budget 64 GiB, "
                                  "one cold pass per step" % (N, d, N * (d * 4 + 4) / 1e9, K),
                      "executor": "grouped", "chunk_points": best}, steps, warmup)
    line.update({"value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["wall_ms"], 2),
                 "dtype": "f32", "p50_ms": round(m["p50_ms"], 2), "p99_ms": round(m["p99_ms"], 2),
                 "roofline": {"bound": "host_link", "achieved": round(m["h2d_gbs"], 2),
                              "peak": round(link["h2d"], 2), "unit": "GB/s", "frac": round(m["link_frac"], 4),
                              "peak_nominal": PCIE_NOMINAL_GBS, "peak_d2h": round(link["d2h"], 2),
                              "traffic": None, "kernel": "k_kmeans (H2D copies bound the pass)"},
                 "overlap": m["overlap"],
                 "chunk_sweep": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in res[c].items()}
                                 for c in sweep]})
    return line


def bench_serve(args, L, torch):
    from paper_2202_05549_amd import serve

    return serve.bench(args, L, torch, log, overlap=copy_overlap)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=["jacobi", "stencil1d", "gemm_ooc", "batch", "serve", "kmeans",
                                           "kmeans_ooc", "jacobi_tiled", "disk", "rtc"],
                    default="jacobi")
    ap.add_argument("--kmeans-points", type=int, default=1_000_000_000,
                    help="kmeans_ooc: points in host memory (default 10^9)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sb-band", type=int, default=0,
                    help="gemm_ooc: superblock rows per band of the banded issue order (0 = serpentine order)")
    ap.add_argument("--rows", type=int, default=0,
                    help="Jacobi tile variant (lt_kernel_tune: 8/16/32, 132/164/228, 302/304/308; 0 = default)")
    ap.add_argument("--executor", choices=["all", "grouped", "drain", "plain"], default="all",
                    help="jacobi: executors to run (all = grouped, drain and plain); batch: drain = the "
                         "batched and graph legs only")
    ap.add_argument("--compute-streams", type=int, default=0,
                    help="gemm_ooc: compute streams of the context (0 = 1)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB float32 device copy first (the reference kernel for HBM counter scaling)")
    ap.add_argument("--kma-variant", type=int, default=0,
                    help="kmeans: assignment body (lt_kernel_tune, d = 16): 0 = default (centres in SGPRs), "
                         "1 = centres broadcast from LDS, 2 = two points per lane")
    ap.add_argument("--kmu-variant", type=int, default=0,
                    help="kmeans: centre-update body (lt_kernel_tune): 0 = default (d 16/32: one feature per "
                         "lane, two LDS copies per wave), 1 = four features per lane, 2 = two features per lane")
    ap.add_argument("--d2h-kernel", type=int, default=0,
                    help="serve: write-backs into pinned homes through the library's row-copy kernel (1) or "
                         "hipMemcpy*Async (0)")
    ap.add_argument("--tuned", default="",
                    help="batch: fixed SB:WG:FLUSH:VEC:TILE instead of the autotuning sweep")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving trace at the full size ranges (GEMM to 65536, k-means to 1e9 points)")
    args = ap.parse_args()
    args.steps_given = args.steps is not None
    args.warmup_given = args.warmup is not None
    if args.steps is None:
        args.steps = 10
    if args.warmup is None:
        args.warmup = 2
    if args.gpus != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not implemented "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2202_05549_amd as L

    if args.calibrate_copy:
        calibration_copy(torch)
    fn = {"jacobi": bench_jacobi, "stencil1d": bench_stencil1d, "gemm_ooc": bench_gemm_ooc, "batch": bench_batch,
          "serve": bench_serve, "kmeans": bench_kmeans, "kmeans_ooc": bench_kmeans_ooc,
          "jacobi_tiled": bench_jacobi_tiled, "rtc": bench_rtc,
          "disk": bench_disk}[args.workload]
    line = fn(args, L, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
