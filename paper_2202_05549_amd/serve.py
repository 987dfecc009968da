"""Serving driver over the C-ABI request loop (lt_server_*).

``Server`` wraps one lt_server.  ``replay`` feeds a request trace to it on
the wall clock (each request is submitted at its arrival time) and polls
for completions; latency is completion time minus arrival time.  ``bench``
is the serving leg of bench.py: the same trace served with continuous
batching (several admitted requests overlapping, inputs resident across
requests) and plain (first come first served, one request at a time, inputs
uploaded again for every request).
"""
from __future__ import annotations

import ctypes as C
import json
import math
import time

import numpy as np

from . import (LT_OK, LT_REQ_GEMM, LT_REQ_JACOBI, LT_REQ_KMEANS, LtError, check, lt_completion,
               lt_now, lt_request, lt_server_config, lt_server_create, lt_server_destroy, lt_server_drain,
               lt_server_poll, lt_server_submit)

KINDS = {"jacobi": LT_REQ_JACOBI, "kmeans": LT_REQ_KMEANS, "gemm": LT_REQ_GEMM}


class Server:
    def __init__(self, ctx, max_active=8, keep_resident=True, admit_bytes=0, chunk_rows=0, gemm_tile=0,
                 lookahead=0, max_bypass=0):
        cfg = lt_server_config()
        cfg.max_active = max_active
        cfg.keep_resident = 1 if keep_resident else 0
        cfg.admit_bytes = admit_bytes
        cfg.chunk_rows = chunk_rows
        cfg.gemm_tile = gemm_tile
        cfg.lookahead = lookahead
        cfg.max_bypass = max_bypass
        self.ctx = ctx
        self.h = C.c_void_p()
        check(ctx.h, lt_server_create(ctx.h, C.byref(cfg), C.byref(self.h)))
        self._buf = (lt_completion * 256)()

    def submit(self, kind, dataset, size, in0, in1=None, out=None, d=0, K=0, sweeps=0):
        r = lt_request()
        r.kind = KINDS[kind] if isinstance(kind, str) else kind
        r.dataset = dataset
        r.size = size
        r.d = d
        r.K = K
        r.sweeps = sweeps
        r.in0 = in0.ctypes.data
        r.in1 = in1.ctypes.data if in1 is not None else None
        r.out = out.ctypes.data
        rid = C.c_uint64()
        check(self.ctx.h, lt_server_submit(self.h, C.byref(r), C.byref(rid)))
        return rid.value

    def _collect(self, fn):
        out = []
        while True:
            n = C.c_int32()
            check(self.ctx.h, fn(self.h, self._buf, len(self._buf), C.byref(n)))
            for i in range(n.value):
                c = self._buf[i]
                out.append({"id": c.id, "status": c.status, "kind": c.kind, "t_submit": c.t_submit,
                            "t_admit": c.t_admit, "t_done": c.t_done, "footprint": c.footprint,
                            "cache_hit": bool(c.cache_hit)})
            if n.value < len(self._buf):
                return out

    def poll(self):
        return self._collect(lt_server_poll)

    def drain(self):
        return self._collect(lt_server_drain)

    def close(self):
        if self.h:
            st = lt_server_destroy(self.h)
            self.h = None
            if st != LT_OK:
                raise LtError(st, "server destroy")


def replay(server, trace, submit_fn, realtime=True, poll_interval=2e-4, progress=None):
    """Submits trace requests at their arrival times (seconds from start) and
    polls until all complete.  ``submit_fn(server, req) -> id``;
    ``progress(done, total)`` (optional) is called after each completion.
    Returns (completions by request index, start time on lt_now's clock)."""
    start = lt_now()
    pending = {}
    done = {}
    i = 0
    while i < len(trace) or pending:
        now = lt_now() - start
        while i < len(trace) and (not realtime or trace[i]["t"] <= now):
            pending[submit_fn(server, trace[i])] = i
            i += 1
        for c in server.poll():
            done[pending.pop(c["id"])] = c
            if progress:
                progress(len(done), len(trace))
        if i < len(trace) and realtime:
            wait = trace[i]["t"] - (lt_now() - start)
            if wait > 0 and not pending:
                time.sleep(min(wait, 0.01))
        elif pending:
            time.sleep(poll_interval)
    return done, start


def request_bytes(req):
    """Algorithmic bytes of one request (the work it must move at least once)."""
    n = req["size"]
    if req["kind"] == "jacobi":
        return 8 * n * n * req.get("sweeps", 10)
    if req["kind"] == "kmeans":
        return n * (16 * 4 + 4)
    return 3 * 4 * n * n


def request_flops(req):
    n = req["size"]
    if req["kind"] == "gemm":
        return 2.0 * n ** 3
    if req["kind"] == "kmeans":
        return 3.0 * 64 * 16 * n
    return 4.0 * n * n * req.get("sweeps", 10)


class HostBuffers:
    """Host buffers of the serving datasets: pinned (lt_host_alloc) while
    the pinned total stays within ``pin_bytes``, pageable numpy memory
    beyond it (copies from pageable memory go through the HIP runtime's own
    staging).  None = no cap."""

    def __init__(self, ctx, pin_bytes=None):
        self.ctx = ctx
        self.cap = pin_bytes
        self.pinned_bytes = 0
        self.pageable_bytes = 0

    def alloc(self, shape, dtype=np.float32):
        nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
        if self.cap is None or self.pinned_bytes + nbytes <= self.cap:
            self.pinned_bytes += nbytes
            return self.ctx.pinned(shape, dtype)
        self.pageable_bytes += nbytes
        return np.empty(shape, dtype=dtype)


def _dataset_bytes(r):
    n = r["size"]
    if r["kind"] == "kmeans":
        return n * (16 * 4 + 4)
    return (2 if r["kind"] == "jacobi" else 3) * 4 * n * n


def _unique(trace):
    """One request per (kind, dataset), smallest footprint first, so that a
    pinned cap leaves only the largest datasets in pageable memory."""
    seen = {}
    for r in trace:
        seen.setdefault((r["kind"], r["dataset"]), r)
    return sorted(seen.values(), key=_dataset_bytes)


def make_datasets(ctx, trace, seed=4, host=None):
    """Host inputs for every (kind, dataset) of the trace."""
    import synthetic

    host = host or HostBuffers(ctx)
    data = {}
    for r in _unique(trace):
        key = (r["kind"], r["dataset"])
        n = r["size"]
        if r["kind"] == "jacobi":
            f = host.alloc((n, n))
            synthetic.jacobi2d_input(n, seed=seed * 1000 + r["dataset"], out=f)
            data[key] = (f, None)
        elif r["kind"] == "kmeans":
            # drawn in bands straight into the host buffer (up to 1e9 points)
            xp = host.alloc((n, 16))
            _, mu = synthetic.kmeans_blobs_banded(n, 16, 64, seed=seed * 1000 + r["dataset"], out=xp)
            cp = ctx.pinned(mu.shape)
            cp[...] = mu
            data[key] = (xp, cp)
        else:
            a = host.alloc((n, n))
            b = host.alloc((n, n))
            synthetic.dense_normal((n, n), [seed, r["dataset"], n, 0], out=a)
            synthetic.dense_normal((n, n), [seed, r["dataset"], n, 1], out=b)
            data[key] = (a, b)
    return data


def submit_with(data, outs):
    """``outs``: dict keyed by (kind, dataset), or a callable taking the
    request and returning its output buffer."""
    def fn(server, r):
        in0, in1 = data[(r["kind"], r["dataset"])]
        out = outs(r) if callable(outs) else outs[(r["kind"], r["dataset"])]
        if r["kind"] == "jacobi":
            return server.submit("jacobi", r["dataset"], r["size"], in0, out=out, sweeps=r.get("sweeps", 10))
        if r["kind"] == "kmeans":
            return server.submit("kmeans", r["dataset"], r["size"], in0, in1, out=out, d=16, K=64)
        return server.submit("gemm", r["dataset"], r["size"], in0, in1, out=out)
    return fn


def output_buffers(ctx, trace, host=None):
    host = host or HostBuffers(ctx)
    outs = {}
    for r in _unique(trace):
        key = (r["kind"], r["dataset"])
        n = r["size"]
        if r["kind"] == "kmeans":
            outs[key] = host.alloc((n,), np.int32)
        else:
            outs[key] = host.alloc((n, n))
    return outs


def summarize(trace, done, start):
    lat = []
    t_first = min(trace[i]["t"] for i in done)
    t_last = max(c["t_done"] - start for c in done.values())
    byts = sum(request_bytes(trace[i]) for i in done)
    flops = sum(request_flops(trace[i]) for i in done)
    for i, c in done.items():
        lat.append(c["t_done"] - start - trace[i]["t"])
    lat = np.array(lat)
    makespan = t_last - t_first
    wait = np.array([c["t_admit"] - c["t_submit"] for c in done.values()])
    service = np.array([c["t_done"] - c["t_admit"] for c in done.values()])
    return {"requests": len(done), "makespan_s": makespan, "req_per_s": len(done) / makespan,
            "gbs": byts / makespan / 1e9, "tflops": flops / makespan / 1e12,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_wait_ms": float(wait.mean() * 1e3), "mean_service_ms": float(service.mean() * 1e3),
            "cache_hits": int(sum(c["cache_hit"] for c in done.values())),
            "errors": int(sum(c["status"] != 0 for c in done.values()))}


def bench(args, L, torch, log, overlap=None):
    """``overlap(spans)``, when given, summarizes the device-clock spans of
    each mode (kernel and host-link copy busy time)."""
    import synthetic

    full = getattr(args, "serve_full", False)
    # the full size ranges with 8 datasets per kind; the default run keeps
    # the ranges below 16384 / 1e8 / 16384 and 4 datasets per kind so that it
    # ends in a minute
    count, pool = (128, 8) if full else (64, 4)
    ranges = dict(jacobi_range=(1024, 32768 if full else 16384), kmeans_range=(1e5, 1e9 if full else 1e8),
                  gemm_range=(1024, 65536 if full else 16384))
    trace = synthetic.serving_trace(count=count, rate=200.0, seed=4, pool=pool, **ranges)
    for r in trace:
        r["sweeps"] = 10
    budget = 64 << 30
    res = {}
    # two compute streams: with the H2D and D2H streams that makes four,
    # the number of hardware queues a process gets by default; more streams
    # would share queues and order unrelated work behind each other
    d2h_kernel = getattr(args, "d2h_kernel", 0)
    ctx = L.Context(device_budget_bytes=budget, n_compute_streams=2, stage_threshold_bytes=8 << 30,
                    sb_order=L.LT_ORDER_SERPENTINE, d2h_kernel=d2h_kernel)
    slots = 16
    try:
        log("serving: generating %d datasets in pinned host memory" % len({(r["kind"], r["dataset"]) for r in trace}))
        # the full trace's datasets (about 130 GB) exceed what one process
        # can pin on the GPU machine (hipHostMalloc fails beyond about 64 GiB in
        # total): the largest inputs then stay in pageable memory.  Outputs
        # are pinned first: a copy into pageable memory blocks the issuing
        # thread until it is done
        host = HostBuffers(ctx, pin_bytes=(56 << 30) if full else None)
        outs = output_buffers(ctx, trace, host=host)
        data = make_datasets(ctx, trace, host=host)
        host_gb = (host.pinned_bytes + host.pageable_bytes) / 1e9
        log("serving: %.1f GB of inputs and outputs (%.1f GB pinned, %.1f GB pageable)"
            % (host_gb, host.pinned_bytes / 1e9, host.pageable_bytes / 1e9))
        # warm-up outside the timed traces: one small request of each kind on
        # datasets the trace never uses (device arena, code objects, streams)
        warm = [{"id": i, "t": 0.0, "kind": k, "dataset": 1000 + i, "size": n, "sweeps": 2}
                for i, (k, n) in enumerate((("jacobi", 512), ("kmeans", 4096), ("gemm", 512)))]
        wdata, wouts = make_datasets(ctx, warm), output_buffers(ctx, warm)
        srv = Server(ctx, max_active=slots, keep_resident=False, admit_bytes=budget)
        try:
            replay(srv, warm, submit_with(wdata, wouts), realtime=False)
        finally:
            srv.close()
        ctx.sync()
        # continuous batching with cached datasets first among the first 64
        # queued requests, the same in arrival order, and plain (one request
        # at a time, in arrival order, inputs uploaded for every request)
        for mode, (act, keep, look) in (("continuous", (slots, True, 64)), ("continuous_fcfs", (slots, True, 0)),
                                        ("plain", (1, False, 0))):
            log("serving %s: %d requests, Poisson 200/s" % (mode, count))
            srv = Server(ctx, max_active=act, keep_resident=keep, admit_bytes=budget, lookahead=look)
            ctx.reset_stats()
            if overlap:
                ctx.profile(True)
                ctx.profile_reset()
            def progress(k, total):
                if k % 16 == 0 or k == total:
                    log("%s: %d of %d requests done" % (mode, k, total))

            try:
                done, start = replay(srv, trace, submit_with(data, outs), progress=progress)
            finally:
                srv.close()
            ctx.sync()
            st = ctx.stats()
            res[mode] = summarize(trace, done, start)
            res[mode].update({"h2d_gb": st["bytes_h2d"] / 1e9, "d2h_gb": st["bytes_d2h"] / 1e9,
                              "dispatches": st["dispatches"]})
            if overlap:
                res[mode]["device_time"] = overlap(ctx.profile_spans())
                ctx.profile(False)
            log("%s: %s" % (mode, json.dumps(res[mode])))
    finally:
        ctx.close()
    m = res["continuous"]
    line = {"metric": "effective GB/s (% HBM or host-link roofline), plain vs batched; p50/p99 latency",
            "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "data": "synthetic",
            "config": {"workload": "serving: %d requests, Poisson 200/s seed 4, kinds uniform over Jacobi "
                                   "(n %d..%d, 10 sweeps), k-means assignment (N %.0e..%.0e, d=16, K=64) and GEMM "
                                   "(n %d..%d), %d datasets per kind with Zipf(1.1) popularity, device budget "
                                   "64 GiB, inputs and outputs in host memory (%.1f GB: %.1f GB pinned, "
                                   "%.1f GB pageable)"
                                   % (count, ranges["jacobi_range"][0], ranges["jacobi_range"][1],
                                      ranges["kmeans_range"][0], ranges["kmeans_range"][1],
                                      ranges["gemm_range"][0], ranges["gemm_range"][1], pool, host_gb,
                                      host.pinned_bytes / 1e9, host.pageable_bytes / 1e9),
                       "executor": "continuous batching, %d slots, resident datasets, cached datasets first "
                                   "among the first 64 queued (at most 256 bypasses)" % slots,
                       "write_backs": "row-copy kernel" if d2h_kernel else "hipMemcpyAsync"},
            "value": round(m["gbs"], 2), "unit": "GB/s", "ms_per_step": round(m["makespan_s"] * 1e3, 2),
            "dtype": "f32+i32", "p50_ms": round(m["p50_ms"], 2), "p99_ms": round(m["p99_ms"], 2),
            "req_per_s": round(m["req_per_s"], 3), "tflops": round(m["tflops"], 2),
            "plain": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in res["plain"].items()},
            "continuous_fcfs": {k: (round(v, 3) if isinstance(v, float) else v)
                                for k, v in res["continuous_fcfs"].items()},
            "served_over_plain": round(res["plain"]["makespan_s"] / m["makespan_s"], 3),
            "fcfs_over_plain": round(res["plain"]["makespan_s"] / res["continuous_fcfs"]["makespan_s"], 3),
            "cache_hits": m["cache_hits"], "h2d_gb": round(m["h2d_gb"], 2), "d2h_gb": round(m["d2h_gb"], 2),
            "device_time": m.get("device_time")}
    return line
