"""CPU tests of the serving loop's host logic (dry-run context, no GPU).

In a dry run no device work is issued and every fence has passed, so these
tests check admission order, the dataset cache, footprints and argument
validation of lt_server_* -- the request results themselves are checked on
the GPU.
"""
import numpy as np
import pytest

import paper_2202_05549_amd as L
from paper_2202_05549_amd import serve


def dry(**kw):
    kw.setdefault("device_budget_bytes", 1 << 30)
    return L.Context(dry_run=1, **kw)


def _bufs(kind, n, d=16, K=64):
    if kind == "jacobi":
        return np.zeros((n, n), np.float32), None, np.zeros((n, n), np.float32)
    if kind == "kmeans":
        return np.zeros((n, d), np.float32), np.zeros((K, d), np.float32), np.zeros(n, np.int32)
    return np.zeros((n, n), np.float32), np.zeros((n, n), np.float32), np.zeros((n, n), np.float32)


def _submit(srv, kind, ds, n, sweeps=3):
    a, b, o = _bufs(kind, n)
    if kind == "jacobi":
        return srv.submit(kind, ds, n, a, out=o, sweeps=sweeps), (a, b, o)
    if kind == "kmeans":
        return srv.submit(kind, ds, n, a, b, out=o, d=16, K=64), (a, b, o)
    return srv.submit(kind, ds, n, a, b, out=o), (a, b, o)


def test_every_request_completes_once_in_order():
    ctx = dry()
    srv = serve.Server(ctx, max_active=3, keep_resident=True, chunk_rows=64, gemm_tile=64)
    keep = []
    ids = []
    plan = [("jacobi", 0, 128), ("kmeans", 1, 1000), ("gemm", 0, 128), ("jacobi", 0, 128), ("gemm", 2, 192)]
    for kind, ds, n in plan:
        rid, bufs = _submit(srv, kind, ds, n)
        ids.append(rid)
        keep.append(bufs)
    done = srv.poll() + srv.drain()
    srv.close()
    ctx.close()
    assert sorted(c["id"] for c in done) == sorted(ids)
    assert len({c["id"] for c in done}) == len(ids)
    assert all(c["status"] == 0 for c in done)
    by = {c["id"]: c for c in done}
    for rid, (kind, _, _) in zip(ids, plan):
        assert by[rid]["kind"] == serve.KINDS[kind]
        assert by[rid]["t_submit"] <= by[rid]["t_admit"] <= by[rid]["t_done"]
    # admission is first come, first served
    adm = [by[r]["t_admit"] for r in ids]
    assert adm == sorted(adm)


def test_dataset_cache_hits_only_when_resident():
    for keep, expect in ((True, [False, True, False, True]), (False, [False, False, False, False])):
        ctx = dry()
        srv = serve.Server(ctx, max_active=2, keep_resident=keep, chunk_rows=64, gemm_tile=64)
        bufs = []
        ids = []
        # same dataset and size twice -> hit; a new dataset -> miss
        for kind, ds, n in (("kmeans", 0, 500), ("kmeans", 0, 500), ("kmeans", 1, 500), ("kmeans", 1, 500)):
            rid, b = _submit(srv, kind, ds, n)
            ids.append(rid)
            bufs.append(b)
        done = {c["id"]: c for c in srv.drain()}
        srv.close()
        ctx.close()
        assert [done[r]["cache_hit"] for r in ids] == expect


def test_footprints():
    ctx = dry()
    srv = serve.Server(ctx, max_active=1, keep_resident=False, chunk_rows=64, gemm_tile=64)
    bufs = []
    ids = {}
    for kind, n, sweeps in (("jacobi", 100, 1), ("jacobi", 100, 2), ("jacobi", 100, 10), ("kmeans", 1000, 0),
                            ("gemm", 96, 0)):
        rid, b = _submit(srv, kind, 0, n, sweeps=sweeps)
        ids[rid] = (kind, n, sweeps)
        bufs.append(b)
    done = srv.drain()
    srv.close()
    ctx.close()
    want = {("jacobi", 100, 1): 100 * 100 * 4 * 2, ("jacobi", 100, 2): 100 * 100 * 4 * 3,
            ("jacobi", 100, 10): 100 * 100 * 4 * 4, ("kmeans", 1000, 0): 1000 * (16 * 4 + 4) + 64 * 16 * 4,
            ("gemm", 96, 0): 3 * 96 * 96 * 4}
    for c in done:
        assert c["footprint"] == want[ids[c["id"]]]


def test_invalid_requests_are_rejected():
    ctx = dry()
    srv = serve.Server(ctx, max_active=2)
    a = np.zeros((8, 8), np.float32)
    with pytest.raises(L.LtError):
        srv.submit("jacobi", 0, 8, a, out=a, sweeps=0)
    with pytest.raises(L.LtError):
        srv.submit("kmeans", 0, 8, a, a, out=a, d=0, K=4)
    with pytest.raises(L.LtError):
        srv.submit("kmeans", 0, 8, a, a, out=a, d=4, K=300)
    with pytest.raises(L.LtError):
        srv.submit("gemm", 0, 8, a, None, out=a)
    with pytest.raises(L.LtError):
        srv.submit(7, 0, 8, a, a, out=a)
    assert srv.drain() == []
    srv.close()
    ctx.close()


def test_trace_replay_dry():
    import synthetic

    trace = synthetic.serving_trace(count=12, rate=1e6, seed=5, pool=2, jacobi_range=(64, 200),
                                    kmeans_range=(1000, 5000), gemm_range=(64, 200))
    ctx = dry()
    srv = serve.Server(ctx, max_active=4, keep_resident=True, chunk_rows=64, gemm_tile=64)
    data = {}
    outs = {}
    for r in trace:
        key = (r["kind"], r["dataset"])
        if key not in data:
            a, b, o = _bufs(r["kind"], r["size"])
            data[key] = (a, b)
            outs[key] = o
        r["sweeps"] = 2
    done, start = serve.replay(srv, trace, serve.submit_with(data, outs), realtime=False)
    srv.close()
    ctx.close()
    assert sorted(done) == list(range(len(trace)))
    s = serve.summarize(trace, done, start)
    assert s["requests"] == len(trace) and s["errors"] == 0
    # every repeated (kind, dataset) after its first request is a hit
    seen = set()
    for i, r in enumerate(trace):
        key = (r["kind"], r["dataset"])
        assert done[i]["cache_hit"] == (key in seen)
        seen.add(key)
