"""GPU tests of the serving loop: every request's result equals the oracle,
and equals the result of the same request served alone (bit for bit: the
same tasks run the same bodies whatever else is admitted)."""
import sys

import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import paper_2202_05549_amd as L
    return L


def _trace():
    tr = synthetic.serving_trace(count=14, rate=2000.0, seed=21, pool=3, jacobi_range=(200, 700),
                                 kmeans_range=(5000, 300000), gemm_range=(100, 900))
    for r in tr:
        r["sweeps"] = 4
    return tr


def _serve(L, trace, max_active, keep, budget=1 << 30, realtime=True, chunk_rows=0, lookahead=0):
    from paper_2202_05549_amd import serve

    outs = {}
    with L.Context(device_budget_bytes=budget, n_compute_streams=2) as ctx:
        data = serve.make_datasets(ctx, trace, seed=21)

        def out_for(r):
            n = r["size"]
            buf = np.full((n,), -1, np.int32) if r["kind"] == "kmeans" else np.full((n, n), np.nan, np.float32)
            outs[r["id"]] = buf
            return buf

        srv = serve.Server(ctx, max_active=max_active, keep_resident=keep, chunk_rows=chunk_rows, gemm_tile=256,
                           lookahead=lookahead)
        try:
            done, _ = serve.replay(srv, trace, serve.submit_with(data, out_for), realtime=realtime)
        finally:
            srv.close()
        ctx.sync()
        host = {k: (np.array(v[0]), None if v[1] is None else np.array(v[1])) for k, v in data.items()}
    assert len(done) == len(trace)
    assert all(c["status"] == 0 for c in done.values())
    return outs, host, done


def _check_oracle(trace, outs, host):
    for r in trace:
        in0, in1 = host[(r["kind"], r["dataset"])]
        got = outs[r["id"]]
        if r["kind"] == "jacobi":
            assert np.array_equal(got, oracle.jacobi2d(in0, r["sweeps"])), r
        elif r["kind"] == "kmeans":
            assert np.array_equal(got, oracle.kmeans_assign(in0, in1)), r
        else:
            ref = oracle.gemm(in0, in1)
            scale = oracle.gemm(np.abs(in0), np.abs(in1))
            assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-30), r


def test_served_results_match_oracle_and_alone(L):
    trace = _trace()
    say("serve mixed", [(r["kind"], r["size"]) for r in trace])
    mixed, host, done = _serve(L, trace, max_active=6, keep=True)
    _check_oracle(trace, mixed, host)
    assert sum(c["cache_hit"] for c in done.values()) > 0
    # admitted requests overlapped: some request was admitted before an
    # earlier one finished
    ts = sorted(done.values(), key=lambda c: c["t_admit"])
    assert any(b["t_admit"] < a["t_done"] for a, b in zip(ts, ts[1:]))
    say("serve alone")
    alone, _, _ = _serve(L, trace, max_active=1, keep=False, realtime=False)
    for r in trace:
        assert np.array_equal(mixed[r["id"]], alone[r["id"]], equal_nan=False), r


def test_serving_under_a_small_budget_spills(L):
    # admission by footprint with a budget smaller than several requests
    trace = _trace()
    say("serve small budget")
    outs, host, done = _serve(L, trace, max_active=4, keep=True, budget=4 << 20, chunk_rows=4096)
    _check_oracle(trace, outs, host)


def test_lookahead_admits_cached_datasets_first_with_the_same_results(L):
    # one slot, everything queued behind a long first request (Jacobi 8192^2,
    # 100 sweeps: milliseconds on the device, longer than submitting the
    # rest): with a lookahead, a queued request on a dataset already cached
    # goes before older ones on other datasets; results are the oracle's and
    # those of the arrival-order run
    blocker = {"id": 0, "t": 0.0, "kind": "jacobi", "dataset": 99, "size": 8192, "sweeps": 100}
    trace = [blocker] + [dict(r, id=r["id"] + 1, t=0.0) for r in _trace()]
    say("serve lookahead")
    la, host, done = _serve(L, trace, max_active=1, keep=True, realtime=False, lookahead=8)
    _check_oracle(trace[1:], la, host)
    fcfs, _, done_f = _serve(L, trace, max_active=1, keep=True, realtime=False)
    for r in trace:
        assert np.array_equal(la[r["id"]], fcfs[r["id"]]), r
    order = [i for i, _ in sorted(done.items(), key=lambda kv: kv[1]["t_admit"])]
    order_f = [i for i, _ in sorted(done_f.items(), key=lambda kv: kv[1]["t_admit"])]
    assert order_f == sorted(order_f)          # arrival order
    assert order[0] == 0 and order != sorted(order)   # some request went ahead
    assert sum(c["cache_hit"] for c in done.values()) >= sum(c["cache_hit"] for c in done_f.values())
    # no request waited behind more than max_bypass (4 x 8) later ones
    pos = {i: k for k, i in enumerate(order)}
    for i in order:
        assert sum(1 for j in order if j > i and pos[j] < pos[i]) <= 32
