"""GPU parity of the serving configuration's largest requests, at full size
and in the launch configuration the serving bench times: a 2-D Jacobi
request of 32768^2 points (10 sweeps) and a k-means assignment request of
10^9 points (64 GB of points, more than the device budget is ever given to
one array here, read from pageable memory through the bounce ring), both
served by one continuous-batching server with a 64 GiB device budget.

The outputs are too large for the oracle to recompute whole, so:
  * sampled outputs, each computed by the oracle on its own: a Jacobi point
    after s sweeps depends only on the inputs within distance s, so the
    oracle's s sweeps over the (2s + 1)^2 window around it (clipped at the
    grid's edges, where the zero boundary is real) give it exactly; a label
    is the oracle's assignment of that point;
  * properties of every output: all labels in [0, K), all Jacobi values
    finite and within the inputs' range [0, 1).
Bit-exact: Jacobi in float32 with the same association order, labels from
the same float32 fma chain (a differing label must be a float64 near-tie).
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import paper_2202_05549_amd as L
    return L


def test_largest_served_jacobi_and_kmeans_requests_sampled(L):
    from paper_2202_05549_amd import serve

    sweeps, n, N, K = 10, 32768, 10 ** 9, 64
    trace = [{"id": 0, "t": 0.0, "kind": "jacobi", "dataset": 0, "size": n, "sweeps": sweeps},
             {"id": 1, "t": 0.0, "kind": "kmeans", "dataset": 0, "size": N}]
    say("serve full-size jacobi", n, "and kmeans", N)
    with L.Context(device_budget_bytes=64 << 30, n_compute_streams=2, stage_threshold_bytes=8 << 30,
                   sb_order=L.LT_ORDER_SERPENTINE) as ctx:
        # as in the serving bench: outputs pinned first, then the inputs up
        # to 56 GiB pinned in all; the 64 GB of points stay pageable
        host = serve.HostBuffers(ctx, pin_bytes=56 << 30)
        outs = serve.output_buffers(ctx, trace, host=host)
        data = serve.make_datasets(ctx, trace, host=host)
        assert host.pageable_bytes >= N * 16 * 4
        srv = serve.Server(ctx, max_active=16, keep_resident=True, admit_bytes=64 << 30)
        try:
            done, _ = serve.replay(srv, trace, serve.submit_with(data, outs), realtime=False)
        finally:
            srv.close()
        ctx.sync()
        assert len(done) == 2 and all(c["status"] == 0 for c in done.values())
        x0, _ = data[("jacobi", 0)]
        y = outs[("jacobi", 0)]
        X, mu = data[("kmeans", 0)]
        lab = outs[("kmeans", 0)]
        rng = np.random.default_rng(7)

        say("jacobi samples")
        # corners, edges and random interior points
        pts = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (5, n // 2), (n // 2, n - 3)]
        pts += [tuple(p) for p in rng.integers(0, n, (2042, 2))]
        for r, c in pts:
            r0, r1 = max(0, r - sweeps), min(n, r + sweeps + 1)
            c0, c1 = max(0, c - sweeps), min(n, c + sweeps + 1)
            w = oracle.jacobi2d(np.ascontiguousarray(x0[r0:r1, c0:c1]), sweeps)
            assert w[r - r0, c - c0] == y[r, c], (r, c)
        assert np.isfinite(y).all() and float(y.min()) >= 0.0 and float(y.max()) < 1.0

        say("kmeans samples")
        idx = np.unique(np.concatenate([[0, N - 1], rng.integers(0, N, 8190)]))
        ref = oracle.kmeans_assign(np.ascontiguousarray(X[idx]), np.asarray(mu))
        got = np.asarray(lab[idx])
        for p in np.nonzero(got != ref)[0]:
            da = oracle.kmeans_dist64(X[idx[p]], mu[ref[p]])
            db = oracle.kmeans_dist64(X[idx[p]], mu[got[p]])
            assert abs(da - db) <= 1e-5 * max(da, db), int(idx[p])
        # every label valid, in 2^27-point slices to bound temporaries
        for s in range(0, N, 1 << 27):
            part = np.asarray(lab[s:s + (1 << 27)])
            assert part.min() >= 0 and part.max() < K, s
