"""GPU parity of the batched path: many launches drained by one persistent
kernel.  Each launch's result must equal the oracle and the unbatched path
bit for bit (same bodies, same arithmetic)."""
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


def _mix(L, count, hi_log2, sb, batched, seed=3, drain_wg=0):
    plan = synthetic.batch_plan(count, seed=seed, hi_log2=hi_log2)
    data = [synthetic.batch_data(k, n, i, seed=seed) for i, (k, n) in enumerate(plan)]
    outs = []
    with L.Context(device_budget_bytes=4 << 30, drain_workgroups=drain_wg) as ctx:
        arrs = []
        for (k, n), v in zip(plan, data):
            if k == 0:
                x = ctx.array([n], chunk=[sb])
                y = ctx.array([n], chunk=[sb])
            else:
                x = ctx.array([n], np.int32, chunk=[sb])
                y = ctx.array([256], np.int32)
                y.fill(-7)
            x.write(v)
            arrs.append((y, x))
        ctx.sync()
        names = ["stencil1d_f32" if k == 0 else "hist256_i32" for k, _ in plan]
        args = L.Context.arg_table(count, [[n for _, n in plan], [a[0] for a in arrs], [a[1] for a in arrs]])
        grids = np.array([[n] for _, n in plan], dtype=np.int64)
        if batched:
            ctx.batch_begin()
        ctx.launch_many(names, grids, [1], [sb], args)
        if batched:
            ctx.batch_end()
        ctx.sync()
        outs = [a[0].read() for a in arrs]
    return plan, data, outs


@pytest.mark.parametrize("sb", [1 << 12, 1 << 16, 12345])
def test_batched_mix_matches_oracle_and_plain(L, sb):
    say("batch mix", sb)
    plan, data, got = _mix(L, 96, 18.0, sb, batched=True)
    _, _, plain = _mix(L, 96, 18.0, sb, batched=False)
    for (k, n), v, g, p in zip(plan, data, got, plain):
        ref = oracle.stencil1d(v) if k == 0 else oracle.hist256(v)
        assert np.array_equal(g, ref), (k, n)
        assert np.array_equal(g, p), (k, n)


def test_batched_mix_small_drain(L):
    # few workgroups: waits inside the drain are exercised more
    say("batch mix small drain")
    plan, data, got = _mix(L, 40, 16.0, 1 << 12, batched=True, drain_wg=3)
    for (k, n), v, g in zip(plan, data, got):
        ref = oracle.stencil1d(v) if k == 0 else oracle.hist256(v)
        assert np.array_equal(g, ref)


@pytest.mark.parametrize("wg", [0, 7])
def test_batched_stencil_pingpong_dependencies(L, wg):
    # 12 launches that each read the previous one's output: every task waits
    # on its three predecessors inside the drain
    n = 300_001
    say("batch pingpong", wg)
    x0 = synthetic.stencil1d_input(n, 8)
    with L.Context(device_budget_bytes=1 << 30, drain_workgroups=wg) as ctx:
        a = ctx.array([n], chunk=[20000])
        b = ctx.array([n], chunk=[20000])
        a.write(x0)
        ctx.batch_begin()
        inp, out = a, b
        for _ in range(12):
            ctx.launch("stencil1d_f32", [n], [1], [20000], args=[n, out, inp])
            inp, out = out, inp
        ctx.batch_end()
        ctx.sync()
        got = inp.read()
    assert np.array_equal(got, oracle.stencil1d_iter(x0, 12))


@pytest.mark.parametrize("n,m,sb", [(1000, 1500, 64), (1000, 1024, 256), (777, 2048, 384), (300, 4096, 128)])
def test_batched_jacobi_sweeps(L, n, m, sb):
    # superblocks smaller than a drain tile (ragged tiles), and larger ones
    # whose full tiles take the marching path, with ragged last tasks
    say("batch jacobi", n, m, sb)
    x0 = synthetic.jacobi2d_input(n, m, seed=14)
    with L.Context(device_budget_bytes=1 << 30) as ctx:
        a = ctx.array([n, m], chunk=[sb, 0])
        b = ctx.array([n, m], chunk=[sb, 0])
        a.write(x0)
        ctx.batch_begin()
        inp, out = a, b
        for _ in range(9):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], [sb, 0], args=[n, m, out, inp])
            inp, out = out, inp
        ctx.batch_end()
        ctx.sync()
        got = inp.read()
    assert np.array_equal(got, oracle.jacobi2d(x0, 9))


def test_batch_after_unbatched_work_and_touch(L):
    # work issued before the batch (a fill and a plain launch) must complete
    # before the batched tasks that depend on it
    n = 100_000
    say("batch ordering")
    with L.Context(device_budget_bytes=1 << 30) as ctx:
        y = ctx.array([n], np.int32, chunk=[7000])
        y.fill(5)
        ctx.launch("touch_i32", [n], [1], [7000], args=[n, y])
        ctx.batch_begin()
        for _ in range(3):
            ctx.launch("touch_i32", [n], [1], [7000], args=[n, y])
        ctx.batch_end()
        ctx.launch("touch_i32", [n], [1], [7000], args=[n, y])
        ctx.sync()
        got = y.read()
    assert np.all(got == 10)


def test_auto_flushed_batch_matches(L):
    say("batch auto flush")
    plan = synthetic.batch_plan(60, seed=5, hi_log2=17.0)
    data = [synthetic.batch_data(k, n, i, seed=5) for i, (k, n) in enumerate(plan)]
    with L.Context(device_budget_bytes=2 << 30, batch_flush_tasks=7) as ctx:
        arrs = []
        for (k, n), v in zip(plan, data):
            x = ctx.array([n], np.float32 if k == 0 else np.int32, chunk=[4096])
            y = ctx.array([n] if k == 0 else [256], np.float32 if k == 0 else np.int32, chunk=[4096] if k == 0 else None)
            x.write(v)
            arrs.append((y, x))
        ctx.batch_begin()
        for (k, n), (y, x) in zip(plan, arrs):
            ctx.launch("stencil1d_f32" if k == 0 else "hist256_i32", [n], [1], [4096], args=[n, y, x])
        ctx.batch_end()
        ctx.sync()
        assert ctx.stats()["dispatches"] > 4  # several drains
        for (k, n), v, (y, x) in zip(plan, data, arrs):
            ref = oracle.stencil1d(v) if k == 0 else oracle.hist256(v)
            assert np.array_equal(y.read(), ref)


def test_graph_replays_with_eager_work_between(L):
    # a graph of two stencil launches (x -> y -> x) and one histogram; every
    # replay is checked against the eager result, with eager launches and
    # synchronizations between the replays
    n = 200_003
    say("graph replay")
    x0 = synthetic.stencil1d_input(n, 9)
    v = synthetic.zipf_values(150_000, np.random.default_rng(9))
    with L.Context(device_budget_bytes=1 << 30) as ctx:
        x = ctx.array([n], chunk=[30000])
        y = ctx.array([n], chunk=[30000])
        hv = ctx.array([v.size], np.int32, chunk=[40000])
        h = ctx.array([256], np.int32)
        z = ctx.array([1000], np.int32)
        x.write(x0)
        hv.write(v)
        z.fill(0)
        ctx.graph_begin()
        ctx.launch("stencil1d_f32", [n], [1], [30000], args=[n, y, x])
        ctx.launch("stencil1d_f32", [n], [1], [30000], args=[n, x, y])
        ctx.launch("hist256_i32", [v.size], [1], [40000], args=[v.size, h, hv])
        g = ctx.graph_end()
        cur = x0
        for rep in range(4):
            h.fill(77)
            ctx.graph_launch(g)
            ctx.launch("touch_i32", [1000], [1], [100], args=[1000, z])  # eager work
            ctx.sync()
            cur = oracle.stencil1d_iter(cur, 2)
            assert np.array_equal(x.read(), cur), rep
            assert np.array_equal(h.read(), oracle.hist256(v)), rep
        assert np.all(z.read() == 4)
        ctx.graph_destroy(g)
        ctx.sync()
