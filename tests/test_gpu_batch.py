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


def _mix(L, count, hi_log2, sb, batched, seed=3, drain_wg=0, drain_tile=0):
    plan = synthetic.batch_plan(count, seed=seed, hi_log2=hi_log2)
    data = [synthetic.batch_data(k, n, i, seed=seed) for i, (k, n) in enumerate(plan)]
    outs = []
    with L.Context(device_budget_bytes=4 << 30, drain_workgroups=drain_wg, drain_tile=drain_tile) as ctx:
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


@pytest.mark.parametrize("tile", [4096, 12288, 1 << 18])
def test_batched_mix_drain_tile_sizes(L, tile):
    # tasks cut into interleaved tiles of other sizes: the same results
    say("batch mix drain tile", tile)
    plan, data, got = _mix(L, 48, 20.0, 1 << 20, batched=True, drain_tile=tile)
    for (k, n), v, g in zip(plan, data, got):
        ref = oracle.stencil1d(v) if k == 0 else oracle.hist256(v)
        assert np.array_equal(g, ref), (k, n)


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


@pytest.mark.parametrize("n,m,sb", [(1000, 1500, 64), (1000, 1024, 256), (777, 2048, 384), (300, 4096, 128),
                                    (1000, 1500, 256)])
def test_batched_jacobi_sweeps(L, n, m, sb):
    # superblocks smaller than a drain tile (ragged tiles), and larger ones
    # whose full tiles take the marching path, with ragged last tasks; 1500
    # columns end a marching tile inside its second wave
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


def test_batch_near_the_budget_matches_oracle(L):
    # the arrays take the whole budget but 1 MiB: the batch's queue area fits
    # beside them, and no chunk a queued task addresses may be evicted for it
    n = 1 << 20
    say("batch near budget")
    x0 = [synthetic.stencil1d_input(n, 60 + i) for i in range(2)]
    with L.Context(device_budget_bytes=4 * n * 4 + (1 << 20)) as ctx:
        xs = [ctx.array([n], chunk=[1 << 18]) for _ in range(4)]
        xs[0].write(x0[0])
        xs[2].write(x0[1])
        ctx.sync()
        ctx.batch_begin()
        ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[1], xs[0]])
        ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[3], xs[2]])
        ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[0], xs[1]])
        ctx.batch_end()
        ctx.sync()
        s = ctx.stats()
        assert s["evictions_dirty"] == 0 and s["evictions_clean"] == 0
        got0, got3 = xs[0].read(), xs[3].read()
    assert np.array_equal(got0, oracle.stencil1d_iter(x0[0], 2))
    assert np.array_equal(got3, oracle.stencil1d(x0[1]))


def _c4_subset(count=8192, take=112, big=8, seed=3):
    """Launch indices of the 8192-launch batching mix (sizes 2^10..2^24):
    ``big`` launches above 2^22 elements and ``take`` others, drawn with a
    fixed seed, in program order."""
    plan = synthetic.batch_plan(count, seed=seed)
    pick = np.random.default_rng(77)
    large = [i for i, (_, n) in enumerate(plan) if n > (1 << 22)]
    rest = [i for i, (_, n) in enumerate(plan) if n <= (1 << 22)]
    idx = sorted(set(pick.choice(large, big, replace=False).tolist()) |
                 set(pick.choice(rest, take, replace=False).tolist()))
    return [(i, plan[i][0], plan[i][1]) for i in idx]


@pytest.mark.parametrize("sb", [1 << 24, 1 << 22])
def test_c4_mix_at_benchmark_superblocks_batched_and_replayed(L, sb):
    # launches of the 8192-launch mix at the superblocks the benchmark runs
    # (2^24: one task per launch, up to 256 drain tiles of 65536 elements, so
    # a histogram task flushes many tiles into one partial; 2^22: several
    # tasks and partials per launch), inputs from the seeded recipe.  Every
    # launch matches the oracle batched, and on each of two graph replays.
    sub = _c4_subset()
    assert sum(1 for _, _, n in sub if n > (1 << 22)) >= 8
    say("c4 subset", len(sub), "launches, sb", sb, "elements", sum(n for _, _, n in sub))
    data = [synthetic.batch_data(k, n, i, seed=3) for i, k, n in sub]
    refs = [oracle.stencil1d(v) if k == 0 else oracle.hist256(v) for (_, k, _), v in zip(sub, data)]
    with L.Context(device_budget_bytes=8 << 30) as ctx:
        arrs = []
        for (_, k, n), v in zip(sub, data):
            if k == 0:
                x = ctx.array([n], chunk=[sb])
                y = ctx.array([n], chunk=[sb])
            else:
                x = ctx.array([n], np.int32, chunk=[sb])
                y = ctx.array([256], np.int32)
            x.write(v)
            arrs.append((y, x))
        names = ["stencil1d_f32" if k == 0 else "hist256_i32" for _, k, _ in sub]
        args = L.Context.arg_table(len(sub), [[n for _, _, n in sub], [a[0] for a in arrs], [a[1] for a in arrs]])
        grids = np.array([[n] for _, _, n in sub], dtype=np.int64)

        def clear():
            for (_, k, _), (y, _) in zip(sub, arrs):
                y.fill(np.float32(np.nan) if k == 0 else np.int32(-5))
            ctx.sync()

        def check(tag):
            for (i, k, n), (y, _), ref in zip(sub, arrs, refs):
                assert np.array_equal(y.read(), ref), (tag, i, k, n)

        clear()
        ctx.batch_begin()
        ctx.launch_many(names, grids, [256], [sb], args)
        ctx.batch_end()
        ctx.sync()
        check("batched")
        ctx.graph_begin()
        ctx.launch_many(names, grids, [256], [sb], args)
        g = ctx.graph_end()
        for rep in range(2):
            clear()
            ctx.graph_launch(g)
            ctx.sync()
            check("replay %d" % rep)
        ctx.graph_destroy(g)
        ctx.sync()
