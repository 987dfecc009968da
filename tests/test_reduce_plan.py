"""CPU (dry-run) tests of the planner for float reductions.

A body that spreads one superblock over several workgroups gets one partial
slot per workgroup; the planner sizes the partials accordingly and folds
them with a slot fold and a combine per reduce argument.  No device work.
"""
import numpy as np
import pytest

import paper_2202_05549_amd as L


def dry(**kw):
    kw.setdefault("device_budget_bytes", 1 << 30)
    kw.setdefault("trace", 1)
    return L.Context(dry_run=1, **kw)


def _kmu_slots(points, d, tile=4096):
    # one slot per 4096-point tile, at most 512 for d = 16 and 32 (two LDS
    # copies per wave: two workgroups per CU), else 1024
    cap = 512 if d in (16, 32) else 1024
    return max(1, min(cap, -(-points // tile)))


@pytest.mark.parametrize("N,sb,d", [(300000, 65536, 16), (777, 256, 16), (20000, 1 << 20, 16),
                                    (3000000, 1 << 22, 16), (5000000, 1 << 23, 8)])
def test_kmeans_update_plan(N, sb, d):
    K = 64
    with dry() as ctx:
        x = ctx.array([N, d])
        lb = ctx.array([N], np.int32)
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        lid = ctx.launch("kmeans_update_f32", [N], [1], [sb], args=[N, d, K, sums, counts, x, lb])
        tasks = ctx.tasks(lid)
        ex = [t for t in tasks if t.kind == L.LT_TASK_EXEC]
        comb = [t for t in tasks if t.kind == L.LT_TASK_COMBINE]
        nsb = -(-N // sb)
        assert len(ex) == nsb and len(comb) == 2  # one combine per reduce argument
        # each combine waits for every superblock task
        for c in comb:
            assert set(ctx.deps(c.id)) >= {t.id for t in ex}
        # partial bytes: slots x (K d float64 + K int32) per task; the two
        # partial blocks appear in the trace as allocations with no owner
        # chunk, and are not filled (the body stores every slot whole)
        want = [0, 0]
        for t in ex:
            s = _kmu_slots(min(t.sb_hi[0], N) - t.sb_lo[0], d)
            want[0] += s * K * d * 8
            want[1] += s * K * 4
        tr = ctx.trace()
        parts = sorted(int(op.bytes) for op in tr if op.kind == 6 and op.chunk == 0)
        assert parts == sorted((w + 255) // 256 * 256 for w in want)
        assert not [op for op in tr if op.kind == 4]
        ctx.sync()


def test_float_slots_refused_inside_a_batch():
    N, d, K = 50000, 16, 64
    with dry() as ctx:
        x = ctx.array([N, d])
        lb = ctx.array([N], np.int32)
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        ctx.batch_begin()
        with pytest.raises(L.LtError) as e:
            ctx.launch("kmeans_update_f32", [N], [1], [N], args=[N, d, K, sums, counts, x, lb])
        assert e.value.status == L.LT_ERR_UNSUPPORTED
        ctx.batch_end()


def test_rowreduce_partials_per_column_superblock():
    n, m = 300, 5000
    with dry() as ctx:
        a = ctx.array([n, m])
        out = ctx.array([n])
        lid = ctx.launch("rowreduce_f32", [n, m], [1, 64], [64, 2048], args=[n, m, out, a],
                         kernel_annotation="global [i, j] => read A[i, j], reduce(min) out[i]")
        tasks = ctx.tasks(lid)
        ex = [t for t in tasks if t.kind == L.LT_TASK_EXEC]
        assert len(ex) == 5 * 3
        # every task's partial is its own rows of out
        for t in ex:
            regs = ctx.regions(t.id)
            r = [g for g in regs if g.arg == 2][0]
            assert (r.lo[0], r.hi[0]) == (t.sb_lo[0], min(t.sb_hi[0], n))
        ctx.sync()


@pytest.mark.parametrize("n,sb", [(1_000_003, 1 << 20), (65536, 65536), (70000, 1 << 16), (5, 4), (40_000_000, 1 << 25)])
def test_hist_slots_outside_batches_one_partial_inside(n, sb):
    # outside a batch: one 256-bin slot per 64 Ki elements of a superblock
    # (at most 1024), stored whole by the body, so no fill; inside a batch:
    # one partial per superblock, cleared with the batch's counters
    def slots(e):
        return 1 if e <= 0 else min(1024, -(-e // 65536))

    with dry() as ctx:
        v = ctx.array([n], np.int32)
        h = ctx.array([256], np.int32)
        ctx.clear_trace()
        lid = ctx.launch("hist256_i32", [n], [1], [sb], args=[n, h, v])
        ex = [t for t in ctx.tasks(lid) if t.kind == L.LT_TASK_EXEC]
        want = sum(slots(min(t.sb_hi[0], n) - t.sb_lo[0]) for t in ex) * 256 * 4
        tr = ctx.trace()
        parts = [int(op.bytes) for op in tr if op.kind == 6 and op.chunk == 0]
        assert parts == [(want + 255) // 256 * 256]
        assert not [op for op in tr if op.kind == 4]
        ctx.sync()
        ctx.clear_trace()
        ctx.batch_begin()
        ctx.launch("hist256_i32", [n], [1], [sb], args=[n, h, v])
        ctx.batch_end()
        ctx.sync()
        st = ctx.stats()
        assert st["dispatches"] >= 1
