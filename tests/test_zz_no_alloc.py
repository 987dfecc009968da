"""lt_batch_end_noalloc: the open batch issued from the library's fixed
device scratch.  Its results must equal lt_batch_end's (and the oracle's)
bit for bit, on consecutive calls that reuse the scratch, the second with a
smaller batch; a batch too large for the scratch is refused and stays
issuable."""
import sys

import numpy as np
import pytest

import oracle
import synthetic


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import paper_2202_05549_amd as L
    return L


def _run_batch(L, ctx, plan, data, sb, noalloc, jac=None):
    """Launches the mix (and optionally Jacobi sweeps) in one batch; returns
    every output read back."""
    arrs = []
    for (k, n), v in zip(plan, data):
        if k == 0:
            x = ctx.array([n], chunk=[sb])
            y = ctx.array([n], chunk=[sb])
            y.fill(np.float32(np.nan))
        else:
            x = ctx.array([n], np.int32, chunk=[sb])
            y = ctx.array([256], np.int32)
            y.fill(np.int32(-3))
        x.write(v)
        arrs.append((y, x))
    ja = None
    if jac is not None:
        f0, sweeps = jac
        a = ctx.array(list(f0.shape), chunk=[64, 0])
        b = ctx.array(list(f0.shape), chunk=[64, 0])
        a.write(f0)
        ja = (a, b)
    ctx.sync()
    names = ["stencil1d_f32" if k == 0 else "hist256_i32" for k, _ in plan]
    args = L.Context.arg_table(len(plan), [[n for _, n in plan], [a[0] for a in arrs], [a[1] for a in arrs]])
    grids = np.array([[n] for _, n in plan], dtype=np.int64)
    ctx.batch_begin()
    ctx.launch_many(names, grids, [256], [sb], args)
    if ja is not None:
        r, c = jac[0].shape
        for t in range(jac[1]):
            src, dst = (ja[0], ja[1]) if t % 2 == 0 else (ja[1], ja[0])
            ctx.launch("jacobi2d_f32", [r, c], [1, 1], [64, 0], args=[r, c, dst, src])
    if noalloc:
        ctx.batch_end_noalloc()
    else:
        ctx.batch_end()
    ctx.sync()
    outs = [y.read() for y, _ in arrs]
    if ja is not None:
        outs.append((ja[0] if jac[1] % 2 == 0 else ja[1]).read())
    for y, x in arrs:
        y.destroy()
        x.destroy()
    if ja is not None:
        ja[0].destroy()
        ja[1].destroy()
    ctx.sync()
    return outs


@pytest.mark.gpu
def test_noalloc_batch_equals_batch_end_on_two_calls():
    import paper_2202_05549_amd as L

    # first call: 80 launches up to 2^20 elements at superblock 2^16 (multi
    # task launches, several histogram partials per launch) plus 6 Jacobi
    # sweeps; second call: a smaller batch through the same scratch
    big = synthetic.batch_plan(80, seed=11, hi_log2=20.0)
    small = synthetic.batch_plan(12, seed=12, hi_log2=14.0)
    big_data = [synthetic.batch_data(k, n, i, seed=11) for i, (k, n) in enumerate(big)]
    small_data = [synthetic.batch_data(k, n, i, seed=12) for i, (k, n) in enumerate(small)]
    f0 = synthetic.jacobi2d_input(300, 517, seed=13)
    with L.Context(device_budget_bytes=2 << 30) as ctx:
        for tag, plan, data, sb, jac in (("big", big, big_data, 1 << 16, (f0, 6)),
                                         ("small", small, small_data, 1 << 12, None)):
            say("no-alloc batch", tag, len(plan), "launches")
            ref_outs = _run_batch(L, ctx, plan, data, sb, noalloc=False, jac=jac)
            got_outs = _run_batch(L, ctx, plan, data, sb, noalloc=True, jac=jac)
            assert len(ref_outs) == len(got_outs)
            for i, ((k, n), v) in enumerate(zip(plan, data)):
                want = oracle.stencil1d(v) if k == 0 else oracle.hist256(v)
                assert np.array_equal(ref_outs[i], want), (tag, i, k, n)
                assert np.array_equal(got_outs[i], ref_outs[i]), (tag, i, k, n)
            if jac is not None:
                want = oracle.jacobi2d(f0, jac[1])
                assert np.array_equal(ref_outs[-1], want), tag
                assert np.array_equal(got_outs[-1], want), tag


@pytest.mark.gpu
def test_noalloc_batch_in_a_fresh_context_then_smaller():
    import paper_2202_05549_amd as L

    # a fresh context on the same device reuses the scratch the earlier
    # calls (if any) left behind: counters are cleared per call
    plan = synthetic.batch_plan(30, seed=21, hi_log2=18.0)
    data = [synthetic.batch_data(k, n, i, seed=21) for i, (k, n) in enumerate(plan)]
    for count in (30, 7):
        say("no-alloc fresh context", count)
        with L.Context(device_budget_bytes=1 << 30) as ctx:
            got = _run_batch(L, ctx, plan[:count], data[:count], 1 << 13, noalloc=True)
            ref = _run_batch(L, ctx, plan[:count], data[:count], 1 << 13, noalloc=False)
        for i, ((k, n), v) in enumerate(zip(plan[:count], data[:count])):
            assert np.array_equal(got[i], ref[i]), (count, i, k, n)


def test_noalloc_batch_too_large_is_refused_and_stays_open():
    import paper_2202_05549_amd as L

    # 32768 histogram superblocks: 32768 x (192 B task + 1 KiB partial) is
    # more than the 32 MiB scratch
    ctx = L.Context(dry_run=1, device_budget_bytes=1 << 30)
    n = 1 << 22
    v = ctx.array([n], np.int32, chunk=[1 << 16])
    h = ctx.array([256], np.int32)
    ctx.batch_begin()
    ctx.launch("hist256_i32", [n], [128], [128], args=[n, h, v])
    with pytest.raises(L.LtError) as e:
        ctx.batch_end_noalloc()
    assert e.value.status == L.LT_ERR_BUDGET
    assert "32 MiB" in str(e.value) or "33554432" in str(e.value)
    # still open: the usual issue takes it
    before = ctx.stats()["dispatches"]
    ctx.batch_end()
    ctx.sync()
    assert ctx.stats()["dispatches"] > before
    ctx.close()


def test_noalloc_batch_needs_a_device():
    import paper_2202_05549_amd as L

    ctx = L.Context(dry_run=1, device_budget_bytes=1 << 30)
    n = 1 << 12
    x = ctx.array([n])
    y = ctx.array([n])
    ctx.batch_begin()
    ctx.launch("stencil1d_f32", [n], [256], [1024], args=[n, y, x])
    with pytest.raises(L.LtError) as e:
        ctx.batch_end_noalloc()
    assert e.value.status == L.LT_ERR_UNSUPPORTED
    ctx.batch_end()
    ctx.sync()
    ctx.close()
