"""GPU parity of halo (overlapping) distributions.

Arrays stored as STENCIL chunks (cores plus replica halos) must give the
results of the plain definition bit for bit, whatever the tiling, the
superblocks, the executor or the spilling: replicas are refreshed from
their owners before they are read, writes go to the owners' cores, and
reads of whole arrays take each element from its owner.
"""
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


def _jacobi(ctx, x0, chunk, halo, sweeps, sb, host=False):
    n, m = x0.shape
    if host:
        ha = ctx.pinned((n, m))
        ha[...] = x0
        hb = ctx.pinned((n, m))
        hb[...] = 0
        a = ctx.array_host(ha, chunk=chunk, halo=halo)
        b = ctx.array_host(hb, chunk=chunk, halo=halo)
    else:
        a = ctx.array([n, m], chunk=chunk, halo=halo)
        b = ctx.array([n, m], chunk=chunk, halo=halo)
        a.write(x0)
        b.fill(0.0)
    inp, out = a, b
    for _ in range(sweeps):
        ctx.launch("jacobi2d_f32", [n, m], [1, 1], sb, args=[n, m, out, inp])
        inp, out = out, inp
    ctx.sync()
    return inp.read()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape,chunk,halo,sb", [
    ((512, 768), [128, 256], [1, 1], [128, 256]),     # tiles with a one-element halo
    ((500, 700), [96, 200], [2, 1], [96, 200]),       # ragged, wider halo
    ((300, 1000), [64, 0], [1, 0], [64, 0]),          # row slabs with a halo
    ((400, 640), [100, 160], [1, 1], [50, 320]),      # superblocks not aligned to the tiles
])
def test_jacobi_halo_tiles_bit_exact(L, mode, shape, chunk, halo, sb):
    say("jacobi halo", mode, shape, chunk, halo, sb)
    x0 = synthetic.jacobi2d_input(*shape, seed=21)
    with L.Context(device_budget_bytes=1 << 30, exec_mode=mode) as ctx:
        got = _jacobi(ctx, x0, chunk, halo, 6, sb)
        st = ctx.stats()
    assert np.array_equal(got, oracle.jacobi2d(x0, 6))
    if sb == chunk:
        assert st["assembled_regions"] == 0 and st["halo_copies"] > 0


@pytest.mark.parametrize("host", [False, True])
def test_jacobi_halo_out_of_core(L, host):
    # tiles streamed through a budget of a few tiles: replicas come from
    # owners on the device or, after they were written back, from the host
    n, m = 1024, 1024
    say("jacobi halo spill", host)
    x0 = synthetic.jacobi2d_input(n, m, seed=22)
    tile = 256 * 256 * 4
    with L.Context(device_budget_bytes=12 * tile, stage_threshold_bytes=1 << 40) as ctx:
        got = _jacobi(ctx, x0, [256, 256], [1, 1], 5, [256, 256], host=host)
        st = ctx.stats()
    assert np.array_equal(got, oracle.jacobi2d(x0, 5))
    # host-backed tiles reload their halo with the owners' written-back cores
    # from the home buffer; spill buffers keep their own halo and refresh it
    assert st["evictions_dirty"] > 0 and (host or st["halo_copies"] > 0)


@pytest.mark.parametrize("order,band", [(1, 0), (2, 2), (2, 3)])
def test_jacobi_halo_out_of_core_issue_orders(L, order, band):
    # the out-of-core halo tiles under the serpentine and banded issue orders:
    # replica refreshes and reloads follow the order of the superblocks, and
    # the result is the oracle's bit for bit under every order
    n, m = 1024, 1280
    say("jacobi halo spill order", order, band)
    x0 = synthetic.jacobi2d_input(n, m, seed=23)
    tile = 256 * 256 * 4
    with L.Context(device_budget_bytes=14 * tile, stage_threshold_bytes=1 << 40, sb_order=order,
                   sb_band=band) as ctx:
        got = _jacobi(ctx, x0, [256, 256], [1, 1], 4, [256, 256])
        st = ctx.stats()
    assert np.array_equal(got, oracle.jacobi2d(x0, 4))
    assert st["evictions_dirty"] > 0


@pytest.mark.parametrize("halo", [1, 3])
def test_stencil1d_halo_bit_exact(L, halo):
    n = 100003
    say("stencil1d halo", halo)
    x0 = synthetic.stencil1d_input(n, 5)
    with L.Context(device_budget_bytes=1 << 30, exec_mode=1) as ctx:
        x = ctx.array([n], chunk=[10000], halo=[halo])
        y = ctx.array([n], chunk=[10000], halo=[halo])
        x.write(x0)
        for sb in (10000, 7000, 10000):  # aligned, then reads spanning chunks beyond the halo
            ctx.launch("stencil1d_f32", [n], [1], [sb], args=[n, y, x])
            x, y = y, x
        ctx.sync()
        got = x.read()
    ref = x0
    for _ in range(3):
        ref = oracle.stencil1d(ref)
    assert np.array_equal(got, ref)


def test_touch_on_halo_array_writes_owners_once(L):
    # writes whose regions straddle tiles are scattered to the owners' cores;
    # replicas never leak into a whole-array read
    n, m = 300, 500
    say("touch halo")
    with L.Context(device_budget_bytes=1 << 30) as ctx:
        y = ctx.array([n * m], np.int32, chunk=[7000], halo=[5])
        y.fill(0)
        for sb in (7000, 3000, 4096):
            ctx.launch("touch_i32", [n * m], [1], [sb], args=[n * m, y])
        ctx.sync()
        got = y.read()
    assert np.all(got == 3)


# ------------------------------------------------------------ disk tier

@pytest.mark.parametrize("halo", [None, [1, 1]])
def test_jacobi_through_the_disk_tier(L, halo, tmp_path):
    # device budget of 20 of the 32 tiles and a host budget of 6 more: the
    # other spill buffers live in the spill file and come back on demand
    n, m = 1024, 1024
    say("jacobi disk tier", halo)
    x0 = synthetic.jacobi2d_input(n, m, seed=23)
    tile = 256 * 256 * 4
    with L.Context(device_budget_bytes=20 * tile, host_budget_bytes=6 * tile, spill_dir=str(tmp_path),
                   stage_threshold_bytes=1 << 40) as ctx:
        a = ctx.array([n, m], chunk=[256, 256], halo=halo)
        b = ctx.array([n, m], chunk=[256, 256], halo=halo)
        a.write(x0)
        b.fill(0.0)
        inp, out = a, b
        for _ in range(5):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], [256, 256], args=[n, m, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
        st = ctx.stats()
    assert st["bytes_disk_write"] > 0 and st["bytes_disk_read"] > 0
    assert st["host_spill_bytes"] <= 6 * tile
    assert np.array_equal(got, oracle.jacobi2d(x0, 5))


@pytest.mark.parametrize("shape,chunk,halo", [
    ((512, 768), [128, 256], [1, 1]),   # tiles: eight neighbours per interior tile
    ((300, 1000), [64, 0], [1, 0]),     # row slabs
])
def test_batched_jacobi_on_halo_arrays_bit_exact(L, shape, chunk, halo):
    # sweeps queued in one open batch read replicas that the previous sweep
    # writes: the runtime issues the batch before refreshing them, so the
    # result is the plain definition's
    say("batched halo jacobi", shape, chunk, halo)
    n, m = shape
    x0 = synthetic.jacobi2d_input(n, m, seed=44)
    sb = [chunk[0], chunk[1] or m]
    with L.Context(device_budget_bytes=1 << 30) as ctx:
        a = ctx.array([n, m], chunk=chunk, halo=halo)
        b = ctx.array([n, m], chunk=chunk, halo=halo)
        a.write(x0)
        b.fill(0.0)
        ctx.sync()
        ctx.batch_begin()
        inp, out = a, b
        for _ in range(5):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], sb, args=[n, m, out, inp])
            inp, out = out, inp
        ctx.batch_end()
        ctx.sync()
        assert ctx.stats()["halo_copies"] > 0
        got = inp.read()
    assert np.array_equal(got, oracle.jacobi2d(x0, 5))
