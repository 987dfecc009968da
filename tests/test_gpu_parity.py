"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Float kernels are compared bit for bit: each body fixes its float32
operation order and the oracle follows the same order, so the only admissible
difference is none (the workload tolerance, max-rel 1e-5, is the fallback
and is never needed).  Integer results are bit-exact by definition.
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


def ctx_of(L, **kw):
    kw.setdefault("device_budget_bytes", 4 << 30)
    return L.Context(**kw)


# ------------------------------------------------------------------- touch

@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n,block,sb,chunk", [(1000, 16, 64, 100), (4096, 1, 1000, 512), (70001, 64, 4096, 0)])
def test_touch_every_index_exactly_once(L, mode, n, block, sb, chunk):
    say("touch", mode, n, block, sb, chunk)
    with ctx_of(L, exec_mode=mode) as ctx:
        y = ctx.array([n], np.int32, chunk=[chunk])
        y.fill(0)
        ctx.launch("touch_i32", [n], [block], [sb], args=[n, y])
        ctx.launch("touch_i32", [n], [block], [sb], args=[n, y])
        ctx.sync()
        got = y.read()
    exp = oracle.touch(oracle.touch(np.zeros(n, np.int32), n), n)
    assert np.array_equal(got, exp)


# --------------------------------------------------------------- stencil1d

@pytest.mark.parametrize("mode", [0, 1])
def test_stencil1d_config1_bit_exact(L, mode):
    # 1-D 3-point stencil, 2^20 float32 ~U(-1,1) seed 0, 8 chunks of 2^17
    n = 1 << 20
    say("stencil1d config", mode)
    x0 = synthetic.stencil1d_input(n, 0)
    with ctx_of(L, exec_mode=mode) as ctx:
        x = ctx.array([n], chunk=[1 << 17])
        y = ctx.array([n], chunk=[1 << 17])
        x.write(x0)
        lid = ctx.launch("stencil1d_f32", [n], [256], [1 << 17], args=[n, y, x])
        assert len(ctx.tasks(lid)) == 8
        ctx.sync()
        got = y.read()
    assert np.array_equal(got, oracle.stencil1d(x0))


@pytest.mark.parametrize("n,chunk,block,sb", [(1000003, 99991, 1, 77777), (5, 2, 1, 1), (4099, 4096, 4, 8),
                                              (123457, 1 << 14, 32, 96),
                                              # tasks above 2^21 elements take the streamed body
                                              (5000011, 0, 1, 2500001), (4194304 + 8191, 0, 1, 4194304 + 8191)])
def test_stencil1d_ragged_bit_exact(L, n, chunk, block, sb):
    say("stencil1d ragged", n, chunk, block, sb)
    x0 = synthetic.stencil1d_input(n, 17)
    for mode in (0, 1):
        with ctx_of(L, exec_mode=mode) as ctx:
            x = ctx.array([n], chunk=[chunk])
            y = ctx.array([n], chunk=[chunk])
            x.write(x0)
            ctx.launch("stencil1d_f32", [n], [block], [sb], args=[n, y, x])
            ctx.sync()
            assert np.array_equal(y.read(), oracle.stencil1d(x0)), mode


def test_paper_host_sample_ten_iterations(L):
    # Sec. 3.6 host sample: n = 1e6, chunks of 64000, superblocks of 64000
    # threads, blocks of 16, ten launches with input and output swapped
    n = 1_000_000
    say("host sample")
    x0 = synthetic.stencil1d_input(n, 3)
    with ctx_of(L) as ctx:
        a = ctx.array([n], chunk=[64000])
        b = ctx.array([n], chunk=[64000])
        a.write(x0)
        inp, out = a, b
        for _ in range(10):
            ctx.launch("stencil1d_f32", [n], [16], [64000], args=[n, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
    assert np.array_equal(got, oracle.stencil1d_iter(x0, 10))


@pytest.mark.parametrize("budget_chunks", [4, 7])
def test_stencil1d_out_of_core_matches(L, budget_chunks):
    # device budget of a few chunks: chunks spill to pinned host memory and
    # come back; the result must not change (distribution/budget invariance)
    chunk = 1 << 16
    n = 24 * chunk + 123
    say("stencil1d spill", budget_chunks)
    x0 = synthetic.stencil1d_input(n, 5)
    with ctx_of(L, device_budget_bytes=budget_chunks * chunk * 4 + 4096) as ctx:
        a = ctx.array([n], chunk=[chunk])
        b = ctx.array([n], chunk=[chunk])
        a.write(x0)
        inp, out = a, b
        for _ in range(5):
            ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
        st = ctx.stats()
    assert st["evictions_dirty"] > 0 and st["bytes_h2d"] > 0
    assert st["peak_resident_bytes"] <= budget_chunks * chunk * 4 + 4096
    assert np.array_equal(got, oracle.stencil1d_iter(x0, 5))


# ----------------------------------------------------------------- jacobi

@pytest.mark.parametrize("shape,chunk,sb,mode", [
    ((300, 517), (37, 0), (37, 0), 0),
    ((300, 517), (37, 0), (37, 0), 1),
    ((256, 1024), (64, 0), (32, 0), 1),
    ((129, 300), (0, 64), (16, 0), 0),      # column chunks: regions assembled
    ((129, 300), (40, 100), (40, 100), 0),  # tiles: halo regions span tiles
    ((1, 1), (0, 0), (0, 0), 0),
    ((3, 1027), (1, 0), (1, 0), 1),
])
def test_jacobi_small_bit_exact(L, shape, chunk, sb, mode):
    say("jacobi", shape, chunk, sb, mode)
    n, m = shape
    x0 = synthetic.jacobi2d_input(n, m, seed=9)
    with ctx_of(L, exec_mode=mode) as ctx:
        a = ctx.array([n, m], chunk=list(chunk))
        b = ctx.array([n, m], chunk=list(chunk))
        a.write(x0)
        inp, out = a, b
        for _ in range(5):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], list(sb), args=[n, m, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
    assert np.array_equal(got, oracle.jacobi2d(x0, 5))


@pytest.mark.parametrize("variant", [8, 16, 32, 132, 164, 228, 302, 304, 308])
@pytest.mark.parametrize("shape,chunk,sb", [((1000, 2051), (96, 0), (96, 0)), ((777, 1024), (0, 0), (256, 0)),
                                            ((300, 4096), (128, 0), (128, 1024)), ((513, 515), (0, 0), (0, 0)),
                                            ((600, 1500), (0, 0), (256, 0))])
def test_jacobi_tile_variants_bit_exact(L, variant, shape, chunk, sb):
    # every tiling of the body (rows loaded at once, marched in groups of 8,
    # or stacked bands per wave) gives the same bits, on full and ragged tiles
    # (1500 columns: a full-height tile whose columns end inside a wave)
    say("jacobi variant", variant, shape, chunk, sb)
    n, m = shape
    x0 = synthetic.jacobi2d_input(n, m, seed=11)
    with ctx_of(L, exec_mode=1) as ctx:
        ctx.tune("jacobi2d_f32", variant)
        a = ctx.array([n, m], chunk=list(chunk))
        b = ctx.array([n, m], chunk=list(chunk))
        a.write(x0)
        inp, out = a, b
        for _ in range(3):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], list(sb), args=[n, m, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
    assert np.array_equal(got, oracle.jacobi2d(x0, 3))


@pytest.mark.parametrize("policy", [0, 1])
def test_jacobi_out_of_core_matches(L, policy):
    # both eviction policies (next use, LRU) give the oracle's bits
    n, m = 1024, 1024
    say("jacobi spill", policy)
    x0 = synthetic.jacobi2d_input(n, m, seed=10)
    with ctx_of(L, device_budget_bytes=10 * 64 * m * 4, evict_policy=policy) as ctx:
        a = ctx.array([n, m], chunk=[64, 0])
        b = ctx.array([n, m], chunk=[64, 0])
        a.write(x0)
        inp, out = a, b
        for _ in range(4):
            ctx.launch("jacobi2d_f32", [n, m], [1, 256], [64, 0], args=[n, m, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
        assert ctx.stats()["evictions_dirty"] > 0
    assert np.array_equal(got, oracle.jacobi2d(x0, 4))


@pytest.mark.parametrize("mode", [0, 1])
def test_jacobi_config2_full_size_bit_exact(L, mode):
    # 2-D Jacobi 16384^2 ~U(0,1) seed 1, 100 ping-pong sweeps, 512-row
    # chunks and superblocks (the benchmark configuration)
    n = 16384
    sweeps = 100
    say("jacobi config2", mode)
    x0 = synthetic.jacobi2d_input(n, seed=1)
    with ctx_of(L, exec_mode=mode) as ctx:
        a = ctx.array([n, n], chunk=[512, 0])
        b = ctx.array([n, n], chunk=[512, 0])
        a.write(x0)
        inp, out = a, b
        for _ in range(sweeps):
            ctx.launch("jacobi2d_f32", [n, n], [1, 256], [512, 0], args=[n, n, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
    if "ref" not in _C2:
        _C2["ref"] = oracle.jacobi2d(x0, sweeps, inplace=True)
    assert np.array_equal(got, _C2["ref"])


_C2 = {}


# ---------------------------------------------------------------- hist256

@pytest.mark.parametrize("n,chunk,sb", [(1_000_003, 1 << 16, 1 << 16), (777, 100, 64), (1 << 22, 1 << 20, 1 << 19),
                                        (1 << 26, 1 << 24, 1 << 26), (70 << 20, 0, 0)])
def test_hist256_bit_exact_and_overwrites_target(L, n, chunk, sb):
    say("hist", n, chunk, sb)
    v = synthetic.zipf_values(n, np.random.default_rng(12))
    with ctx_of(L) as ctx:
        va = ctx.array([n], np.int32, chunk=[chunk])
        h = ctx.array([256], np.int32)
        va.write(v)
        h.fill(12345)  # reduce(+) overwrites the target
        ctx.launch("hist256_i32", [n], [1], [sb], args=[n, h, va])
        ctx.sync()
        got = h.read()
    assert np.array_equal(got, oracle.hist256(v))


@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("hchunk", [0, 64])
def test_hist256_reductions_into_one_target_keep_program_order(L, batched, hchunk):
    # three histogram launches into one h, with a plain read of h (its bins
    # are the values of a histogram into g) and a read-modify-write of h
    # between them, all issued without a sync.  Each fold overwrites h, so
    # only program order gives g = hist(H1) and h = H3.
    say("hist ordering", batched, hchunk)
    rng = np.random.default_rng(41)
    sizes = (1000, 5003, 300_001)
    vs = [synthetic.zipf_values(n, rng) for n in sizes]
    with ctx_of(L) as ctx:
        va = [ctx.array([n], np.int32, chunk=[4096]) for n in sizes]
        for a, v in zip(va, vs):
            a.write(v)
        h = ctx.array([256], np.int32, chunk=[hchunk])
        g = ctx.array([256], np.int32)
        h.fill(-1)
        g.fill(-1)
        ctx.sync()
        if batched:
            ctx.batch_begin()
        ctx.launch("hist256_i32", [sizes[0]], [1], [512], args=[sizes[0], h, va[0]])
        ctx.launch("hist256_i32", [256], [1], [64], args=[256, g, h])
        ctx.launch("hist256_i32", [sizes[1]], [1], [2048], args=[sizes[1], h, va[1]])
        ctx.launch("touch_i32", [256], [1], [128], args=[256, h])
        ctx.launch("hist256_i32", [sizes[2]], [1], [65536], args=[sizes[2], h, va[2]])
        if batched:
            ctx.batch_end()
        ctx.sync()
        got_g, got_h = g.read(), h.read()
    h1 = oracle.hist256(vs[0])
    assert h1.max() < 256  # the bins of H1 are valid histogram values
    assert np.array_equal(got_g, oracle.hist256(h1))
    assert np.array_equal(got_h, oracle.hist256(vs[2]))


# ----------------------------------------------------------------- k-means

@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("N,d,K,chunk", [(100_003, 16, 64, 1 << 14), (5000, 3, 7, 999), (4096, 32, 256, 0),
                                         (70_001, 16, 256, 1 << 14), (300, 16, 1, 0), (1000, 16, 5, 333),
                                         (20_001, 32, 48, 4096), (9_999, 8, 33, 1000), (7_777, 4, 129, 0)])
def test_kmeans_assign_labels_bit_exact(L, variant, N, d, K, chunk):
    # d = 4, 8, 16 and 32: the default body reads the centres through scalar
    # loads, variant 1 broadcasts them from LDS; at d = 16 variant 2 takes
    # two points per lane
    # (superblocks of 333 points leave lanes whose second point is past the
    # superblock)
    say("kmeans", variant, N, d, K)
    X, mu, _ = synthetic.kmeans_blobs(N, d, K, seed=13)
    with ctx_of(L) as ctx:
        ctx.tune("kmeans_assign_f32", variant)
        xa = ctx.array([N, d], chunk=[chunk, 0])
        ca = ctx.array([K, d])
        lab = ctx.array([N], np.int32, chunk=[chunk])
        xa.write(X)
        ca.write(mu)
        ctx.launch("kmeans_assign_f32", [N], [1], [chunk if chunk else 0], args=[N, d, K, lab, xa, ca])
        ctx.sync()
        got = lab.read()
    assert np.array_equal(got, oracle.kmeans_assign(X, mu))


# -------------------------------------------------------------------- GEMM
# Tolerance (componentwise, from the float32 error of a length-K dot product
# and the workload's 1e-5): |C - C_ref| <= 1e-5 * (|A| |B|) elementwise, with
# C_ref and |A||B| in float64.

def _gemm_case(L, M, N, K, chunkA, chunkB, chunkC, sb, seed=21, ident=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, K), dtype=np.float32)
    B = np.eye(K, N, dtype=np.float32) if ident else rng.standard_normal((K, N), dtype=np.float32)
    with ctx_of(L) as ctx:
        a = ctx.array([M, K], chunk=list(chunkA))
        b = ctx.array([K, N], chunk=list(chunkB))
        c = ctx.array([M, N], chunk=list(chunkC))
        a.write(A)
        b.write(B)
        c.fill(np.nan)
        ctx.launch("gemm_f32", [M, N], [1, 1], list(sb), args=[M, N, K, c, a, b])
        ctx.sync()
        got = c.read()
    return A, B, got


@pytest.mark.parametrize("M,N,K,chunkA,chunkB,chunkC,sb", [
    (300, 260, 77, (128, 0), (0, 100), (128, 100), (128, 100)),
    (256, 256, 64, (0, 0), (0, 0), (0, 0), (0, 0)),
    (513, 257, 129, (200, 0), (0, 0), (0, 0), (256, 0)),   # odd strides: scalar loads
    (64, 1000, 1, (0, 0), (0, 500), (64, 500), (64, 500)),
])
def test_gemm_small_componentwise(L, M, N, K, chunkA, chunkB, chunkC, sb):
    say("gemm", M, N, K, sb)
    A, B, got = _gemm_case(L, M, N, K, chunkA, chunkB, chunkC, sb)
    ref = oracle.gemm(A, B)
    scale = oracle.gemm(np.abs(A), np.abs(B))
    assert not np.isnan(got).any()
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-30)


@pytest.mark.parametrize("M,N,K,sb,ndisp", [
    (300, 260, 77, (128, 100), 2),    # 3 x 3 = 9 superblocks: a dispatch of 8 tasks, then 1
    (520, 530, 96, (256, 256), 2),    # 3 x 3 superblocks, ragged edge blocks in the last row and column
    (1100, 300, 64, (256, 300), 1),   # 5 superblocks of whole rows, the last one 76 rows
])
def test_gemm_grouped_dispatch(L, M, N, K, sb, ndisp):
    # LT_EXEC_GROUPED: superblocks of one launch without edges among them share
    # a dispatch and each workgroup finds its task in the table.  C is chunked
    # like the superblocks, so no two tasks write one chunk.
    say("gemm grouped", M, N, K, sb)
    rng = np.random.default_rng(23)
    A = rng.standard_normal((M, K), dtype=np.float32)
    B = rng.standard_normal((K, N), dtype=np.float32)
    with ctx_of(L, exec_mode=1) as ctx:
        a = ctx.array([M, K])
        b = ctx.array([K, N])
        c = ctx.array([M, N], chunk=list(sb))
        a.write(A)
        b.write(B)
        c.fill(np.nan)
        d0 = ctx.stats()["dispatches"]
        ctx.launch("gemm_f32", [M, N], [1, 1], list(sb), args=[M, N, K, c, a, b])
        ctx.sync()
        assert ctx.stats()["dispatches"] - d0 == ndisp
        got = c.read()
    ref = oracle.gemm(A, B)
    scale = oracle.gemm(np.abs(A), np.abs(B))
    assert not np.isnan(got).any()
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-30)


def test_gemm_identity_is_exact(L):
    say("gemm identity")
    A, B, got = _gemm_case(L, 512, 384, 384, (256, 0), (0, 128), (256, 128), (256, 128), ident=True)
    assert np.array_equal(got, A[:, :384])


def test_gemm_one_4096_tile_sampled(L):
    M = N = 4096
    K = 8192
    say("gemm 4096 tile")
    A, B, got = _gemm_case(L, M, N, K, (4096, 0), (0, 4096), (4096, 4096), (4096, 4096), seed=2)
    rng = np.random.default_rng(5)
    ii = rng.integers(0, M, 2048)
    jj = rng.integers(0, N, 2048)
    val, av = oracle.gemm_entries(A, B, ii, jj)
    assert np.all(np.abs(got[ii, jj] - val) <= 1e-5 * av)
    assert oracle.freivalds(A, B, got, panel=256) < 1e-5


def test_gemm_whole_4096_tile_elementwise(L):
    # one 4096^2 superblock with K = 4096: the shape of one out-of-core tile
    # dispatch, which runs the full block grid (groups of 8 block rows, each
    # XCD's blocks an 8 x 4 patch); every element against the float64 product
    M = N = K = 4096
    say("gemm whole 4096 tile")
    A, B, got = _gemm_case(L, M, N, K, (4096, 0), (0, 4096), (4096, 4096), (4096, 4096), seed=31)
    assert not np.isnan(got).any()
    ref = oracle.gemm(A, B)
    scale = oracle.gemm(np.abs(A), np.abs(B))
    err = np.abs(got - ref) / scale
    say("gemm whole 4096 tile: worst componentwise error %.3g" % err.max())
    assert err.max() <= 1e-5


def test_gemm_config3_out_of_core(L):
    # C = A B, FP32, 65536^2 operands (16 GiB each) in pinned host memory,
    # device budget 16 GiB, 4096^2 superblocks in serpentine order: A is split
    # in 4096-row panels, B in 4096-column panels, C in 4096^2 tiles.  C
    # starts as NaN, so a tile that is never written cannot pass.  Checked by
    # Freivalds at full size per 4096-column panel (each panel its own probe
    # vector, so the scale is one panel's, not a whole row's) and 4096 sampled
    # entries against float64.
    n, T = 65536, 4096
    say("gemm config3: allocating 48 GiB pinned host memory")
    with ctx_of(L, device_budget_bytes=16 << 30, stage_threshold_bytes=8 << 30,
                sb_order=L.LT_ORDER_SERPENTINE) as ctx:
        A = ctx.pinned((n, n))
        B = ctx.pinned((n, n))
        Cm = ctx.pinned((n, n))
        say("gemm config3: generating operands")
        synthetic.gemm_operand(0, n, T, out=A, workers=16)
        synthetic.gemm_operand(1, n, T, out=B, workers=16)
        for r0 in range(0, n, T):
            Cm[r0:r0 + T].fill(np.nan)
        a = ctx.array_host(A, chunk=[T, 0])
        b = ctx.array_host(B, chunk=[0, T])
        c = ctx.array_host(Cm, chunk=[T, T])
        say("gemm config3: launching")
        ctx.launch("gemm_f32", [n, n], [1, 1], [T, T], args=[n, n, n, c, a, b])
        ctx.sync()
        st = ctx.stats()
        say("gemm config3: H2D GiB %.1f D2H GiB %.1f" % (st["bytes_h2d"] / 2**30, st["bytes_d2h"] / 2**30))
        assert st["peak_resident_bytes"] <= 16 << 30
        assert st["evictions_dirty"] > 0
        rng = np.random.default_rng(7)
        ii = rng.integers(0, n, 4096)
        jj = rng.integers(0, n, 4096)
        for r0 in range(0, n, T):
            assert not np.isnan(Cm[r0:r0 + T]).any(), r0
        val, av = oracle.gemm_entries(A, B, ii, jj)
        assert np.all(np.abs(Cm[ii, jj] - val) <= 1e-5 * av)
        say("gemm config3: Freivalds per 4096-column panel")
        worst = oracle.freivalds(A, B, Cm, trials=2, panel=T)
        say("gemm config3: Freivalds worst ratio %.3g" % worst)
        assert worst < 1e-5


def test_gemm_out_of_core_issue_orders(L):
    # C = A B with host-home operands, 8 x 8 superblocks (the last row and
    # column ragged) and a device budget of five A/B panels, so chunks are
    # evicted and reloaded: every issue order gives the same C, bit for bit,
    # within the componentwise bound of the float64 product
    n, T = 1000, 128
    rng = np.random.default_rng(29)
    A0 = rng.standard_normal((n, n), dtype=np.float32)
    B0 = rng.standard_normal((n, n), dtype=np.float32)
    ref = oracle.gemm(A0, B0)
    scale = oracle.gemm(np.abs(A0), np.abs(B0))
    outs = []
    for order, band in ((L.LT_ORDER_SERPENTINE, 0), (L.LT_ORDER_BANDS, 2), (L.LT_ORDER_BANDS, 3)):
        say("gemm out-of-core order", order, band)
        with ctx_of(L, device_budget_bytes=5 * T * n * 4, sb_order=order, sb_band=band) as ctx:
            A = ctx.pinned((n, n))
            B = ctx.pinned((n, n))
            Cm = ctx.pinned((n, n))
            A[:] = A0
            B[:] = B0
            Cm[:] = np.nan
            a = ctx.array_host(A, chunk=[T, 0])
            b = ctx.array_host(B, chunk=[0, T])
            c = ctx.array_host(Cm, chunk=[T, T])
            ctx.launch("gemm_f32", [n, n], [1, 1], [T, T], args=[n, n, n, c, a, b])
            ctx.sync()
            st = ctx.stats()
            assert st["peak_resident_bytes"] <= 5 * T * n * 4
            assert st["evictions_clean"] + st["evictions_dirty"] > 0
            outs.append(Cm.copy())
    assert not np.isnan(outs[0]).any()
    assert np.all(np.abs(outs[0] - ref) <= 1e-5 * scale + 1e-30)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 1023, 1025])
def test_stencil1d_degenerate_sizes(L, n):
    say("stencil1d tiny", n)
    x0 = synthetic.stencil1d_input(n, 3)
    for mode in (0, 1):
        with ctx_of(L, exec_mode=mode) as ctx:
            x = ctx.array([n])
            y = ctx.array([n])
            x.write(x0)
            y.fill(9.0)
            ctx.launch("stencil1d_f32", [n], [1], [max(1, n // 2)], args=[n, y, x])
            ctx.sync()
            assert np.array_equal(y.read(), oracle.stencil1d(x0)), (n, mode)


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (5, 1), (2, 2), (3, 257), (17, 4)])
def test_jacobi_degenerate_shapes(L, shape):
    n, m = shape
    say("jacobi tiny", shape)
    x0 = synthetic.jacobi2d_input(n, m, seed=8)
    with ctx_of(L) as ctx:
        a = ctx.array([n, m])
        b = ctx.array([n, m])
        a.write(x0)
        inp, out = a, b
        for _ in range(3):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], [max(1, n // 2), 0], args=[n, m, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = inp.read()
    assert np.array_equal(got, oracle.jacobi2d(x0, 3))


def test_empty_grid_launch_is_a_no_op(L):
    n = 64
    say("empty grid")
    with ctx_of(L) as ctx:
        x = ctx.array([n])
        y = ctx.array([n])
        x.fill(1.0)
        y.fill(7.0)
        ctx.launch("stencil1d_f32", [0], [1], [1], args=[n, y, x])
        ctx.sync()
        assert np.all(y.read() == 7.0)


# --------------------------------------------------------------- denormals
# The oracle never flushes subnormals; the HIP code is built without
# flush-to-zero, so the stencils stay bit-exact on subnormal data.

def test_stencil1d_subnormal_inputs_bit_exact(L):
    n = 4099
    say("stencil1d subnormal")
    rng = np.random.default_rng(77)
    x0 = (rng.uniform(-1, 1, n) * 2.0 ** -140).astype(np.float32)
    assert np.count_nonzero(np.abs(x0) < np.finfo(np.float32).tiny) > n // 2
    with ctx_of(L) as ctx:
        x = ctx.array([n], chunk=[1024])
        y = ctx.array([n], chunk=[1024])
        x.write(x0)
        ctx.launch("stencil1d_f32", [n], [1], [1024], args=[n, y, x])
        ctx.sync()
        got = y.read()
    ref = oracle.stencil1d(x0)
    assert np.count_nonzero(ref) > 0
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_jacobi_subnormal_inputs_bit_exact(L):
    n, m = 130, 1024
    say("jacobi subnormal")
    rng = np.random.default_rng(78)
    x0 = (rng.uniform(0, 1, (n, m)) * 2.0 ** -138).astype(np.float32)
    with ctx_of(L) as ctx:
        a = ctx.array([n, m], chunk=[64, 0])
        b = ctx.array([n, m], chunk=[64, 0])
        a.write(x0)
        ctx.launch("jacobi2d_f32", [n, m], [1, 1], [64, 0], args=[n, m, b, a])
        ctx.sync()
        got = b.read()
    ref = oracle.jacobi2d(x0, 1)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_gemm_subnormal_products_kept(L):
    # products of 2^-70 x 2^-70 = 2^-140 are float32 subnormals, and so is
    # their sum over K = 256 (2^-132); the FP32 matrix cores keep them
    M = N = K = 256
    say("gemm subnormal")
    A = np.full((M, K), 2.0 ** -70, np.float32)
    B = np.full((K, N), 2.0 ** -70, np.float32)
    with ctx_of(L) as ctx:
        a = ctx.array([M, K])
        b = ctx.array([K, N])
        c = ctx.array([M, N])
        a.write(A)
        b.write(B)
        ctx.launch("gemm_f32", [M, N], [1, 1], [M, N], args=[M, N, K, c, a, b])
        ctx.sync()
        got = c.read()
    exact = np.float32(K * 2.0 ** -140)   # 2^-132, a subnormal, exactly representable
    assert exact != 0 and exact < np.finfo(np.float32).tiny
    assert np.all(got == exact)


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("shape,chunk", [((300, 517), (64, 128)), ((257, 1024), (64, 0)), ((33, 7), (5, 3))])
def test_host_backed_write_back_paths(L, pinned, engine, shape, chunk):
    # results written back into the home buffer through a copy kernel
    # (pinned home, d2h_kernel 1: rows of any pitch and width, 16-, 4- and
    # 1-byte words) or the copy engine, out of core so that write-backs
    # happen during the launches and at the sync
    n, m = shape
    say("write-back paths", shape, chunk, pinned, engine)
    x0 = synthetic.jacobi2d_input(n, m, seed=31)
    tile = chunk[0] * (chunk[1] or m) * 4
    with ctx_of(L, device_budget_bytes=16 * tile + (1 << 20), d2h_kernel=1 - engine) as ctx:
        A = ctx.pinned((n, m)) if pinned else np.empty((n, m), np.float32)
        B = ctx.pinned((n, m)) if pinned else np.empty((n, m), np.float32)
        A[...] = x0
        B[...] = np.nan
        a = ctx.array_host(A, chunk=list(chunk))
        b = ctx.array_host(B, chunk=list(chunk))
        inp, out = a, b
        for _ in range(3):
            ctx.launch("jacobi2d_f32", [n, m], [1, 1], list(chunk), args=[n, m, out, inp])
            inp, out = out, inp
        ctx.sync()
        got = np.array(B if inp is b else A)
    assert np.array_equal(got, oracle.jacobi2d(x0, 3))


@pytest.mark.parametrize("n,chunk", [(3_000_001, 1 << 19), (40_000_000, 1 << 25)])
def test_stencil1d_pageable_home_out_of_core(L, n, chunk):
    # a 1-D host-backed array over pageable memory, larger than the device
    # budget: its chunks reach the device through the pinned bounce ring
    # (pieces of up to 64 MiB of one row)
    say("stencil pageable home", n, chunk)
    x0 = synthetic.stencil1d_input(n, 7)
    A = x0.copy()
    B = np.full(n, np.nan, np.float32)
    with ctx_of(L, device_budget_bytes=6 * chunk * 4 + (1 << 20)) as ctx:
        a = ctx.array_host(A, chunk=[chunk])
        b = ctx.array_host(B, chunk=[chunk])
        inp, out = a, b
        for _ in range(3):
            ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, out, inp])
            inp, out = out, inp
        ctx.sync()
        st = ctx.stats()
        got = np.array(B if inp is b else A)
    assert st["bytes_h2d"] > 0
    assert np.array_equal(got, oracle.stencil1d_iter(x0, 3))
