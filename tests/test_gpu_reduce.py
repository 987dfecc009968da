"""GPU parity of float reductions and the k-means centre update.

reduce(f) with f in {+, *, min, max} on float32 data (the row reduction of
Sec. 2.3), and the K-Means benchmark's centre update (per-cluster sums and
counts by reduce(+), then new centres), against the float64 oracle.

Tolerances, derived from the arithmetic:
  * min and max are exact: the result is one of the inputs, bit for bit.
  * Row +: each superblock's partial is a float64 fold rounded once to
    float32, and the P partials of a row are added in float32, so
    |gpu - exact| <= (P + 2) u sum_j |a_ij|, u = 2^-24 (the float64 part adds
    at most m 2^-53 sum |a|, far below one u).
  * Row *: the same count of float32 roundings, relative to |product|.
  * k-means sums are float64 folds in another order than the oracle's:
    |gpu - oracle| <= 2 N 2^-53 sum |x|; counts are integers and exact.
  * Centres: sums / counts in float64 rounded once to float32 on both sides,
    from float64 sums that agree to ~1e-13 relative: equal, or one float32
    ulp apart when the two sums straddle a rounding boundary.
Every float fold has a fixed order, so a repeated launch is bit-identical.
"""
import sys

import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


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


ROW_ANNOT = "global [i, j] => read A[i, j], reduce(%s) out[i]"


def _row_input(op, n, m, seed):
    rng = np.random.default_rng([31, seed])
    if op == "*":
        return rng.uniform(0.99, 1.0101, (n, m)).astype(np.float32)
    return rng.uniform(-1.0, 1.0, (n, m)).astype(np.float32)


def _rowreduce(L, ctx, A, op, sb, chunk=None, block=(1, 64)):
    n, m = A.shape
    a = ctx.array([n, m], chunk=chunk or [0, 0])
    out = ctx.array([n])
    a.write(A)
    out.fill(7.0)  # overwritten: reduce targets take the fold, not old + fold
    ctx.launch("rowreduce_f32", [n, m], list(block), list(sb), args=[n, m, out, a],
               kernel_annotation=ROW_ANNOT % op)
    ctx.sync()
    return out.read()


def _check_row(op, A, got, sb_cols):
    ref, sa = oracle.reduce_rows(A, op)
    P = -(-A.shape[1] // sb_cols)
    if op in ("min", "max"):
        assert np.array_equal(got.astype(np.float64), ref)
    elif op == "+":
        err = np.abs(got.astype(np.float64) - ref)
        assert np.all(err <= (P + 2) * U * sa), float((err / np.maximum(sa, 1e-300)).max())
    else:
        err = np.abs(got.astype(np.float64) - ref)
        assert np.all(err <= (P + 2) * U * np.abs(ref))


@pytest.mark.parametrize("op", ["+", "*", "min", "max"])
@pytest.mark.parametrize("n,m,sb", [(300, 5000, (64, 2048)), (7, 70001, (8, 70016)), (1000, 37, (128, 64)),
                                    (513, 4099, (512, 1024)), (50, 20000, (16, 1024))])
def test_rowreduce_ops_against_oracle(L, op, n, m, sb):
    # 20000 columns in superblocks of 1024: 20 partials per row, folded by
    # the combine in groups of 8 (8 + 8 + 4)
    say("rowreduce", op, n, m, sb)
    A = _row_input(op, n, m, n + m)
    with ctx_of(L) as ctx:
        got = _rowreduce(L, ctx, A, op, sb)
        again = _rowreduce(L, ctx, A, op, sb)
    _check_row(op, A, got, sb[1])
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))  # fixed fold order


@pytest.mark.parametrize("op", ["+", "max"])
def test_rowreduce_independent_of_distribution_and_mode(L, op):
    # same superblocks: the result is bit-identical whether A is one slab,
    # row chunks, column chunks (assembled temporaries, unaligned rows) or
    # tiles, and under either executor
    n, m, sb = 260, 3000, (64, 1024)
    say("rowreduce distributions", op)
    A = _row_input(op, n, m, 5)
    outs = []
    for mode in (0, 1):
        for chunk in ([0, 0], [100, 0], [0, 700], [90, 1100]):
            with ctx_of(L, exec_mode=mode) as ctx:
                outs.append(_rowreduce(L, ctx, A, op, sb, chunk=chunk))
    _check_row(op, A, outs[0], sb[1])
    for o in outs[1:]:
        assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32))


def test_rowreduce_subgrid_leaves_other_rows(L):
    # rows only partly covered by the grid keep the fold of what was covered
    n, m = 64, 256
    A = _row_input("+", n, m, 9)
    say("rowreduce sub-grid")
    with ctx_of(L) as ctx:
        a = ctx.array([n, m])
        out = ctx.array([n])
        a.write(A)
        out.fill(5.0)
        # grid of 32 rows: out[i] for i >= 32 is outside every region and stays
        ctx.launch("rowreduce_f32", [32, m], [1, 64], [16, 128], args=[n, m, out, a],
                   kernel_annotation=ROW_ANNOT % "min")
        ctx.sync()
        got = out.read()
    assert np.array_equal(got[:32].astype(np.float64), oracle.reduce_rows(A[:32], "min")[0])
    assert np.all(got[32:] == 5.0)


# ------------------------------------------------------------ k-means update

def _update(L, ctx, X, lab, K, sb, chunk=None):
    N, d = X.shape
    x = ctx.array([N, d], chunk=chunk or [0, 0])
    lb = ctx.array([N], np.int32, chunk=[chunk[0]] if chunk else [0])
    sums = ctx.array([K, d], np.float64)
    counts = ctx.array([K], np.int32)
    x.write(X)
    lb.write(lab)
    sums.fill(3.0)
    counts.fill(3)
    ctx.launch("kmeans_update_f32", [N], [1], [sb], args=[N, d, K, sums, counts, x, lb])
    ctx.sync()
    return sums.read(), counts.read()


@pytest.mark.parametrize("N,d,K,sb", [(312345, 16, 64, 65536), (100000, 3, 5, 100000), (50001, 32, 48, 4096),
                                      (20000, 16, 96, 1 << 20), (777, 4, 40, 256), (30001, 1, 7, 8192),
                                      (30001, 2, 256, 8192), (40000, 5, 33, 16384), (40000, 12, 100, 16383),
                                      (9000, 8, 64, 1000)])
def test_kmeans_update_against_oracle(L, N, d, K, sb):
    say("kmeans update", N, d, K, sb)
    X, _, z = synthetic.kmeans_blobs(N, d, K, seed=12)
    lab = z.copy()
    lab[::97] = -1  # labels outside [0, K) are skipped
    lab[5::131] = K + 3
    with ctx_of(L) as ctx:
        sums, counts = _update(L, ctx, X, lab, K, sb)
        sums2, counts2 = _update(L, ctx, X, lab, K, sb)
    rs, rc, ra = oracle.kmeans_update(X, lab, K)
    assert np.array_equal(counts.astype(np.int64), rc)
    assert np.all(np.abs(sums - rs) <= 2 * N * 2.0 ** -53 * ra)
    assert np.array_equal(sums.view(np.uint64), sums2.view(np.uint64)) and np.array_equal(counts, counts2)


def test_kmeans_update_spilled_inputs_bit_identical(L):
    # host-backed points streamed through a small device budget give the
    # same bits as the resident run with the same superblocks
    N, d, K, sb = 400000, 16, 64, 50000
    say("kmeans update spilled")
    X, _, z = synthetic.kmeans_blobs(N, d, K, seed=13)
    with ctx_of(L) as ctx:
        ref_s, ref_c = _update(L, ctx, X, z, K, sb, chunk=[sb, 0])
    with ctx_of(L, device_budget_bytes=24 << 20) as ctx:
        xh = ctx.pinned((N, d))
        xh[...] = X
        lh = ctx.pinned((N,), np.int32)
        lh[...] = z
        x = ctx.array_host(xh, chunk=[sb, 0])
        lb = ctx.array_host(lh, chunk=[sb])
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        ctx.launch("kmeans_update_f32", [N], [1], [sb], args=[N, d, K, sums, counts, x, lb])
        ctx.sync()
        s, c = sums.read(), counts.read()
        assert ctx.stats()["bytes_h2d"] > 0
    assert np.array_equal(s.view(np.uint64), ref_s.view(np.uint64)) and np.array_equal(c, ref_c)


def test_kmeans_centres_and_empty_cluster(L):
    N, d, K = 60000, 16, 65
    say("kmeans centres")
    X, mu, z = synthetic.kmeans_blobs(N, d, K - 1, seed=14)
    cen0 = np.vstack([mu, np.full((1, d), 42.0, np.float32)])  # cluster K-1 gets no points
    with ctx_of(L) as ctx:
        x = ctx.array([N, d])
        lb = ctx.array([N], np.int32)
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        cen = ctx.array([K, d])
        x.write(X)
        lb.write(z)
        cen.write(cen0)
        ctx.launch("kmeans_update_f32", [N], [256], [16384], args=[N, d, K, sums, counts, x, lb])
        ctx.launch("kmeans_centres_f32", [K, d], [1, 16], [K, d], args=[K, d, cen, sums, counts])
        ctx.sync()
        got = cen.read()
    rs, rc, _ = oracle.kmeans_update(X, z, K)
    ref = oracle.kmeans_centres(rs, rc, cen0)
    assert np.all(got[K - 1] == 42.0)
    ulps = np.abs(got.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1


def test_kmeans_lloyd_five_rounds(L):
    # the K-Means benchmark loop: assignment then centre update, 5 rounds,
    # from perturbed means; labels must match the oracle's run bit for bit
    # except at float64 near-ties, centres within one float32 ulp
    N, d, K, iters, sb = 200000, 16, 64, 5, 32768
    say("kmeans lloyd")
    X, mu, _ = synthetic.kmeans_blobs(N, d, K, seed=15)
    cen0 = (mu + np.random.default_rng(16).normal(0, 1.5, mu.shape)).astype(np.float32)
    ref = oracle.kmeans_lloyd(X, cen0, iters)
    with ctx_of(L) as ctx:
        x = ctx.array([N, d], chunk=[sb, 0])
        lb = ctx.array([N], np.int32, chunk=[sb])
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        cen = ctx.array([K, d])
        x.write(X)
        cen.write(cen0)
        prev = cen0
        for it in range(iters):
            ctx.launch("kmeans_assign_f32", [N], [256], [sb], args=[N, d, K, lb, x, cen])
            ctx.launch("kmeans_update_f32", [N], [1], [sb], args=[N, d, K, sums, counts, x, lb])
            ctx.launch("kmeans_centres_f32", [K, d], [1, 16], [K, d], args=[K, d, cen, sums, counts])
            ctx.sync()
            lab_g, cen_g = lb.read(), cen.read()
            # labels: the oracle's assignment from the centres this round
            # started from (the GPU's previous centres); a differing label
            # must be a near-tie in float64
            lab_r = oracle.kmeans_assign(X, prev)
            bad = np.nonzero(lab_g != lab_r)[0]
            for p in bad:
                da = oracle.kmeans_dist64(X[p], prev[lab_r[p]])
                db = oracle.kmeans_dist64(X[p], prev[lab_g[p]])
                assert abs(da - db) <= 1e-5 * max(da, db), (it, p)
            # centres, every round: the oracle's update of the GPU's labels
            rs, rc, _ = oracle.kmeans_update(X, lab_g, K)
            cen_r = oracle.kmeans_centres(rs, rc, prev)
            ulps = np.abs(cen_g.view(np.int32).astype(np.int64) - cen_r.view(np.int32).astype(np.int64))
            assert ulps.max() <= 1, it
            if it == 0:
                # the first round starts from the same centres as the oracle's loop
                assert np.array_equal(lab_g, ref[0][0]) or len(bad) > 0
            prev = cen_g


@pytest.mark.parametrize("d", [8, 16, 32])
def test_kmeans_update_lane_widths_bit_identical(L, d):
    # two or four features per lane (tuning variants 2 and 1) add the same
    # values in the same order
    N, K, sb = 70001, 40 if d == 32 else 64, 16384
    say("kmeans update lane widths", d)
    X, _, z = synthetic.kmeans_blobs(N, d, K, seed=21)
    outs = []
    for variant in (1, 2):
        with ctx_of(L) as ctx:
            if variant:
                ctx.tune("kmeans_update_f32", variant)
            outs.append(_update(L, ctx, X, z, K, sb))
    assert np.array_equal(outs[0][0].view(np.uint64), outs[1][0].view(np.uint64))
    assert np.array_equal(outs[0][1], outs[1][1])
    rs, rc, ra = oracle.kmeans_update(X, z, K)
    assert np.array_equal(outs[0][1].astype(np.int64), rc)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("N,d,K,sb", [(312345, 16, 64, 65536), (50001, 32, 48, 4096), (20000, 16, 96, 1 << 20),
                                      (4093, 16, 7, 1000), (9000, 32, 2, 2500)])
def test_kmeans_update_d16_d32_kernels(L, variant, N, d, K, sb):
    # d = 16 and 32: the default body (one feature per lane, two interleaved
    # LDS copies per wave) and variant 1 (four features per lane, one copy)
    # sum in different fixed orders: both within the float64 bound of the
    # oracle and bit-identical run to run.  Superblocks of 1000 and 2500
    # points leave partial tiles (the clamped load path); K = 96 at d = 16
    # and K = 48 at d = 32 need more than 64 KiB of LDS
    say("kmeans update d16/d32 kernels", variant, N, d, K, sb)
    X, _, z = synthetic.kmeans_blobs(N, d, K, seed=23)
    lab = z.copy()
    lab[::89] = -1
    lab[7::113] = K + 1
    with ctx_of(L) as ctx:
        ctx.tune("kmeans_update_f32", variant)
        sums, counts = _update(L, ctx, X, lab, K, sb)
        sums2, counts2 = _update(L, ctx, X, lab, K, sb)
    rs, rc, ra = oracle.kmeans_update(X, lab, K)
    assert np.array_equal(counts.astype(np.int64), rc)
    assert np.all(np.abs(sums - rs) <= 2 * N * 2.0 ** -53 * ra)
    assert np.array_equal(sums.view(np.uint64), sums2.view(np.uint64)) and np.array_equal(counts, counts2)


@pytest.mark.parametrize("N,d,K", [(1, 4, 1), (3, 16, 5), (7, 3, 64), (2, 32, 2)])
def test_kmeans_degenerate_sizes(L, N, d, K):
    # one point, more clusters than points, clusters left empty
    say("kmeans tiny", N, d, K)
    rng = np.random.default_rng([22, N, d, K])
    X = rng.standard_normal((N, d)).astype(np.float32)
    cen0 = rng.standard_normal((K, d)).astype(np.float32)
    with ctx_of(L) as ctx:
        x = ctx.array([N, d])
        cen = ctx.array([K, d])
        lb = ctx.array([N], np.int32)
        sums = ctx.array([K, d], np.float64)
        counts = ctx.array([K], np.int32)
        x.write(X)
        cen.write(cen0)
        ctx.launch("kmeans_assign_f32", [N], [1], [0], args=[N, d, K, lb, x, cen])
        ctx.launch("kmeans_update_f32", [N], [1], [0], args=[N, d, K, sums, counts, x, lb])
        ctx.launch("kmeans_centres_f32", [K, d], [1, 1], [K, d], args=[K, d, cen, sums, counts])
        ctx.sync()
        lab, s, c, got = lb.read(), sums.read(), counts.read(), cen.read()
    ref_lab = oracle.kmeans_assign(X, cen0)
    assert np.array_equal(lab, ref_lab)
    rs, rc, ra = oracle.kmeans_update(X, ref_lab, K)
    assert np.array_equal(c.astype(np.int64), rc)
    assert np.all(np.abs(s - rs) <= 2 * N * 2.0 ** -53 * ra)
    ref = oracle.kmeans_centres(rs, rc, cen0)
    ulps = np.abs(got.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1
