"""Pins of the CPU oracle against facts it does not compute itself.

Each test checks one oracle routine against something fixed outside it: a
closed form, an exact-arithmetic evaluation with the float32 rounding bound,
a textbook special case, or a library routine on a special case (exact
integer products, ``bincount``).  They run without a GPU.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthetic

U = 2.0 ** -24  # float32 unit roundoff


# ------------------------------------------------------------------ stencil1d

@pytest.mark.parametrize("c", [1.0, 0.75, -2.5, 3.0, 1024.0, 2.0 ** -20])
def test_stencil1d_constant_field_is_fixed_in_interior(c):
    n = 1000
    y = oracle.stencil1d(np.full(n, c, np.float32))
    assert np.all(y[1:-1] == np.float32(c))
    # the two ends see one zero neighbour: (c + 0)/4 + c/2 = 3c/4, exact here
    assert y[0] == np.float32(0.75 * c) and y[-1] == np.float32(0.75 * c)


def test_stencil1d_linear_ramp_is_fixed_in_interior():
    n = 1 << 16
    x = np.arange(n, dtype=np.float32)
    y = oracle.stencil1d(x)
    assert np.array_equal(y[1:-1], x[1:-1])
    assert y[0] == np.float32(0.25)
    assert y[-1] == np.float32((n - 2) / 4 + (n - 1) / 2)


@pytest.mark.parametrize("k", [1, 3, 17])
def test_stencil1d_eigenmode(k):
    # x_i = sin(pi k (i+1)/(n+1)) vanishes at i = -1 and i = n, so the stencil
    # with zero outside maps it to (1/2 + cos(pi k/(n+1))/2) x exactly.
    n = 4096
    i = np.arange(n)
    x64 = np.sin(np.pi * k * (i + 1) / (n + 1))
    lam = 0.5 + 0.5 * np.cos(np.pi * k / (n + 1))
    y = oracle.stencil1d(x64.astype(np.float32)).astype(np.float64)
    # input rounding (<= u per entry, operator norm 1) plus two roundings
    assert np.max(np.abs(y - lam * x64)) <= 4 * U


def test_stencil1d_exact_arithmetic_bound():
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, 97).astype(np.float32)
    y = oracle.stencil1d(x)
    n = x.size
    for i in range(n):
        a = Fraction(float(x[i - 1])) if i > 0 else Fraction(0)
        b = Fraction(float(x[i]))
        c = Fraction(float(x[i + 1])) if i + 1 < n else Fraction(0)
        exact = (a + c) / 4 + b / 2
        bound = U * (abs(float(a + c)) / 4 + abs(float(exact))) * (1 + 4 * U)
        assert abs(float(Fraction(float(y[i])) - exact)) <= bound, i


# ------------------------------------------------------------------ jacobi2d

def test_jacobi_constant_field_after_t_sweeps():
    N, c, t = 40, 1.0, 7
    y = oracle.jacobi2d(np.full((N, N), c, np.float32), t)
    r = np.arange(N)
    d = np.minimum.outer(np.minimum(r, N - 1 - r), np.minimum(r, N - 1 - r))
    assert np.all(y[d >= t] == np.float32(c))
    one = oracle.jacobi2d_sweep(np.full((N, N), c, np.float32))
    assert one[0, 0] == 0.5 and one[0, N - 1] == 0.5 and one[N - 1, 0] == 0.5
    assert np.all(one[0, 1:-1] == 0.75) and np.all(one[1:-1, 0] == 0.75)
    assert np.all(one[1:-1, 1:-1] == 1.0)


def test_jacobi_exact_arithmetic_bound_one_sweep():
    rng = np.random.default_rng(11)
    n, m = 9, 13
    x = rng.uniform(-1, 1, (n, m)).astype(np.float32)
    y = oracle.jacobi2d_sweep(x)

    def g(r, c):
        return Fraction(float(x[r, c])) if 0 <= r < n and 0 <= c < m else Fraction(0)

    for r in range(n):
        for c in range(m):
            V = g(r - 1, c) + g(r + 1, c)
            H = g(r, c - 1) + g(r, c + 1)
            exact = (V + H) / 4
            bound = U * (abs(float(V)) + abs(float(H)) + abs(float(V + H))) / 4 * (1 + 4 * U)
            assert abs(float(Fraction(float(y[r, c])) - exact)) <= bound, (r, c)


@pytest.mark.parametrize("N", [64, 255])
def test_jacobi_eigenmode_decay(N):
    # u = sin(pi (r+1)/(N+1)) sin(pi (c+1)/(N+1)) is an eigenvector of the
    # four-neighbour mean with zero outside, eigenvalue cos(pi/(N+1)).
    t = 100
    r = np.arange(N)
    s = np.sin(np.pi * (r + 1) / (N + 1))
    u0 = np.outer(s, s)
    lam = np.cos(np.pi / (N + 1))
    y = oracle.jacobi2d(u0.astype(np.float32), t).astype(np.float64)
    ref = lam ** t * u0
    # worst case three roundings per sweep on non-negative data
    assert np.max(np.abs(y - ref)) <= (3 * t + 2) * U * np.max(ref) * 1.01
    assert np.max(np.abs(y - ref)) < 1e-5 * np.max(ref) * 3


def test_jacobi_pingpong_parity_of_result_buffer():
    x = synthetic.jacobi2d_input(32, seed=5)
    one = oracle.jacobi2d_sweep(x)
    two = oracle.jacobi2d_sweep(one)
    assert np.array_equal(oracle.jacobi2d(x, 1), one)
    assert np.array_equal(oracle.jacobi2d(x, 2), two)


# ---------------------------------------------------------------------- GEMM

def test_gemm_integer_matrices_exact():
    rng = np.random.default_rng(3)
    A = rng.integers(-8, 9, (37, 53))
    B = rng.integers(-8, 9, (53, 29))
    Cm = oracle.gemm(A.astype(np.float32), B.astype(np.float32))
    assert np.array_equal(Cm, (A @ B).astype(np.float64))


def test_gemm_identity_operands():
    A = synthetic.gemm_tile(0, 0, 0, 64)
    I = np.eye(64, dtype=np.float32)
    assert np.array_equal(oracle.gemm(A, I), A.astype(np.float64))
    assert np.array_equal(oracle.gemm(I, A), A.astype(np.float64))


def test_gemm_leading_dimension_views():
    rng = np.random.default_rng(4)
    A = rng.integers(-3, 4, (20, 30)).astype(np.float32)
    B = rng.integers(-3, 4, (30, 40)).astype(np.float32)
    full = oracle.gemm(A, B)
    sub = oracle.gemm(A[5:15, :], B[:, 10:25])
    assert np.array_equal(sub, full[5:15, 10:25])


def test_gemm_entries_and_freivalds_detect_error():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((96, 80), dtype=np.float32)
    B = rng.standard_normal((80, 72), dtype=np.float32)
    Cf = oracle.gemm(A, B)
    ii = rng.integers(0, 96, 50)
    jj = rng.integers(0, 72, 50)
    val, av = oracle.gemm_entries(A, B, ii, jj)
    assert np.allclose(val, Cf[ii, jj], rtol=0, atol=1e-12)
    assert np.all(av >= np.abs(val) - 1e-12)
    C32 = Cf.astype(np.float32)
    assert oracle.freivalds(A, B, C32) < 1e-6
    # the row-sum scale makes Freivalds blind to errors far below 1e-5 of a
    # whole row of |A||B|; a unit error in one entry is well above it
    bad = C32.copy()
    bad[17, 33] += 1.0
    assert oracle.freivalds(A, B, bad) > 1e-5


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_freivalds_fails_on_non_finite_entries(bad):
    # one non-finite entry anywhere (here in the last row and column) must
    # fail the check, with or without column panels
    rng = np.random.default_rng(15)
    A = rng.standard_normal((64, 48), dtype=np.float32)
    B = rng.standard_normal((48, 80), dtype=np.float32)
    C32 = oracle.gemm(A, B).astype(np.float32)
    assert oracle.freivalds(A, B, C32, panel=16) < 1e-6
    C32[63, 79] = bad
    assert oracle.freivalds(A, B, C32) == np.inf
    assert oracle.freivalds(A, B, C32, panel=16) == np.inf


def test_freivalds_matches_a_direct_residual_on_one_panel():
    # with a single trial and one panel the ratio is exactly
    # |(C - A B)[:, panel] r| / (|A| |B|)[:, panel] 1 for the drawn signs:
    # recomputed here from the full float64 product, independent of the
    # thin products the check uses
    rng = np.random.default_rng(16)
    A = rng.standard_normal((40, 30), dtype=np.float32)
    B = rng.standard_normal((30, 24), dtype=np.float32)
    E = np.zeros((40, 24), dtype=np.float64)
    E[7, 13] = 0.5
    Cm = (oracle.gemm(A, B) + E).astype(np.float32)
    got = oracle.freivalds(A, B, Cm, trials=1, seed=99, panel=8)
    r_all = np.random.default_rng(99).choice(np.array([-1.0, 1.0]), (24, 1))[:, 0]
    resid = np.zeros((40, 3))
    scale = np.zeros((40, 3))
    ref = oracle.gemm(A, B)
    absref = oracle.gemm(np.abs(A), np.abs(B))
    for c in range(3):
        sl = slice(8 * c, 8 * c + 8)
        resid[:, c] = np.abs((Cm.astype(np.float64)[:, sl] - ref[:, sl]) @ r_all[sl])
        scale[:, c] = absref[:, sl].sum(axis=1)
    assert got == pytest.approx((resid / scale).max(), rel=1e-6)


def test_freivalds_panels_see_a_wrong_block_that_whole_rows_miss():
    # a 32 x 32 block of C off by 1e-2 of |C| per entry: against the scale of
    # a whole 2048-column row the residual stays under the 1e-5 threshold;
    # against one 128-column panel it is far above it
    rng = np.random.default_rng(17)
    n = 2048
    A = rng.standard_normal((n, n), dtype=np.float32)
    B = rng.standard_normal((n, n), dtype=np.float32)
    Cm = oracle.gemm(A, B).astype(np.float32)
    assert oracle.freivalds(A, B, Cm, trials=1, panel=128) < 1e-6
    blk = Cm[512:544, 1024:1056]
    blk += np.float32(1e-2) * np.abs(blk) + np.float32(0.1)
    whole = oracle.freivalds(A, B, Cm, trials=2)
    panels = oracle.freivalds(A, B, Cm, trials=2, panel=128)
    assert panels > 1e-5
    assert whole < 1e-5
    assert panels > 8 * whole


# ----------------------------------------------------------------- histogram

def test_hist_counts_sum_and_bincount():
    rng = np.random.default_rng(6)
    v = synthetic.zipf_values(100_003, rng)
    h = oracle.hist256(v)
    assert h.sum() == v.size
    assert np.array_equal(h, np.bincount(v, minlength=256).astype(np.int32))


def test_hist_constant_and_out_of_range():
    v = np.full(1000, 77, np.int32)
    h = oracle.hist256(v)
    assert h[77] == 1000 and h.sum() == 1000
    w = np.array([-1, 256, 1 << 20, 5], np.int32)
    h2 = oracle.hist256(w)
    assert h2[5] == 1 and h2.sum() == 1


# ------------------------------------------------------------------- k-means

def test_kmeans_points_at_centres_take_own_label():
    rng = np.random.default_rng(8)
    Cen = rng.uniform(-10, 10, (64, 16)).astype(np.float32)
    lab = oracle.kmeans_assign(Cen.copy(), Cen)
    assert np.array_equal(lab, np.arange(64, dtype=np.int32))


def test_kmeans_tie_goes_to_smallest_index():
    Cen = np.array([[1, 0], [0, 1], [1, 0]], np.float32)
    X = np.array([[1, 0], [0.5, 0.5], [0, 1]], np.float32)
    # point 1 is equidistant from all; point 0 ties between centres 0 and 2
    assert list(oracle.kmeans_assign(X, Cen)) == [0, 0, 1]


def test_kmeans_matches_float64_argmin_on_blobs():
    X, mu, _ = synthetic.kmeans_blobs(5000, 16, 64, seed=9)
    lab = oracle.kmeans_assign(X, mu)
    d = ((X.astype(np.float64)[:, None, :] - mu.astype(np.float64)[None]) ** 2).sum(-1)
    ref = np.argmin(d, axis=1)
    srt = np.sort(d, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-4 * srt[:, 1]
    assert np.array_equal(lab[clear], ref[clear])
    p = int(np.argmax(clear))
    assert abs(oracle.kmeans_dist64(X[p], mu[lab[p]]) - d[p, lab[p]]) < 1e-9 * d[p, lab[p]] + 1e-12


# ------------------------------------------------------------------- touch

# ----------------------------------------------------------------- reductions

@pytest.mark.parametrize("op,np_fn", [("+", np.sum), ("min", np.min), ("max", np.max)])
def test_reduce_rows_matches_numpy_folds(op, np_fn):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((37, 1001)).astype(np.float32)
    out, sa = oracle.reduce_rows(A, op)
    ref = np_fn(A.astype(np.float64), axis=1)
    if op == "+":
        # float64 sums of 1001 float32 values: both within 1001 u64 sum|a|
        assert np.all(np.abs(out - ref) <= 1001 * 2.0 ** -53 * sa)
        assert np.allclose(sa, np.abs(A.astype(np.float64)).sum(axis=1))
    else:
        assert np.array_equal(out, ref)  # min and max are exact


def test_reduce_rows_closed_forms():
    m = 4096
    ramp = np.tile(np.arange(m, dtype=np.float32), (3, 1))
    out, _ = oracle.reduce_rows(ramp, "+")
    assert np.all(out == m * (m - 1) / 2)  # exact: integers below 2^53
    # products of powers of two are exact: 2^(sum of exponents)
    e = np.random.default_rng(2).integers(-3, 4, (5, 60))
    P = np.ldexp(np.ones_like(e, dtype=np.float32), e)
    prod, _ = oracle.reduce_rows(P, "*")
    assert np.array_equal(prod, np.ldexp(1.0, e.sum(axis=1)))
    # a sign flip: the max of -A is minus the min of A
    A = np.random.default_rng(3).uniform(-5, 5, (4, 100)).astype(np.float32)
    assert np.array_equal(oracle.reduce_rows(-A, "max")[0], -oracle.reduce_rows(A, "min")[0])


def test_reduce_rows_empty_fold_is_identity():
    A = np.zeros((3, 0), np.float32)
    assert np.array_equal(oracle.reduce_rows(A, "+")[0], np.zeros(3))
    assert np.array_equal(oracle.reduce_rows(A, "*")[0], np.ones(3))
    assert np.all(oracle.reduce_rows(A, "min")[0] == np.inf)
    assert np.all(oracle.reduce_rows(A, "max")[0] == -np.inf)


def test_kmeans_update_matches_bincount():
    rng = np.random.default_rng(5)
    N, d, K = 20000, 7, 13
    X = rng.standard_normal((N, d)).astype(np.float32)
    lab = rng.integers(0, K, N).astype(np.int32)
    sums, counts, abss = oracle.kmeans_update(X, lab, K)
    assert np.array_equal(counts, np.bincount(lab, minlength=K))
    assert counts.sum() == N
    for j in range(d):
        ref = np.bincount(lab, weights=X[:, j].astype(np.float64), minlength=K)
        assert np.all(np.abs(sums[:, j] - ref) <= N * 2.0 ** -53 * abss[:, j])
        aref = np.bincount(lab, weights=np.abs(X[:, j]).astype(np.float64), minlength=K)
        assert np.allclose(abss[:, j], aref, rtol=1e-12)
    # every point lands in exactly one cluster: cluster sums add up to column sums
    assert np.allclose(sums.sum(axis=0), X.astype(np.float64).sum(axis=0), rtol=0, atol=1e-9 * np.abs(X).sum())


def test_kmeans_update_points_at_integer_centres_exact():
    # centres with small integer coordinates; points exactly at them: sums are
    # counts times the centre, exactly, and the new centres equal the old ones
    K, d = 9, 5
    cen = np.arange(K * d, dtype=np.float32).reshape(K, d) - 20
    z = np.random.default_rng(6).integers(0, K - 1, 3000).astype(np.int32)  # cluster K-1 stays empty
    X = cen[z]
    lab = oracle.kmeans_assign(X, cen)
    assert np.array_equal(lab, z)
    sums, counts, _ = oracle.kmeans_update(X, lab, K)
    assert np.array_equal(sums, counts[:, None] * cen.astype(np.float64))
    assert counts[K - 1] == 0
    moved = cen.copy()
    moved[K - 1] = 99.0  # an empty cluster keeps whatever centre it had
    new = oracle.kmeans_centres(sums, counts, moved)
    assert np.array_equal(new[:K - 1], cen[:K - 1]) and np.all(new[K - 1] == 99.0)


def test_kmeans_update_ignores_out_of_range_labels():
    X = np.ones((6, 2), np.float32)
    lab = np.array([0, 1, -1, 2, 5, 1], np.int32)
    sums, counts, _ = oracle.kmeans_update(X, lab, 3)
    assert list(counts) == [1, 2, 1] and sums[1, 0] == 2.0


def test_kmeans_lloyd_on_separated_blobs():
    # started from the true means of well-separated blobs, the first round
    # labels every point with its own blob and moves each centre to the mean
    # of its blob's points; the within-cluster sum of squares never increases
    X, mu, z = synthetic.kmeans_blobs(30000, 16, 64, seed=8)
    rounds = oracle.kmeans_lloyd(X, mu, 5)
    lab1, _, counts1, cen1 = rounds[0]
    assert np.array_equal(lab1, z)
    X64 = X.astype(np.float64)
    for k in range(64):
        if counts1[k]:
            ref = X64[z == k].mean(axis=0)
            assert np.all(np.abs(cen1[k] - ref) <= 2 * np.abs(ref) * 2.0 ** -24 + 1e-12)
    sse = []
    cen = mu
    for lab, _, _, new in rounds:
        sse.append(float(((X64 - cen.astype(np.float64)[lab]) ** 2).sum()))
        cen = new
    assert all(b <= a * (1 + 1e-9) for a, b in zip(sse, sse[1:]))


def test_touch_exactly_once_within_n():
    y = oracle.touch(np.zeros(100, np.int32), grid=128)
    assert np.all(y == 1)
    y = oracle.touch(np.zeros(100, np.int32), grid=60)
    assert np.all(y[:60] == 1) and np.all(y[60:] == 0)


# --------------------------------------------------------------- synthetic

def test_zipf_law_normaliser():
    cdf = synthetic.zipf_cdf()
    w = np.arange(1, 257, dtype=np.float64) ** -1.1
    assert abs(w.sum() - 4.8421) < 1e-3
    assert abs(cdf[0] - 0.2065) < 1e-3
    v = synthetic.zipf_values(200_000, np.random.default_rng(1))
    assert v.min() >= 0 and v.max() <= 255
    assert abs((v == 0).mean() - 0.2065) < 5e-3


def test_batch_plan_sizes_log_uniform():
    plan = synthetic.batch_plan(8192)
    ns = np.array([n for _, n in plan])
    assert ns.min() >= 1 << 10 and ns.max() < 1 << 24
    kinds = np.array([k for k, _ in plan])
    assert 0.45 < kinds.mean() < 0.55
    assert abs(np.median(np.log2(ns)) - 17) < 0.3


def test_zipf_sampler_is_the_inverse_cdf():
    # the generator's cell table gives exactly searchsorted(cdf, u, "right")
    # (clipped to 255) for the uniform draws of the same generator
    cdf = synthetic.zipf_cdf()
    for seed in (0, 3, 11):
        u = np.random.default_rng(seed).random(2_000_000)
        ref = np.minimum(np.searchsorted(cdf, u, side="right"), 255).astype(np.int32)
        assert np.array_equal(synthetic.zipf_values(2_000_000, np.random.default_rng(seed)), ref)
