"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (``paper_2202_05549_amd``)
never imports it, and the two share no code: the oracle has its own C
routines (``oracle.c``) and its own annotation reader (``planner.py``).

Numpy-level wrappers around ``liboracle.so``.  ``build()`` compiles it with
gcc (``-O2 -fopenmp -ffp-contract=off``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-o", tmp,
                               src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        i64, p, i32 = C.c_int64, C.c_void_p, C.c_int
        L.or_stencil1d_f32.argtypes = [i64, p, p]
        L.or_jacobi2d_sweep_f32.argtypes = [i64, i64, p, p]
        L.or_jacobi2d_f32.argtypes = [i64, i64, i32, p, p]
        L.or_jacobi2d_f32.restype = i32
        L.or_gemm_f64.argtypes = [i64, i64, i64, p, i64, p, i64, p, i64]
        L.or_gemm_entries_f64.argtypes = [i64, p, i64, p, i64, i64, p, p, p, p]
        L.or_matvec_f64.argtypes = [i64, i64, p, i64, p, p, i32]
        L.or_matmul_thin_f64.argtypes = [i64, i64, p, i64, i64, p, p, i32]
        L.or_hist256_i32.argtypes = [i64, p, p]
        L.or_kmeans_assign_f32.argtypes = [i64, i64, i64, p, p, p]
        L.or_kmeans_dist_f64.argtypes = [i64, p, p]
        L.or_kmeans_dist_f64.restype = C.c_double
        L.or_reduce_rows_f64.argtypes = [i64, i64, i32, p, p, p]
        L.or_kmeans_update_f64.argtypes = [i64, i64, i64, p, p, p, p, p]
        L.or_kmeans_centres_f32.argtypes = [i64, i64, p, p, p]
        L.or_touch_i32.argtypes = [i64, i64, p]
        L.or_num_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"] or a.ndim == 0
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ kernels


def stencil1d(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().or_stencil1d_f32(x.size, _ptr(x), _ptr(y))
    return y


def stencil1d_iter(x: np.ndarray, iters: int) -> np.ndarray:
    """``iters`` launches with input and output swapped after each."""
    a = np.ascontiguousarray(x, dtype=np.float32).copy()
    b = np.empty_like(a)
    for _ in range(iters):
        lib().or_stencil1d_f32(a.size, _ptr(a), _ptr(b))
        a, b = b, a
    return a


def jacobi2d_sweep(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().or_jacobi2d_sweep_f32(x.shape[0], x.shape[1], _ptr(x), _ptr(y))
    return y


def jacobi2d(x0: np.ndarray, sweeps: int, inplace: bool = False):
    """Result of ``sweeps`` ping-pong sweeps starting from x0.

    With ``inplace`` the input buffer is reused as the first ping-pong buffer
    (saves one copy of a large field).
    """
    a = x0 if inplace else np.array(x0, dtype=np.float32, copy=True)
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    b = np.empty_like(a)
    w = lib().or_jacobi2d_f32(a.shape[0], a.shape[1], sweeps, _ptr(a), _ptr(b))
    return a if w == 0 else b


def gemm(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """float64-accumulated A @ B for float32 A, B (any leading dimension)."""
    assert A.dtype == np.float32 and B.dtype == np.float32
    assert A.strides[1] == 4 and B.strides[1] == 4
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    Cm = np.empty((M, N), dtype=np.float64)
    lib().or_gemm_f64(M, N, K, C.c_void_p(A.ctypes.data), A.strides[0] // 4,
                      C.c_void_p(B.ctypes.data), B.strides[0] // 4, _ptr(Cm), N)
    return Cm


def gemm_entries(A: np.ndarray, B: np.ndarray, ii, jj):
    """(value, |A||B| value) of selected entries of A @ B, in float64."""
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    val = np.empty(ii.size, dtype=np.float64)
    av = np.empty(ii.size, dtype=np.float64)
    K = A.shape[1]
    lib().or_gemm_entries_f64(K, C.c_void_p(A.ctypes.data), A.strides[0] // 4,
                              C.c_void_p(B.ctypes.data), B.strides[0] // 4,
                              ii.size, _ptr(ii), _ptr(jj), _ptr(val), _ptr(av))
    return val, av


def matvec(A: np.ndarray, x: np.ndarray, absval: bool = False) -> np.ndarray:
    assert A.dtype == np.float32 and A.strides[1] == 4
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.shape[0], dtype=np.float64)
    lib().or_matvec_f64(A.shape[0], A.shape[1], C.c_void_p(A.ctypes.data),
                        A.strides[0] // 4, _ptr(x), _ptr(y), int(absval))
    return y


def matmul_thin(A: np.ndarray, X: np.ndarray, absval: bool = False) -> np.ndarray:
    """op(A) X in float64 for float32 A (unit column stride) and a float64
    X with few columns; op takes |a| when ``absval``."""
    assert A.dtype == np.float32 and A.strides[1] == 4
    X = np.ascontiguousarray(X, dtype=np.float64)
    assert X.shape[0] == A.shape[1]
    Y = np.empty((A.shape[0], X.shape[1]), dtype=np.float64)
    lib().or_matmul_thin_f64(A.shape[0], A.shape[1], C.c_void_p(A.ctypes.data), A.strides[0] // 4,
                             X.shape[1], _ptr(X), _ptr(Y), int(absval))
    return Y


def freivalds(A, B, Cm, trials: int = 3, seed: int = 12345, panel: int = 0):
    """Randomized check of Cm = A B in float64 (Freivalds' algorithm).

    Each trial draws r in {-1, +1}^n and compares, row by row, Cm r with
    A (B r); the residual |(Cm r - A (B r))_i| is divided by the scale
    (|A| (|B| 1))_i, so a correct float32 product scores of the order of the
    float32 unit roundoff times sqrt(K).  With ``panel`` > 0 the columns are
    checked in panels of that width, each with its own r supported on the
    panel only: the scale then covers one panel instead of all n columns, so
    an error confined to a small block of C is not diluted by the whole row.
    Returns the worst ratio over rows, panels and trials.  A non-finite
    entry of Cm makes its row of Cm R non-finite (NaN times the zero of
    another panel is still NaN), and any non-finite ratio returns +inf, so a
    NaN-filled or unwritten part of C can never pass.
    """
    rng = np.random.default_rng(seed)
    n = B.shape[1]
    w = n if panel <= 0 else min(panel, n)
    starts = list(range(0, n, w))
    # column c of R is the indicator of panel c (for the scale) or the random
    # signs on panel c (for a trial): one pass over each matrix per trial
    ind = np.zeros((n, len(starts)), dtype=np.float64)
    for c, j0 in enumerate(starts):
        ind[j0:j0 + w, c] = 1.0
    scale = matmul_thin(A, matmul_thin(B, ind, absval=True), absval=True)
    worst = 0.0
    for _ in range(trials):
        R = ind * rng.choice(np.array([-1.0, 1.0]), (n, 1))
        lhs = matmul_thin(Cm, R)
        rhs = matmul_thin(A, matmul_thin(B, R))
        ratio = np.abs(lhs - rhs) / np.maximum(scale, np.finfo(np.float64).tiny)
        if not np.isfinite(ratio).all():
            return float("inf")
        worst = max(worst, float(ratio.max()))
    return worst


def hist256(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.int32)
    h = np.empty(256, dtype=np.int32)
    lib().or_hist256_i32(v.size, _ptr(v), _ptr(h))
    return h


def kmeans_assign(X: np.ndarray, Cen: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    Cen = np.ascontiguousarray(Cen, dtype=np.float32)
    lab = np.empty(X.shape[0], dtype=np.int32)
    lib().or_kmeans_assign_f32(X.shape[0], X.shape[1], Cen.shape[0], _ptr(X),
                               _ptr(Cen), _ptr(lab))
    return lab


def kmeans_dist64(x: np.ndarray, c: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    c = np.ascontiguousarray(c, dtype=np.float32)
    return float(lib().or_kmeans_dist_f64(x.size, _ptr(x), _ptr(c)))


REDUCE_OPS = {"+": 0, "*": 1, "min": 2, "max": 3}


def reduce_rows(A: np.ndarray, op: str = "+"):
    """Row fold out[i] = op over j of A[i, j] in float64 (Sec. 2.3 example).
    Returns (out float64 (n,), sum_j |A[i, j]| float64 (n,))."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    n, m = A.shape
    out = np.empty(n, dtype=np.float64)
    sa = np.empty(n, dtype=np.float64)
    lib().or_reduce_rows_f64(n, m, REDUCE_OPS[op], _ptr(A), _ptr(out), _ptr(sa))
    return out, sa


def kmeans_update(X: np.ndarray, lab: np.ndarray, K: int):
    """Per-cluster sums (float64 (K, d)), counts (int64 (K,)) and sums of
    absolute values (float64 (K, d)) of the points with each label."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    N, d = X.shape
    sums = np.empty((K, d), dtype=np.float64)
    counts = np.empty(K, dtype=np.int64)
    abss = np.empty((K, d), dtype=np.float64)
    lib().or_kmeans_update_f64(N, d, K, _ptr(X), _ptr(lab), _ptr(sums), _ptr(counts), _ptr(abss))
    return sums, counts, abss


def kmeans_centres(sums: np.ndarray, counts: np.ndarray, cen: np.ndarray) -> np.ndarray:
    """New float32 centres sums / counts (rounded once); empty clusters keep
    the centre in ``cen``.  Returns a new array."""
    sums = np.ascontiguousarray(sums, dtype=np.float64)
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    out = np.array(cen, dtype=np.float32, copy=True)
    K, d = out.shape
    lib().or_kmeans_centres_f32(K, d, _ptr(sums), _ptr(counts), _ptr(out))
    return out


def kmeans_lloyd(X: np.ndarray, cen0: np.ndarray, iters: int):
    """The K-Means benchmark's loop: ``iters`` rounds of assignment then
    centre update.  Returns a list of (labels, sums, counts, centres) per
    round."""
    cen = np.array(cen0, dtype=np.float32, copy=True)
    out = []
    for _ in range(iters):
        lab = kmeans_assign(X, cen)
        sums, counts, _ = kmeans_update(X, lab, cen.shape[0])
        cen = kmeans_centres(sums, counts, cen)
        out.append((lab, sums, counts, cen))
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


def touch(y: np.ndarray, grid: int) -> np.ndarray:
    y = np.array(y, dtype=np.int32, copy=True)
    lib().or_touch_i32(y.size, grid, _ptr(y))
    return y
