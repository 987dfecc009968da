"""Seeded synthetic inputs for the annotated-launch workloads.

This module only draws random numbers and lays them out.  It holds none of the
method's arithmetic (no stencil, no product, no histogram, no distance), so
both the CPU oracle and the GPU path may take their inputs from here.

Every generator is deterministic in its seed.  numpy's ``default_rng`` (PCG64)
is the only random source; sub-streams are seeded with a list ``[seed, ...]``
so that a tile or a request can be regenerated on its own.

Workloads (shapes and laws of the five benchmark configurations):

* 1-D stencil input: float32 ~ U(-1, 1), length 2**20, seed 0.
* 2-D Jacobi field: float32 ~ U[0, 1), 16384 x 16384, seed 1.
* GEMM operands: float32 ~ N(0, 1), 65536 x 65536, built tile by tile from
  ``default_rng([2, m, I, J])`` (m = 0 for A, 1 for B) so any tile can be
  recomputed independently of the others.
* Batching mix: 8192 launches; kind ~ Bernoulli(1/2) (0 = stencil,
  1 = histogram); size n = floor(2**U(10, 24)); stencil data ~ U(-1, 1);
  histogram values int32 from a Zipf(s = 1.1) law bounded to 0..255, drawn by
  inverse CDF.  Seed 3.
* Serving trace: Poisson arrivals (rate 200/s, seed 4) of Jacobi, k-means and
  GEMM requests; k-means points are Gaussian blobs around 64 centres in 16-D.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# ---------------------------------------------------------------- 1-D stencil


def stencil1d_input(n: int = 1 << 20, seed: int = 0) -> np.ndarray:
    """x ~ U(-1, 1) float32 of length n."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n).astype(np.float32)


# ------------------------------------------------------------------ 2-D Jacobi


def jacobi2d_input(n: int = 16384, m: int | None = None, seed: int = 1,
                   out: np.ndarray | None = None) -> np.ndarray:
    """X0 ~ U[0, 1) float32 of shape (n, m), row-major.

    Rows are drawn in bands from independent sub-streams ``[seed, band]`` so a
    large field can be produced by several threads and still be reproducible.
    """
    m = n if m is None else m
    if out is None:
        out = np.empty((n, m), dtype=np.float32)
    band = 512
    nb = (n + band - 1) // band

    def fill(b):
        r0, r1 = b * band, min(n, (b + 1) * band)
        np.random.default_rng([seed, b]).random((r1 - r0, m), dtype=np.float32,
                                                out=out[r0:r1])

    if nb == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(max_workers=8) as ex:
            list(ex.map(fill, range(nb)))
    return out


# ----------------------------------------------------------------------- GEMM


def gemm_tile(m: int, I: int, J: int, tile: int, seed: int = 2) -> np.ndarray:
    """One tile of operand m (0 = A, 1 = B) at tile coordinates (I, J)."""
    return np.random.default_rng([seed, m, I, J]).standard_normal(
        (tile, tile), dtype=np.float32)


def gemm_operand(m: int, n: int, tile: int, seed: int = 2,
                 out: np.ndarray | None = None, workers: int = 8) -> np.ndarray:
    """Operand m of an n x n GEMM, assembled row-major from seeded tiles.

    ``out`` may be any writable float32 (n, n) buffer, e.g. a view of pinned
    host memory.
    """
    assert n % tile == 0
    if out is None:
        out = np.empty((n, n), dtype=np.float32)
    nt = n // tile

    def fill(idx):
        I, J = divmod(idx, nt)
        out[I * tile:(I + 1) * tile, J * tile:(J + 1) * tile] = gemm_tile(m, I, J, tile, seed)

    if nt * nt == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fill, range(nt * nt)))
    return out


# ---------------------------------------------------------------- histogram

ZIPF_S = 1.1
HIST_BINS = 256


def zipf_cdf(s: float = ZIPF_S, nbins: int = HIST_BINS) -> np.ndarray:
    """CDF of the bounded Zipf law P(v = k) proportional to (k + 1)**-s."""
    w = (np.arange(1, nbins + 1, dtype=np.float64)) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


_ZIPF_TABLES = {}


def _zipf_table(s: float, nbins: int, cells: int = 1 << 16):
    """Per cell [j / cells, (j + 1) / cells) of the unit interval: the number
    of CDF entries <= j / cells, and the most entries any cell spans."""
    key = (s, nbins, cells)
    if key not in _ZIPF_TABLES:
        cdf = zipf_cdf(s, nbins)
        lo = np.searchsorted(cdf, np.arange(cells, dtype=np.float64) / cells, side="right")
        hi = np.searchsorted(cdf, np.arange(1, cells + 1, dtype=np.float64) / cells, side="right")
        _ZIPF_TABLES[key] = (cdf, lo.astype(np.int32), int((hi - lo).max()), cells)
    return _ZIPF_TABLES[key]


def zipf_values(n: int, rng: np.random.Generator, s: float = ZIPF_S,
                nbins: int = HIST_BINS) -> np.ndarray:
    """n int32 values in [0, nbins) drawn by inverse CDF from bounded Zipf(s):
    value = the number of CDF entries <= u for u ~ U[0, 1) (searchsorted with
    side "right", clipped to nbins - 1), found through a cell table and at
    most `span` exact comparisons against the CDF."""
    cdf, lo, span, cells = _zipf_table(s, nbins)
    u = rng.random(n)
    v = lo[(u * cells).astype(np.int64)]
    cdf_ext = np.append(cdf, np.inf)
    for _ in range(span):
        v += cdf_ext[v] <= u
    np.minimum(v, nbins - 1, out=v)
    return v.astype(np.int32)


# ----------------------------------------------------------------- batching


def batch_plan(count: int = 8192, seed: int = 3, lo_log2: float = 10.0,
               hi_log2: float = 24.0):
    """Kinds and sizes of the batching mix: list of (kind, n).

    kind 0 = 1-D stencil (float32), kind 1 = 256-bin histogram (int32).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(2))
        n = int(math.floor(2.0 ** rng.uniform(lo_log2, hi_log2)))
        out.append((kind, n))
    return out


def batch_data(kind: int, n: int, launch: int, seed: int = 3) -> np.ndarray:
    """Input array of launch ``launch`` in the batching mix."""
    rng = np.random.default_rng([seed, launch])
    if kind == 0:
        return rng.uniform(-1.0, 1.0, n).astype(np.float32)
    return zipf_values(n, rng)


# ------------------------------------------------------------------- k-means


def kmeans_blobs(N: int, d: int = 16, K: int = 64, seed: int = 4,
                 spread: float = 10.0):
    """Gaussian blobs: K means ~ U(-spread, spread)^d, points mu_z + N(0, I).

    Returns (X float32 (N, d), centres float32 (K, d), z int32 (N,)).
    """
    rng = np.random.default_rng([seed, N, d, K])
    mu = rng.uniform(-spread, spread, (K, d)).astype(np.float32)
    z = rng.integers(0, K, N).astype(np.int32)
    X = (mu[z] + rng.standard_normal((N, d), dtype=np.float32)).astype(np.float32)
    return X, mu, z


def kmeans_blobs_banded(N: int, d: int = 16, K: int = 64, seed: int = 4, spread: float = 10.0,
                        out: np.ndarray | None = None, band: int = 1 << 22, workers: int = 16):
    """Gaussian blobs for large N, drawn in bands of ``band`` points by a pool
    of threads straight into ``out`` (e.g. pinned host memory): K means
    ~ U(-spread, spread)^d from sub-stream [seed, N, d, K]; band b's labels z
    (uniform over K) and N(0, I) offsets from sub-stream [seed, N, d, K, b].
    The same law as ``kmeans_blobs``, other streams.  Returns (X, means)."""
    mu = np.random.default_rng([seed, N, d, K]).uniform(-spread, spread, (K, d)).astype(np.float32)
    if out is None:
        out = np.empty((N, d), dtype=np.float32)

    def fill(b):
        r0 = b * band
        r1 = min(N, r0 + band)
        rng = np.random.default_rng([seed, N, d, K, b])
        z = rng.integers(0, K, r1 - r0)
        rng.standard_normal((r1 - r0, d), dtype=np.float32, out=out[r0:r1])
        out[r0:r1] += mu[z]

    nb = (N + band - 1) // band
    if nb == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fill, range(nb)))
    return out, mu


# ------------------------------------------------------------------- serving


def dense_normal(shape, seed, out=None, band: int = 4096) -> np.ndarray:
    """~N(0, 1) float32 of ``shape`` (2-D), row bands from sub-streams
    ``[*seed, band]`` (serving GEMM operands of arbitrary size)."""
    seed = list(seed) if isinstance(seed, (list, tuple)) else [seed]
    if out is None:
        out = np.empty(shape, dtype=np.float32)
    for b, r0 in enumerate(range(0, shape[0], band)):
        r1 = min(shape[0], r0 + band)
        np.random.default_rng(seed + [b]).standard_normal((r1 - r0, shape[1]), dtype=np.float32,
                                                            out=out[r0:r1])
    return out



def serving_trace(count: int = 512, rate: float = 200.0, seed: int = 4,
                  jacobi_range=(1024, 32768), kmeans_range=(1e5, 1e9),
                  gemm_range=(1024, 65536), pool: int = 8):
    """Poisson request trace.

    Each request is a dict with arrival time ``t`` (s), ``kind`` in
    {"jacobi", "kmeans", "gemm"}, a size drawn log-uniformly from the kind's
    range, and ``dataset``: an index into a pool of ``pool`` datasets per kind
    with Zipf(1.1) popularity, so repeated requests can reuse resident arrays.
    Sizes are a property of the dataset, so a repeated dataset has one size.
    """
    rng = np.random.default_rng(seed)
    kinds = ("jacobi", "kmeans", "gemm")
    ranges = {"jacobi": jacobi_range, "kmeans": kmeans_range, "gemm": gemm_range}
    sizes = {}
    for k in kinds:
        lo, hi = ranges[k]
        u = np.random.default_rng([seed, kinds.index(k)]).uniform(
            math.log(lo), math.log(hi), pool)
        sizes[k] = [int(math.exp(x)) for x in u]
    pop = zipf_cdf(1.1, pool)
    t = 0.0
    out = []
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        kind = kinds[int(rng.integers(3))]
        ds = int(np.searchsorted(pop, rng.random(), side="right"))
        ds = min(ds, pool - 1)
        out.append({"id": r, "t": t, "kind": kind, "dataset": ds,
                    "size": sizes[kind][ds]})
    return out
