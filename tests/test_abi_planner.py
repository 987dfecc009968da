"""CPU tests of the C ABI and the planner (no GPU).

The library must load and export every symbol include/lt.h declares.  The
planner runs in dry-run contexts (planning and memory simulation only, no
device work) and its regions, superblocks and dependency edges are checked
against the brute-force planner oracle.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2202_05549_amd as L
from oracle import planner as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "lt.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    decl = set(re.findall(r"\b(lt_[a-z_0-9]+)\s*\(", hdr))
    assert len(decl) >= 25
    lib = C.CDLL(L.LIB_PATH)
    missing = [d for d in sorted(decl) if not hasattr(lib, d)]
    assert not missing, missing
    # the binding covers every declared call
    assert decl <= set(L.exported_symbols()) | {"lt_config_init"}


def dry(**kw):
    kw.setdefault("device_budget_bytes", 1 << 30)
    return L.Context(dry_run=1, **kw)


def _box(r, nd):
    return [(int(r.lo[a]), int(r.hi[a]) - 1) for a in range(nd)]


# ------------------------------------------------------------ regions (T2)

ANNOTS_1D = [
    "global i => read x[i-1:i+1], write y[i]",
    "global i => read x[2*i:2*i+3], write y[i]",
    "global i => read x[-3*i+40:-3*i+42], write y[i]",
    "global i, block b => read x[b:b+2], write y[i]",
    "global i, local t => read x[t], write y[i]",
    "global i, block b, local t => read x[4*b+t-1 : 4*b+t+5], write y[i]",
    "global i => read x[:], write y[i]",
    "global i => read x[5:], write y[i]",
    "global i => read x[:i], write y[i]",
]


@pytest.mark.parametrize("annot", ANNOTS_1D)
@pytest.mark.parametrize("n,block,sb", [(64, 4, 8), (61, 4, 12), (40, 1, 7)])
def test_regions_match_bruteforce_1d(annot, n, block, sb):
    ctx = dry()
    x = ctx.array([n], np.float32)
    y = ctx.array([n], np.float32)
    lid = ctx.launch("stencil1d_f32", [n], [block], [sb], args=[n, y, x], kernel_annotation=annot)
    grid_r = -(-n // block) * block
    sbs = P.superblocks([n], [block], [sb])
    tasks = ctx.tasks(lid)
    assert len(tasks) == len(sbs)
    for t, (lo, hi) in zip(tasks, sbs):
        assert (t.sb_lo[0], t.sb_hi[0]) == (lo[0], hi[0])
        regs = {r.arg: r for r in ctx.regions(t.id)}
        for arg, name in ((1, "y"), (2, "x")):
            exp = P.region(annot, name, [n], lo, hi, [block])
            got = _box(regs[arg], 1) if arg in regs else None
            assert got == (None if exp is None else [tuple(e) for e in exp]), (name, lo, hi)
    assert tasks[-1].sb_hi[0] == grid_r
    ctx.close()


ANNOTS_2D = [
    "global [r, c] => read x[r-1:r+1, c-1:c+1], write y[r, c]",
    "global [r, c] => read x[c, r], write y[r, c]",
    "global [r, c] => read x[r+c-2:r+c, 2*c-r], write y[r, c]",
    "global [r, c], block [br, bc], local [lr, lc] => read x[br*2+lc, :], write y[r, c]",
]


@pytest.mark.parametrize("annot", ANNOTS_2D)
def test_regions_match_bruteforce_2d(annot):
    n, m = 11, 13
    ctx = dry()
    x = ctx.array([n, m], np.float32)
    y = ctx.array([n, m], np.float32)
    block, sb = [2, 3], [4, 6]
    lid = ctx.launch("jacobi2d_f32", [n, m], block, sb, args=[n, m, y, x], kernel_annotation=annot)
    sbs = P.superblocks([n, m], block, sb)
    tasks = ctx.tasks(lid)
    assert len(tasks) == len(sbs)
    for t, (lo, hi) in zip(tasks, sbs):
        regs = {r.arg: r for r in ctx.regions(t.id)}
        for arg, name in ((2, "y"), (3, "x")):
            exp = P.region(annot, name, [n, m], lo, hi, block)
            got = _box(regs[arg], 2) if arg in regs else None
            assert got == (None if exp is None else [tuple(e) for e in exp]), (name, lo, hi)
            if exp is not None:
                pts = P.accessed_elements(annot, name, [n, m], lo, hi, block)
                for p in pts:
                    assert all(exp[a][0] <= p[a] <= exp[a][1] for a in range(2))
    ctx.close()


def test_worked_example_wrapper_offsets():
    # Sec. 3.5 wrapper: superblock starting at thread 1024 reads input from
    # 1023 and writes output from 1024
    ctx = dry()
    n = 4096
    x = ctx.array([n]); y = ctx.array([n])
    lid = ctx.launch("stencil1d_f32", [n], [1], [1024], args=[n, y, x],
                     kernel_annotation="global i => read x[i-1:i+1], write y[i]")
    t = ctx.tasks(lid)[1]
    regs = {r.arg: r for r in ctx.regions(t.id)}
    assert regs[2].lo[0] == 1023 and regs[1].lo[0] == 1024
    assert regs[2].hi[0] == 2049 and regs[1].hi[0] == 2048
    ctx.close()


# ----------------------------------------------------- superblocks (T3)

@pytest.mark.parametrize("grid,block,sb", [([1000000], [16], [64000]), ([100], [16], [32]),
                                           ([7, 9], [2, 3], [4, 3]), ([33, 17], [4, 4], [0, 8])])
def test_superblocks_partition_grid(grid, block, sb):
    ctx = dry()
    nd = len(grid)
    if nd == 1:
        x = ctx.array(grid); y = ctx.array(grid)
        lid = ctx.launch("stencil1d_f32", grid, block, sb, args=[grid[0], y, x])
    else:
        x = ctx.array(grid); y = ctx.array(grid)
        lid = ctx.launch("jacobi2d_f32", grid, block, sb, args=[grid[0], grid[1], y, x])
    got = [(tuple(t.sb_lo[:nd]), tuple(t.sb_hi[:nd])) for t in ctx.tasks(lid)]
    assert got == P.superblocks(grid, block, sb)
    ctx.close()


@pytest.mark.parametrize("grid,sb", [((1000, 700), (100, 100)), ((64, 64), (8, 16)), ((30, 500), (10, 100)),
                                     ((7, 9), (1, 1))])
@pytest.mark.parametrize("order,band", [(0, 0), (1, 0), (2, 0), (2, 1), (2, 3), (2, 4), (2, 50)])
def test_superblock_issue_orders(grid, sb, order, band):
    # every order issues each superblock of the row-major partition once;
    # serpentine reverses odd rows; bands visit h rows column by column, the
    # rows of a column consecutively, snaking, odd bands right to left
    ctx = dry(sb_order=order, sb_band=band)
    x = ctx.array(list(grid)); y = ctx.array(list(grid))
    lid = ctx.launch("jacobi2d_f32", list(grid), [1, 1], list(sb), args=[grid[0], grid[1], y, x])
    got = [(tuple(t.sb_lo[:2]), tuple(t.sb_hi[:2])) for t in ctx.tasks(lid)]
    ctx.close()
    want = P.superblocks(list(grid), [1, 1], list(sb))
    assert sorted(got) == sorted(want) and len(got) == len(want)
    rows = -(-grid[0] // sb[0])
    cols = -(-grid[1] // sb[1])
    ij = [(lo[0] // sb[0], lo[1] // sb[1]) for lo, _ in got]
    if order == 0:
        assert ij == [(i, j) for i in range(rows) for j in range(cols)]
    elif order == 1:
        assert ij == [(i, j if i % 2 == 0 else cols - 1 - j) for i in range(rows) for j in range(cols)]
    else:
        h = band if band > 0 else 2
        k = 0
        for bnd, r0 in enumerate(range(0, rows, h)):
            hb = min(h, rows - r0)
            last_row = None
            col_seq = range(cols) if bnd % 2 == 0 else range(cols - 1, -1, -1)
            for c in col_seq:
                col = ij[k:k + hb]
                k += hb
                assert all(j == c for _, j in col)
                assert sorted(i for i, _ in col) == list(range(r0, r0 + hb))
                if last_row is not None:
                    assert col[0][0] == last_row        # the snake turns on the row it ended on
                last_row = col[-1][0]
        assert k == len(ij)


@pytest.mark.parametrize("shape", [[0], [64, 0], [0, 64], [4, 4, 0]])
def test_zero_extent_arrays_are_rejected(shape):
    # an array has at least one element along every axis; an empty launch grid
    # is the way to express no work
    ctx = dry()
    with pytest.raises(L.LtError, match="must be > 0"):
        ctx.array(shape)
    ctx.close()


def test_unknown_config_keys_are_rejected():
    with pytest.raises(TypeError, match="sb_bnd"):
        dry(sb_bnd=2)
    ctx = dry()
    with pytest.raises(TypeError, match="evict_polcy"):
        ctx.configure(evict_polcy=1)
    ctx.close()


def test_superblock_order_validation():
    with pytest.raises(L.LtError):
        dry(sb_order=3)
    with pytest.raises(L.LtError):
        dry(sb_order=2, sb_band=-1)
    ctx = dry()
    with pytest.raises(L.LtError):
        ctx.configure(sb_order=-1)
    ctx.configure(sb_order=L.LT_ORDER_BANDS, sb_band=4)
    ctx.close()


# ------------------------------------------------------------- DAG (T4)

def _launch_seq(ctx, rng, n, arrays, steps, hist=None, first=()):
    """Random stencil/touch launches on tiny arrays, and with ``hist`` =
    (h, values, h2) also histogram reductions into the shared target h,
    read-modify-writes of h, and plain reads of h (a histogram of h's bins
    into h2).  ``first`` fixes the kinds of the first launches.  Returns the oracle task list in program order
    (each launch expanded as the planner lays it out, reductions folded by a
    task of their own) and the planner's task ids in the same order."""
    tasks, ids = [], []
    annots = ["global i => read x[i-1:i+1], write y[i]", "global i => read x[i], write y[i]",
              "global i => read x[:], write y[i]", "global i => read x[i+2:i+3], write y[i]"]
    modes = {0: "read", 1: "write", 2: "readwrite", 3: "reduce"}
    ops = {0: "+", 1: "*", 2: "min", 3: "max"}

    def record(lid, arr_of):
        sbs, sb_ids, tail = [], [], []
        for t in ctx.tasks(lid):
            acc = [(arr_of(r).id, modes[r.mode], ops[r.op] if r.mode == 3 else None, _box(r, 1))
                   for r in ctx.regions(t.id)]
            if t.kind == L.LT_TASK_COMBINE:
                tail.append(t.id)
            else:
                sbs.append(acc)
                sb_ids.append(t.id)
        expanded = P.launch_tasks(lid, sbs)
        assert len(expanded) == len(sb_ids) + len(tail)
        tasks.extend(expanded)
        ids.extend(sb_ids + tail)

    nkinds = 6 if hist is not None else 3
    for step in range(steps):
        kind = first[step] if step < len(first) else rng.integers(nkinds)
        sb = int(rng.choice([4, 8, 12]))
        if kind < 2:
            a, b = rng.choice(len(arrays), 2, replace=False)
            annot = annots[rng.integers(len(annots))]
            lid = ctx.launch("stencil1d_f32", [n], [4], [sb], args=[n, arrays[b], arrays[a]],
                             kernel_annotation=annot)
            record(lid, lambda r, a=a, b=b: arrays[a] if r.arg == 2 else arrays[b])
        elif kind == 2:
            a = rng.integers(len(arrays))
            lid = ctx.launch("stencil1d_f32", [n], [4], [sb], args=[n, arrays[a], arrays[a]],
                             kernel_annotation="global i => readwrite y[i], read x[i]")
            record(lid, lambda r, a=a: arrays[a])
        elif kind == 3:
            h, vals, _ = hist
            v = vals[rng.integers(len(vals))]
            lid = ctx.launch("hist256_i32", [n], [4], [sb], args=[n, h, v])
            record(lid, lambda r, h=h, v=v: h if r.arg == 1 else v)
        elif kind == 4:
            h, _, _ = hist
            lid = ctx.launch("touch_i32", [256], [4], [int(rng.choice([64, 256]))], args=[256, h])
            record(lid, lambda r, h=h: h)
        else:
            # a plain read of h: its bins are the values of another histogram
            h, _, h2 = hist
            lid = ctx.launch("hist256_i32", [256], [4], [int(rng.choice([64, 256]))], args=[256, h2, h])
            record(lid, lambda r, h=h, h2=h2: h2 if r.arg == 1 else h)
    return tasks, ids


def _closure_contains_required(ctx, tasks, ids):
    pos = {tid: k for k, tid in enumerate(ids)}
    preds = {k: set() for k in range(len(ids))}
    for k, tid in enumerate(ids):
        for d in ctx.deps(tid):
            if d in pos:
                assert pos[d] < k  # edges point backwards: acyclic
                preds[k].add(pos[d])
    reach = {}
    for k in range(len(ids)):
        r = set(preds[k])
        for p in preds[k]:
            r |= reach[p]
        reach[k] = r
    for p, q in P.required_orderings(tasks):
        assert p in reach[q], (p, q)


@pytest.mark.parametrize("halo", [None, 1, 3])
@pytest.mark.parametrize("seed", range(6))
def test_dag_contains_every_required_ordering(seed, halo):
    rng = np.random.default_rng(seed)
    ctx = dry()
    n = 40
    arrays = [ctx.array([n], chunk=[int(rng.choice([5, 8, 40]))], halo=None if halo is None else [halo])
              for _ in range(3)]
    tasks, ids = _launch_seq(ctx, rng, n, arrays, 6)
    _closure_contains_required(ctx, tasks, ids)
    ctx.close()


@pytest.mark.parametrize("seed", range(8))
def test_dag_orders_reductions_into_one_target(seed):
    # histogram launches into one target h, mixed with read-modify-writes of
    # h and stencil launches: a later fold must follow every earlier fold,
    # read and write of h (the target is overwritten per launch)
    rng = np.random.default_rng(100 + seed)
    ctx = dry()
    n = 40
    arrays = [ctx.array([n], chunk=[int(rng.choice([5, 8, 40]))]) for _ in range(3)]
    h = ctx.array([256], np.int32, chunk=[int(rng.choice([64, 256]))])
    vals = [ctx.array([n], np.int32, chunk=[int(rng.choice([8, 40]))]) for _ in range(2)]
    h2 = ctx.array([256], np.int32)
    # fold, read of h, read-modify-write, fold again; then random launches
    tasks, ids = _launch_seq(ctx, rng, n, arrays, 12, hist=(h, vals, h2), first=(3, 5, 3, 4, 3))
    assert any(len(t["accesses"]) and t["accesses"][-1][0] == h.id and t["accesses"][-1][1] == "write"
               for t in tasks)
    _closure_contains_required(ctx, tasks, ids)
    ctx.close()


# -------------------------------------------------------- memory (T5)

def test_budget_is_respected_and_spill_traffic_accounted():
    chunk = 1 << 16  # 256 KiB chunks
    n = 16 * chunk
    ctx = dry(device_budget_bytes=6 * chunk * 4, trace=1, stage_threshold_bytes=1 << 40)
    x = ctx.array([n], chunk=[chunk]); y = ctx.array([n], chunk=[chunk])
    for it in range(3):
        ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
        x, y = y, x
    ctx.sync()
    tr = ctx.trace()
    cap = 6 * chunk * 4
    assert max(r.resident for r in tr) <= cap
    s = ctx.stats()
    assert s["peak_resident_bytes"] <= cap
    assert s["evictions_dirty"] > 0 and s["bytes_d2h"] > 0
    ctx.close()


def test_task_larger_than_budget_rejected():
    ctx = dry(device_budget_bytes=1 << 20)
    n = 1 << 20
    x = ctx.array([n]); y = ctx.array([n])
    with pytest.raises(L.LtError) as e:
        ctx.launch("stencil1d_f32", [n], [256], [0], args=[n, y, x])
    assert e.value.status == L.LT_ERR_BUDGET
    ctx.close()


def test_full_overwrite_skips_load():
    # a write-only access that covers a whole spilled chunk does not reload it
    chunk = 1 << 14
    n = 8 * chunk
    ctx = dry(device_budget_bytes=4 * chunk * 4, trace=1)
    x = ctx.array([n], chunk=[chunk]); y = ctx.array([n], chunk=[chunk])
    ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
    ctx.sync()
    h2d_chunks = {r.chunk for r in ctx.trace() if r.kind == 1}
    # x chunks were never written (undefined) and y chunks are fully
    # overwritten: nothing is loaded
    assert not h2d_chunks
    ctx.close()


# ------------------------------------------------------- errors (T9)

def test_errors_are_reported():
    ctx = dry()
    n = 64
    x = ctx.array([n]); y = ctx.array([n]); h = ctx.array([256], np.int32)
    bad = [
        (dict(annotation="global i => read x[i*i], write y[i]"), L.LT_ERR_PARSE),
        (dict(annotation="global i => read x[q], write y[i]"), L.LT_ERR_PARSE),
        (dict(annotation="global i => reduce(-) y[i], read x[i]"), L.LT_ERR_PARSE),
        (dict(annotation="global i => read x[i]"), L.LT_ERR_PARSE),
        (dict(annotation="global [i, j] => read x[i], write y[j]"), L.LT_ERR_PARSE),
    ]
    for kw, code in bad:
        with pytest.raises(L.LtError) as e:
            ctx.launch("stencil1d_f32", [n], [4], [8], args=[n, y, x], **kw)
        assert e.value.status == code, kw
    with pytest.raises(L.LtError) as e:
        ctx.launch("stencil1d_f32", [n], [4], [6], args=[n, y, x])  # not a multiple
    assert e.value.status == L.LT_ERR_INVALID
    with pytest.raises(L.LtError) as e:
        ctx.launch("stencil1d_f32", [n], [4], [8], args=[n, h, x])  # dtype
    assert e.value.status == L.LT_ERR_INVALID
    with pytest.raises(L.LtError) as e:
        ctx.launch("stencil1d_f32", [n], [4], [8], args=[n, y])  # arity
    assert e.value.status == L.LT_ERR_INVALID
    with pytest.raises(L.LtError):
        ctx.kernel("no_such_kernel")
    y.destroy()
    with pytest.raises(L.LtError):
        ctx.launch("stencil1d_f32", [n], [4], [8], args=[n, x, x])  # fine: in place
        ctx.launch("stencil1d_f32", [n], [4], [8], args=[n, L.Array(ctx, None, np.float32, (n,)), x])
    ctx.close()


def test_custom_distribution_validation():
    ctx = dry()
    with pytest.raises(L.LtError):
        ctx.array([10], boxes=[((0,), (6,)), ((5,), (10,))])  # overlap
    with pytest.raises(L.LtError):
        ctx.array([10], boxes=[((0,), (4,)), ((5,), (10,))])  # gap
    a = ctx.array([10], boxes=[((4,), (10,)), ((0,), (4,))])
    assert a.id > 0
    ctx.close()


# ------------------------------------------------- halo distributions (f2)

def _jacobi_sweeps(ctx, n, m, chunk, halo, sweeps, sb):
    a = ctx.array([n, m], chunk=chunk, halo=halo)
    b = ctx.array([n, m], chunk=chunk, halo=halo)
    a.fill(1.0)
    b.fill(0.0)
    inp, out = a, b
    for _ in range(sweeps):
        ctx.launch("jacobi2d_f32", [n, m], [1, 64], sb, args=[n, m, out, inp])
        inp, out = out, inp
    ctx.sync()


def test_halo_reads_are_served_by_one_chunk():
    n, m = 256, 512
    ctx = dry()
    _jacobi_sweeps(ctx, n, m, [64, 128], [1, 1], 4, [64, 128])
    s = ctx.stats()
    # every tile's halo read fits the tile's stored box: no assembled copies
    assert s["assembled_regions"] == 0
    # after the first sweep each written tile's neighbours refresh their replicas:
    # 16 tiles, 3 sweeps that read freshly written data, one piece per neighbour
    # (4 edge + 4 corner neighbours for interior tiles)
    nb = 0
    for i in range(4):
        for j in range(4):
            nb += sum(1 for di in (-1, 0, 1) for dj in (-1, 0, 1)
                      if (di or dj) and 0 <= i + di < 4 and 0 <= j + dj < 4)
    assert s["halo_copies"] == 3 * nb
    ctx.close()
    # the same tiles without a halo assemble every read from up to 9 chunks
    ctx = dry()
    _jacobi_sweeps(ctx, n, m, [64, 128], None, 4, [64, 128])
    s = ctx.stats()
    assert s["assembled_regions"] == 4 * 16 and s["halo_copies"] == 0
    ctx.close()


def test_halo_refreshes_are_batched_per_launch():
    # grouped executor: one refresh dispatch and one kernel dispatch per sweep
    n, m = 256, 512
    ctx = dry(exec_mode=1)
    a = ctx.array([n, m], chunk=[64, 128], halo=[1, 1])
    b = ctx.array([n, m], chunk=[64, 128], halo=[1, 1])
    a.fill(1.0)
    b.fill(0.0)
    ctx.reset_stats()
    inp, out = a, b
    for _ in range(4):
        ctx.launch("jacobi2d_f32", [n, m], [1, 64], [64, 128], args=[n, m, out, inp])
        inp, out = out, inp
    ctx.sync()
    s = ctx.stats()
    assert s["dispatches"] == 4 + 3 and s["bytes_d2d"] == 0 and s["assembled_regions"] == 0
    ctx.close()


@pytest.mark.parametrize("M,N,K,sb,ndisp", [
    (300, 260, 77, (128, 100), 2),   # 9 tasks, 8 per GEMM dispatch
    (520, 530, 96, (256, 256), 2),
    (1100, 300, 64, (256, 300), 1),
])
def test_gemm_groups_superblocks_without_edges(M, N, K, sb, ndisp):
    # grouped executor: superblocks with no edges among them share dispatches
    # of up to 8 tasks; with C in one chunk, every task writes that chunk, so
    # each depends on the one before and gets a dispatch of its own
    for chunk_c, want in ((list(sb), ndisp), ([0, 0], 9 if ndisp == 2 else 5)):
        ctx = dry(exec_mode=1)
        a = ctx.array([M, K])
        b = ctx.array([K, N])
        c = ctx.array([M, N], chunk=chunk_c)
        a.fill(0.0)
        b.fill(0.0)
        c.fill(0.0)
        ctx.reset_stats()
        ctx.launch("gemm_f32", [M, N], [1, 1], list(sb), args=[M, N, K, c, a, b])
        ctx.sync()
        assert ctx.stats()["dispatches"] == want, (chunk_c, ctx.stats())
        ctx.close()


def test_halo_stores_cores_with_replicas():
    ctx = dry()
    x = ctx.array([100], chunk=[30], halo=[2])
    y = ctx.array([100], chunk=[30], halo=[2])
    x.fill(0.0)
    lid = ctx.launch("stencil1d_f32", [100], [1], [30], args=[100, y, x])
    for t in ctx.tasks(lid):
        for r in ctx.regions(t.id):
            assert r.resolved == 0  # direct views
    ctx.sync()
    ctx.close()


def test_halo_distribution_validation():
    ctx = dry()
    with pytest.raises(L.LtError) as e:
        ctx.array([100], chunk=[30], halo=[-1])
    assert e.value.status == L.LT_ERR_INVALID
    ctx.close()


# --------------------------------------------------------- disk tier (f4)

def test_disk_tier_keeps_spill_memory_under_the_host_budget():
    chunk = 1 << 14
    n = 16 * chunk
    hb = 3 * chunk * 4
    ctx = dry(device_budget_bytes=4 * chunk * 4, host_budget_bytes=hb, trace=1, stage_threshold_bytes=1 << 40)
    x = ctx.array([n], chunk=[chunk])
    y = ctx.array([n], chunk=[chunk])
    x.fill(1.0)
    y.fill(0.0)
    for _ in range(4):
        ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
        x, y = y, x
    ctx.sync()
    s = ctx.stats()
    assert s["host_spill_bytes"] <= hb
    assert s["bytes_disk_write"] > 0 and s["bytes_disk_read"] > 0
    tr = ctx.trace()
    writes = sum(r.bytes for r in tr if r.kind == 8)
    reads = sum(r.bytes for r in tr if r.kind == 9)
    assert writes == s["bytes_disk_write"] and reads == s["bytes_disk_read"]
    # a chunk only comes back from disk after it went there
    assert reads <= writes
    ctx.close()


def test_disk_tier_off_without_host_budget():
    chunk = 1 << 14
    n = 16 * chunk
    ctx = dry(device_budget_bytes=4 * chunk * 4, stage_threshold_bytes=1 << 40)
    x = ctx.array([n], chunk=[chunk])
    y = ctx.array([n], chunk=[chunk])
    x.fill(1.0)
    for _ in range(3):
        ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
        x, y = y, x
    ctx.sync()
    s = ctx.stats()
    assert s["bytes_disk_write"] == 0 and s["host_spill_bytes"] > 0
    ctx.close()


def test_host_budget_smaller_than_a_chunk_is_an_error():
    chunk = 1 << 14
    n = 8 * chunk
    ctx = dry(device_budget_bytes=3 * chunk * 4, host_budget_bytes=chunk, stage_threshold_bytes=1 << 40)
    x = ctx.array([n], chunk=[chunk])
    y = ctx.array([n], chunk=[chunk])
    with pytest.raises(L.LtError) as e:
        x.fill(1.0)  # spilling the filled chunks already needs a spill buffer
        for _ in range(3):
            ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
            x, y = y, x
        ctx.sync()
    assert e.value.status == L.LT_ERR_BUDGET


# ------------------------------------------------------------ eviction policy

def _ooc_gemm_h2d(policy):
    # the out-of-core GEMM pattern at small scale: 8 x 8 C tiles, A row panels
    # and B column panels of 8 tiles, a budget of 12 panels for 24 panels' data
    n, T = 4096, 512
    tile = T * T * 4
    ctx = dry(device_budget_bytes=12 * 8 * tile, stage_threshold_bytes=1 << 40,
              sb_order=L.LT_ORDER_SERPENTINE, evict_policy=policy, trace=1)
    a = ctx.array([n, n], chunk=[T, 0])
    b = ctx.array([n, n], chunk=[0, T])
    c = ctx.array([n, n], chunk=[T, T])
    a.fill(1.0)
    b.fill(1.0)
    ctx.sync()
    ctx.reset_stats()
    ctx.clear_trace()
    ctx.launch("gemm_f32", [n, n], [1, 1], [T, T], args=[n, n, n, c, a, b])
    ctx.sync()
    s = ctx.stats()
    ctx.close()
    return s["bytes_h2d"], s["evictions_clean"] + s["evictions_dirty"]


def test_next_use_eviction_moves_no_more_than_lru():
    nu, nu_ev = _ooc_gemm_h2d(L.LT_EVICT_NEXT_USE)
    lru, lru_ev = _ooc_gemm_h2d(L.LT_EVICT_LRU)
    assert nu_ev > 0 and lru_ev > 0  # the budget binds under both
    assert nu <= lru, (nu, lru)


def test_banded_order_reuses_panels():
    # out-of-core GEMM with host-home operands, 16 x 16 C tiles and a device
    # budget smaller than B: bands of h superblock rows use each B panel for h
    # tiles in a row, so the product loads fewer panels than in serpentine
    # order (at a budget of 16 panels these are the ratios of the 65536^3
    # product with 16 GiB: 77, 67, 51 panels of which 32 are compulsory)
    n, T = 4096, 256
    panel = (n // T) * T * T * 4
    A = np.zeros((n, n), np.float32)
    B = np.zeros((n, n), np.float32)
    Cm = np.zeros((n, n), np.float32)

    def h2d(budget, order, band):
        ctx = dry(device_budget_bytes=budget * panel, stage_threshold_bytes=1 << 40, sb_order=order, sb_band=band)
        a = ctx.array_host(A, chunk=[T, 0])
        b = ctx.array_host(B, chunk=[0, T])
        c = ctx.array_host(Cm, chunk=[T, T])
        ctx.launch("gemm_f32", [n, n], [1, 1], [T, T], args=[n, n, n, c, a, b])
        ctx.sync()
        s = ctx.stats()
        ctx.close()
        assert s["bytes_d2h"] == n * n * 4          # C written back once
        return s["bytes_h2d"] / panel

    for budget in (10, 16):
        serp = h2d(budget, L.LT_ORDER_SERPENTINE, 0)
        b2 = h2d(budget, L.LT_ORDER_BANDS, 2)
        b4 = h2d(budget, L.LT_ORDER_BANDS, 4)
        assert 32 <= b4 < b2 < serp, (budget, serp, b2, b4)
    assert b4 <= 0.7 * serp


def test_evict_policy_validated():
    with pytest.raises(L.LtError):
        dry(evict_policy=7)
    ctx = dry()
    with pytest.raises(L.LtError):
        ctx.configure(evict_policy=-1)
    ctx.configure(evict_policy=L.LT_EVICT_LRU)
    ctx.close()


def test_scattered_runs_move_on_device_instead_of_reloading():
    # out-of-core Jacobi with a budget of 8 row slabs: each task reads a run of
    # three neighbouring slabs, which must sit contiguously.  Runs whose
    # members are resident but scattered move device-to-device, so each sweep
    # loads every input slab about once from the host
    n, rows, sweeps = 2048, 128, 6
    slab = rows * n * 4
    ctx = dry(device_budget_bytes=8 * slab, stage_threshold_bytes=4 * slab)
    a = ctx.array([n, n], chunk=[rows, 0])
    b = ctx.array([n, n], chunk=[rows, 0])
    a.fill(1.0)
    b.fill(0.0)
    ctx.sync()
    ctx.reset_stats()
    inp, out = a, b
    for _ in range(sweeps):
        ctx.launch("jacobi2d_f32", [n, n], [1, 256], [rows, 0], args=[n, n, out, inp])
        inp, out = out, inp
    ctx.sync()
    s = ctx.stats()
    ctx.close()
    field = n * n * 4
    assert s["bytes_d2d"] > 0
    assert s["bytes_h2d"] <= 1.15 * sweeps * field, s["bytes_h2d"] / (sweeps * field)
    assert s["bytes_d2h"] <= 1.15 * sweeps * field


def test_pinned_pool_recycles_spill_buffers_within_the_host_budget():
    # repeated demotion and reload cycles through the disk tier reuse pooled
    # pinned buffers; held spill memory never exceeds the host budget
    chunk = 1 << 14
    n = 16 * chunk
    hb = 4 * chunk * 4
    ctx = dry(device_budget_bytes=4 * chunk * 4, host_budget_bytes=hb, stage_threshold_bytes=1 << 40)
    x = ctx.array([n], chunk=[chunk])
    y = ctx.array([n], chunk=[chunk])
    x.fill(1.0)
    y.fill(0.0)
    peak = 0
    for _ in range(6):
        ctx.launch("stencil1d_f32", [n], [256], [chunk], args=[n, y, x])
        x, y = y, x
        peak = max(peak, ctx.stats()["host_spill_bytes"])
    ctx.sync()
    s = ctx.stats()
    ctx.close()
    assert peak <= hb and s["host_spill_bytes"] <= hb
    assert s["bytes_disk_write"] > 0 and s["bytes_disk_read"] > 0


@pytest.mark.parametrize("chunk,halo", [([64, 0], [1, 0]), ([64, 128], [1, 1])])
def test_batched_halo_pingpong_refreshes_like_the_plain_path(chunk, halo):
    # a sweep reads replicas whose owners the previous sweep, queued in the
    # same open batch, writes: the batch is issued first, so every replica is
    # refreshed exactly as on the plain path
    n, m = 256, 512

    def run(batched):
        ctx = dry()
        a = ctx.array([n, m], chunk=chunk, halo=halo)
        b = ctx.array([n, m], chunk=chunk, halo=halo)
        a.fill(1.0)
        b.fill(0.0)
        ctx.sync()
        ctx.reset_stats()
        if batched:
            ctx.batch_begin()
        inp, out = a, b
        for _ in range(4):
            ctx.launch("jacobi2d_f32", [n, m], [1, 64], chunk[:1] + [chunk[1] or m], args=[n, m, out, inp])
            inp, out = out, inp
        if batched:
            ctx.batch_end()
        ctx.sync()
        s = ctx.stats()
        ctx.close()
        return s

    plain, batched = run(False), run(True)
    assert plain["halo_copies"] > 0
    if chunk[1] == 0:
        assert plain["halo_copies"] == 18  # 3 sweeps x 6 row pieces of 4 slabs
    assert batched["halo_copies"] == plain["halo_copies"]
    assert batched["assembled_regions"] == 0


def test_graph_refuses_halo_replica_reads():
    ctx = dry()
    a = ctx.array([256, 512], chunk=[64, 0], halo=[1, 0])
    b = ctx.array([256, 512], chunk=[64, 0], halo=[1, 0])
    a.fill(1.0)
    ctx.graph_begin()
    with pytest.raises(L.LtError, match="halo replicas") as e:
        ctx.launch("jacobi2d_f32", [256, 512], [1, 64], [64, 512], args=[256, 512, b, a])
    assert e.value.status == L.LT_ERR_UNSUPPORTED
    ctx.close()


def test_batch_queue_never_evicts_a_queued_chunk():
    # four resident 4 MiB arrays fill the budget exactly; a batch of two
    # stencil launches over them needs room for its queue.  The chunks the
    # queued tasks address are pinned, so nothing is evicted and the batch
    # fails cleanly with LT_ERR_BUDGET (reported again, sticky, at lt_sync).
    n = 1 << 20
    ctx = dry(device_budget_bytes=4 * n * 4)
    xs = [ctx.array([n], chunk=[1 << 18]) for _ in range(4)]
    for x in xs:
        x.fill(0.5)
    ctx.sync()
    ctx.reset_stats()
    ctx.batch_begin()
    ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[1], xs[0]])
    ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[3], xs[2]])
    with pytest.raises(L.LtError) as e:
        ctx.batch_end()
    assert e.value.status == L.LT_ERR_BUDGET
    s = ctx.stats()
    assert s["evictions_dirty"] == 0 and s["evictions_clean"] == 0
    with pytest.raises(L.LtError) as e:
        ctx.sync()
    assert e.value.status == L.LT_ERR_BUDGET
    # with one spare megabyte the same batch is issued
    ctx.close()
    ctx = dry(device_budget_bytes=4 * n * 4 + (1 << 20))
    xs = [ctx.array([n], chunk=[1 << 18]) for _ in range(4)]
    for x in xs:
        x.fill(0.5)
    ctx.batch_begin()
    ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[1], xs[0]])
    ctx.launch("stencil1d_f32", [n], [256], [1 << 18], args=[n, xs[3], xs[2]])
    ctx.batch_end()
    ctx.sync()
    s = ctx.stats()
    assert s["evictions_dirty"] == 0 and s["evictions_clean"] == 0
    ctx.close()
