"""Pins of the brute-force planner oracle (oracle/planner.py).

The annotation reader is pinned to the strings the paper prints (Sec. 2.3,
Sec. 3.6) and the region enumerator to the worked offsets of the generated
wrapper (Sec. 3.5) and hand-derived boxes (tests/golden/regions.json).
"""
import json
import os

import pytest

from oracle import planner as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _expr_text(node):
    if node is None:
        return None
    k = node[0]
    if k == "num":
        return str(node[1])
    if k == "var":
        return node[1]
    if k == "neg":
        return "-" + _expr_text(node[1])
    return _expr_text(node[1]) + k + _expr_text(node[2])


@pytest.mark.parametrize("case", _load("annotations.json")["cases"],
                         ids=lambda c: c["cite"])
def test_paper_annotations_parse(case):
    bindings, accesses = P.parse(case["text"])
    assert [[k, n] for k, n in bindings] == case["bindings"]
    got = []
    for a in accesses:
        idx = []
        for ix in a["index"]:
            if ix[0] == "point":
                t = _expr_text(ix[1])
                idx.append(["point", t, t])
            else:
                idx.append(["slice", _expr_text(ix[1]), _expr_text(ix[2])])
        got.append([a["mode"], a["op"], a["array"], idx])
    assert got == case["expect"]


@pytest.mark.parametrize("case", _load("annotations.json")["reject"],
                         ids=lambda c: c["text"])
def test_invalid_annotations_rejected(case):
    # the oracle evaluates lazily: a non-linear index parses but the product
    # rejects it; the oracle must at least fail to evaluate unknown names and
    # bad modes.  Non-linearity is checked by evaluating on two thread sets.
    text = case["text"]
    try:
        b, acc = P.parse(text)
    except P.AnnotError:
        return
    # parsed: must be non-linear (i*i) or use an unbound name
    with pytest.raises((P.AnnotError, AssertionError)):
        r1 = P.region(text, acc[0]["array"], [64], [0], [4], [1])
        r2 = P.region(text, acc[0]["array"], [64], [4], [8], [1])
        # linear accesses shift by the same amount as the superblock
        assert r2[0][0] - r1[0][0] == 4 and r2[0][1] - r1[0][1] == 4


@pytest.mark.parametrize("case", _load("regions.json")["cases"],
                         ids=lambda c: c["cite"])
def test_worked_regions(case):
    for arr, shape in case["arrays"].items():
        got = P.region(case["text"], arr, shape, case["sb_lo"], case["sb_hi"],
                       case["block"])
        exp = case["expect"][arr]
        assert (None if got is None else [list(x) for x in got]) == exp


def test_region_covers_all_accessed_elements():
    text = "global [i, j] => read A[i-1:i+1, j-2:j], write B[i, j]"
    shape = [9, 11]
    for sb in P.superblocks([9, 11], [3, 4], [3, 4]):
        box = P.region(text, "A", shape, sb[0], sb[1], [3, 4])
        pts = P.accessed_elements(text, "A", shape, sb[0], sb[1], [3, 4])
        for p in pts:
            assert all(box[a][0] <= p[a] <= box[a][1] for a in range(2))
        # tight: each face of the box is touched
        for a in range(2):
            assert min(p[a] for p in pts) == box[a][0]
            assert max(p[a] for p in pts) == box[a][1]


@pytest.mark.parametrize("grid,block,sb", [
    ([100], [16], [32]), ([7, 9], [2, 3], [4, 3]), ([5, 4, 3], [1, 2, 3], [2, 2, 3]),
    ([1000000], [16], [64000]),
])
def test_superblocks_cover_each_thread_exactly_once(grid, block, sb):
    sbs = P.superblocks(grid, block, sb)
    rounded = [-(-g // b) * b for g, b in zip(grid, block)]
    total = 1
    for r in rounded:
        total *= r
    vol = 0
    for lo, hi in sbs:
        v = 1
        for a in range(len(grid)):
            assert lo[a] % block[a] == 0
            v *= hi[a] - lo[a]
        vol += v
    assert vol == total
    if total <= 10000:
        seen = {}
        for lo, hi in sbs:
            for t in P.superblock_threads(lo, hi):
                seen[t] = seen.get(t, 0) + 1
        assert len(seen) == total and set(seen.values()) == {1}


def test_conflict_table():
    assert not P.conflicting("read", None, "read", None)
    assert P.conflicting("read", None, "write", None)
    assert P.conflicting("write", None, "read", None)
    assert P.conflicting("write", None, "write", None)
    assert P.conflicting("readwrite", None, "read", None)
    # same-operator reductions commute inside one launch only: a later
    # launch's fold overwrites the target
    assert not P.conflicting("reduce", "+", "reduce", "+", same_launch=True)
    assert P.conflicting("reduce", "+", "reduce", "+")
    assert P.conflicting("reduce", "+", "reduce", "+", same_launch=False)
    assert P.conflicting("reduce", "+", "reduce", "max", same_launch=True)
    assert P.conflicting("reduce", "+", "read", None)


def test_required_orderings_stencil_pingpong():
    # two launches of the Sec. 3.6 stencil (input/output swapped), two
    # superblocks each: launch-2 task k must follow launch-1 tasks touching
    # its halo (write-read) and the ones that read what it overwrites.
    n = 8
    t = "global i => read x[i-1:i+1], write y[i]"
    tasks = []
    for (src, dst) in (("a", "b"), ("b", "a")):
        for lo, hi in P.superblocks([n], [1], [4]):
            rx = P.region(t, "x", [n], lo, hi, [1])
            ry = P.region(t, "y", [n], lo, hi, [1])
            tasks.append({"accesses": [(src, "read", None, rx), (dst, "write", None, ry)]})
    req = P.required_orderings(tasks)
    assert set(req) == {(0, 2), (1, 2), (0, 3), (1, 3)}


def test_required_orderings_two_reductions_into_one_target():
    # two histogram launches into one h (two superblocks each), with a read
    # of h between them: under the overwrite reading the second launch's fold
    # must follow the first one's and the read, and the read must follow the
    # first fold; superblocks of one launch stay unordered
    n = 8
    t = "global i => read v[i], reduce(+) h[:]"
    shape_h = [256]
    tasks = []
    for L, src in ((1, "v1"), (3, "v2")):
        sbs = []
        for lo, hi in P.superblocks([n], [1], [4]):
            rv = P.region(t, "v", [n], lo, hi, [1])
            rh = P.region(t, "h", shape_h, lo, hi, [1])
            sbs.append([(src, "read", None, rv), ("h", "reduce", "+", rh)])
        tasks += P.launch_tasks(L, sbs)
        if L == 1:
            tasks.append({"launch": 2, "accesses": [("h", "read", None, ((0, 255),))]})
    # tasks: 0, 1 = launch 1 superblocks; 2 = its fold; 3 = the read;
    # 4, 5 = launch 3 superblocks; 6 = its fold
    req = set(P.required_orderings(tasks))
    assert {(0, 2), (1, 2), (2, 3), (2, 6), (3, 6), (4, 6), (5, 6)} <= req
    assert (0, 1) not in req and (4, 5) not in req
    # the superblocks of launch 3 write private partials: nothing orders them
    # after launch 1 or the read
    assert not any(q in (4, 5) for _, q in req)
    # flat (unexpanded) superblock accesses from different launches conflict
    flat = [{"launch": 1, "accesses": [("h", "reduce", "+", ((0, 255),))]},
            {"launch": 2, "accesses": [("h", "reduce", "+", ((0, 255),))]},
            {"launch": 2, "accesses": [("h", "reduce", "+", ((0, 255),))]}]
    assert set(P.required_orderings(flat)) == {(0, 1), (0, 2)}
