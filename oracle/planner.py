"""Brute-force planner oracle -- TEST INFRASTRUCTURE ONLY.

Checks what the planner derives from a data annotation, by enumerating every
thread of a (tiny) superblock and every element it touches.  Pure Python
loops; meant for grids of at most a few thousand threads.

Semantics (Sec. 2.3 "Data Annotations"):

* Left of ``=>`` the annotation binds variables to the thread's ``global``
  index, its thread-block index (``block``) or its index inside the block
  (``local``).  A bracketed list binds several axes; the list runs from the
  slowest axis to the fastest (``global [i, j]``: i is the row, j the
  column), matching row-major arrays whose last index is contiguous.
* Right of ``=>`` each item names an access mode (``read``, ``write``,
  ``readwrite`` or ``reduce(f)`` with f in ``+ * min max``), an array and one
  index per array axis.  An index is an expression, or a slice ``lo:hi``
  that covers lo..hi inclusive (Fortran style); an omitted lo is 0 and an
  omitted hi is the last index of that axis.
* Expressions must be linear in the bound variables; integer literals and
  named integer scalars of the kernel may appear as constants.

The access region of a superblock for one array (Sec. 2.3, Sec. 2.4) is the
dense bounding box of everything its threads touch, clipped here to the
array's domain; an empty clip means the superblock does not touch the array.
"""
from __future__ import annotations

import itertools
import re

_TOKEN = re.compile(r"\s*(=>|[A-Za-z_][A-Za-z_0-9]*|\d+|[\[\](),:+\-*])")


class AnnotError(ValueError):
    pass


def _tokens(s: str):
    pos = 0
    out = []
    s = s.strip()
    while pos < len(s):
        m = _TOKEN.match(s, pos)
        if not m:
            if s[pos:].strip() == "":
                break
            raise AnnotError("bad character at %d: %r" % (pos, s[pos:pos + 8]))
        out.append(m.group(1))
        pos = m.end()
    return out


class _Reader:
    """Reads the annotation into a small tree; expressions stay as token lists
    evaluated later by a recursive evaluator over concrete integers."""

    def __init__(self, text: str):
        self.t = _tokens(text)
        self.k = 0

    def peek(self):
        return self.t[self.k] if self.k < len(self.t) else None

    def take(self, want=None):
        tok = self.peek()
        if tok is None or (want is not None and tok != want):
            raise AnnotError("expected %r, found %r" % (want, tok))
        self.k += 1
        return tok

    def names(self):
        if self.peek() == "[":
            self.take("[")
            out = [self.take()]
            while self.peek() == ",":
                self.take(",")
                out.append(self.take())
            self.take("]")
            return out
        return [self.take()]

    # expression tree: ("num", v) | ("var", name) | (op, a, b) | ("neg", a)
    def expr(self):
        node = self.term()
        while self.peek() in ("+", "-"):
            op = self.take()
            node = (op, node, self.term())
        return node

    def term(self):
        node = self.unary()
        while self.peek() == "*":
            self.take("*")
            node = ("*", node, self.unary())
        return node

    def unary(self):
        if self.peek() == "-":
            self.take("-")
            return ("neg", self.unary())
        if self.peek() == "+":
            self.take("+")
            return self.unary()
        if self.peek() == "(":
            self.take("(")
            e = self.expr()
            self.take(")")
            return e
        tok = self.take()
        if tok.isdigit():
            return ("num", int(tok))
        if re.match(r"[A-Za-z_]", tok):
            return ("var", tok)
        raise AnnotError("unexpected %r" % tok)

    def index(self):
        lo = hi = None
        if self.peek() == ":":
            self.take(":")
            if self.peek() not in (",", "]"):
                hi = self.expr()
            return ("slice", lo, hi)
        lo = self.expr()
        if self.peek() == ":":
            self.take(":")
            if self.peek() not in (",", "]"):
                hi = self.expr()
            return ("slice", lo, hi)
        return ("point", lo)

    def parse(self):
        bindings = []  # (kind, [names])
        while True:
            kind = self.take()
            if kind not in ("global", "block", "local"):
                raise AnnotError("unknown binding %r" % kind)
            bindings.append((kind, self.names()))
            if self.peek() == "=>":
                break
            self.take(",")
        self.take("=>")
        accesses = []
        while True:
            mode = self.take()
            op = None
            if mode == "reduce":
                self.take("(")
                op = self.take()
                if op not in ("+", "*", "min", "max"):
                    raise AnnotError("bad reduction %r" % op)
                self.take(")")
            elif mode not in ("read", "write", "readwrite"):
                raise AnnotError("bad mode %r" % mode)
            name = self.take()
            self.take("[")
            idx = [self.index()]
            while self.peek() == ",":
                self.take(",")
                idx.append(self.index())
            self.take("]")
            accesses.append({"mode": mode, "op": op, "array": name, "index": idx})
            if self.peek() is None:
                break
            self.take(",")
        return bindings, accesses


def parse(text: str):
    """Returns (bindings, accesses) or raises AnnotError."""
    return _Reader(text).parse()


def _eval(node, env):
    kind = node[0]
    if kind == "num":
        return node[1]
    if kind == "var":
        if node[1] not in env:
            raise AnnotError("unknown name %r" % node[1])
        return env[node[1]]
    if kind == "neg":
        return -_eval(node[1], env)
    a, b = _eval(node[1], env), _eval(node[2], env)
    return a + b if kind == "+" else a - b if kind == "-" else a * b


def _thread_env(bindings, t, block):
    env = {}
    nd = len(t)
    for kind, names in bindings:
        if len(names) != nd:
            raise AnnotError("binding arity %d != grid dims %d" % (len(names), nd))
        for ax, nm in enumerate(names):
            if kind == "global":
                env[nm] = t[ax]
            elif kind == "block":
                env[nm] = t[ax] // block[ax]
            else:
                env[nm] = t[ax] % block[ax]
    return env


def thread_access_box(access, env, shape):
    """Per-axis inclusive (lo, hi) of one thread's access, before clipping."""
    box = []
    for ax, ix in enumerate(access["index"]):
        if ix[0] == "point":
            v = _eval(ix[1], env)
            box.append((v, v))
        else:
            lo = 0 if ix[1] is None else _eval(ix[1], env)
            hi = shape[ax] - 1 if ix[2] is None else _eval(ix[2], env)
            box.append((lo, hi))
    return box


def superblock_threads(sb_lo, sb_hi):
    """All thread indices of a superblock given as half-open per-axis bounds."""
    return itertools.product(*[range(a, b) for a, b in zip(sb_lo, sb_hi)])


def region(text, array, shape, sb_lo, sb_hi, block, scalars=None):
    """Inclusive per-axis (lo, hi) access region of ``array`` for a superblock,
    clipped to the domain, or None when the superblock touches nothing.

    Computed as the bounding box of every thread's access box (threads whose
    slice is empty contribute nothing), then clipped to [0, shape-1].
    """
    bindings, accesses = parse(text)
    acc = [a for a in accesses if a["array"] == array]
    if not acc:
        return None
    nd = len(shape)
    lo = [None] * nd
    hi = [None] * nd
    for t in superblock_threads(sb_lo, sb_hi):
        env = dict(scalars or {})
        env.update(_thread_env(bindings, t, block))
        for a in acc:
            if len(a["index"]) != nd:
                raise AnnotError("index arity")
            box = thread_access_box(a, env, shape)
            if any(l > h for l, h in box):
                continue
            for ax, (l, h) in enumerate(box):
                lo[ax] = l if lo[ax] is None else min(lo[ax], l)
                hi[ax] = h if hi[ax] is None else max(hi[ax], h)
    if lo[0] is None:
        return None
    out = []
    for ax in range(nd):
        l, h = max(lo[ax], 0), min(hi[ax], shape[ax] - 1)
        if l > h:
            return None
        out.append((l, h))
    return out


def accessed_elements(text, array, shape, sb_lo, sb_hi, block, scalars=None):
    """Set of in-domain element indices of ``array`` touched by the superblock."""
    bindings, accesses = parse(text)
    acc = [a for a in accesses if a["array"] == array]
    out = set()
    for t in superblock_threads(sb_lo, sb_hi):
        env = dict(scalars or {})
        env.update(_thread_env(bindings, t, block))
        for a in acc:
            box = thread_access_box(a, env, shape)
            rngs = []
            for ax, (l, h) in enumerate(box):
                rngs.append(range(max(l, 0), min(h, shape[ax] - 1) + 1))
            out.update(itertools.product(*rngs))
    return out


def modes_of(text, array):
    """Access modes (with reduction op) the annotation uses for ``array``."""
    _, accesses = parse(text)
    return [(a["mode"], a["op"]) for a in accesses if a["array"] == array]


def superblocks(grid, block, sb):
    """Split a thread grid into superblocks (Sec. 2.1): grids are rounded up to
    whole blocks; superblocks are boxes of ``sb`` threads (a multiple of the
    block) tiling the rounded grid; the last one on each axis may be short.
    Returns a list of (lo, hi) half-open thread boxes in row-major order.
    """
    nd = len(grid)
    axes = []
    for ax in range(nd):
        g = -(-grid[ax] // block[ax]) * block[ax]
        s = sb[ax] if sb[ax] > 0 else g
        axes.append([(a, min(a + s, g)) for a in range(0, g, s)])
    out = []
    for combo in itertools.product(*axes):
        out.append((tuple(c[0] for c in combo), tuple(c[1] for c in combo)))
    return out


def conflicting(mode_a, op_a, mode_b, op_b, same_launch=False):
    """Do two accesses to overlapping elements need an ordering (Sec. 2.4:
    read-write, write-write and write-read conflicts)?  Two reads never do.
    Two reductions with the same operator commute only inside one launch:
    a launch's fold overwrites its target (reduce(f) is write-like, Sec. 2.3,
    and the target is the fold of that launch's contributions alone), so
    reductions from different launches into one element keep program
    order."""
    if mode_a == "read" and mode_b == "read":
        return False
    if mode_a == "reduce" and mode_b == "reduce" and op_a == op_b and same_launch:
        return False
    return True


def launch_tasks(launch, sb_accesses):
    """Tasks of one launch as the planner of Sec. 2.4 lays them out.

    ``sb_accesses`` holds, per superblock in issue order, its accesses
    (array, mode, op, inclusive box).  Each superblock is one task.  A
    reduce access does not touch the target: the superblock writes a private
    temporary ("partial", launch, array, superblock) instead, and one
    reduction task per reduced array, after the superblock tasks, reads all
    of that array's partials and writes the union of their boxes in the
    target (the fold overwrites it).  Returns task dicts for
    ``required_orderings``.
    """
    tasks = []
    reduced = {}
    for k, acc in enumerate(sb_accesses):
        mine = []
        for (ar, mode, op, box) in acc:
            if mode == "reduce":
                part = ("partial", launch, ar, k)
                mine.append((part, "write", None, ((0, 0),)))
                reduced.setdefault(ar, []).append((part, box))
            else:
                mine.append((ar, mode, op, box))
        tasks.append({"launch": launch, "accesses": mine})
    for ar, parts in reduced.items():
        lo = [min(b[a][0] for _, b in parts) for a in range(len(parts[0][1]))]
        hi = [max(b[a][1] for _, b in parts) for a in range(len(parts[0][1]))]
        acc = [(p, "read", None, ((0, 0),)) for p, _ in parts]
        acc.append((ar, "write", None, tuple(zip(lo, hi))))
        tasks.append({"launch": launch, "accesses": acc})
    return tasks


def boxes_overlap(a, b):
    return all(max(x[0], y[0]) <= min(x[1], y[1]) for x, y in zip(a, b))


def required_orderings(tasks):
    """Pairs (p, q), p < q, of tasks in program order that must stay ordered.

    ``tasks`` is a list of dicts {"accesses": [(array, mode, op, box)]} with
    inclusive boxes and an optional "launch" key.  Two tasks must be ordered
    when they touch overlapping parts of one array and the two accesses
    conflict (tasks without a launch key count as different launches).
    """
    out = []
    for q in range(len(tasks)):
        for p in range(q):
            need = False
            lp, lq = tasks[p].get("launch"), tasks[q].get("launch")
            same = lp is not None and lp == lq
            for (ar, ma, oa, ba) in tasks[p]["accesses"]:
                for (br, mb, ob, bb) in tasks[q]["accesses"]:
                    if ar == br and conflicting(ma, oa, mb, ob, same) and boxes_overlap(ba, bb):
                        need = True
            if need:
                out.append((p, q))
    return out
