"""Autotuner for launch and batch parameters.

The paper leaves chunk and superblock sizes to the programmer (it found
roughly 50 MB - 5 GB chunks to work, Sec. 4.3) and names automatic selection
as future work.  This tuner times candidate settings of a workload on the
GPU, through the C ABI only, and keeps the fastest: the superblock (chunk)
size of batched launches, the drain kernel's workgroup count, and the rows
per tile of the Jacobi body.  Results are cached in a JSON file keyed by a
workload signature, so a later run reuses them without timing again.
"""
from __future__ import annotations

import itertools
import json
import os
import time

DEFAULT_CACHE = os.environ.get("LT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "lt_tune.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(signature: str, space: dict, run, reps: int = 2, cache: str | None = DEFAULT_CACHE,
         retune: bool = False, log=None, strategy: str = "grid", start: dict | None = None,
         confirm: int = 0, tol: float = 0.0):
    """Returns the fastest point of ``space`` for ``run``.

    ``space`` maps parameter names to candidate lists; ``run(**params)``
    performs one step of the workload and returns its duration in seconds
    (it may also time internally).  Each point is run ``reps`` times and the
    minimum kept; a point is never timed twice by the search.

    ``strategy``:
      * ``"grid"``: every point of the product of the lists.
      * ``"descent"``: coordinate descent from ``start`` (default: the first
        candidate of every list).  Each pass tries every candidate of one
        parameter at a time with the others fixed and moves to the fastest
        when it beats the current point by more than ``tol`` (a fraction);
        passes repeat until one moves nothing.  It times the sum of the list
        lengths per pass instead of their product.

    With ``confirm`` > 0 the ``confirm`` + 1 fastest points found are timed
    ``reps`` more times each, and the minimum over all their timings decides:
    one lucky sample then does not pick the winner.  With a cache path, a
    stored choice for ``signature`` is returned without timing unless
    ``retune``.
    """
    if strategy not in ("grid", "descent"):
        raise ValueError("unknown strategy %r" % strategy)
    for n, vals in space.items():
        if not vals:
            raise ValueError("no candidates for %r" % n)
    if cache and not retune:
        hit = _load(cache).get(signature)
        if hit is not None:
            return hit["best"]
    names = sorted(space)
    seen = {}
    results = []

    def key(params):
        return tuple(params[n] for n in names)

    def cost(params):
        k = key(params)
        if k not in seen:
            t = min(run(**params) for _ in range(reps))
            seen[k] = t
            results.append({"params": dict(params), "seconds": t})
            if log:
                log("tune %s %s: %.3f ms" % (signature, params, t * 1e3))
        return seen[k]

    if strategy == "grid":
        for values in itertools.product(*[space[n] for n in names]):
            cost(dict(zip(names, values)))
    else:
        cur = {n: space[n][0] for n in names}
        if start:
            unknown = set(start) - set(names)
            if unknown:
                raise ValueError("start names unknown parameters %s" % sorted(unknown))
            cur.update(start)
        cost(cur)
        moved = True
        while moved:
            moved = False
            for n in names:
                best_v, best_t = cur[n], cost(cur)
                for v in space[n]:
                    t = cost(dict(cur, **{n: v}))
                    if t < best_t * (1.0 - tol):
                        best_v, best_t = v, t
                if best_v != cur[n]:
                    cur[n] = best_v
                    moved = True
    ranked = sorted(seen, key=seen.get)
    if confirm > 0:
        for k in ranked[:confirm + 1]:
            params = dict(zip(names, k))
            t = min(run(**params) for _ in range(reps))
            if log:
                log("tune %s %s: %.3f ms (confirm)" % (signature, params, t * 1e3))
            seen[k] = min(seen[k], t)
        ranked = sorted(ranked[:confirm + 1], key=seen.get)
    best = dict(zip(names, ranked[0]))
    best_t = seen[ranked[0]]
    if cache:
        data = _load(cache)
        data[signature] = {"best": best, "seconds": best_t, "trials": results, "time": time.time(),
                           "strategy": strategy}
        _store(cache, data)
    return best
