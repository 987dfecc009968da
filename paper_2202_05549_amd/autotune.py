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
         retune: bool = False, log=None):
    """Returns the fastest point of ``space`` for ``run``.

    ``space`` maps parameter names to candidate lists; ``run(**params)``
    performs one step of the workload and returns its duration in seconds
    (it may also time internally).  Each point is run ``reps`` times and the
    minimum kept.  With a cache path, a stored choice for ``signature`` is
    returned without timing unless ``retune``.
    """
    if cache and not retune:
        hit = _load(cache).get(signature)
        if hit is not None:
            return hit["best"]
    names = sorted(space)
    results = []
    best, best_t = None, float("inf")
    for values in itertools.product(*[space[n] for n in names]):
        params = dict(zip(names, values))
        t = min(run(**params) for _ in range(reps))
        results.append({"params": params, "seconds": t})
        if log:
            log("tune %s %s: %.3f ms" % (signature, params, t * 1e3))
        if t < best_t:
            best, best_t = params, t
    if cache:
        data = _load(cache)
        data[signature] = {"best": best, "seconds": best_t, "trials": results, "time": time.time()}
        _store(cache, data)
    return best
