"""Host tests of the autotuner's search: grid and coordinate descent find
the fastest point of synthetic cost surfaces, never time a point twice,
keep the minimum over repetitions and confirmations, and reuse the cache."""
import itertools

import pytest

from paper_2202_05549_amd import autotune

SPACE = {"sb": [1 << 20, 1 << 22, 1 << 24], "wg": [512, 1024, 2048], "vec": [2, 4], "tile": [0, 16384, 32768]}


def separable(sb, wg, vec, tile):
    # a bowl in each parameter: optimum at sb 2^22, wg 1024, vec 4, tile 16384
    return (1.0 + abs(sb.bit_length() - 23) * 0.3 + abs(wg - 1024) / 1024 * 0.2 + (vec == 2) * 0.05
            + abs(tile - 16384) / 16384 * 0.1)


def counting(f):
    calls = []

    def run(**p):
        calls.append(tuple(sorted(p.items())))
        return f(**p)
    return run, calls


def test_grid_finds_global_minimum_and_times_each_point_once():
    run, calls = counting(separable)
    best = autotune.tune("g", SPACE, run, reps=1, cache=None)
    assert best == {"sb": 1 << 22, "wg": 1024, "vec": 4, "tile": 16384}
    assert len(calls) == 3 * 3 * 2 * 3 and len(set(calls)) == len(calls)


def test_descent_finds_separable_minimum_with_fewer_timings():
    run, calls = counting(separable)
    best = autotune.tune("d", SPACE, run, reps=1, cache=None, strategy="descent")
    assert best == {"sb": 1 << 22, "wg": 1024, "vec": 4, "tile": 16384}
    assert len(set(calls)) == len(calls)          # memoised
    assert len(calls) < 3 * 3 * 2 * 3 // 2


def test_descent_from_start_and_tolerance():
    run, calls = counting(separable)
    start = {"sb": 1 << 22, "wg": 1024, "vec": 4, "tile": 16384}
    best = autotune.tune("d", SPACE, run, reps=1, cache=None, strategy="descent", start=start)
    assert best == start
    # a move must beat the current point by more than tol: with a huge
    # tolerance descent never moves, so it times one pass around the start
    # (1 + 2 + 2 + 1 + 2 points) and returns the fastest of those
    run2, calls2 = counting(separable)
    far = {"sb": 1 << 20, "wg": 512, "vec": 2, "tile": 0}
    best = autotune.tune("d", SPACE, run2, reps=1, cache=None, strategy="descent", start=far, tol=0.9)
    assert len(calls2) == 8
    one_pass = [dict(far, **{n: v}) for n in SPACE for v in SPACE[n]]
    assert best == min(one_pass, key=lambda p: separable(**p))
    with pytest.raises(ValueError):
        autotune.tune("d", SPACE, run2, cache=None, strategy="descent", start={"nope": 1})


def test_descent_reaches_a_coordinate_wise_minimum_on_a_coupled_surface():
    # non-separable: the best tile depends on sb; descent must end where no
    # single-parameter move helps
    def coupled(sb, wg, vec, tile):
        return separable(sb, wg, vec, tile) + (0.4 if (sb == 1 << 24) != (tile == 32768) else 0.0)
    run, _ = counting(coupled)
    best = autotune.tune("c", SPACE, run, reps=1, cache=None, strategy="descent")
    t = coupled(**best)
    for n, vals in SPACE.items():
        for v in vals:
            assert coupled(**dict(best, **{n: v})) >= t


def test_reps_and_confirm_keep_the_minimum():
    # point A is fast but noisy: its first sample is slow; B is steady.
    # With reps=1 and no confirmation B wins on the first samples; with a
    # confirmation round A's later samples are seen and A wins.
    samples = {"A": iter([3.0, 1.0, 1.0, 1.0]), "B": itertools.repeat(2.0)}

    def run(p):
        return next(samples[p])
    space = {"p": ["A", "B"]}
    assert autotune.tune("n", space, run, reps=1, cache=None) == {"p": "B"}
    samples["A"] = iter([3.0, 1.0, 1.0, 1.0])
    assert autotune.tune("n", space, run, reps=1, cache=None, confirm=1) == {"p": "A"}
    samples["A"] = iter([3.0, 1.0, 1.0, 1.0])
    assert autotune.tune("n", space, run, reps=2, cache=None) == {"p": "A"}


def test_cache_hit_skips_timing(tmp_path):
    path = str(tmp_path / "tune.json")
    run, calls = counting(separable)
    best = autotune.tune("sig", SPACE, run, reps=1, cache=path, strategy="descent")
    n = len(calls)
    again = autotune.tune("sig", SPACE, run, reps=1, cache=path, strategy="descent")
    assert again == best and len(calls) == n
    autotune.tune("sig", SPACE, run, reps=1, cache=path, retune=True, strategy="descent")
    assert len(calls) == 2 * n


def test_bad_arguments():
    with pytest.raises(ValueError):
        autotune.tune("x", {"a": []}, lambda a: 1.0, cache=None)
    with pytest.raises(ValueError):
        autotune.tune("x", {"a": [1]}, lambda a: 1.0, cache=None, strategy="random")
