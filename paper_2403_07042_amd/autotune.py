"""Autotuner for the solver's launch knobs, with a JSON cache.

Knobs: the tile edges of the two products of a step (qme_set_tiles) and the
k-splits of the products (qme_set_split: the tail of the lower-triangle
product, every tile of a launch too small for the device) for a single
instance, and graph replay / instance order for a batch.  Every
candidate is timed on the real step (median of several trials of a few steps,
on a scratch copy of the state so the caller's state does not advance) and
the fastest is applied.  Results are cached per (GPU architecture,
precision, N, ld) in $QME_TUNE_CACHE (default ~/.cache/qme_mi355x/tune.json).

With the split off, tile choice among tiles of one matrix-core shape never
changes results: FP32 64- and 128-tiles (32x32 MFMA) and FP64 32- and
64-tiles (16x16 MFMA) accumulate each output element over k in the same
order, so their products are bitwise identical; FP32 32-tiles use the 16x16
MFMA, which groups the k sum differently (FP rounding only).  A split
regroups the k sum of the split tiles (FP rounding only, deterministic for a
given configuration).
"""
from __future__ import annotations

import json
import os
import statistics
import time

CACHE_ENV = "QME_TUNE_CACHE"

TILES = {
    "fp32": [(32, 32), (32, 64), (64, 32), (64, 64), (64, 128), (128, 64), (128, 128)],
    "fp64": [(32, 32), (32, 64), (64, 32), (64, 64)],
    "bf16x3": [(64, 64)],
}


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(
        os.path.expanduser("~"), ".cache", "qme_mi355x", "tune.json")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(precision: str, ld: int):
    """Tile pairs valid for this precision whose edges divide ld."""
    return [t for t in TILES[precision] if ld % t[0] == 0 and ld % t[1] == 0]


def solver_key(arch: str, precision: str, n: int, ld: int) -> str:
    return f"{arch}|{precision}|n={n}|ld={ld}"


def _arch(torch) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name))


def _time(torch, fn, trials: int) -> float:
    times = []
    for _ in range(trials):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return statistics.median(times)


def tune_solver(sol, steps: int = 4, trials: int = 3, use_cache: bool = True,
                path: str | None = None):
    """Pick and apply the fastest (tile1, tile2, split) for this solver;
    returns it."""
    torch = sol.torch
    key = solver_key(_arch(torch), sol.precision, sol.n, sol.ld)
    cache = load_cache(path) if use_cache else {}
    if key in cache and "split" in cache[key]:
        best = tuple(cache[key]["tiles"]) + (bool(cache[key]["split"]),)
        sol.set_tiles(*best[:2])
        sol.set_split(best[2])
        return best
    scratch = sol.state.clone()
    results = {}
    for tiles in candidates(sol.precision, sol.ld):
        for split in (True, False):
            sol.set_tiles(*tiles)
            sol.set_split(split)
            sol.step(1, state=scratch)                   # warm-up
            results[tiles + (split,)] = _time(torch, lambda: sol.step(steps, state=scratch), trials)
    best = min(results, key=results.get)
    sol.set_tiles(*best[:2])
    sol.set_split(best[2])
    del scratch
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"tiles": list(best[:2]), "split": best[2],
                      "seconds_per_step": {f"{a}x{b}{'/split' if sp else ''}": t / steps
                                           for (a, b, sp), t in results.items()}}
        save_cache(cache, path)
    return best


def tune_batch(batch, steps: int = 2, trials: int = 3):
    """Pick and apply the fastest (use_graph, largest_first) for a batch.
    Runs advance the batch's states by the steps timed (callers tune before
    setting their initial states, or re-set them afterwards)."""
    torch = batch.torch
    options = [(True, True), (True, False), (False, True)]
    results = {}
    for use_graph, largest in options:
        batch.config(use_graph=use_graph, largest_first=largest)
        batch.step(steps)                                 # warm-up / capture
        results[(use_graph, largest)] = _time(torch, lambda: batch.step(steps), trials)
    best = min(results, key=results.get)
    batch.config(use_graph=best[0], largest_first=best[1])
    return best, results
