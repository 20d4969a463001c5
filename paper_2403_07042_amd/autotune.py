"""Autotuner for the solver's launch knobs, with a JSON cache.

Knobs: the tile edges of the two products of a step (qme_set_tiles) and the
k-splits of the products (qme_set_split: the tail of the lower-triangle
product, every tile of a launch too small for the device) for a single
instance; for a batch, the tile edges per instance size (32 or 64 for each
product), graph replay and instance order.  Every
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
    "bf16x3": [(64, 64), (128, 64)],
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


BATCH_TILES = [(32, 32), (32, 64), (64, 32), (64, 64)]


def batch_key(arch: str, batch) -> str:
    sizes = {}
    for s in batch.solvers:
        sizes[s.n] = sizes.get(s.n, 0) + 1
    mix = ",".join(f"{n}x{c}" for n, c in sorted(sizes.items()))
    return f"{arch}|batch|fp32|{mix}"


def tune_batch(batch, steps: int = 2, trials: int = 3, tiles: bool = True,
               use_cache: bool = False, path: str | None = None):
    """Pick and apply the fastest batch configuration: the tile edges of the
    two products per instance size (32 or 64 each; all instances of one N
    share them), then graph replay on/off and the instance order.  Sizes
    are tuned one at a time, largest first, each over the four tile pairs
    with the other sizes held (coordinate descent on the whole batched
    step).  Runs advance the batch's states by the steps timed (callers tune
    before setting their initial states, or re-set them afterwards).
    Returns (best, results): best = (use_graph, largest_first, {N: tiles})."""
    torch = batch.torch
    key = batch_key(_arch(torch), batch)
    if use_cache:
        entry = load_cache(path).get(key)
        if entry:
            per_n = {int(n): tuple(t) for n, t in entry["tiles"].items()}
            for s in batch.solvers:
                s.set_tiles(*per_n[s.n])
            batch.config(use_graph=entry["use_graph"], largest_first=entry["largest_first"])
            return (entry["use_graph"], entry["largest_first"], per_n), {}
    results = {}

    def timed(use_graph, largest):
        batch.config(use_graph=use_graph, largest_first=largest)
        batch.step(steps)                                 # warm-up / capture
        return _time(torch, lambda: batch.step(steps), trials)

    sizes = sorted({s.n for s in batch.solvers}, reverse=True)
    per_n = {n: next((s.tile1, s.tile2) for s in batch.solvers if s.n == n) for n in sizes}
    per_n = {n: (t if t in BATCH_TILES else (64, 64)) for n, t in per_n.items()}

    def apply(assign):
        for s in batch.solvers:
            s.set_tiles(*assign[s.n])

    if tiles:
        for n in sizes:
            best_t, best_time = None, None
            for t in BATCH_TILES:
                trial = dict(per_n)
                trial[n] = t
                apply(trial)
                sec = timed(True, True)
                results[("tiles", n, t)] = sec
                if best_time is None or sec < best_time:
                    best_t, best_time = t, sec
            per_n[n] = best_t
    apply(per_n)
    for use_graph, largest in [(True, True), (True, False), (False, True)]:
        results[(use_graph, largest)] = timed(use_graph, largest)
    best_order = min([k for k in results if len(k) == 2], key=results.get)
    batch.config(use_graph=best_order[0], largest_first=best_order[1])
    best = (best_order[0], best_order[1], dict(per_n))
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"use_graph": best[0], "largest_first": best[1],
                      "tiles": {str(n): list(t) for n, t in per_n.items()},
                      "seconds_per_batched_step": {
                          (f"{k[1]}:{k[2][0]}x{k[2][1]}" if k[0] == "tiles" else
                           f"graph={k[0]},largest_first={k[1]}"): v / steps
                          for k, v in results.items()}}
        save_cache(cache, path)
    return best, results
