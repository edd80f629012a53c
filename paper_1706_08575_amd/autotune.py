"""Autotuner for the spreading launch: tile edge (for batches, tile and
records per task) chosen by timing candidates on the caller's own data,
remembered in a JSON cache keyed by the workload's shape.

Keys are plain strings: single plans by (dimension, precision, W, sigma, n,
log2 of samples per grid cell rounded to half steps); batches by (W, sigma,
R) and the sorted list of (n, density bucket) of their items, written out.
The neighbour-bin shape of the weight sum is not tuned here: it follows
from the raster's mean density (about 4.5 samples per bin), a rule measured
once on the SAS rasters.
The cache lives at $FTCG_TUNING_CACHE (default: ~/.cache/ftcg_tuning.json);
every measurement is the mean of the library's own event timings of the
spreading step over `reps` executions after one warm-up.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

PLAN_TILES = (16, 32, 64, 128)
BATCH_TILES = (16, 32, 64)
BATCH_CHUNKS = (1024, 4096, 16384)


def cache_path() -> str:
    return os.environ.get("FTCG_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ftcg_tuning.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + f".{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass   # a read-only home only loses the memory of the result


def density_bucket(m: int, n: int, sigma: float) -> float:
    cells = (sigma * n) ** 2
    return round(2.0 * math.log2(max(m, 1) / cells)) / 2.0


def plan_key(dim: int, dtype: str, W: int, sigma: float, n: int, m: int) -> str:
    return f"plan/d{dim}/{dtype}/W{W}/s{sigma:g}/n{n}/dens{density_bucket(m, n, sigma):+.1f}"


def batch_key(W: int, sigma: float, R: float, sizes, ms) -> str:
    mix = sorted((int(n), density_bucket(int(m), int(n), sigma)) for n, m in zip(sizes, ms))
    items = ",".join(f"{n}:{d:+.1f}" for n, d in mix)
    return f"batch/W{W}/s{sigma:g}/R{R:g}/items{len(mix)}/{items}"


def _spread_ms(obj, run, reps: int) -> float:
    run()
    torch.cuda.synchronize()
    obj.enable_timing(True)
    obj.timing()
    for _ in range(reps):
        run()
    t = obj.timing()
    obj.enable_timing(False)
    ms, cnt = t.get("spread", (0.0, 0))
    return ms / max(cnt, 1)


def tune_plan(plan, k: torch.Tensor, fhat: torch.Tensor, tiles=PLAN_TILES, reps: int = 3, use_cache: bool = True):
    """Pick the spreading launch of `plan` for raster k, values fhat: the tile
    edge with the plan's LDS accumulation. Leaves the plan tuned and with its
    points set. Returns ((tile, accum), {"tile/accum": ms})."""
    dtype = "f32" if plan.cdtype == torch.complex64 else "f64"
    key = plan_key(plan.dim, dtype, plan.W, plan.sigma, plan.n, int(k.shape[0]))
    cache = _load() if use_cache else {}
    if use_cache and key in cache and "accum" in cache[key]:
        tile, accum = int(cache[key]["tile"]), cache[key]["accum"]
        plan.set_tuning(tile, accum, 1)
        plan.set_points(k)
        return (tile, accum), cache[key].get("ms", {})
    base = "fixed" if dtype == "f32" else "f64"
    cands = [(t, base) for t in tiles if t >= 2 * plan.W]
    times = {}
    for t, accum in cands:
        try:
            plan.set_tuning(t, accum, 1)
        except Exception:
            continue
        plan.set_points(k)
        times[(t, accum)] = _spread_ms(plan, lambda: plan.execute(fhat), reps)
    best = min(times, key=times.get)
    plan.set_tuning(best[0], best[1], 1)
    plan.set_points(k)
    ms = {f"{a}/{b}": v for (a, b), v in times.items()}
    if use_cache:
        cache[key] = {"tile": best[0], "accum": best[1], "ms": ms, "when": time.time()}
        _store(cache)
    return best, ms


def tune_batch(batch, m, k: torch.Tensor, fhat: torch.Tensor, tiles=BATCH_TILES, chunks=BATCH_CHUNKS,
               reps: int = 3, use_cache: bool = True):
    """Pick (tile, records per task) of a Batch by timing whole executions.
    Leaves the batch tuned with its points set. Returns ((tile, chunk), {(tile, chunk): ms})."""
    key = batch_key(batch.W, batch.sigma, batch.R, batch.sizes, m)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        tile, chunk = int(cache[key]["tile"]), int(cache[key]["chunk"])
        batch.set_tuning(tile=tile, chunk=chunk)
        batch.set_points(m, k)
        return (tile, chunk), {}
    times = {}
    out = None
    for t in tiles:
        for c in chunks:
            batch.set_tuning(tile=t, chunk=c)
            batch.set_points(m, k)
            out = batch.execute(fhat, out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                out = batch.execute(fhat, out)
            torch.cuda.synchronize()
            times[(t, c)] = (time.perf_counter() - t0) / reps * 1e3
    best = min(times, key=times.get)
    batch.set_tuning(tile=best[0], chunk=best[1])
    batch.set_points(m, k)
    if use_cache:
        cache[key] = {"tile": best[0], "chunk": best[1],
                      "ms": {f"{a}x{b}": v for (a, b), v in times.items()}, "when": time.time()}
        _store(cache)
    return best, times
