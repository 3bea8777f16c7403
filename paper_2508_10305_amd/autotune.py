"""Autotuner for the batched form's launch geometry.

Picks the persistent grid (workgroups per compute unit) and the number of
consecutive blocks a wave takes per work-queue grab by timing graph replays
of the actual batch, and caches the choice per device and batch shape
(total blocks and blocks per job, in powers of two) in a JSON file.  The
stream bytes do not depend on the choice: only the launch shape changes.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning", "batch_launch.json")

GRID_PER_CU = (2, 4, 8, 16)
TILES = (1, 2, 4)


def shape_key(device_name: str, block_size: int, total_blocks: int, njobs: int) -> str:
    tb = int(math.log2(max(1, total_blocks)))
    per = int(math.log2(max(1, total_blocks // max(1, njobs))))
    return f"{device_name}|B{block_size}|blocks2^{tb}|perjob2^{per}"


def load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def tune(run: Callable[[int, int], float], cus: int, key: str, reps: int = 1,
         use_cache: bool = True, log: Optional[Callable[[str], None]] = None) -> dict:
    """`run(grid, tile)` builds a batch with that geometry and returns the
    measured milliseconds of one compress + decompress round.  Returns
    {"grid", "tile", "ms", "table"} and records it in the cache."""
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]
    table = []
    # persistent grids of 2..16 workgroups per CU x tile, and grid 0: one
    # workgroup per block (no persistent loop)
    shapes = [(g * cus, t) for g in GRID_PER_CU for t in TILES] + [(0, 1)]
    for grid, t in shapes:
        ms = min(run(grid, t) for _ in range(reps))
        table.append({"grid": grid, "tile": t, "ms": ms})
        if log:
            log(f"[tune] grid={grid} tile={t}: {ms:.3f} ms")
    best = min(table, key=lambda r: r["ms"])
    rec = {"grid": best["grid"], "tile": best["tile"], "ms": best["ms"], "table": table}
    cache[key] = rec
    if use_cache:
        save_cache(cache)
    return rec
