"""Autotuner of the update kernel's tile shape.

For a domain and precision, every tile shape the library offers (``cc_grid.tile`` ids) is timed on
the domain's own state with HIP events around the update kernel, and the fastest is kept.  Results
are cached in a JSON file keyed by precision and grid size, so later runs reuse them.  Results of
the stage do not depend on the tile shape (the kernel's arithmetic is the same for every shape).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")
# id -> (TX, TY, TZ) of the update kernel's tile; ids 9-12 repeat a shape with registers capped
# for 6 or 8 waves per SIMD; ids 13-19 give every thread two or four points spaced evenly in k (13-15, 17, 18: two;
# 16, 19: four); id 20 is the two-pass update (p' and lattice velocities computed once into the
# grid's stage workspace, then one point per thread)
TILE_IDS = {1: (4, 4, 16), 2: (8, 4, 16), 3: (4, 8, 16), 4: (8, 8, 8), 5: (2, 4, 32), 6: (4, 4, 32),
            7: (8, 8, 16), 8: (2, 2, 64), 9: (8, 8, 8), 10: (8, 8, 8), 11: (4, 4, 16), 12: (4, 8, 16),
            13: (8, 8, 16), 14: (8, 8, 16), 15: (8, 8, 8), 16: (8, 8, 8), 17: (4, 4, 16), 18: (8, 8, 8),
            19: (8, 8, 16), 20: (1, 1, 1)}
TILE_MINW = {9: 6, 10: 8, 11: 8, 12: 6, 13: 4, 14: 6, 15: 6, 16: 8, 17: 8, 18: 4, 19: 6}
# id -> template arguments of k_stage_tiled: threads per tile (TX, TY, TZ), minimum waves, points per
# thread along k
TILE_TEMPLATE = {0: (8, 8, 8, 1, 1), 1: (4, 4, 16, 1, 1), 2: (8, 4, 16, 1, 1), 3: (4, 8, 16, 1, 1),
                 4: (8, 8, 8, 1, 1), 5: (2, 4, 32, 1, 1), 6: (4, 4, 32, 1, 1), 7: (8, 8, 16, 1, 1),
                 8: (2, 2, 64, 1, 1), 9: (8, 8, 8, 6, 1), 10: (8, 8, 8, 8, 1), 11: (4, 4, 16, 8, 1),
                 12: (4, 8, 16, 6, 1), 13: (8, 8, 8, 4, 2), 14: (8, 8, 8, 6, 2), 15: (8, 8, 4, 6, 2),
                 16: (8, 8, 2, 8, 4), 17: (4, 4, 8, 8, 2), 18: (8, 8, 4, 4, 2), 19: (8, 8, 4, 6, 4)}


def kernel_names(tile: int, prec: str, small: bool = False):
    """rocprofv3 names (without arguments) of the two launches of one update stage on a grid with a
    known band height: the points at or above their column's band top over the whole grid (the
    kernel without the band paths), then the points below it in one-wave tiles (8x8x1; 4x4x4 on a
    grid with ``small`` = fewer than 8 columns in x or y)."""
    t = "double" if prec == "f64" else "float"
    tx, ty, tz, w, kp = TILE_TEMPLATE[tile]
    band = "4, 4, 4" if small else "8, 8, 1"
    return (f"cc::k_stage_tiled<{t}, {tx}, {ty}, {tz}, 0, {w}, {kp}, true, 1>",
            f"cc::k_stage_tiled<{t}, {band}, 0, 1, 1, false, 2>")


def key(dom) -> str:
    prec = "f64" if dom.prec == 0 else "f32"
    return f"{prec}:{dom.cfg.nx}x{dom.cfg.ny}x{dom.cfg.nz}"


def load_cache(path: str = CACHE) -> Dict[str, dict]:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def cached_tile(dom, path: str = CACHE) -> Optional[int]:
    ent = load_cache(path).get(key(dom))
    return int(ent["tile"]) if ent else None


def tune(dom, q, reps: int = 5, path: Optional[str] = CACHE, dt: float = 0.05) -> dict:
    """Time the update kernel (stage-2 form: q_n and q_s distinct) for every tile id on ``dom``.

    ``q`` is a valid state of ``dom``.  Returns {"tile": best id, "ms": {id: ms per launch}} and,
    when ``path`` is given, stores it in the cache.  The domain's tile is left at the best id."""
    a, b = dom.new_state(), dom.new_state()
    for f in q.t:
        a.t[f].copy_(q.t[f])
    dom.rk_stage(q, q, b, dt / 3.0)  # a valid stage-1 state to read
    stream = torch.cuda.current_stream()
    out = dom.new_state()
    times = {}
    for tid in TILE_IDS:
        dom.grid.tile = tid
        dom.rk_update(a, b, out, dt / 2.0)  # warm-up
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(stream)
            dom.rk_update(a, b, out, dt / 2.0)
            e1.record(stream)
        torch.cuda.synchronize()
        times[tid] = sorted(e0.elapsed_time(e1) for e0, e1 in ev)[reps // 2]
    best = min(times, key=times.get)
    dom.grid.tile = best
    res = {"tile": best, "shape": TILE_IDS[best], "ms": times}
    if path:
        cache = load_cache(path)
        cache[key(dom)] = {"tile": best, "shape": list(TILE_IDS[best]),
                           "ms": {str(k): round(v, 5) for k, v in times.items()}}
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res

