"""Autotuner of the update kernel's tile shapes: single grids, ensemble batches and refined grids.

For a single grid every tile shape the library offers (``cc_grid.tile`` ids) is timed on the
domain's own state with HIP events around the update launches, and the fastest is kept.  Batches
(ensembles of independent domains) and refined grids time the batch tile shapes on their own blocks.
Results are cached in a JSON file keyed by what was tuned (kind, precision, sizes) and by a hash of
the kernel sources, so a cached choice is reused only for the kernels it was measured on.  The
stage's results do not depend on the tile shape (the arithmetic is the same for every shape).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("cc_kernels.hpp", "cc_stage.hip", "cc_stream.hip",
                                                          "cc_batch.hip")]

# id -> (TX, TY, TZ) of the update kernel's tile; ids 9-12 repeat a shape with registers capped
# for 6 or 8 waves per SIMD; ids 13-19 give every thread two or four points spaced evenly in k (13-15, 17, 18: two;
# 16, 19: four); id 20 is the two-pass update (p' and lattice velocities computed once into the
# grid's stage workspace, then one point per thread)
TILE_IDS = {1: (4, 4, 16), 2: (8, 4, 16), 3: (4, 8, 16), 4: (8, 8, 8), 5: (2, 4, 32), 6: (4, 4, 32),
            7: (8, 8, 16), 8: (2, 2, 64), 9: (8, 8, 8), 10: (8, 8, 8), 11: (4, 4, 16), 12: (4, 8, 16),
            13: (8, 8, 16), 14: (8, 8, 16), 15: (8, 8, 8), 16: (8, 8, 8), 17: (4, 4, 16), 18: (8, 8, 8),
            19: (8, 8, 16), 20: (1, 1, 1),
            21: (8, 32), 22: (8, 32), 23: (8, 16), 24: (8, 32), 25: (8, 32), 26: (8, 16), 27: (16, 16),
            28: (16, 16), 29: (16, 32)}
# ids 21-29: streaming forms of the regular points, (TY, TZ) threads over a j-k cross-section
# marching along x through chunks of STREAM_CHUNK planes with STREAM_NBAR barriers per plane
STREAM_CHUNK = {21: 32, 22: 32, 23: 32, 24: 64, 25: 64, 26: 32, 27: 32, 28: 32, 29: 32}
STREAM_NBAR = {21: 2, 22: 1, 23: 1, 24: 2, 25: 1, 26: 2, 27: 1, 28: 2, 29: 2}
TILE_MINW = {9: 6, 10: 8, 11: 8, 12: 6, 13: 4, 14: 6, 15: 6, 16: 8, 17: 8, 18: 4, 19: 6}
# id -> template arguments of k_stage_tiled: threads per tile (TX, TY, TZ), minimum waves, points per
# thread along k
TILE_TEMPLATE = {0: (8, 8, 8, 1, 1), 1: (4, 4, 16, 1, 1), 2: (8, 4, 16, 1, 1), 3: (4, 8, 16, 1, 1),
                 4: (8, 8, 8, 1, 1), 5: (2, 4, 32, 1, 1), 6: (4, 4, 32, 1, 1), 7: (8, 8, 16, 1, 1),
                 8: (2, 2, 64, 1, 1), 9: (8, 8, 8, 6, 1), 10: (8, 8, 8, 8, 1), 11: (4, 4, 16, 8, 1),
                 12: (4, 8, 16, 6, 1), 13: (8, 8, 8, 4, 2), 14: (8, 8, 8, 6, 2), 15: (8, 8, 4, 6, 2),
                 16: (8, 8, 2, 8, 4), 17: (4, 4, 8, 8, 2), 18: (8, 8, 4, 4, 2), 19: (8, 8, 4, 6, 4)}
# tile ids a batch (ensemble or refined grid) accepts
BATCH_TILES = (0, 1, 6, 7, 8, 9, 11, 12)
BATCH_CANDIDATES = (0, 1, 6, 7, 9, 11, 12, 21, 22, 23, 24, 25, 26, 27, 28, 29)  # streaming forms: whole grids only
REFINED_CANDIDATES = (1, 6, 9, 11)


def kernel_names(tile: int, prec: str, small: bool = False):
    """rocprofv3 names (without arguments) of the launches of one update stage on a grid with a
    known band height.  Tiled shapes: the points at or above their column's band top over the whole
    grid (the kernel without the band paths), then the points below it in one-wave tiles (8x8x1;
    4x4x4 on a grid with ``small`` = fewer than 8 columns in x or y).  The two-pass form (id 20):
    the prepare pass and the point pass."""
    t = "double" if prec == "f64" else "float"
    if tile == 20:
        return (f"cc::k_prepare<{t}>", f"cc::k_stage_points<{t}, 0>")
    band = "4, 4, 4" if small else "8, 8, 1"
    if tile in STREAM_CHUNK:
        ty, tz = TILE_IDS[tile]
        w = 4 if prec == "f32" else 1
        return (f"cc::k_stage_stream<{t}, {ty}, {tz}, {STREAM_CHUNK[tile]}, {w}, {STREAM_NBAR[tile]}>",
                f"cc::k_stage_tiled<{t}, {band}, 0, 1, 1, false, 2>")
    tx, ty, tz, w, kp = TILE_TEMPLATE[tile]
    return (f"cc::k_stage_tiled<{t}, {tx}, {ty}, {tz}, 0, {w}, {kp}, true, 1>",
            f"cc::k_stage_tiled<{t}, {band}, 0, 1, 1, false, 2>")


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def _prec(p) -> str:
    if isinstance(p, str):
        return p
    return "f64" if p == 0 else "f32"


def key(dom) -> str:
    return f"grid:{_prec(dom.prec)}:{dom.cfg.nx}x{dom.cfg.ny}x{dom.cfg.nz}"


def load_cache(path: str = CACHE) -> Dict[str, dict]:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _lookup(k: str, path: Optional[str]) -> Optional[dict]:
    ent = load_cache(path).get(k) if path else None
    if ent and ent.get("source_hash") == source_hash():
        return ent
    return None


def _store(k: str, best: int, times: Dict[int, float], path: Optional[str]):
    if not path:
        return
    cache = load_cache(path)
    cache[k] = {"tile": int(best), "ms": {str(t): round(v, 5) for t, v in times.items()},
                "source_hash": source_hash()}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_tile(dom, path: str = CACHE) -> Optional[int]:
    ent = _lookup(key(dom), path)
    return int(ent["tile"]) if ent else None


def tune(dom, q, reps: int = 5, path: Optional[str] = CACHE, dt: float = 0.05, force: bool = False,
         candidates: Optional[Iterable[int]] = None) -> dict:
    """Tile id of the single-grid update on ``dom`` (stage-2 form: q_n and q_s distinct).

    A cached choice for the same grid size, precision and kernel sources is reused unless ``force``;
    otherwise every candidate is timed (median of ``reps`` launches after one warm-up) and the
    result cached.  ``q`` is a valid state of ``dom``.  The domain's tile is set to the choice.
    Returns {"tile", "ms": {id: ms}, "source": "cache" | "timed"}."""
    import torch
    ent = None if force else _lookup(key(dom), path)
    if ent:
        dom.grid.tile = int(ent["tile"])
        return {"tile": int(ent["tile"]), "ms": {int(k): v for k, v in ent["ms"].items()}, "source": "cache"}
    a, b = dom.new_state(), dom.new_state()
    for f in q.t:
        a.t[f].copy_(q.t[f])
    dom.rk_stage(q, q, b, dt / 3.0)  # a valid stage-1 state to read
    stream = torch.cuda.current_stream()
    out = dom.new_state()
    times = {}
    for tid in (candidates or TILE_IDS):
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
    _store(key(dom), best, times, path)
    return {"tile": best, "ms": times, "source": "timed"}


def tune_batch(doms, states, dt: float, prec: str, path: Optional[str] = CACHE, force: bool = False,
               candidates: Iterable[int] = BATCH_CANDIDATES) -> dict:
    """Tile id of a batch of independent domains: each candidate steps the batch eagerly (one step,
    then two timed steps with HIP events); the states are advanced by the timing runs."""
    import torch
    from . import cutcell as CC
    sizes = hashlib.sha256(json.dumps([[d.cfg.nx, d.cfg.ny, d.cfg.nz] for d in doms]).encode()).hexdigest()[:12]
    k = f"batch:{_prec(prec)}:{len(doms)}:{sizes}"
    ent = None if force else _lookup(k, path)
    if ent:
        return {"tile": int(ent["tile"]), "ms": {int(t): v for t, v in ent["ms"].items()}, "source": "cache"}
    stream = torch.cuda.current_stream()
    times = {}
    for tile in candidates:
        b = CC.Batch(doms, states, tile=tile)
        b.step(dt, 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(dt, 2)
        e1.record(stream)
        torch.cuda.synchronize()
        times[tile] = e0.elapsed_time(e1)
        b.close()
    best = min(times, key=times.get)
    _store(k, best, times, path)
    return {"tile": best, "ms": times, "source": "timed"}


def tune_refined(layout, prec: str, path: Optional[str] = CACHE, force: bool = False,
                 candidates: Iterable[int] = REFINED_CANDIDATES) -> dict:
    """Tile id of a refined grid: each candidate builds the hierarchy and times one eager level-0
    step (after one untimed step) with HIP events."""
    import torch
    from . import cutcell as CC
    desc = json.dumps([[int(b.level), [int(v) for v in b.org], [int(v) for v in b.size]] for b in layout.blocks])
    k = f"refined:{_prec(prec)}:{len(layout.blocks)}:{hashlib.sha256(desc.encode()).hexdigest()[:12]}"
    ent = None if force else _lookup(k, path)
    if ent:
        return {"tile": int(ent["tile"]), "ms": {int(t): v for t, v in ent["ms"].items()}, "source": "cache"}
    stream = torch.cuda.current_stream()
    times = {}
    for tile in candidates:
        h = CC.Hierarchy(layout, prec, "cuda:0", tile=tile)
        h.step(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        times[tile] = e0.elapsed_time(e1)
        h.close()
        del h
    best = min(times, key=times.get)
    _store(k, best, times, path)
    return {"tile": best, "ms": times, "source": "timed"}
