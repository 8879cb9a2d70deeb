"""Benchmark of the cut-cell Runge-Kutta stage on one MI355X.

Workload: the 256 x 256 x 128 bell-hill domain (dx = dy = 100 m, dz = 50 m, h0 = 400 m, a = 2 km,
theta' noise from seed 0, dt = 0.05 s).  A "step" is one three-stage Runge-Kutta step: per stage the
fused tendency+update kernel and the velocity-diagnostic kernel.  The metric is interior
cell-updates per second per stage (nx*ny*nz cells x 3 stages per step), for the FP32 perturbation
form (headline) and the plain FP64 path (reported beside it).

The roofline object describes the dominant kernel, the fused update of one stage, which runs as two
back-to-back launches of the same kernel template: every point at or above its column's band top
(over the whole grid, the band paths compiled out), then the points below it (cut, merged and
next-to-terrain cells; lattice points not predicted) in one-wave tiles.  Its algorithmic bytes per stage (5 fields read
and written per cell, plus q_n read in stages 2 and 3) are divided by the stage's update duration,
measured with HIP events around the two launches on the launch stream, against the 8 TB/s HBM peak.  Measured HBM traffic
comes from a committed rocprofv3 counter summary when it was taken on the current kernel source.
The CPU baseline times the FP64 oracle on this machine's host cores on four steps of the workload.

The refined line (both precisions) runs the three-level hemisphere grid of blocks (25 level-0 steps in
one graph launch; cell-updates count the blocks' own cells x their level's steps x 3 stages).
The ensemble line (both precisions) advances 64 independent domains of uneven size through 50 steps
with one captured graph of the batched kernels.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f32|f64] [--no-cpu] [--no-ensemble] [--no-amr]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_update_bell256.json")
STAGE_SRC = os.path.join(ROOT, "paper_1509_02572_amd", "csrc", "cc_kernels.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(STAGE_SRC, "rb").read()).hexdigest()[:16]


def run_gpu(cfg, prec: str, steps: int, warmup: int, tile: int = 0):
    import torch
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W

    from paper_1509_02572_amd import autotune
    dom = CC.Domain(cfg, prec, "cuda:0")
    q = dom.init_state(W.theta_noise(cfg))
    if tile:
        dom.grid.tile = tile  # fixed tile shape (profiling runs)
        tuned = {"tile": tile}
    else:
        tuned = autotune.tune(dom, q, path=None, dt=cfg.dt)  # untimed: picks the tile shape
        log(f"bench: {prec} tile timings (ms per update launch): "
            + ", ".join(f"{k}{autotune.TILE_IDS[k]}w{autotune.TILE_MINW.get(k, 0)}={v:.4f}"
                        for k, v in tuned["ms"].items()))
    a, b, c = q, dom.new_state(), dom.new_state()
    dt = cfg.dt
    esz = 8 if prec == "f64" else 4
    ncell = cfg.nx * cfg.ny * cfg.nz
    stream = torch.cuda.current_stream()

    def step(a, b, c, ev=None):
        # stage s: update kernel (timed with events when ev is given) + diagnostics
        for s, (qs, qo, cdt) in enumerate(((a, b, dt / 3.0), (b, c, dt / 2.0), (c, b, dt))):
            if ev is not None:
                ev.append((torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True), s))
                ev[-1][0].record(stream)
            dom.rk_update(a, qs, qo, cdt, final_stage=(s == 2))
            if ev is not None:
                ev[-1][1].record(stream)
            dom.diagnose(qo)
        return b, a, c

    for _ in range(warmup):
        a, b, c = step(a, b, c)
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b, c = step(a, b, c, ev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = dom.check()
    if st[:5].any():
        raise RuntimeError(f"device status counters set: {st}")
    secs = t1 - t0
    upd_ms = [e0.elapsed_time(e1) for e0, e1, _ in ev]
    # algorithmic bytes: stage 1 reads q_s (= q_n) and writes q_out; stages 2-3 also read q_n; the
    # float form's final stage also reads and writes the low-order parts of rho' and (rho theta)'
    lo = 16 if prec == "f32" else 0
    bytes_per = [ncell * (5 * esz * (2 if s == 0 else 3) + (lo if s == 2 else 0)) for _, _, s in ev]
    avg_ms = sum(upd_ms) / len(upd_ms)
    avg_bytes = sum(bytes_per) / len(bytes_per)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": " + ".join(autotune.kernel_names(tuned["tile"], prec)),
            "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(avg_bytes)}
    if os.path.exists(TRAFFIC_FILE):  # counters taken on this kernel source and tile shape
        tr = json.load(open(TRAFFIC_FILE))
        ent = tr.get(prec, {}).get(str(tuned["tile"]))
        if ent and tr.get("kernel_source_sha256_16") == kernel_hash():
            roof["traffic"] = ent["hbm_bytes_per_launch"]
    value = ncell * 3 * steps / secs
    red = dom.reduce(a)
    roof["tile"] = list(autotune.TILE_IDS[tuned["tile"]])
    roof["tile_min_waves_per_simd"] = autotune.TILE_MINW.get(tuned["tile"], 0)
    return {"value": value, "ms_per_step": secs / steps * 1e3, "roofline": roof,
            "mass_total": float(red[2]), "mass_pert": float(red[0])}


def run_ensemble(prec: str, warmup: int):
    """The 64-member ensemble: every member advanced through all its steps by one graph launch of
    the batched kernels (one update and one diagnostic launch per stage for the whole batch)."""
    import torch
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W
    cfgs = W.ensemble(64, 0)
    doms = [CC.Domain(c, prec, "cuda:0") for c in cfgs]
    states = [d.init_state() for d in doms]
    dt, nsteps = cfgs[0].dt, cfgs[0].nsteps
    stream = torch.cuda.current_stream()
    # tile shape of the batch: one eager step per candidate, timed with events
    times = {}
    for tile in (0, 1, 6, 7, 9, 11, 12):
        b = CC.Batch(doms, states, tile=tile)
        b.step(dt, 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(dt, 2)
        e1.record(stream)
        torch.cuda.synchronize()
        times[tile] = e0.elapsed_time(e1)
        b.close()
    tile = min(times, key=times.get)
    batch = CC.Batch(doms, states, tile=tile)
    for _ in range(max(warmup, 1)):
        batch.step(dt, nsteps, use_graph=True)  # the first call captures the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    batch.step(dt, nsteps, use_graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = batch.check()
    if st[:5].any():
        raise RuntimeError(f"device status counters set: {st}")
    cells = batch.cells
    batch.close()
    return {"value": cells * 3 * nsteps / secs, "unit": "cell-updates/s", "cells": cells,
            "steps": nsteps, "ms_per_step": secs / nsteps * 1e3, "graph_ms": e0.elapsed_time(e1),
            "tile": tile, "tile_ms_per_2_steps": {str(k): round(v, 4) for k, v in times.items()}}


def run_amr(prec: str, warmup: int, layout=None):
    """The refined hemisphere (three levels of blocks, ghost cells integrated on, fine-first
    subcycling with flux matching): all its level-0 steps in one graph launch.  Cell-updates count
    own cells only (each level's cells x its steps x 3 stages); ghost work is overhead."""
    import torch
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W
    lay = layout if layout is not None else W.amr_hemisphere(2000)
    t0 = time.perf_counter()
    h = CC.Hierarchy(lay, prec, "cuda:0", tile=11)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    nsteps = lay.base.nsteps
    stream = torch.cuda.current_stream()
    for _ in range(max(warmup, 1)):
        h.step(1, use_graph=True)  # captures the single-step graphs (both starting buffers)
        h.step(1, use_graph=True)
    h.step(nsteps, use_graph=True)  # captures the timed sequence
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    h.step(nsteps, use_graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = h.check()
    if st[:6].any():
        raise RuntimeError(f"device status counters set: {st}")
    updates = sum(lay.cells(l) * (1 << l) for l in range(lay.levels)) * 3 * nsteps
    box = sum(int(d.cfg.nx * d.cfg.ny * d.cfg.nz) for d in h.doms)
    h.close()
    return {"value": updates / secs, "unit": "cell-updates/s", "blocks": len(lay.blocks),
            "own_cells_per_level": [lay.cells(l) for l in range(lay.levels)], "box_cells": box,
            "steps_level0": nsteps, "ms_per_level0_step": secs / nsteps * 1e3, "graph_ms": e0.elapsed_time(e1),
            "setup_s": round(setup, 1)}


def run_cpu_baseline(cfg):
    """FP64 oracle on the host cores: four full steps (three stages each) of the same workload,
    about 10 s of CPU work."""
    from oracle import oracle as O
    from paper_1509_02572_amd import workloads as W
    O.build(force=False)
    o = O.Oracle(cfg).merge()
    q = o.init_state(W.theta_noise(cfg))
    threads = O.set_threads(0)
    nsteps = 4
    t0 = time.perf_counter()
    o.run(q, cfg.dt, nsteps)
    secs = time.perf_counter() - t0
    n = cfg.nx * cfg.ny * cfg.nz
    return {"value": n * 3 * nsteps / secs, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsteps} RK steps (3 stages each) of the {cfg.nx}x{cfg.ny}x{cfg.nz} workload, FP64, "
                      f"{secs:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="fixed update-kernel tile id (default: autotuned)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the cut-cell stage is measured on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    from paper_1509_02572_amd import workloads as W
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration: 3 copies of 1 GiB (1 GiB read + 1 GiB written each)")
        del src, dst
    cfg = W.get("bell256")
    other = "f64" if args.prec == "f32" else "f32"
    log(f"bench: {cfg.name} {cfg.nx}x{cfg.ny}x{cfg.nz} prec={args.prec} steps={args.steps} warmup={args.warmup}")
    head = run_gpu(cfg, args.prec, args.steps, args.warmup, args.tile)
    log(f"bench: {args.prec} {head['value']:.4g} cell-updates/s, {head['ms_per_step']:.3f} ms/step")
    side = run_gpu(cfg, other, args.steps, args.warmup, args.tile)
    log(f"bench: {other} {side['value']:.4g} cell-updates/s, {side['ms_per_step']:.3f} ms/step")
    f64 = head if args.prec == "f64" else side
    amr = {}
    if not args.no_amr:
        from paper_1509_02572_amd import workloads as W
        lay = W.amr_hemisphere(2000)
        for p in (args.prec, other):
            amr[p] = run_amr(p, args.warmup, lay)
            log(f"bench: refined hemisphere {p} {amr[p]['value']:.4g} cell-updates/s, "
                f"{amr[p]['ms_per_level0_step']:.2f} ms per level-0 step")
    ens = {}
    if not args.no_ensemble:
        for p in (args.prec, other):
            ens[p] = run_ensemble(p, args.warmup)
            log(f"bench: ensemble {p} {ens[p]['value']:.4g} cell-updates/s, {ens[p]['ms_per_step']:.3f} ms/step")
    out = {
        "metric": "cell-updates/s per RK stage",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": "bell256: 256x256x128 cells, dx=dy=100 m, dz=50 m, bell hill h0=400 m "
                               "a=2 km, N=0.01 1/s, U=10 m/s, theta' noise N(0,0.01 K) seed 0, dt=0.05 s",
                   "precision": "FP32 perturbation (FP64 base state and sums)" if args.prec == "f32" else "FP64",
                   "cells": cfg.nx * cfg.ny * cfg.nz, "stages_per_step": 3},
        "roofline": head["roofline"],
        other: {"value": side["value"], "ms_per_step": side["ms_per_step"], "roofline": side["roofline"]},
        "speedup_vs_fp64": head["value"] / f64["value"],
    }
    if amr:
        out["refined"] = {"workload": "hemisphere R=1 km on 128x128x64 level-0 cells at 200 m (25.6x25.6x12.8 km), "
                                      "levels 1 (100 m) and 2 (50 m), 8^3-cell bricks, 6 ghost cells, dt(0)=0.2 s, "
                                      "25 level-0 steps per graph launch",
                          **amr}
    if ens:
        out["ensemble"] = {"workload": "64 periodic domains, nx,ny~U{48..96}, nz~U{48..64}, dx=dy=dz=100 m, "
                                       "1-5 Gaussian hills each (seed 0), dt=0.09 s, 50 steps per graph launch",
                           **ens}
    if not args.no_cpu:
        log("bench: timing the CPU oracle baseline")
        out["cpu_baseline"] = run_cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
