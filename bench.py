"""Benchmark of the cut-cell Runge-Kutta stage on one MI355X.

Headline workload: the 512 x 512 x 160 hemisphere domain (dx = dy = dz = 50 m, R = 1 km, N = 0.01 1/s,
U = 10 m/s, no noise, dt = 0.05 s), the largest single-grid configuration.  A "step" is one
three-stage Runge-Kutta step: per stage the fused tendency+update and the velocity-diagnostic
kernel.  The metric is interior cell-updates per second per stage (nx*ny*nz cells x 3 stages per
step), for the FP32 perturbation form (headline) and the plain FP64 path (reported beside it).  The
256 x 256 x 128 bell-hill domain (theta' noise, seed 0) is reported as a second line.

The roofline object describes the dominant kernel, the fused update of one stage (the regular-point
launch over the whole grid plus the band-point launch below the band height).  Its algorithmic bytes
are those the method must move per cell-stage: stage 1 reads q_s (= q_n) and writes q_out, 5 fields
each (40 B in the FP32 form, 80 B in FP64); stages 2-3 also read q_n (60 B / 120 B).  The FP32 form's
final stage also moves the low-order parts of rho' and (rho theta)' (+16 B/cell), reported as overhead
and not counted.  They are divided by the stage's update duration, measured with HIP events around
the launches on the launch stream, against the 8 TB/s HBM peak.  Measured HBM traffic comes from a
committed rocprofv3 counter summary when it was taken on the current kernel source.

The refined line (both precisions) runs the three-level hemisphere grid of blocks (25 level-0 steps in
one graph launch; cell-updates count the blocks' own cells x their level's steps x 3 stages).
The ensemble line (both precisions) advances 64 independent domains of uneven size through 50 steps
with one captured graph of the batched kernels.  Both carry a roofline object over their graph time
with the same per-cell algorithmic bytes (own cells only).

The CPU baseline times the FP64 oracle on this machine's host cores on one step of the headline
workload; --cpu-sweep also times one stage at 1, 2, 4, ... host threads.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f32|f64] [--workload hemi512|bell256]
                       [--no-cpu] [--no-ensemble] [--no-amr] [--no-second] [--cpu-sweep]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "hemi512": "hemi512: 512x512x160 cells at dx=dy=dz=50 m, hemisphere R=1 km, N=0.01 1/s, U=10 m/s, "
               "no noise, dt=0.05 s",
    "bell256": "bell256: 256x256x128 cells, dx=dy=100 m, dz=50 m, bell hill h0=400 m a=2 km, N=0.01 1/s, "
               "U=10 m/s, theta' noise N(0,0.01 K) seed 0, dt=0.05 s",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the stage kernels' sources (the traffic counters are valid only for the same code)."""
    from paper_1509_02572_amd import autotune
    return autotune.source_hash()


def traffic_file(name: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_update_{name}.json")


def algorithmic_bytes(prec: str, stage: int) -> int:
    """Bytes per cell the method must move in RK stage `stage` (0, 1, 2): read q_s (stage 1: q_s is
    q_n) and write q_out, stages 2-3 also read q_n; 5 fields of 4 B (FP32 form) or 8 B (FP64)."""
    esz = 8 if prec == "f64" else 4
    return 5 * esz * (2 if stage == 0 else 3)


def lo_overhead_bytes(prec: str, stage: int) -> int:
    """Extra bytes per cell of the FP32 form's final stage: the low-order parts of rho' and (rho
    theta)' read from q_n and written to q_out (not part of the algorithmic count)."""
    return 16 if (prec == "f32" and stage == 2) else 0


def roofline(bytes_per_launch: float, ms: float, **extra) -> dict:
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    out.update(extra)
    return out


def run_gpu(cfg, prec: str, steps: int, warmup: int, tile: int = 0):
    import torch
    from paper_1509_02572_amd import autotune
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W

    dom = CC.Domain(cfg, prec, "cuda:0")
    q = dom.init_state(W.theta_noise(cfg))
    if tile:
        dom.grid.tile = tile  # fixed tile shape (profiling runs)
        tuned = {"tile": tile, "source": "fixed"}
    else:
        tuned = autotune.tune(dom, q, dt=cfg.dt)  # untimed: picks the tile shape (or reads the cache)
        log(f"bench: {cfg.name} {prec} tile {tuned['tile']} ({tuned['source']}); ms per update launch: "
            + ", ".join(f"{k}={v:.4f}" for k, v in tuned["ms"].items()))
    a, b, c = q, dom.new_state(), dom.new_state()
    dt = cfg.dt
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
    upd = [(e0.elapsed_time(e1), s) for e0, e1, s in ev]
    avg_ms = sum(m for m, _ in upd) / len(upd)
    avg_bytes = sum(ncell * algorithmic_bytes(prec, s) for _, s in upd) / len(upd)
    over = sum(ncell * lo_overhead_bytes(prec, s) for _, s in upd) / len(upd)
    per_stage = {}
    for s in range(3):
        ms = [m for m, t in upd if t == s]
        per_stage[f"stage{s + 1}"] = {"ms": round(sum(ms) / len(ms), 4),
                                      "cell_updates_per_s": ncell / (sum(ms) / len(ms) * 1e-3),
                                      "bytes_per_cell": algorithmic_bytes(prec, s)}
    roof = roofline(avg_bytes, avg_ms, kernel=" + ".join(autotune.kernel_names(tuned["tile"], prec)),
                    avg_launch_ms=round(avg_ms, 4), algorithmic_bytes_per_launch=int(avg_bytes),
                    bytes_per_cell_stage=round(avg_bytes / ncell, 2), overhead_bytes_per_launch=int(over),
                    per_stage=per_stage, tile=tuned["tile"], tile_shape=list(autotune.TILE_IDS[tuned["tile"]]))
    tf = traffic_file(cfg.name)
    if os.path.exists(tf):  # counters taken on this kernel source and tile shape
        tr = json.load(open(tf))
        ent = tr.get(prec, {}).get(str(tuned["tile"]))
        if ent and tr.get("kernel_source_sha256_16") == kernel_hash():
            roof["traffic"] = ent["hbm_bytes_per_launch"]
            roof["traffic_source"] = os.path.relpath(tf, ROOT)
    value = ncell * 3 * steps / secs
    red = dom.reduce(a)
    return {"value": value, "ms_per_step": secs / steps * 1e3, "roofline": roof,
            "mass_total": float(red[2]), "mass_pert": float(red[0])}


def paper_model_config(cfg):
    """The workload with the source terms of the paper's model switched on: fourth-order artificial
    diffusion at 1e-3 1/s in every direction and a sponge over the top third of the domain at
    0.01 1/s at the lid."""
    return cfg.replace(kdh=1e-3, kdv=1e-3, zsp=cfg.z0 + cfg.nz * cfg.dz * 2.0 / 3.0, rsp=0.01)


def run_paper_model(cfg, prec: str, steps: int, warmup: int, tile: int):
    """Two runs of the workload with diffusion and sponge on (paper_model_config): the Runge-Kutta
    stage as in the headline (stage time beside the headline's gives the cost of the source-term
    launch), and the paper's own scheme, leap-frog with the Robert-Asselin filter (weight 0.1) in p'
    form: one update per step, timed with HIP events around each step."""
    import torch
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W
    pc = paper_model_config(cfg)
    dom = CC.Domain(pc, prec, "cuda:0")
    q = dom.init_state(W.theta_noise(pc))
    dom.grid.tile = tile  # the headline's update form
    stream = torch.cuda.current_stream()
    ncell = pc.nx * pc.ny * pc.nz
    esz = 8 if prec == "f64" else 4
    # Runge-Kutta stages with the source terms
    a, b, c = q, dom.new_state(), dom.new_state()
    for _ in range(warmup):
        a, b, c = dom.step(a, b, c, pc.dt)
    ev = []
    for _ in range(steps):
        for s, (qs, qo, cdt) in enumerate(((a, b, pc.dt / 3.0), (b, c, pc.dt / 2.0), (c, b, pc.dt))):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dom.rk_update(a, qs, qo, cdt, final_stage=(s == 2))
            e1.record(stream)
            ev.append((e0, e1))
            dom.diagnose(qo)
        a, b, c = b, a, c
    torch.cuda.synchronize()
    rk_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)
    # leap-frog in p' form
    q = dom.init_state(W.theta_noise(pc))
    dom.pform(q, True)
    qm, q0, qp = dom.new_state(), q, dom.new_state()
    dom.lf_step(None, q0, qp, pc.dt, 0.1, first=True)
    qm, q0, qp = q0, qp, qm
    for _ in range(warmup):
        dom.lf_step(qm, q0, qp, pc.dt, 0.1)
        qm, q0, qp = q0, qp, qm
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dom.lf_step(qm, q0, qp, pc.dt, 0.1)
        e1.record(stream)
        ev.append((e0, e1))
        qm, q0, qp = q0, qp, qm
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = dom.check()
    if st[:5].any():
        raise RuntimeError(f"device status counters set: {st}")
    lf_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)
    # a leap-frog step must read q(n) and qbar(n-1) and write q(n+1) and qbar(n): 20 fields per cell
    lf_bytes = ncell * 20 * esz
    return {"diffusion_per_s": pc.kdh, "sponge": {"bottom_m": pc.zsp, "rate_per_s": pc.rsp},
            "rk3_stage_ms": round(rk_ms, 4), "rk3_cell_updates_per_s": ncell / (rk_ms * 1e-3),
            "leapfrog": {"value": ncell * steps / secs, "unit": "cell-updates/s (one update per step)",
                         "ms_per_step": round(lf_ms, 4), "filter_weight": 0.1,
                         "roofline": roofline(lf_bytes, lf_ms, scope="whole step (p' conversion, update, source "
                                              "terms, finish and filter, diagnostics)",
                                              algorithmic_bytes=int(lf_bytes),
                                              bytes_per_cell=20 * esz)}}


def run_ensemble(prec: str, warmup: int):
    """The 64-member ensemble: every member advanced through all its steps by one graph launch of
    the batched kernels (one update and one diagnostic launch per stage for the whole batch)."""
    import torch
    from paper_1509_02572_amd import autotune
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W
    cfgs = W.ensemble(64, 0)
    doms = [CC.Domain(c, prec, "cuda:0", side_stream=False) for c in cfgs]
    bad = [m for m, d in enumerate(doms) if d.check()[0]]
    if bad:  # the generator does not redraw on an unmergeable cell: treat one as an error
        raise RuntimeError(f"ensemble members with unmergeable cells: {bad}")
    states = [d.init_state() for d in doms]
    dt, nsteps = cfgs[0].dt, cfgs[0].nsteps
    stream = torch.cuda.current_stream()
    tuned = autotune.tune_batch(doms, states, dt, prec)
    batch = CC.Batch(doms, states, tile=tuned["tile"])
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
    gms = e0.elapsed_time(e1)
    # whole graph (updates, band launches, diagnostics) against the algorithmic bytes of its stages
    byts = cells * sum(algorithmic_bytes(prec, s) for s in range(3)) * nsteps
    return {"value": cells * 3 * nsteps / secs, "unit": "cell-updates/s", "cells": cells,
            "redraws": sum(c.redraws for c in cfgs),
            "steps": nsteps, "ms_per_step": secs / nsteps * 1e3, "graph_ms": gms,
            "tile": tuned["tile"], "tile_source": tuned["source"],
            "tile_ms": {str(k): round(v, 4) for k, v in tuned["ms"].items()},
            "roofline": roofline(byts, gms, scope="whole graph (all stages, diagnostics included)",
                                 algorithmic_bytes=int(byts))}


def run_amr(prec: str, warmup: int, layout=None):
    """The refined hemisphere (three levels of blocks, ghost cells integrated on, fine-first
    subcycling with flux matching): all its level-0 steps in one graph launch.  Cell-updates count
    own cells only (each level's cells x its steps x 3 stages); ghost work is overhead."""
    import torch
    from paper_1509_02572_amd import autotune
    from paper_1509_02572_amd import cutcell as CC
    from paper_1509_02572_amd import workloads as W
    lay = layout if layout is not None else W.amr_hemisphere(2000)
    tuned = autotune.tune_refined(lay, prec)
    t0 = time.perf_counter()
    h = CC.Hierarchy(lay, prec, "cuda:0", tile=tuned["tile"])
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
    tables = [CC.amr_batch_info(h.h, l) for l in range(lay.levels)]
    own = sum(lay.cells(l) * (1 << l) for l in range(lay.levels))  # own-cell updates per level-0 stage
    updates = own * 3 * nsteps
    box = sum(int(d.cfg.nx * d.cfg.ny * d.cfg.nz) for d in h.doms)
    h.close()
    gms = e0.elapsed_time(e1)
    byts = own * sum(algorithmic_bytes(prec, s) for s in range(3)) * nsteps
    return {"value": updates / secs, "unit": "cell-updates/s", "blocks": len(lay.blocks),
            "own_cells_per_level": [lay.cells(l) for l in range(lay.levels)], "box_cells": box,
            "steps_level0": nsteps, "ms_per_level0_step": secs / nsteps * 1e3, "graph_ms": gms,
            "setup_s": round(setup, 1), "tile": tuned["tile"], "tile_source": tuned["source"], "levels": tables,
            "roofline": roofline(byts, gms, scope="whole graph (own cells; ghost updates, refills, flux "
                                                  "matching and diagnostics included in the time)",
                                 algorithmic_bytes=int(byts))}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(cfg, sweep: bool = False):
    """FP64 oracle on the host cores: one full step (three stages with their diagnostics) of the
    headline workload.  With `sweep`, one stage is also timed at 1, 2, 4, ... threads."""
    from oracle import oracle as O
    from paper_1509_02572_amd import workloads as W
    O.build(force=False)
    o = O.Oracle(cfg).merge()
    q = o.init_state(W.theta_noise(cfg))
    threads = O.set_threads(0)
    nsteps = 1
    t0 = time.perf_counter()
    o.run(q, cfg.dt, nsteps)
    secs = time.perf_counter() - t0
    n = cfg.nx * cfg.ny * cfg.nz
    out = {"value": n * 3 * nsteps / secs, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{nsteps} RK step (3 stages with diagnostics) of the {cfg.nx}x{cfg.ny}x{cfg.nz} workload, "
                     f"FP64, {secs:.1f} s", "cpu_model": cpu_model()}
    if sweep:
        rows = []
        t = 1
        counts = []
        while t < threads:
            counts.append(t)
            t *= 2
        counts.append(threads)
        buf = o.rk_stage(q, q, cfg.dt / 3.0)  # output state, its pages touched outside the timing
        for t in counts:
            O.set_threads(t)
            t0 = time.perf_counter()
            o.rk_stage(q, q, cfg.dt / 3.0, out=buf)
            rows.append((t, time.perf_counter() - t0))
            log(f"bench: cpu oracle {t} threads: one stage {rows[-1][1]:.2f} s")
        O.set_threads(threads)
        t1 = rows[0][1]
        out["sweep"] = [{"threads": t, "stage_s": round(s, 3), "cell_updates_per_s": n / s,
                         "parallel_efficiency": round(t1 / (t * s), 3)} for t, s in rows]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="hemi512", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweep", action="store_true", help="also time one oracle stage at 1, 2, 4, ... threads")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-second", action="store_true", help="skip the second single-grid workload")
    ap.add_argument("--no-paper-model", action="store_true",
                    help="skip the runs with diffusion and sponge (Runge-Kutta and leap-frog)")
    ap.add_argument("--no-other-prec", action="store_true", help="time the chosen precision only")
    ap.add_argument("--tile", type=int, default=0, help="fixed update-kernel tile id (default: autotuned)")
    ap.add_argument("--only", choices=["refined", "ensemble"], default=None,
                    help="run only the refined-grid or the ensemble part (profiling runs; prints its JSON)")
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
    cfg = W.get(args.workload)
    other = "f64" if args.prec == "f32" else "f32"
    if args.only:
        precs = (args.prec,) if args.no_other_prec else (args.prec, other)
        part = {}
        for p in precs:
            part[p] = run_amr(p, args.warmup) if args.only == "refined" else run_ensemble(p, args.warmup)
            log(f"bench: {args.only} {p} {part[p]['value']:.4g} cell-updates/s")
        print(json.dumps({args.only: part}), flush=True)
        return
    log(f"bench: {cfg.name} {cfg.nx}x{cfg.ny}x{cfg.nz} prec={args.prec} steps={args.steps} warmup={args.warmup}")
    head = run_gpu(cfg, args.prec, args.steps, args.warmup, args.tile)
    log(f"bench: {cfg.name} {args.prec} {head['value']:.4g} cell-updates/s, {head['ms_per_step']:.3f} ms/step, "
        f"frac {head['roofline']['frac']}")
    side = None
    if not args.no_other_prec:
        side = run_gpu(cfg, other, args.steps, args.warmup, args.tile)
        log(f"bench: {cfg.name} {other} {side['value']:.4g} cell-updates/s, {side['ms_per_step']:.3f} ms/step, "
            f"frac {side['roofline']['frac']}")
    paper = {}
    if not args.no_paper_model:
        for p, r in ((args.prec, head), (other, side)):
            if r is None:
                continue
            paper[p] = run_paper_model(cfg, p, min(args.steps, 10), min(args.warmup, 2), r["roofline"]["tile"])
            base_ms = r["roofline"]["avg_launch_ms"]
            if base_ms:
                extra = paper[p]["rk3_stage_ms"] - base_ms
                paper[p]["source_terms_ms_per_stage"] = round(extra, 4)
                # the source-term launch reads q_s and reads and writes q_out: 15 fields per cell
                byts = cfg.nx * cfg.ny * cfg.nz * 15 * (8 if p == "f64" else 4)
                if extra > 0:
                    paper[p]["source_terms_roofline"] = roofline(byts, extra, algorithmic_bytes=int(byts),
                                                                 scope="stage time with minus without")
            log(f"bench: paper model {p}: RK3 stage {paper[p]['rk3_stage_ms']:.3f} ms with diffusion and sponge; "
                f"leap-frog {paper[p]['leapfrog']['value']:.4g} cell-updates/s, "
                f"{paper[p]['leapfrog']['ms_per_step']:.3f} ms/step")
    second = {}
    if not args.no_second:
        name2 = "bell256" if args.workload == "hemi512" else "hemi512"
        cfg2 = W.get(name2)
        for p in (args.prec, other):
            r = run_gpu(cfg2, p, args.steps, args.warmup, args.tile)
            second[p] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "roofline": r["roofline"]}
            log(f"bench: {name2} {p} {r['value']:.4g} cell-updates/s, frac {r['roofline']['frac']}")
        second = {"workload": WORKLOADS[name2], **second}
    amr = {}
    if not args.no_amr:
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
        "config": {"workload": WORKLOADS[args.workload],
                   "precision": "FP32 perturbation (FP64 base state and sums)" if args.prec == "f32" else "FP64",
                   "cells": cfg.nx * cfg.ny * cfg.nz, "stages_per_step": 3},
        "roofline": head["roofline"],
    }
    if side is not None:
        f64 = head if args.prec == "f64" else side
        out[other] = {"value": side["value"], "ms_per_step": side["ms_per_step"], "roofline": side["roofline"]}
        out["speedup_vs_fp64"] = head["value"] / f64["value"]
    if paper:
        out["paper_model"] = {"workload": WORKLOADS[args.workload] + ", with artificial diffusion and sponge", **paper}
    if second:
        out["second_workload"] = second
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
        out["cpu_baseline"] = run_cpu_baseline(cfg, args.cpu_sweep)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
