"""Experiments of the paper run on the GPU path (uniform grids, FP64 by default).

* ``convergence``: the global-accuracy study of Appendix A.  Flow over the cosine hill (h_m = 400 m,
  a = 2 km, centred at (32, 16) km) in the 64 x 32 x 16 km domain of Sec. 3 (U = 10 m/s,
  N = 0.01 1/s, free-slip ground, periodic sides, sponge above 10 km) on uniform grids of
  400, 250, 200 and 100 m, integrated for one hour; the L1 and L2 norms of the errors in u and w
  over the lattice points above the hilltop, taking the 100 m run as the exact solution, and the
  slope of their log-log fit against the grid interval (second order: 2).
* ``lee_wave``: the 1-hour bell-hill run of Sec. 3.1.1 (h_m = 400 m, a = 2 km) on a uniform grid; the
  wavelength of the lee oscillation of w along the x axis through the hill centre at z = 800 m
  (the paper reports about 7 km against 2 pi U / N = 6.3 km from linear theory).

Velocities are evaluated at lattice points as the stored momentum divided by the mean total
density of the eight surrounding cells.  The coarse lattice points sample the reference run by
trilinear interpolation between its lattice points (exact where the lattices coincide: 400 and
200 m; the 250 m points fall half-way between 100 m points on every other index).

Choices the paper leaves open (stated again in the design notes): the time step (a fixed acoustic
Courant number, dt = delta / 800 s), the artificial-diffusion rate (1e-3 1/s in every direction:
the hyper-diffusion coefficient kd delta^4 then vanishes as delta^4 and does not limit the order),
the sponge (Rayleigh damping rising as sin^2 from 10 km to a rate of 0.01 1/s at the lid), and the
evaluation region (every lattice point above the hilltop height, up to the lid, over the whole
horizontal domain).

* ``refined``: the refined-grid experiment of Sec. 3.2.  Flow over the hemisphere of Sec. 3.1.2
  (radius 1 km at (32, 16) km) on cubes of 20^3 cells: level 0 alone (400 m, 64 cubes), levels 0-1
  (148 cubes, 200 m around the hill) and levels 0-2 (232 cubes, 100 m nearest the hill), against the
  uniform 100 m grid (4096 cubes) as reference; w is compared on the x-z section through the hill
  centre and on the horizontal slices at z = 1200 m and 2400 m, per region of the level-2 layout.
  Every run carries the artificial diffusion (``--kd``, 1e-3 1/s by default) and the sponge of the
  other studies (above 10 km), and the refined layouts keep 12 ghost layers, which the diffusion's
  reach of two cells per stage needs over two fine steps.

Both run with the three-stage Runge-Kutta scheme of the (rho theta)' form, or with ``--scheme lf``
with the paper's leap-frog and Robert-Asselin filter in p' form (filter weight ``--nu``).

Usage:  python -m paper_1509_02572_amd.studies convergence [--t-end 3600] [--scheme rk3|lf] [--out FILE]
        python -m paper_1509_02572_amd.studies lee-wave [--delta 100] [--t-end 3600] [--scheme rk3|lf] [--out FILE]
        python -m paper_1509_02572_amd.studies refined [--t-end 3600] [--kd 1e-3] [--max-level 2] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, Optional, Sequence

import numpy as np

from . import workloads as W

LX, LY, LZ = 64000.0, 32000.0, 16000.0  # domain of Sec. 3 [m]
HILL_TOP = 400.0
KD = 1e-3  # artificial-diffusion rate [1/s]
ZSP, RSP = 10000.0, 0.01  # sponge bottom [m] and rate at the lid [1/s]
NU = 0.1  # Robert-Asselin filter weight of the leap-frog scheme
MIN_SPACING = 2000.0  # lee-wave maxima closer than this [m] count as one


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def domain_config(name: str, hill: W.Hill, delta: float, t_end: float, kd: float = KD, rsp: float = RSP,
                  zsp: float = ZSP) -> W.Config:
    """Uniform grid of spacing delta over the 64 x 32 x 16 km domain, hill centred at (32, 16) km
    (terrain heights are sampled with the hill centre on the lattice corner (nx/2, ny/2))."""
    nx, ny, nz = (int(round(L / delta)) for L in (LX, LY, LZ))
    dt = delta / 800.0
    return W.Config(name, nx, ny, nz, delta, delta, delta, hill, u0=10.0, v0=0.0, bvn=0.01, theta0=300.0,
                    dt=dt, nsteps=int(round(t_end / dt)), kdh=kd, kdv=kd, zsp=zsp, rsp=rsp)


def cosine_config(delta: float, t_end: float = 3600.0, **kw) -> W.Config:
    return domain_config(f"cosine{int(delta)}", W.Hill("cosine", HILL_TOP, 2000.0), delta, t_end, **kw)


def bell_config(delta: float, t_end: float = 3600.0, **kw) -> W.Config:
    return domain_config(f"bell{int(delta)}", W.Hill("bell", 400.0, 2000.0), delta, t_end, **kw)


def integrate(cfg: W.Config, prec: str = "f64", every: float = 30.0, scheme: str = "rk3", nu: float = NU):
    """Run cfg.nsteps steps from the initial state; progress on stderr every `every` seconds.
    scheme "rk3": three-stage Runge-Kutta, (rho theta)' form; "lf": the paper's leap-frog with the
    Robert-Asselin filter (weight nu) in p' form (the returned state is q^N)."""
    import torch
    from . import autotune
    from . import cutcell as CC
    dom = CC.Domain(cfg, prec)
    q = dom.init_state()
    tile = autotune.tune(dom, q, dt=cfg.dt, path=None)["tile"]  # untimed: the fastest update form
    r0 = dom.reduce(q)
    a, b, c = q, dom.new_state(), dom.new_state()
    if scheme == "lf":
        dom.pform(a, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for n in range(cfg.nsteps):
        if scheme == "rk3":
            a, b, c = dom.step(a, b, c, cfg.dt)
        else:  # (qbar(n-1), q(n), scratch) in (c, a, b)
            dom.lf_step(c, a, b, cfg.dt, nu, first=(n == 0))
            c, a, b = a, b, c
        if (n + 1) % 200 == 0:
            if (n + 1) % 1600 == 0 and dom.check()[2]:  # stop at the first non-finite value
                raise RuntimeError(f"{cfg.name}: non-finite values by step {n + 1} (t = {(n + 1) * cfg.dt:.0f} s)")
            torch.cuda.synchronize()
            now = time.perf_counter()
            if now - last >= every:
                log(f"  {cfg.name}: step {n + 1}/{cfg.nsteps} (t = {(n + 1) * cfg.dt:.0f} s, {now - t0:.0f} s wall)")
                last = now
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    r1 = dom.reduce(a)
    st = dom.check()
    if st[:5].any():
        raise RuntimeError(f"{cfg.name}: device status counters set: {st}")
    info = {"nx": cfg.nx, "ny": cfg.ny, "nz": cfg.nz, "delta": cfg.dx, "dt": cfg.dt, "steps": cfg.nsteps,
            "scheme": scheme, "tile": tile, "wall_s": round(secs, 2),
            "cell_updates_per_s": cfg.ncells * (3 if scheme == "rk3" else 1) * cfg.nsteps / secs,
            "mass_drift_rel": float(abs(r1[0] - r0[0]) / r0[2])}
    log(f"  {cfg.name}: {cfg.nsteps} steps in {secs:.1f} s, mass drift {info['mass_drift_rel']:.1e}")
    return dom, a, info


def lattice_velocity(dom, q) -> Dict[str, np.ndarray]:
    """u and w at lattice points (I, J, K), K >= 1: momentum over the mean total density of the eight
    surrounding cells (host arrays (nx, ny, nz); K = 0 is left at zero)."""
    s = dom.state_numpy(q)
    rhob = dom.base[: dom.cfg.nz].cpu().numpy()
    rho = s["rho"] + rhob[None, None, :]
    r = rho + np.roll(rho, 1, axis=0)
    r = r + np.roll(r, 1, axis=1)
    rc = np.zeros_like(r)
    rc[:, :, 1:] = (r[:, :, 1:] + r[:, :, :-1]) / 8.0
    out = {}
    for f, m in (("u", "mu"), ("w", "mw")):
        mom = s[m]
        if dom.prec != 0 and f == "u":  # float form: rho u stored as the perturbation from rhobar_c u0
            rbc = np.zeros(dom.cfg.nz)
            rbc[1:] = 0.5 * (rhob[:-1] + rhob[1:])
            mom = mom + rbc[None, None, :] * dom.cfg.u0
        v = np.zeros_like(mom)
        v[:, :, 1:] = mom[:, :, 1:] / rc[:, :, 1:]
        out[f] = v
    return out


def _interp_axis(a: np.ndarray, axis: int, pos: np.ndarray, periodic: bool) -> np.ndarray:
    """Linear interpolation of a along `axis` at fractional indices pos."""
    i0 = np.floor(pos + 1e-9).astype(np.int64)
    w = pos - i0
    n = a.shape[axis]
    i1 = i0 + 1
    if periodic:
        i0, i1 = i0 % n, i1 % n
    else:
        i1 = np.minimum(i1, n - 1)
    sh = [1, 1, 1]
    sh[axis] = len(pos)
    w = w.reshape(sh)
    return np.take(a, i0, axis=axis) * (1.0 - w) + np.take(a, i1, axis=axis) * w


def sample_reference(ref: np.ndarray, dref: float, dc: float, shape_c: Sequence[int]) -> np.ndarray:
    """Reference lattice values at the coarse lattice points (I dc, J dc, K dc)."""
    out = ref
    for ax, n in enumerate(shape_c):
        pos = np.arange(n) * dc / dref
        out = _interp_axis(out, ax, pos, periodic=ax < 2)
    return out


BANDS = ((HILL_TOP, 2000.0), (2000.0, 6000.0), (6000.0, ZSP), (ZSP, LZ))


def error_norms(vc: np.ndarray, vref_c: np.ndarray, dc: float) -> Dict[str, object]:
    """L1 and L2 norms (means over the points) of the difference above the hilltop; the same per
    height band (z in (lo, hi]) as a diagnostic."""
    z = np.arange(vc.shape[2]) * dc
    sel = z > HILL_TOP
    d = (vc - vref_c)[:, :, sel]
    out = {"L1": float(np.abs(d).mean()), "L2": float(np.sqrt((d * d).mean())), "points": int(d.size)}
    bands = {}
    for lo, hi in BANDS:
        m = (z > lo) & (z <= hi)
        if not m.any():
            continue
        db = (vc - vref_c)[:, :, m]
        bands[f"{lo:.0f}-{hi:.0f}"] = {"L1": float(np.abs(db).mean()), "L2": float(np.sqrt((db * db).mean()))}
    out["bands"] = bands
    return out


def convergence(deltas=(400.0, 250.0, 200.0), ref: float = 100.0, t_end: float = 3600.0, prec: str = "f64",
                out: Optional[str] = None, scheme: str = "rk3", nu: float = NU) -> dict:
    import torch
    log(f"convergence: cosine hill, deltas {deltas}, reference {ref} m, t_end {t_end} s, {prec}, {scheme}")
    cfg = cosine_config(ref, t_end)
    dom, q, info_ref = integrate(cfg, prec, scheme=scheme, nu=nu)
    vref = lattice_velocity(dom, q)
    del dom, q
    torch.cuda.empty_cache()
    res = {"case": "cosine hill h_m=400 m a=2 km at (32,16) km, 64x32x16 km, U=10 m/s, N=0.01 1/s",
           "t_end_s": t_end, "prec": prec, "scheme": scheme, "nu": nu if scheme == "lf" else None, "kd_per_s": KD,
           "sponge": {"bottom_m": ZSP, "rate_per_s": RSP},
           "reference": info_ref, "runs": {}}
    for dc in deltas:
        c = cosine_config(dc, t_end)
        d, qc, info = integrate(c, prec, scheme=scheme, nu=nu)
        vc = lattice_velocity(d, qc)
        for f in ("u", "w"):
            info[f] = error_norms(vc[f], sample_reference(vref[f], ref, dc, vc[f].shape), dc)
        log(f"  delta {dc:.0f} m: u L1 {info['u']['L1']:.3e} L2 {info['u']['L2']:.3e}; "
            f"w L1 {info['w']['L1']:.3e} L2 {info['w']['L2']:.3e}")
        res["runs"][str(int(dc))] = info
        del d, qc
        torch.cuda.empty_cache()
    ld = np.log(np.array(deltas))
    res["slopes"] = {}
    for f in ("u", "w"):
        for nrm in ("L1", "L2"):
            e = np.array([res["runs"][str(int(dc))][f][nrm] for dc in deltas])
            res["slopes"][f"{f}_{nrm}"] = round(float(np.polyfit(ld, np.log(e), 1)[0]), 3)
    log("  slopes: " + ", ".join(f"{k} {v:.2f}" for k, v in res["slopes"].items()))
    if out:
        json.dump(res, open(out, "w"), indent=1)
    return res


def lee_wavelength(w_line: np.ndarray, dx: float, x0: float, x_from: float, x_to: float) -> Dict[str, object]:
    """Spacing of the successive maxima of w along x in [x_from, x_to] downstream of the hill centre x0
    (a maximum: positive, larger than the two neighbours on each side, located by a parabola through
    three points; of maxima closer than MIN_SPACING the larger is kept, so small ripples on a crest do
    not count); the wavelength is the mean spacing."""
    x = np.arange(len(w_line)) * dx
    peaks = []
    for n in range(2, len(w_line) - 2):
        if not (x0 + x_from <= x[n] <= x0 + x_to):
            continue
        a, b, c = w_line[n - 1], w_line[n], w_line[n + 1]
        if b > a and b >= c and b > w_line[n - 2] and b >= w_line[n + 2] and b > 0.0:
            den = a - 2.0 * b + c
            xp = x[n] + (0.5 * dx * (a - c) / den if den != 0.0 else 0.0) - x0
            if peaks and xp - peaks[-1][0] < MIN_SPACING:
                if b > peaks[-1][1]:
                    peaks[-1] = (xp, b)
                continue
            peaks.append((xp, b))
    peaks = [p for p, _ in peaks]
    sp = np.diff(peaks)
    return {"wavelength_m": float(sp.mean()) if len(sp) else float("nan"),
            "maxima_m": [round(float(p), 1) for p in peaks], "spacings_m": [round(float(v), 1) for v in sp]}


def lee_wave(delta: float = 100.0, t_end: float = 3600.0, prec: str = "f64", out: Optional[str] = None,
             scheme: str = "rk3", nu: float = NU) -> dict:
    log(f"lee wave: bell hill, delta {delta} m, t_end {t_end} s, {prec}, {scheme}")
    cfg = bell_config(delta, t_end)
    dom, q, info = integrate(cfg, prec, scheme=scheme, nu=nu)
    v = lattice_velocity(dom, q)
    K = int(round(800.0 / delta))
    jc, ic = cfg.ny // 2, cfg.nx // 2
    line = v["w"][:, jc, K]
    res = {"case": "bell hill h_m=400 m a=2 km, 64x32x16 km, U=10 m/s, N=0.01 1/s", "t_end_s": t_end,
           "prec": prec, "run": info, "z_m": K * delta,
           "lee": lee_wavelength(line, delta, ic * delta, 2000.0, 30000.0),
           "linear_theory_m": 2.0 * math.pi * cfg.u0 / cfg.bvn,
           "w_max_800m": float(np.abs(v["w"][:, :, K]).max())}
    x = np.arange(cfg.nx) * delta - ic * delta
    step = max(1, int(round(500.0 / delta)))
    res["w_profile_800m"] = [[round(float(a), 1), round(float(b), 5)] for a, b in zip(x[::step], line[::step])]
    log(f"  lee wavelength at z = {K * delta:.0f} m: {res['lee']['wavelength_m']:.0f} m (maxima at "
        f"{res['lee']['maxima_m']} m downstream); 2 pi U/N = {res['linear_theory_m']:.0f} m")
    if out:
        json.dump(res, open(out, "w"), indent=1)
    return res


# ---- the refined-grid experiment (Sec. 3.2) ----

def trilinear(arr: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Values of arr (nx, ny, nz) at fractional indices p (N, 3); every p + 1 lies inside arr."""
    i0 = np.floor(p + 1e-9).astype(np.int64)
    w = p - i0
    out = np.zeros(len(p))
    for c in range(8):
        o = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        wt = np.prod(np.where(o[None, :] == 1, w, 1.0 - w), axis=1)
        idx = i0 + o[None, :]
        out += wt * arr[idx[:, 0], idx[:, 1], idx[:, 2]]
    return out


def sample_blocks(blocks, targets: np.ndarray, delta0: float) -> np.ndarray:
    """Lattice values at target positions (N, 3) [m] from blocks given as (level, own_lo, own_hi,
    box_org, arr): own range and box origin in level-l global lattice indices, arr the box's lattice
    values.  Each target takes the finest block whose own range holds it (trilinear within the box);
    NaN where none does."""
    out = np.full(len(targets), np.nan)
    done = np.zeros(len(targets), dtype=bool)
    for lev in sorted({b[0] for b in blocks}, reverse=True):
        g = targets / (delta0 / (1 << lev))
        for level, lo, hi, org, arr in blocks:
            if level != lev:
                continue
            m = ~done & np.all((g >= np.array(lo) - 1e-9) & (g < np.array(hi) - 1e-9), axis=1)
            if not m.any():
                continue
            out[m] = trilinear(arr, g[m] - np.array(org, dtype=np.float64)[None, :])
            done |= m
    return out


def uniform_as_block(arr: np.ndarray) -> tuple:
    """A periodic uniform grid's lattice values as one level-0 block (padded by one lattice point in x
    and y with the periodic copies, so interpolation reaches the far side)."""
    pad = np.concatenate([arr, arr[:1]], axis=0)
    pad = np.concatenate([pad, pad[:, :1]], axis=1)
    return (0, (0, 0, 0), arr.shape, (0, 0, 0), pad)


def refined_targets(delta: float = 100.0, zmax: float = 10000.0) -> Dict[str, np.ndarray]:
    """Comparison points: the x-z section through the hill centre (y = 16 km, 0 < z <= zmax) and the
    horizontal slices at z = 1200 m and 2400 m, on the reference lattice."""
    x = np.arange(int(round(LX / delta))) * delta
    y = np.arange(int(round(LY / delta))) * delta
    z = np.arange(1, int(round(zmax / delta)) + 1) * delta
    X, Z = np.meshgrid(x, z, indexing="ij")
    xz = np.stack([X.ravel(), np.full(X.size, LY / 2), Z.ravel()], axis=1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    sl = {f"z{int(h)}": np.stack([X.ravel(), Y.ravel(), np.full(X.size, h)], axis=1) for h in (1200.0, 2400.0)}
    return {"xz": xz, **sl}


def region_of(targets: np.ndarray, levels: int = 3) -> np.ndarray:
    """Finest level of the ``levels``-level layout covering each target (0, 1, 2)."""
    reg = np.zeros(len(targets), dtype=np.int64)
    cube0 = W.CBCM_CUBE * 400.0
    for lev, ((x0, x1), (y0, y1), (z0, z1)) in enumerate(W.cbcm_regions(levels)):
        c = cube0 / (1 << lev)
        m = ((targets[:, 0] >= x0 * c) & (targets[:, 0] < x1 * c) & (targets[:, 1] >= y0 * c)
             & (targets[:, 1] < y1 * c) & (targets[:, 2] >= z0 * c) & (targets[:, 2] < z1 * c))
        reg[m] = lev + 1
    return reg


def diff_norms(w: np.ndarray, wref: np.ndarray, reg: np.ndarray) -> Dict[str, object]:
    """RMS and maximum of w - wref, over all points and per region (finest level of the level-2
    layout there), with the RMS of wref for scale."""
    out = {}
    for name, m in (("all", np.ones(len(w), dtype=bool)), ("L0", reg == 0), ("L1", reg == 1), ("L2", reg == 2)):
        if not m.any():
            continue
        d = w[m] - wref[m]
        out[name] = {"rms": float(np.sqrt(np.mean(d * d))), "max": float(np.abs(d).max()),
                     "ref_rms": float(np.sqrt(np.mean(wref[m] ** 2))), "points": int(m.sum())}
    return out


def integrate_refined(layout, prec: str = "f64", t_end: float = 3600.0, chunk: int = 25, every: float = 30.0):
    """Run a refined layout for t_end (level-0 steps of layout.base.dt, chunk steps per graph launch)."""
    import torch
    from . import autotune
    from . import cutcell as CC
    tile = autotune.tune_refined(layout, prec, path=None)["tile"]
    h = CC.Hierarchy(layout, prec, "cuda:0", tile=tile)
    n0 = int(round(t_end / layout.base.dt))
    torch.cuda.synchronize()
    t0 = last = time.perf_counter()
    done = 0
    while done < n0:
        k = min(chunk, n0 - done)
        h.step(k, use_graph=True)
        done += k
        if done % (8 * chunk) == 0 and h.check()[2]:  # stop at the first non-finite own value
            raise RuntimeError(f"refined layout: non-finite values by level-0 step {done}")
        torch.cuda.synchronize()
        now = time.perf_counter()
        if now - last >= every:
            log(f"  refined {len(layout.blocks)} cubes: level-0 step {done}/{n0} ({now - t0:.0f} s wall)")
            last = now
    secs = time.perf_counter() - t0
    st = h.check()
    if st[:6].any():
        raise RuntimeError(f"refined layout: device status counters set: {st}")
    info = {"cubes": len(layout.blocks), "levels": layout.levels, "tile": tile, "level0_steps": n0,
            "dt0": layout.base.dt, "own_cells": layout.cells(), "wall_s": round(secs, 2)}
    log(f"  refined {len(layout.blocks)} cubes: {n0} level-0 steps in {secs:.1f} s")
    return h, info


def hierarchy_blocks(h) -> list:
    """The lattice w of every block of a hierarchy as sample_blocks entries."""
    out = []
    for m, (b, q) in enumerate(zip(h.layout.blocks, h.current())):
        org, size, gb, gt = h.layout.box(b)
        w = lattice_velocity(h.doms[m], q)["w"]
        out.append((b.level, b.org, tuple(o + s for o, s in zip(b.org, b.size)), org, w))
    return out


def refined(t_end: float = 3600.0, prec: str = "f64", out: Optional[str] = None, kd: float = KD,
            max_level: int = 2, min_level: int = 0, ref_file: Optional[str] = None) -> dict:
    """The runs of levels min_level .. max_level against the uniform 100 m reference; ref_file (npz)
    keeps the reference's samples for later calls with the same t_end and kd."""
    import torch
    from . import cutcell as CC
    log(f"refined-grid experiment: hemisphere, t_end {t_end} s, {prec}")
    tg = refined_targets()
    reg = {k: region_of(v) for k, v in tg.items()}
    res = {"case": "hemisphere r=1 km at (32,16) km, 64x32x16 km, U=10 m/s, N=0.01 1/s, cubes of 20^3 cells, "
                   f"diffusion {kd} 1/s, sponge above {ZSP:.0f} m", "t_end_s": t_end, "prec": prec, "kd_per_s": kd,
           "sponge": {"bottom_m": ZSP, "rate_per_s": RSP}, "runs": {}}
    # reference: uniform 100 m
    base = W.cbcm_hemisphere(1).base.replace(kdh=kd, kdv=kd, zsp=ZSP, rsp=RSP)
    ref_cfg = base.replace(name="cbcm_uniform100", nx=640, ny=320, nz=160, dx=100.0, dy=100.0, dz=100.0,
                           dt=0.125, nsteps=int(round(t_end / 0.125)), H=None)
    import os
    if ref_file and os.path.exists(ref_file):
        z = np.load(ref_file)
        assert float(z["t_end"]) == t_end and float(z["kd"]) == kd, "reference of another run"
        wref = {k: z[k] for k in tg}
        res["reference"] = json.loads(str(z["info"]))
    else:
        dom, q, info = integrate(ref_cfg, prec)
        blk = [uniform_as_block(lattice_velocity(dom, q)["w"])]
        wref = {k: sample_blocks(blk, v, 100.0) for k, v in tg.items()}
        res["reference"] = dict(info, cubes=4096)
        if ref_file:
            np.savez(ref_file, t_end=t_end, kd=kd, info=json.dumps(res["reference"]), **wref)
        del dom, q, blk
        torch.cuda.empty_cache()
    if min_level == 0:
        # level 0 alone: the uniform 400 m grid (one level of cubes steps like the uniform grid, bitwise)
        c0 = base.replace(name="cbcm_level0", nsteps=int(round(t_end / base.dt)), H=None)
        dom, q, info = integrate(c0, prec)
        blk = [uniform_as_block(lattice_velocity(dom, q)["w"])]
        info = dict(info, cubes=64)
        info["w"] = {k: diff_norms(sample_blocks(blk, v, 400.0), wref[k], reg[k]) for k, v in tg.items()}
        res["runs"]["level0"] = info
        del dom, q, blk
        torch.cuda.empty_cache()
    for levels in range(max(2, min_level + 1), max_level + 2):
        lay = W.cbcm_hemisphere(levels, ghost=12)
        lay.base = lay.base.replace(kdh=kd, kdv=kd, zsp=ZSP, rsp=RSP)
        h, info = integrate_refined(lay, prec, t_end)
        blk = hierarchy_blocks(h)
        info["w"] = {k: diff_norms(sample_blocks(blk, v, 400.0), wref[k], reg[k]) for k, v in tg.items()}
        res["runs"][f"level{levels - 1}"] = info
        h.close()
        del h, blk
        torch.cuda.empty_cache()
    for name, r in res["runs"].items():
        log(f"  {name}: " + "; ".join(f"{k} rms {v['all']['rms']:.3e} (L0 {v.get('L0', {}).get('rms', 0):.2e}, "
                                      f"L1 {v.get('L1', {}).get('rms', 0):.2e}, L2 {v.get('L2', {}).get('rms', 0):.2e})"
                                      for k, v in r["w"].items()))
    if out:
        json.dump(res, open(out, "w"), indent=1)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("convergence")
    c.add_argument("--t-end", type=float, default=3600.0)
    c.add_argument("--prec", default="f64", choices=["f32", "f64"])
    c.add_argument("--deltas", default="400,250,200")
    c.add_argument("--ref", type=float, default=100.0)
    c.add_argument("--out", default=None)
    c.add_argument("--scheme", default="rk3", choices=["rk3", "lf"])
    c.add_argument("--nu", type=float, default=NU)
    lw = sub.add_parser("lee-wave")
    lw.add_argument("--delta", type=float, default=100.0)
    lw.add_argument("--t-end", type=float, default=3600.0)
    lw.add_argument("--prec", default="f64", choices=["f32", "f64"])
    lw.add_argument("--out", default=None)
    lw.add_argument("--scheme", default="rk3", choices=["rk3", "lf"])
    lw.add_argument("--nu", type=float, default=NU)
    rf = sub.add_parser("refined")
    rf.add_argument("--t-end", type=float, default=3600.0)
    rf.add_argument("--prec", default="f64", choices=["f32", "f64"])
    rf.add_argument("--out", default=None)
    rf.add_argument("--kd", type=float, default=KD)
    rf.add_argument("--max-level", type=int, default=2, choices=[0, 1, 2])
    rf.add_argument("--min-level", type=int, default=0, choices=[0, 1, 2])
    rf.add_argument("--ref-file", default=None, help="npz keeping the reference's samples between calls")
    a = ap.parse_args(argv)
    if a.cmd == "refined":
        r = refined(a.t_end, a.prec, a.out, a.kd, a.max_level, a.min_level, a.ref_file)
        print(json.dumps({k: v for k, v in r.items()}))
        return
    if a.cmd == "convergence":
        r = convergence(tuple(float(x) for x in a.deltas.split(",")), a.ref, a.t_end, a.prec, a.out, a.scheme,
                        a.nu)
    else:
        r = lee_wave(a.delta, a.t_end, a.prec, a.out, a.scheme, a.nu)
    print(json.dumps({k: v for k, v in r.items() if k != "w_profile_800m"}))


if __name__ == "__main__":
    main()
