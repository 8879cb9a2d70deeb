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

Both run with the three-stage Runge-Kutta scheme of the (rho theta)' form, or with ``--scheme lf``
with the paper's leap-frog and Robert-Asselin filter in p' form (filter weight ``--nu``).

Usage:  python -m paper_1509_02572_amd.studies convergence [--t-end 3600] [--scheme rk3|lf] [--out FILE]
        python -m paper_1509_02572_amd.studies lee-wave [--delta 100] [--t-end 3600] [--scheme rk3|lf] [--out FILE]
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
    a = ap.parse_args(argv)
    if a.cmd == "convergence":
        r = convergence(tuple(float(x) for x in a.deltas.split(",")), a.ref, a.t_end, a.prec, a.out, a.scheme,
                        a.nu)
    else:
        r = lee_wave(a.delta, a.t_end, a.prec, a.out, a.scheme, a.nu)
    print(json.dumps({k: v for k, v in r.items() if k != "w_profile_800m"}))


if __name__ == "__main__":
    main()
