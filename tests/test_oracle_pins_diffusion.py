"""Pins of the oracle's fourth-order artificial diffusion (no GPU).

The paper adds a fourth-order artificial diffusion to every prognostic equation (Sec. 2.1), computed
with a 5-point stencil per direction (Sec. 2.2), and a second-order term where the stencil lacks
fluid neighbours, with the terrain as boundary (Sec. 2.4); it gives no coefficient.  The oracle
writes it in flux form (see cutcell_oracle.c).  The pins:

* a discrete Fourier mode is damped at exactly the rate -k 16 sin^4(kappa dx / 2) in x, y and z
  (scalars and momentum), away from the ground and the lid;
* a linear profile in z feels the second-order fallback only at the two levels next to the ground
  and to the lid, in closed form (+-4 k b), and nothing in between;
* a face-list scatter form (every face visited once, its flux added to both sides) reproduces the
  oracle's per-group gather on steep random terrain with merged cells;
* mass and (rho theta)' stay conserved over steps with diffusion on steep terrain.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_02572_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


KH, KV = 0.7, 0.3  # rates [1/s]; large values make the diffusion dominate the checks


def _flat(nx=16, ny=12, nz=16, **kw):
    return W.Config("flatdiff", nx, ny, nz, 100.0, 80.0, 50.0, W.Hill("flat"), u0=0.0, v0=0.0, dt=0.05, **kw)


def _diffusion_only(cfg, q):
    """Tendency with diffusion minus tendency without: the diffusion term alone."""
    a = O.Oracle(cfg.replace(kdh=KH, kdv=KV)).merge().tendency(q)
    b = O.Oracle(cfg).merge().tendency(q)
    return {f: a[f] - b[f] for f in O.FIELDS}


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fourier_mode_damping_rate(axis):
    cfg = _flat()
    o = O.Oracle(cfg).merge()
    n = (cfg.nx, cfg.ny, cfg.nz)[axis]
    m = 3
    idx = np.arange(n)
    if axis < 2:  # periodic: cos(2 pi m i / n)
        wave = np.cos(2 * np.pi * m * idx / n)
        kappa_d = 2 * np.pi * m / n
    else:  # any cosine; checked on levels with the full stencil only
        wave = np.cos(0.7 * idx)
        kappa_d = 0.7
    shape = [1, 1, 1]
    shape[axis] = n
    field = np.broadcast_to(wave.reshape(shape), o.shape)
    q = O.State(o.shape)
    q.a["rho"][...] = 1e-3 * field
    q.a["rth"][...] = 0.2 * field
    pred = o.vcls == O.PRED
    for c, f in enumerate(("mu", "mv", "mw")):
        q.a[f][pred] = (0.5 + c) * 1e-3 * field[pred]
    d = _diffusion_only(cfg, q)
    rate = -(KV if axis == 2 else KH) * 16.0 * math.sin(kappa_d / 2.0) ** 4
    K = np.broadcast_to(np.arange(cfg.nz)[None, None, :], o.shape)
    cells = (K >= 2) & (K <= cfg.nz - 3) if axis == 2 else np.ones(o.shape, bool)
    points = pred & ((K >= 3) & (K <= cfg.nz - 3) if axis == 2 else (K >= 1))
    for f in ("rho", "rth"):
        want = rate * q.a[f][cells]
        assert np.abs(d[f][cells] - want).max() <= 1e-12 * np.abs(want).max(), f
    for f in ("mu", "mv", "mw"):
        want = rate * q.a[f][points]
        assert np.abs(d[f][points] - want).max() <= 1e-12 * np.abs(want).max(), f


def test_linear_profile_sees_fallback_only_at_ground_and_lid():
    cfg = _flat()
    o = O.Oracle(cfg).merge()
    nz = cfg.nz
    b = 2e-4
    K = np.arange(nz)[None, None, :] * np.ones(o.shape)
    q = O.State(o.shape)
    q.a["rho"][...] = 1e-3 + b * K
    pred = o.vcls == O.PRED
    q.a["mu"][pred] = (3e-3 + b * K)[pred]
    d = _diffusion_only(cfg, q)
    want = np.zeros(nz)
    want[0], want[1], want[nz - 2], want[nz - 1] = 4 * KV * b, -4 * KV * b, 4 * KV * b, -4 * KV * b
    assert np.abs(d["rho"] - want[None, None, :]).max() <= 1e-12 * 4 * KV * b
    # lattice points: predicted at 1 <= K <= nz-1; the ground row and the lid act as boundary
    wm = np.zeros(nz)
    wm[1], wm[2], wm[nz - 2], wm[nz - 1] = 4 * KV * b, -4 * KV * b, 4 * KV * b, -4 * KV * b
    got = d["mu"][pred].reshape(cfg.nx, cfg.ny, nz - 1)
    assert np.abs(got - wm[None, None, 1:]).max() <= 1e-12 * 4 * KV * b
    assert not d["rth"].any() and not d["mv"].any() and not d["mw"].any()


def _steep_random_cfg():
    for seed in range(1, 200):
        H = W.random_corners(6, 6, 6, 100.0, seed, 0.05, 0.6)
        cfg = W.Config("rand", 6, 6, 6, 100.0, 100.0, 100.0, W.Hill("flat"), H=H, u0=3.0, v0=-2.0, dt=0.02)
        o = O.Oracle(cfg).merge()
        d = np.bincount(o.dir.ravel(), minlength=6)
        if o.counts[0] == 0 and d[2:].sum() > 0:
            return cfg
    raise RuntimeError


def test_scatter_form_matches_gather_on_steep_terrain():
    """Every face visited once: its flux (third difference of the four group values straddling it,
    -4 x the first difference when an outer cell is solid or outside, nothing through closed or
    group-internal faces) times rate x aperture, subtracted from the lower group and added to the
    upper one, divided by the group volume."""
    cfg = _steep_random_cfg()
    o = O.Oracle(cfg).merge()
    assert ((o.cls == O.ABSORBED).sum() > 0)
    rs = W.random_state(cfg, 5)
    q = O.State(None, rs)
    d = _diffusion_only(cfg, q)
    nx, ny, nz = o.shape
    master = o.master.reshape(-1)
    V = o.V.reshape(-1)
    acc = {f: np.zeros(nx * ny * nz) for f in ("rho", "rth")}
    lin = lambda i, j, k: ((i % nx) * ny + (j % ny)) * nz + k
    for a in range(3):
        A = (o.Ax, o.Ay, o.Az)[a].reshape(-1)
        rate = KV if a == 2 else KH
        for i in range(nx):
            for j in range(ny):
                for k in range(nz):
                    e = [0, 0, 0]
                    e[a] = 1
                    if a == 2 and k == 0:
                        continue
                    U, L = lin(i, j, k), lin(i - e[0], j - e[1], k - e[2])
                    if A[U] == 0.0 or master[U] == master[L]:
                        continue
                    outer = not (a == 2 and (k - 2 < 0 or k + 1 >= nz))
                    if outer:
                        L2, U2 = lin(i - 2 * e[0], j - 2 * e[1], k - 2 * e[2]), lin(i + e[0], j + e[1], k + e[2])
                        outer = V[L2] > 0 and V[U2] > 0
                    for f in ("rho", "rth"):
                        v = q.a[f].reshape(-1)
                        pl, pu = v[master[L]], v[master[U]]
                        F = ((v[master[U2]] - 3.0 * pu) + 3.0 * pl) - v[master[L2]] if outer else -4.0 * (pu - pl)
                        acc[f][master[L]] += rate * A[U] * F
                        acc[f][master[U]] -= rate * A[U] * F
    masters = ((o.cls == O.OPEN) | (o.cls == O.ORPHAN)).reshape(-1)
    Vg = o.Vgroup.reshape(-1)
    for f in ("rho", "rth"):
        want = -acc[f][masters] / Vg[masters]
        got = d[f].reshape(-1)[masters]
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), f


@pytest.mark.parametrize("name", ["hemi_tiny", "steep_random"])
def test_mass_conserved_with_diffusion(name):
    cfg = (W.get(name) if name != "steep_random" else _steep_random_cfg()).replace(kdh=0.05, kdv=0.05)
    o = O.Oracle(cfg).merge()
    q0 = o.init_state(W.theta_noise(cfg.replace(noise_sigma=0.5, seed=2)))
    r0 = o.reduce(q0)
    q1 = o.run(q0, cfg.dt, 20)
    r1 = o.reduce(q1)
    assert abs(r1[0] - r0[0]) <= 1e-12 * r0[2]
    assert abs(r1[1] - r0[1]) <= 1e-12 * r0[2] * 300
    # and the diffusion is active: the run differs from one without it
    q2 = O.Oracle(cfg.replace(kdh=0.0, kdv=0.0)).merge().run(q0, cfg.dt, 20)
    assert np.abs(q1["rho"] - q2["rho"]).max() > 0
