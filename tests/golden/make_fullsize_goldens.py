"""Write the expected values of the full-size 100-step parity tests (bell256 and hemi512).

Calls only the FP64 CPU oracle (``oracle/``) and the seeded input generators of the package
(``workloads``: terrain, theta' noise).  For each workload it runs the oracle through 100
three-stage Runge-Kutta steps from the initial state and stores, in ``<name>_100steps.npz``:

* ``idx``: linear cell/lattice indices (unpadded nx*ny*nz layout, k fastest) of the sample: every
  point of the terrain band (cells that are cut, merged, absorbed or orphans; lattice points that are
  not predicted, except ground points under flat terrain) and 20 000 uniformly drawn points (PCG64,
  seed 12345);
* ``rho, rth, mu, mv, mw``: the oracle's state at those points after 100 steps;
* ``cls, vcls``: the cell class and lattice-point class of each sampled point;
* ``linf_<field>``, ``l2_<field>``: full-field norms of the final oracle state over the points where
  the field is defined (scalars: non-solid cells; momenta: predicted points ``_pred`` and diagnosed
  points ``_diag``);
* ``reduce0``, ``reduce1``: the conservation sums (M', Theta', M_total, E) of the initial and final
  states;
* ``steps``, ``dt``.

Usage: python tests/golden/make_fullsize_goldens.py [bell256|hemi512 ...]   (OMP threads from the
environment).  bell256 takes about 20 minutes on 8 cores, hemi512 about two hours.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1509_02572_amd import workloads as W  # noqa: E402

STEPS = 100
NRANDOM = 20000


def sample_points(o) -> np.ndarray:
    cls, vcls, V = o.cls.ravel(), o.vcls.ravel(), o.V.ravel()
    H = o.H
    nz = o.cfg.nz
    cut = (V > 0) & (V < 1)
    band_cells = (cls != O.SOLID) & (cut | (cls != O.OPEN))
    hcol = np.repeat(H.ravel(), nz)
    band_lat = (vcls == O.MFACE) | ((vcls == O.GROUND) & (hcol > 0))
    band = np.flatnonzero(band_cells | band_lat)
    rng = np.random.Generator(np.random.PCG64(12345))
    rand = rng.integers(0, cls.size, NRANDOM)
    return np.unique(np.concatenate([band, rand]))


def norms(o, q):
    nonsolid = (o.cls != O.SOLID)
    pred = o.vcls == O.PRED
    out = {}
    for f in ("rho", "rth"):
        v = q[f][nonsolid]
        out[f"linf_{f}"] = np.abs(v).max()
        out[f"l2_{f}"] = np.linalg.norm(v)
    for f in ("mu", "mv", "mw"):
        for name, m in (("pred", pred), ("diag", ~pred)):
            v = q[f][m]
            out[f"linf_{f}_{name}"] = np.abs(v).max() if v.size else 0.0
            out[f"l2_{f}_{name}"] = np.linalg.norm(v)
    return out


def make(name: str) -> str:
    cfg = W.get(name)
    t0 = time.perf_counter()
    o = O.Oracle(cfg).merge()
    assert o.counts[0] == 0, "unmergeable cells"
    q0 = o.init_state(W.theta_noise(cfg))
    r0 = o.reduce(q0)
    print(f"{name}: setup {time.perf_counter() - t0:.1f} s, {O.set_threads(0)} threads", flush=True)
    q = q0
    chunk = 10
    for s in range(0, STEPS, chunk):
        t1 = time.perf_counter()
        q = o.run(q, cfg.dt, chunk)
        print(f"{name}: steps {s + chunk}/{STEPS} ({time.perf_counter() - t1:.1f} s)", flush=True)
    assert o.counts[1] == 0, "corners without a nearest plane"
    r1 = o.reduce(q)
    idx = sample_points(o)
    out = {"idx": idx, "cls": o.cls.ravel()[idx], "vcls": o.vcls.ravel()[idx], "reduce0": r0, "reduce1": r1,
           "steps": np.int64(STEPS), "dt": np.float64(cfg.dt)}
    for f in O.FIELDS:
        out[f] = q[f].ravel()[idx]
    out.update(norms(o, q))
    path = os.path.join(HERE, f"{name}_100steps.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: {idx.size} points -> {path} ({time.perf_counter() - t0:.0f} s total)", flush=True)
    return path


if __name__ == "__main__":
    O.build(force=False)
    for n in sys.argv[1:] or ["bell256", "hemi512"]:
        make(n)
