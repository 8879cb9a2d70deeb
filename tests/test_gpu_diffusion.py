"""GPU fourth-order artificial diffusion (with the second-order fallback near terrain) against the
FP64 CPU oracle: tendency and 100-step states in FP64 at 1e-12, the FP32 form at 1e-5 (L2) with
mass conserved to 1e-12; batches refuse a non-zero rate."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1509_02572_amd import workloads as W

pytestmark = pytest.mark.gpu

CC = None
KH, KV = 0.08, 0.05  # rates [1/s]; dt (32 KH + 16 KV) stays well inside the stable range


@pytest.fixture(scope="module", autouse=True)
def _setup():
    global CC
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1509_02572_amd import cutcell
    CC = cutcell
    CC.lib()
    O.build(force=False)


def _steep_random():
    for seed in range(1, 200):
        H = W.random_corners(6, 6, 6, 100.0, seed, 0.05, 0.6)
        cfg = W.Config("rand", 6, 6, 6, 100.0, 100.0, 100.0, W.Hill("flat"), H=H, u0=3.0, v0=-2.0, dt=0.02)
        o = O.Oracle(cfg).merge()
        d = np.bincount(o.dir.ravel(), minlength=6)
        if o.counts[0] == 0 and d[2:].sum() > 0:
            return cfg
    raise RuntimeError


CASES = {
    "flat": lambda: W.Config("flat", 24, 20, 16, 100.0, 100.0, 50.0, W.Hill("flat"), u0=6.0, v0=1.5, dt=0.05),
    "bell_small": lambda: W.get("bell_small"),
    "hemi_tiny": lambda: W.get("hemi_tiny"),
    "steep_random": _steep_random,
}


def _cfg(name):
    return CASES[name]().replace(kdh=KH, kdv=KV)


@pytest.mark.parametrize("name", list(CASES))
def test_f64_tendency_with_diffusion(name):
    cfg = _cfg(name)
    print(f"case diffusion tendency {name}", flush=True)
    o = O.Oracle(cfg).merge()
    dom = CC.Domain(cfg, "f64")
    rs = W.random_state(cfg, 23)
    qo = O.State(None, rs)
    o.diagnose(qo)
    qg = dom.new_state()
    for f in O.FIELDS:
        qg.t[f].copy_(dom.pad(rs[f]))
    dom.diagnose(qg)
    dref = o.tendency(qo)
    dgot = dom.state_numpy(dom.tendency(qg))
    pred, mast = o.vcls == O.PRED, (o.cls == O.OPEN) | (o.cls == O.ORPHAN)
    for f, m in (("rho", mast), ("rth", mast), ("mu", pred), ("mv", pred), ("mw", pred)):
        scale = np.abs(dref[f][m]).max()
        err = np.abs(dgot[f] - dref[f])[m].max() / scale
        assert err <= 1e-12, (f, err)


@pytest.mark.parametrize("name", ["bell_small", "hemi_tiny", "steep_random"])
def test_f64_state_with_diffusion_after_100_steps(name):
    cfg = _cfg(name)
    print(f"case diffusion f64 100 steps {name}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=0.5, seed=3))
    ref = o.run(o.init_state(noise), cfg.dt, 100)
    dom = CC.Domain(cfg, "f64")
    got = dom.state_numpy(dom.run(dom.init_state(noise), cfg.dt, 100))
    nonsolid, pred = o.cls != O.SOLID, o.vcls == O.PRED
    for f, m in (("rho", nonsolid), ("rth", nonsolid), ("mu", pred), ("mv", pred), ("mw", pred),
                 ("mu", ~pred), ("mw", ~pred)):
        scale = max(np.abs(ref[f][m]).max(), 1e-300)
        err = np.abs(got[f] - ref[f])[m].max() / scale
        assert err <= 1e-12, (f, err)
    assert not dom.check()[:5].any()


@pytest.mark.parametrize("name", ["bell_small", "hemi_tiny"])
def test_f32_with_diffusion_after_100_steps(name):
    cfg = _cfg(name)
    print(f"case diffusion f32 100 steps {name}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=0.5, seed=3))
    ref = o.run(o.init_state(noise), cfg.dt, 100)
    dom = CC.Domain(cfg, "f32")
    q = dom.init_state(noise)
    r0 = dom.reduce(q)
    out = dom.run(q, cfg.dt, 100)
    r1 = dom.reduce(out)
    raw = dom.state_numpy(out)
    pred, nonsolid = o.vcls == O.PRED, o.cls != O.SOLID
    rbc = np.zeros(cfg.nz)
    rbc[1:] = 0.5 * (o.rhob[:-1] + o.rhob[1:])
    full = dict(raw)
    for f, u in (("mu", cfg.u0), ("mv", cfg.v0)):
        full[f] = np.where(pred, raw[f] + rbc[None, None, :] * u, raw[f] + u)
    for f, m in (("rho", nonsolid), ("rth", nonsolid), ("mu", pred), ("mv", pred), ("mw", pred)):
        e = np.linalg.norm((full[f] - ref[f])[m]) / np.linalg.norm(ref[f][m])
        assert e <= 1e-5, (f, e)
    assert abs(r1[0] - r0[0]) <= 1e-12 * r0[2]


def test_batch_runs_the_diffusion():
    cfg = _cfg("bell_small")
    print("case batch diffusion", flush=True)
    # a batch of one member runs the sponge (and diffusion) in flux form over the whole grid: the
    # same terms as the single grid up to rounding order (bar: 1e-12 of each field's total magnitude)
    dom = CC.Domain(cfg, "f64", side_stream=False)
    q0 = dom.init_state(W.theta_noise(cfg.replace(noise_sigma=0.5, seed=9)))
    batch = CC.Batch([dom], [q0])
    batch.step(cfg.dt, 4)
    torch.cuda.synchronize()
    ref = dom.state_numpy(dom.run(q0, cfg.dt, 4))
    got = dom.state_numpy(batch.current()[0])
    nz = cfg.nz
    mom = max(np.abs(ref[f]).max() for f in ("mu", "mv", "mw"))
    base = {"rho": dom.base[:nz].abs().max().item(), "rth": dom.base[nz:2 * nz].abs().max().item()}
    for f in CC.FIELDS:
        scale = np.abs(ref[f]).max() + base[f] if f in base else mom
        assert np.abs(got[f] - ref[f]).max() <= 1e-12 * scale, f
    assert not batch.check()[:5].any()
    batch.close()
