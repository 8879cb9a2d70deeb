"""GPU leap-frog with the Robert-Asselin filter in p' form (Sec. 2.2, eq. heat) against the FP64 CPU
oracle: the p' conversion, a forward first step, 60 steps in FP64 at 1e-12 (with and without
diffusion and sponge, over smooth and steep terrain), the float form at 1e-5 (L2) with mass conserved
to 1e-12; argument checks on the host side."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1509_02572_amd import workloads as W

pytestmark = pytest.mark.gpu

CC = None
NU = 0.1


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
    "hemi_tiny": lambda: W.get("hemi_tiny"),
    "bell_small": lambda: W.get("bell_small"),
    "steep_random": _steep_random,
    "hemi_tiny_diff_sponge": lambda: W.get("hemi_tiny").replace(kdh=0.05, kdv=0.05, zsp=700.0, rsp=0.05),
}


def _masks(o):
    return o.cls != O.SOLID, o.vcls == O.PRED


def _compare(o, got, ref, tol):
    nonsolid, pred = _masks(o)
    for f, m in (("rho", nonsolid), ("rth", nonsolid), ("mu", pred), ("mv", pred), ("mw", pred),
                 ("mu", ~pred), ("mw", ~pred)):
        scale = max(np.abs(ref[f][m]).max(), 1e-300)
        err = np.abs(got[f] - ref[f])[m].max() / scale
        assert err <= tol, (f, err)


def test_f64_pform_conversion():
    cfg = W.get("hemi_tiny")
    print("case lf pform hemi_tiny", flush=True)
    o = O.Oracle(cfg).merge()
    dom = CC.Domain(cfg, "f64")
    rs = W.random_state(cfg, 31)
    q = dom.new_state()
    for f in O.FIELDS:
        q.t[f].copy_(dom.pad(rs[f]))
    dom.pform(q, True)
    ref = o.pform(O.State(None, rs), True)
    got = dom.state_numpy(q)
    ns = o.cls != O.SOLID
    assert np.abs(got["rth"] - ref.a["rth"])[ns].max() <= 1e-13 * np.abs(ref.a["rth"][ns]).max()
    dom.pform(q, False)
    back = dom.state_numpy(q)
    assert np.abs(back["rth"] - rs["rth"])[ns].max() <= 1e-13 * np.abs(rs["rth"]).max()


@pytest.mark.parametrize("name", list(CASES))
def test_f64_leapfrog_against_oracle(name):
    cfg = CASES[name]()
    print(f"case lf f64 {name}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=0.5, seed=9))
    q0 = o.pform(o.init_state(noise), True)
    n = 60
    ref_n, ref_b = o.run_lf(q0, cfg.dt, n, NU)
    dom = CC.Domain(cfg, "f64")
    q = dom.pform(dom.init_state(noise), True)
    got_n, got_b = dom.run_lf(q, cfg.dt, n, NU)
    _compare(o, dom.state_numpy(got_n), ref_n.a, 1e-12)
    nonsolid, pred = _masks(o)
    gb = dom.state_numpy(got_b)
    masters = (o.cls == O.OPEN) | (o.cls == O.ORPHAN)
    for f, m in (("rho", masters), ("rth", masters), ("mu", pred), ("mv", pred), ("mw", pred)):
        err = np.abs(gb[f] - ref_b.a[f])[m].max() / max(np.abs(ref_b.a[f][m]).max(), 1e-300)
        assert err <= 1e-12, ("filtered", f, err)
    assert not dom.check()[:5].any()


def test_f64_forward_first_step():
    cfg = W.get("bell_small")
    print("case lf first step bell_small", flush=True)
    o = O.Oracle(cfg).merge()
    rs = W.random_state(cfg, 17)
    qo = O.State(None, rs)
    o.diagnose(qo)
    qo = o.pform(qo, True)
    ref = o.lf_step(None, qo.copy(), 0.05, NU, first=True)
    dom = CC.Domain(cfg, "f64")
    q = dom.new_state()
    for f in O.FIELDS:
        q.t[f].copy_(dom.pad(qo.a[f]))
    qp = dom.new_state()
    dom.lf_step(None, q, qp, 0.05, NU, first=True)
    _compare(o, dom.state_numpy(qp), ref.a, 1e-12)
    # the first step leaves q_0 untouched
    back = dom.state_numpy(q)
    for f in O.FIELDS:
        assert np.array_equal(back[f], qo.a[f]), f


@pytest.mark.parametrize("name", ["hemi_tiny", "bell_small"])
def test_f32_leapfrog_against_oracle(name):
    cfg = CASES[name]()
    print(f"case lf f32 {name}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=0.5, seed=9))
    n = 60
    qi = o.init_state(noise)
    ref_n, _ = o.run_lf(o.pform(qi, True), cfg.dt, n, NU)
    dom = CC.Domain(cfg, "f32")
    q = dom.init_state(noise)
    r0 = dom.reduce(q)
    dom.pform(q, True)
    got_n, got_b = dom.run_lf(q, cfg.dt, n, NU)
    raw = dom.state_numpy(got_n)
    nonsolid, pred = _masks(o)
    rbc = np.zeros(cfg.nz)
    rbc[1:] = 0.5 * (o.rhob[:-1] + o.rhob[1:])
    full = dict(raw)
    for f, u in (("mu", cfg.u0), ("mv", cfg.v0)):
        full[f] = np.where(pred, raw[f] + rbc[None, None, :] * u, raw[f] + u)
    for f, m in (("rho", nonsolid), ("rth", nonsolid), ("mu", pred), ("mv", pred), ("mw", pred)):
        e = np.linalg.norm((full[f] - ref_n.a[f])[m]) / np.linalg.norm(ref_n.a[f][m])
        assert e <= 1e-5, (f, e)
    # M' is read from rho' alone, which the p' form leaves as it is
    for s in (got_n, got_b):
        r = dom.reduce(s)
        assert abs(r[0] - r0[0]) <= 1e-12 * r0[2], (r[0], r0[0])


def test_lf_argument_checks():
    cfg = W.get("hemi_tiny")
    dom = CC.Domain(cfg, "f64")
    q0, qp = dom.init_state(), dom.new_state()
    with pytest.raises(RuntimeError, match="distinct"):
        dom.lf_step(q0, q0, qp, 0.05, NU)
    with pytest.raises(RuntimeError, match="filter weight"):
        dom.lf_step(qp, q0, dom.new_state(), 0.05, 0.9)
    with pytest.raises(RuntimeError, match="dt must be positive"):
        dom.lf_step(None, q0, qp, -1.0, NU, first=True)
