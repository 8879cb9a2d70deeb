"""GPU (HIP, through the C ABI) versus the FP64 CPU oracle.

Bars: classification and merge map bit-exact; geometry bit-exact; FP64 state within 1e-12 relative
(per field, L-infinity over the points where the field is defined) after 100 steps; FP32
perturbation form within 1e-5 relative (per field, L2) after 100 steps with mass conserved to
1e-12 of the total mass.  Large configurations are compared on sampled points.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1509_02572_amd import workloads as W

pytestmark = pytest.mark.gpu

CC = None


@pytest.fixture(scope="module", autouse=True)
def _setup():
    global CC
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1509_02572_amd import cutcell
    CC = cutcell
    CC.lib()
    O.build(force=False)


def _ragged():
    hills = [(350.0, 600.0, 900.0, 1100.0), (250.0, 400.0, 2600.0, 500.0)]
    return W.Config("ragged", 37, 29, 23, 100.0, 100.0, 50.0, W.Hill("gauss", extra=hills), u0=7.0,
                    v0=2.5, bvn=0.012, dt=0.05)


def _steep_random():
    for seed in range(1, 200):
        H = W.random_corners(6, 6, 6, 100.0, seed, 0.05, 0.6)
        cfg = W.Config("rand", 6, 6, 6, 100.0, 100.0, 100.0, W.Hill("flat"), H=H, u0=3.0, v0=-2.0, dt=0.02)
        o = O.Oracle(cfg).merge()
        d = np.bincount(o.dir.ravel(), minlength=6)
        if o.counts[0] == 0 and d[2:].sum() > 0:
            return cfg
    raise RuntimeError


def _flat():
    # no terrain above the ground: every cell is regular, the band is empty
    return W.Config("flat", 24, 20, 16, 100.0, 100.0, 50.0, W.Hill("flat"), u0=6.0, v0=1.5, dt=0.05)


SMALL = {
    "flat": _flat,
    "bell32": lambda: W.get("bell32"),
    "hemi_tiny": lambda: W.get("hemi_tiny"),
    "bell_small": lambda: W.get("bell_small"),
    "ragged": _ragged,
    "steep_random": _steep_random,
}


def _masters(o):
    return (o.cls == O.OPEN) | (o.cls == O.ORPHAN)


def _compare_state(o, got, ref, tol, what=""):
    """L-infinity relative error per field over the points where it is defined."""
    nonsolid = o.cls != O.SOLID
    pred = o.vcls == O.PRED
    errs = {}
    for f in ("rho", "rth"):
        scale = max(np.abs(ref[f][nonsolid]).max(), 1e-300)
        errs[f] = np.abs(got[f] - ref[f])[nonsolid].max() / scale
    for f in ("mu", "mv", "mw"):
        for name, m in (("pred", pred), ("diag", ~pred)):
            if not m.any():
                continue
            scale = max(np.abs(ref[f][m]).max(), 1e-300)
            errs[f + "_" + name] = np.abs(got[f] - ref[f])[m].max() / scale
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: {bad} (all: {errs})"
    return errs


# ------------------------------------------------------------------------------------------------
# geometry and merge map: bit-exact
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(SMALL))
def test_geometry_and_merge_map_bitexact(name):
    cfg = SMALL[name]()
    print(f"case {name} {cfg.nx}x{cfg.ny}x{cfg.nz}", flush=True)
    o = O.Oracle(cfg).merge()
    dom = CC.Domain(cfg, "f64")
    g = dom.geometry_numpy()
    for k in ("V", "Ax", "Ay", "Az", "hc", "gx", "gy", "cls", "dir", "vcls", "master", "Vgroup"):
        assert np.array_equal(g[k], getattr(o, k)), k
    assert np.abs(g["nrm"] - o.nrm).max() <= 2e-16
    st = dom.check()
    assert st[0] == o.counts[0] and not st[3:5].any()


@pytest.mark.parametrize("name", ["bell256", "hemi512"])
def test_full_size_geometry_and_merge_map_bitexact(name):
    cfg = W.get(name)
    print(f"case {name} {cfg.nx}x{cfg.ny}x{cfg.nz}", flush=True)
    o = O.Oracle(cfg).merge()
    dom = CC.Domain(cfg, "f64")
    g = dom.geometry_numpy()
    for k in ("V", "Ax", "Ay", "Az", "cls", "dir", "vcls", "master", "Vgroup"):
        assert np.array_equal(g[k], getattr(o, k)), k
    assert o.counts[0] == 0 and not dom.check()[:5].any()


# ------------------------------------------------------------------------------------------------
# FP64: initial state, tendency and 100-step parity
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(SMALL))
def test_f64_initial_state_and_tendency(name):
    cfg = SMALL[name]()
    print(f"case {name}", flush=True)
    o = O.Oracle(cfg).merge()
    dom = CC.Domain(cfg, "f64")
    noise = W.theta_noise(cfg.replace(noise_sigma=0.01, seed=3))
    q = dom.init_state(noise)
    q0 = o.init_state(noise)
    _compare_state(o, dom.state_numpy(q), q0.a, 1e-13, "init")
    # tendency of a random state whose diagnosed points are filled by each side's own diagnostics
    rs = W.random_state(cfg, 17)
    qo = O.State(None, rs)
    o.diagnose(qo)
    qg = dom.new_state()
    for f in O.FIELDS:
        qg.t[f].copy_(dom.pad(rs[f]))
    dom.diagnose(qg)
    _compare_state(o, dom.state_numpy(qg), qo.a, 1e-13, "diagnose")
    dref = o.tendency(qo)
    dgot = dom.state_numpy(dom.tendency(qg))
    pred, mast = o.vcls == O.PRED, _masters(o)
    for f, m in (("rho", mast), ("rth", mast), ("mu", pred), ("mv", pred), ("mw", pred)):
        scale = np.abs(dref[f][m]).max()
        assert np.abs(dgot[f] - dref[f])[m].max() <= 1e-12 * scale, f
        assert not dgot[f][~m].any(), f


@pytest.mark.parametrize("name,steps,tile", [("bell32", 100, 0), ("hemi_tiny", 100, 0), ("bell_small", 100, 0),
                                             ("ragged", 100, 0), ("steep_random", 100, 0),
                                             ("hemi_tiny", 100, 5), ("bell_small", 100, 7)])
def test_f64_state_parity_after_steps(name, steps, tile):
    cfg = SMALL[name]()
    print(f"case {name} steps {steps} tile {tile}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=0.01, seed=1))
    ref = o.run(o.init_state(noise), cfg.dt, steps)
    dom = CC.Domain(cfg, "f64", tile=tile)
    got = dom.run(dom.init_state(noise), cfg.dt, steps)
    torch.cuda.synchronize()
    _compare_state(o, dom.state_numpy(got), ref.a, 1e-12, name)
    st = dom.check()
    assert st[0] == o.counts[0] and st[1] == 0 and st[2] == 0
    # conservation sums agree with the oracle's
    rg, ro = dom.reduce(got), o.reduce(ref)
    assert abs(rg[0] - ro[0]) <= 1e-12 * ro[2] and abs(rg[2] - ro[2]) <= 1e-12 * ro[2]
    assert abs(rg[3] - ro[3]) <= 1e-12 * abs(ro[3])


def test_f64_mass_conservation_and_determinism():
    cfg = W.get("bell_small")
    dom = CC.Domain(cfg, "f64")
    noise = W.theta_noise(cfg)
    q = dom.init_state(noise)
    r0 = dom.reduce(q)
    a = dom.run(q, cfg.dt, 50)
    b = dom.run(q, cfg.dt, 50)
    r1 = dom.reduce(a)
    assert abs(r1[0] - r0[0]) <= 1e-12 * r0[2]
    assert abs(r1[1] - r0[1]) <= 1e-12 * r0[2] * 300
    for f in CC.FIELDS:
        assert torch.equal(a.t[f], b.t[f]), f


def test_rest_stays_at_rest_on_gpu():
    cfg = W.get("hemi_tiny").replace(u0=0.0, v0=0.0)
    o = O.Oracle(cfg).merge()
    from tests.test_oracle_pins import _hydrostatic_state
    q = _hydrostatic_state(o)
    dom = CC.Domain(cfg, "f64")
    qg = dom.new_state()
    for f in O.FIELDS:
        qg.t[f].copy_(dom.pad(q[f]))
    dom.diagnose(qg)
    out = dom.state_numpy(dom.run(qg, cfg.dt, 100))
    for f in ("mu", "mv", "mw"):
        assert np.abs(out[f]).max() <= 1e-10, f


# ------------------------------------------------------------------------------------------------
# FP32 perturbation form against the FP64 oracle
# ------------------------------------------------------------------------------------------------

def _full_from_pert(o, got):
    """Convert the float perturbation state to the paper's variables with the oracle's base state."""
    cfg = o.cfg
    pred = o.vcls == O.PRED
    rbc = np.zeros(cfg.nz)
    rbc[1:] = 0.5 * (o.rhob[:-1] + o.rhob[1:])
    out = dict(got)
    for f, u in (("mu", cfg.u0), ("mv", cfg.v0)):
        full = got[f] + u
        full[pred] = got[f][pred] + (rbc[None, None, :] * u * np.ones(o.shape))[pred]
        out[f] = full
    return out


@pytest.mark.parametrize("name,tile", [("bell_small", 0), ("hemi_tiny", 0), ("ragged", 0), ("hemi_tiny", 2)])
def test_f32_perturbation_error_after_100_steps(name, tile):
    cfg = SMALL[name]()
    print(f"case {name} tile {tile}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=0.01, seed=1))
    ref = o.run(o.init_state(noise), cfg.dt, 100)
    dom = CC.Domain(cfg, "f32", tile=tile)
    q = dom.init_state(noise)
    r0 = dom.reduce(q)
    got = dom.run(q, cfg.dt, 100)
    r1 = dom.reduce(got)
    raw = dom.state_numpy(got)
    g = _full_from_pert(o, raw)
    nonsolid, pred = o.cls != O.SOLID, o.vcls == O.PRED
    errs = {}
    for f, m in (("rho", nonsolid), ("rth", nonsolid), ("mu", pred), ("mv", pred), ("mw", pred),
                 ("mu", ~pred), ("mw", ~pred)):
        e = np.linalg.norm((g[f] - ref[f])[m]) / np.linalg.norm(ref[f][m])
        errs[f + ("" if m is nonsolid or m is pred else "_diag")] = e
    # the horizontal momenta above are dominated by rhobar_c U0; their perturbation from it (what
    # the float form stores) is also held to the bar, relative to its own norm
    rbc = np.zeros(cfg.nz)
    rbc[1:] = 0.5 * (o.rhob[:-1] + o.rhob[1:])
    for f, u in (("mu", cfg.u0), ("mv", cfg.v0)):
        pert_ref = (ref[f] - rbc[None, None, :] * u)[pred]
        if np.linalg.norm(pert_ref) > 0:
            errs[f + "_pert"] = np.linalg.norm(raw[f][pred] - pert_ref) / np.linalg.norm(pert_ref)
    print("f32 errors", name, errs, flush=True)
    for k, e in errs.items():
        assert e <= 1e-5, (k, errs)
    # mass is still conserved to 1e-12 of the total mass
    assert abs(r1[0] - r0[0]) <= 1e-12 * r0[2]


# ------------------------------------------------------------------------------------------------
# full-size configurations: one stage of the timed path on sampled points
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name,prec", [("bell256", "f64"), ("hemi512", "f64"), ("bell256", "f32"),
                                       ("hemi512", "f32")])
def test_full_size_stage_on_sampled_points(name, prec):
    cfg = W.get(name)
    print(f"case {name} {prec}", flush=True)
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg)
    q0 = o.init_state(noise)
    rng = np.random.Generator(np.random.PCG64(5))
    # sample the cut band densely and the rest uniformly
    band = np.flatnonzero(((o.V > 0) & (o.V < 1)).ravel() | (o.vcls != O.PRED).ravel() & (o.cls != O.SOLID).ravel())
    pts = np.concatenate([rng.choice(band, min(4000, band.size), replace=False),
                          rng.integers(0, o.V.size, 4000)])
    L = o.tendency_points(q0, pts)
    cdt = cfg.dt / 3.0
    dom = CC.Domain(cfg, prec)
    qn = dom.init_state(noise)
    qo = dom.new_state()
    dom.rk_stage(qn, qn, qo, cdt)
    got = dom.state_numpy(qo)
    if prec == "f32":
        got = _full_from_pert(o, got)
    mast = _masters(o).ravel()[pts]
    pred = (o.vcls == O.PRED).ravel()[pts]
    tol = 1e-12 if prec == "f64" else 1e-5
    for t, (f, m) in enumerate((("rho", mast), ("rth", mast), ("mu", pred), ("mv", pred), ("mw", pred))):
        ref = q0[f].ravel()[pts] + cdt * L[:, t]
        g = got[f].ravel()[pts]
        scale = max(np.abs(ref[m]).max(), 1e-300)
        err = np.abs(g - ref)[m].max() / scale
        print(f"  {f}: rel err {err:.3e}", flush=True)
        assert err <= tol, (f, err)
    assert not dom.check()[:5].any()


# ------------------------------------------------------------------------------------------------
# error paths (forced from the host; every kernel exits normally)
# ------------------------------------------------------------------------------------------------

def test_error_paths():
    # v-shaped valley: unmergeable cells are counted, as in the oracle
    nx, ny, nz, d = 8, 4, 8, 100.0
    I = np.arange(nx)[:, None] + 0 * np.arange(ny)[None, :]
    H = np.minimum(20.0 + 3.0 * d * np.abs(I - 4).astype(float), 0.6 * nz * d)
    cfg = W.Config("vvalley", nx, ny, nz, d, d, d, W.Hill("flat"), H=H)
    o = O.Oracle(cfg).merge()
    dom = CC.Domain(cfg, "f64")
    rc, host = CC.cutcell_check_status(dom.status)
    assert rc == CC.CC_EUNMERGEABLE and host[0] == o.counts[0] > 0
    assert np.array_equal(dom.geometry_numpy()["cls"], o.cls)
    # a non-finite value in the state is reported after a stage
    cfg = W.get("bell32")
    dom = CC.Domain(cfg, "f64")
    q = dom.init_state()
    q.t["rth"][dom.nzs * 40 + 10] = float("nan")
    s = dom.new_state()
    dom.rk_stage(q, q, s, cfg.dt)
    rc, host = CC.cutcell_check_status(dom.status)
    assert rc == CC.CC_ENONFINITE and host[2] > 0
    # terrain above the allowed band is reported by the geometry call
    H = W.terrain(cfg).copy()
    H[3, 3] = cfg.nz * cfg.dz
    dom = CC.Domain(cfg.replace(H=H), "f64")
    rc, host = CC.cutcell_check_status(dom.status)
    assert host[3] == 1
    # host-side argument errors
    with pytest.raises(RuntimeError, match="alias"):
        dom.rk_stage(q, q, q, 0.1)


# ------------------------------------------------------------------------------------------------
# every tile shape the autotuner can pick computes bitwise the same stage
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name,prec", [("bell256", "f32"), ("bell256", "f64"), ("ragged", "f32"),
                                       ("hemi_tiny", "f64")])
def test_tile_shapes_bitwise_identical(name, prec):
    from paper_1509_02572_amd import autotune
    cfg = W.get(name) if name in W.CONFIGS else SMALL[name]()
    print(f"case {name} {prec}", flush=True)
    dom = CC.Domain(cfg, prec)
    q = dom.init_state(W.theta_noise(cfg.replace(noise_sigma=0.01, seed=2)))
    a = dom.new_state()
    dom.rk_stage(q, q, a, cfg.dt / 3.0)  # a state with non-trivial p' and velocities
    ref = None
    for tid in [0] + list(autotune.TILE_IDS):
        dom.grid.tile = tid
        out = dom.new_state()
        dom.rk_stage(q, a, out, cfg.dt / 2.0, final_stage=True)
        if ref is None:
            ref = out
            continue
        for f in ref.t:
            assert torch.equal(out.t[f], ref.t[f]), (tid, f)
    assert not dom.check()[:5].any()


# ------------------------------------------------------------------------------------------------
# the band-point launch over the listed band tiles (grid with a stage workspace) and over every
# tile below the band height (no workspace) compute bitwise the same stage
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name,prec", [("bell_small", "f32"), ("ragged", "f64"), ("steep_random", "f64")])
def test_band_tile_list_matches_full_band_grid(name, prec):
    cfg = SMALL[name]()
    print(f"case {name} {prec}", flush=True)
    listed = CC.Domain(cfg, prec)
    plain = CC.Domain(cfg, prec, stage_ws=False)
    assert listed.geom.nband_tiles >= 0 and plain.geom.nband_tiles == -1
    assert listed.geom.kband == plain.geom.kband
    noise = W.theta_noise(cfg.replace(noise_sigma=0.01, seed=4))
    a = listed.run(listed.init_state(noise), cfg.dt, 3)
    b = plain.run(plain.init_state(noise), cfg.dt, 3)
    torch.cuda.synchronize()
    for f in a.t:
        assert torch.equal(a.t[f], b.t[f]), f
    assert not listed.check()[:5].any() and not plain.check()[:5].any()


# ------------------------------------------------------------------------------------------------
# one step of a single grid captured into a HIP graph (the band-point launch forked to the side
# stream inside the capture) replays bitwise like eager stepping, with eager work between replays
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_single_grid_graph_replays_match_eager(prec):
    cfg = SMALL["bell_small"]()
    print(f"case graph bell_small {prec}", flush=True)
    dom = CC.Domain(cfg, prec)
    x = dom.init_state(W.theta_noise(cfg.replace(noise_sigma=0.01, seed=6)))
    y, z = dom.new_state(), dom.new_state()
    dom.step(x, y, z, cfg.dt)  # eager first call (creates the side stream); x is only read
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dom.step(x, y, z, cfg.dt)
    torch.cuda.synchronize()
    ea, eb, ec = dom.new_state(), dom.new_state(), dom.new_state()
    for rep in range(3):
        for f in x.t:
            ea.t[f].copy_(x.t[f])
        ref = dom.step(ea, eb, ec, cfg.dt)[0]
        g.replay()
        torch.cuda.synchronize()
        for f in x.t:
            assert torch.equal(y.t[f], ref.t[f]), (rep, f)
        for f in x.t:  # the next replay starts from this one's output
            x.t[f].copy_(y.t[f])
        torch.cuda.synchronize()
    assert not dom.check()[:5].any()


def test_flat_terrain_f64_parity():
    """Flat ground: only the regular update runs (no band).  Without terrain the flow stays close to
    the reference state, so the perturbations are driven by a 1 K theta' noise, large enough that
    they stand well above the FP64 rounding of the base-state fluxes the oracle sums and the kernel
    cancels exactly."""
    cfg = _flat()
    o = O.Oracle(cfg).merge()
    noise = W.theta_noise(cfg.replace(noise_sigma=1.0, seed=1))
    ref = o.run(o.init_state(noise), cfg.dt, 20)
    dom = CC.Domain(cfg, "f64")
    got = dom.run(dom.init_state(noise), cfg.dt, 20)
    torch.cuda.synchronize()
    _compare_state(o, dom.state_numpy(got), ref.a, 1e-12, "flat")
    assert not dom.check()[:5].any()


def test_flat_terrain_has_no_band():
    """Over flat ground every point is regular (the ground row of lattice points is never
    predicted and the ground closes the bottom faces): the band height is 1 and no band tile is
    listed, so the update is the regular-point launch alone."""
    dom = CC.Domain(_flat(), "f64")
    assert dom.geom.kband == 1 and dom.geom.nband_tiles == 0
    colk = dom.g["colk"].cpu().numpy().reshape(3, -1)
    assert colk[0].max() == 0 and colk[1].max() == 1


# ------------------------------------------------------------------------------------------------
# two grids stepped at once on two streams (each with its own stage context) match serial stepping
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_two_grids_on_two_streams_match_serial(prec):
    cfgs = [SMALL["bell_small"](), SMALL["ragged"]()]
    print(f"case two streams {prec}", flush=True)
    doms = [CC.Domain(c, prec, tile=21) for c in cfgs]
    noise = [W.theta_noise(c.replace(noise_sigma=0.01, seed=8)) for c in cfgs]
    ref = [d.run(d.init_state(n), c.dt, 4) for d, c, n in zip(doms, cfgs, noise)]
    torch.cuda.synchronize()
    starts = [d.init_state(n) for d, n in zip(doms, noise)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    bufs = [(q, d.new_state(), d.new_state()) for d, q in zip(doms, starts)]
    torch.cuda.synchronize()
    for _ in range(4):  # interleave the two grids' stages on their own streams
        for m in range(2):
            with torch.cuda.stream(streams[m]):
                a, b, c = bufs[m]
                bufs[m] = doms[m].step(a, b, c, cfgs[m].dt)
    torch.cuda.synchronize()
    for m in range(2):
        for f in ref[m].t:
            assert torch.equal(bufs[m][0].t[f], ref[m].t[f]), (m, f)
        assert not doms[m].check()[:5].any()
