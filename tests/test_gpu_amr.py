"""Refined grids (Sec. 2.2) through amr_hierarchy_create / amr_block_step, against the refined-grid
oracle and the properties it is pinned to.

Bars: a single level of blocks reproduces the uniform-grid kernels bitwise; three levels agree with
the oracle to 1e-12 (FP64, L-infinity over own cells relative to the field's maximum) and the float
form to 1e-5 (L2 per field over own cells); mass and
(rho theta)' are conserved to 1e-12 of the total mass (both precisions); graph replays reproduce
eager stepping bitwise.
"""
import numpy as np
import pytest
import torch

from oracle import amr_oracle as A
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


def small_layout():
    base = W.Config("amr_test", 16, 16, 24, 200.0, 200.0, 200.0, W.Hill("hemisphere", 0.0, 600.0), dt=0.2)
    return W.amr_layout(base, levels=3, brick=8, ghost=6, d_fine=300.0, band=400.0, seed=1)


def _gpu_mass(h):
    mp = tp = mt = 0.0
    for m, q in enumerate(h.current()):
        d = h.doms[m]
        (i0, j0, k0), (i1, j1, k1) = h.own[m]
        V = d.unpad(d.g["V"])[i0:i1, j0:j1, k0:k1]
        rhob = d.base[:d.cfg.nz].cpu().numpy()[k0:k1]
        own = h.own_cells(m, q)
        dv = d.cfg.dx * d.cfg.dy * d.cfg.dz
        mp += float((V * own["rho"]).sum()) * dv
        tp += float((V * own["rth"]).sum()) * dv
        mt += float((V * (own["rho"] + rhob[None, None, :])).sum()) * dv
    return mp, tp, mt


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_level_equals_uniform_grid_bitwise(prec):
    base = W.Config("one", 32, 32, 16, 100.0, 100.0, 100.0, W.Hill("bell", 400.0, 600.0), dt=0.1, u0=8.0, v0=3.0)
    lay = W.amr_layout(base, levels=1, brick=8, ghost=6, seed=2)
    print("case single level", prec, len(lay.blocks), flush=True)
    h = CC.Hierarchy(lay, prec)
    h.step(3)
    dom = CC.Domain(base, prec)
    q = dom.run(dom.init_state(), base.dt, 3)
    torch.cuda.synchronize()
    ref = dom.state_numpy(q)
    for m, (b, qb) in enumerate(zip(lay.blocks, h.current())):
        own = h.own_cells(m, qb)
        sl = tuple(slice(o, o + s) for o, s in zip(b.org, b.size))
        for f in CC.FIELDS:
            assert np.array_equal(own[f], ref[f][sl]), (m, f)
    assert not h.check()[:6].any()


def test_three_levels_against_oracle():
    lay = small_layout()
    print("case three levels", len(lay.blocks), flush=True)
    steps = 2
    h = CC.Hierarchy(lay, "f64")
    h.step(steps)
    torch.cuda.synchronize()
    a = A.AmrOracle(lay)
    a.step(steps)
    scale = {f: max(np.abs(a.own_cells(m)[f]).max() for m in range(len(lay.blocks))) for f in A.FIELDS}
    err = {f: 0.0 for f in A.FIELDS}
    for m, qb in enumerate(h.current()):
        got, ref = h.own_cells(m, qb), a.own_cells(m)
        for f in A.FIELDS:
            err[f] = max(err[f], float(np.abs(got[f] - ref[f]).max()) / scale[f])
    print("errors", err, flush=True)
    for f, e in err.items():
        assert e <= 1e-12, (f, err)
    assert not h.check()[:6].any()


def test_three_levels_with_diffusion_against_oracle():
    # every block applies the artificial diffusion and the sponge (rate from the domain's lid height)
    # over its update range; the oracle steps each box with the uniform-grid oracle, whose stage
    # carries both.  The diffusion reaches two
    # cells per stage, so the stale ghost layers advance two per stage: 12 layers keep them away from
    # the own cells over two fine steps (with 6 they reach the own cells, where the box-edge values
    # they carry differ between the two sides by rounding only, but at their own large magnitude)
    base = small_layout().base.replace(kdh=0.05, kdv=0.05, zsp=2400.0, rsp=0.05)
    lay = W.amr_layout(base, levels=3, brick=8, ghost=12, d_fine=300.0, band=400.0, seed=1)
    assert {lay.block_config(b).ztop for b in lay.blocks} == {base.nz * base.dz}
    print("case three levels diffusion", len(lay.blocks), flush=True)
    steps = 2
    h = CC.Hierarchy(lay, "f64")
    h.step(steps)
    torch.cuda.synchronize()
    a = A.AmrOracle(lay)
    a.step(steps)
    plain = A.AmrOracle(W.amr_layout(small_layout().base, levels=3, brick=8, ghost=12, d_fine=300.0, band=400.0,
                                     seed=1))
    plain.step(steps)
    scale = {f: max(np.abs(a.own_cells(m)[f]).max() for m in range(len(lay.blocks))) for f in A.FIELDS}
    err = {f: 0.0 for f in A.FIELDS}
    moved = 0.0
    for m, qb in enumerate(h.current()):
        got, ref = h.own_cells(m, qb), a.own_cells(m)
        for f in A.FIELDS:
            err[f] = max(err[f], float(np.abs(got[f] - ref[f]).max()) / scale[f])
        moved = max(moved, float(np.abs(ref["mw"] - plain.own_cells(m)["mw"]).max()) / scale["mw"])
    print("errors", err, "diffusion effect", moved, flush=True)
    for f, e in err.items():
        assert e <= 1e-12, (f, err)
    assert moved > 1e-9
    assert not h.check()[:6].any()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_uniform_flow_over_flat_ground_stays_uniform(prec):
    # every level keeps uniform inflow over flat ground on its own; the transfers between levels must
    # too, where the fine bricks stand on the ground (coarse-fine faces reaching down to it)
    base = W.Config("flat2", 16, 16, 16, 200.0, 200.0, 200.0, W.Hill("flat"), dt=0.2, u0=10.0, v0=2.0)
    blocks = [W.AmrBlock(0, (8 * x, 8 * y, 8 * z), (8, 8, 8)) for x in range(2) for y in range(2) for z in range(2)
              if (x, y, z) != (0, 0, 0)]
    blocks += [W.AmrBlock(1, (8 * x, 8 * y, 8 * z), (8, 8, 8)) for x in range(2) for y in range(2) for z in range(2)]
    lay = W.AmrLayout(base, 2, 8, 6, [], blocks)
    print("case flat two levels", prec, flush=True)
    h = CC.Hierarchy(lay, prec)
    h.step(2)
    torch.cuda.synchronize()
    for m, (b, qb) in enumerate(zip(lay.blocks, h.current())):
        d = h.doms[m]
        (i0, j0, k0), (i1, j1, k1) = h.own[m]
        own = h.own_cells(m, qb)
        pred = (d.unpad(d.g["vcls"]) == O.PRED)[i0:i1, j0:j1, k0:k1]
        assert np.abs(own["mw"][pred]).max() <= 1e-4, (m, b.level)
    assert not h.check()[:6].any()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_three_levels_conserve_mass(prec):
    lay = small_layout()
    print("case mass", prec, flush=True)
    h = CC.Hierarchy(lay, prec)
    m0 = _gpu_mass(h)
    h.step(3)
    torch.cuda.synchronize()
    m1 = _gpu_mass(h)
    assert abs(m1[0] - m0[0]) <= 1e-12 * m0[2], (m0, m1)
    assert abs(m1[1] - m0[1]) <= 300.0 * 1e-12 * m0[2], (m0, m1)
    assert not h.check()[:6].any()


def test_float_form_against_oracle():
    """The float form of the refined grid against the FP64 refined-grid oracle: L2 over the own
    cells of all blocks, per field, at 1e-5 (rho', (rho theta)' and w, which both forms store
    alike)."""
    lay = small_layout()
    print("case three levels f32 vs oracle", len(lay.blocks), flush=True)
    h32 = CC.Hierarchy(lay, "f32")
    h32.step(3)
    torch.cuda.synchronize()
    a = A.AmrOracle(lay)
    a.step(3)
    num = {f: 0.0 for f in ("rho", "rth", "mw")}
    den = dict(num)
    for m, q32 in enumerate(h32.current()):
        r = a.own_cells(m)
        g = h32.own_cells(m, q32)
        for f in num:
            num[f] += float(((g[f] - r[f]) ** 2).sum())
            den[f] += float((r[f] ** 2).sum())
    errs = {f: (num[f] / den[f]) ** 0.5 for f in num}
    print("f32 vs oracle", errs, flush=True)
    for f, e in errs.items():
        assert e <= 1e-5, (f, errs)


def test_graph_replays_match_eager():
    lay = small_layout()
    eager = CC.Hierarchy(lay, "f32")
    graph = CC.Hierarchy(lay, "f32")
    for rep in range(3):
        eager.step(1)
        graph.step(1, use_graph=True)
        torch.cuda.synchronize()
        for m, (a, b) in enumerate(zip(eager.current(), graph.current())):
            for f in a.t:
                assert torch.equal(a.t[f], b.t[f]), (rep, m, f)
        _ = _gpu_mass(eager)  # eager work between replays
    assert not graph.check()[:6].any()


def test_full_refined_hemisphere_conserves_mass():
    """The refined hemisphere workload (about 1800 blocks over three levels) in the float form: two
    level-0 steps, mass conserved to 1e-12 of the total, no device condition."""
    lay = W.amr_hemisphere(2000)
    print("case refined hemisphere", len(lay.blocks), flush=True)
    h = CC.Hierarchy(lay, "f32", tile=9)
    m0 = _gpu_mass(h)
    h.step(2, use_graph=True)
    torch.cuda.synchronize()
    m1 = _gpu_mass(h)
    assert abs(m1[0] - m0[0]) <= 1e-12 * m0[2], (m0, m1)
    assert not h.check()[:6].any(), h.check()
    h.close()
