"""The allocation-free conservation sums (static device scratch) agree with cutcell_reduce, which
takes a caller workspace, on two calls in a row, the second on a smaller grid."""
import numpy as np
import pytest
import torch

from paper_1509_02572_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_reduce_noalloc_matches_workspace_form(prec):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1509_02572_amd import cutcell as CC
    for name in ("bell_small", "hemi_tiny"):  # the second grid is the smaller one
        cfg = W.get(name)
        print(f"case noalloc {name} {prec}", flush=True)
        dom = CC.Domain(cfg, prec)
        q = dom.run(dom.init_state(W.theta_noise(cfg.replace(noise_sigma=0.01, seed=9))), cfg.dt, 3)
        ref = dom.reduce(q)  # cutcell_reduce with the domain's workspace
        out = torch.full((4,), float("nan"), dtype=torch.float64, device=dom.dev)
        CC.cutcell_reduce_noalloc(dom.grid, dom.phys, dom.geom, dom.base, dom.prec, q.c, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # same kernels, same block count and order: the sums are bitwise equal
        assert np.array_equal(got, ref), (name, got, ref)
        assert np.isfinite(got).all() and got[2] > 0
