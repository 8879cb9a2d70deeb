"""The oracle's conservation sums against exactly rounded sums (math.fsum) of the same terms.

M' = sum over group masters of Vgroup dV rho', Theta' the same with (rho theta)', M_total with the
base density of the master's level added (Sec. 2.4: the merged-cell scheme conserves mass).  The
oracle sums cell by cell with a compensation term; over a million cells its result must stay within
a few rounding errors of the exactly rounded sum (a plain running sum drifts by far more)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_02572_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


@pytest.mark.parametrize("name", ["bell_small", "flat_large"])
def test_mass_sums_match_exactly_rounded_sums(name):
    if name == "flat_large":
        cfg = W.Config("flat_large", 128, 128, 64, 100.0, 100.0, 50.0, W.Hill("cosine", 300.0, 2500.0))
    else:
        cfg = W.get(name)
    o = O.Oracle(cfg).merge()
    rs = W.random_state(cfg, 11)
    q = O.State(None, rs)
    got = o.reduce(q)
    m = ((o.cls == O.OPEN) | (o.cls == O.ORPHAN))
    vg = (o.Vgroup * (cfg.dx * cfg.dy * cfg.dz))[m]
    K = np.broadcast_to(np.arange(cfg.nz)[None, None, :], o.shape)[m]
    rho = q.a["rho"][m]
    want = [math.fsum(vg * rho), math.fsum(vg * q.a["rth"][m]), math.fsum(vg * (o.rhob[K] + rho))]
    mtot = want[2]
    for a, b in zip(got[:3], want):
        assert abs(a - b) <= 4e-16 * mtot, (a, b)
