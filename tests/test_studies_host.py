"""Host logic of the experiment drivers (no GPU): grid set-up of the Appendix A study, sampling of
the reference lattice at coarse points, the error norms and the lee-wave estimator."""
import math

import numpy as np

from paper_1509_02572_amd import studies as S


def test_grids_of_the_convergence_study():
    for d, n in ((400.0, (160, 80, 40)), (250.0, (256, 128, 64)), (200.0, (320, 160, 80)), (100.0, (640, 320, 160))):
        c = S.cosine_config(d)
        assert (c.nx, c.ny, c.nz) == n
        assert c.nsteps * c.dt == 3600.0
        # hill centre on the lattice corner at (32, 16) km
        assert (c.nx // 2) * c.dx == 32000.0 and (c.ny // 2) * c.dy == 16000.0
        assert c.zsp == 10000.0 and c.nz * c.dz == 16000.0


def test_reference_sampling_is_exact_for_trilinear_fields():
    # a field linear in each coordinate (periodic directions: linear within the sampled range is
    # enough away from the wrap) is reproduced exactly at 400, 250 and 200 m points
    nx, ny, nz = 64, 32, 16
    x = np.arange(nx)[:, None, None] * 100.0
    y = np.arange(ny)[None, :, None] * 100.0
    z = np.arange(nz)[None, None, :] * 100.0
    f = 1.0 + 2e-4 * x + 3e-4 * y - 5e-4 * z + 1e-7 * x * z
    for dc in (400.0, 250.0, 200.0):
        sh = (int(6000 // dc), int(3000 // dc), int(1400 // dc))
        g = S.sample_reference(f, 100.0, dc, sh)
        X = np.arange(sh[0])[:, None, None] * dc
        Y = np.arange(sh[1])[None, :, None] * dc
        Z = np.arange(sh[2])[None, None, :] * dc
        assert np.abs(g - (1.0 + 2e-4 * X + 3e-4 * Y - 5e-4 * Z + 1e-7 * X * Z)).max() < 1e-12


def test_error_norms_select_points_above_the_hilltop():
    v = np.zeros((4, 3, 20))
    r = np.zeros_like(v)
    v[:, :, 1] = 5.0  # z = 400 m: not above the hilltop
    v[:, :, 2] = 1.0  # z = 800 m
    e = S.error_norms(v, r, 400.0)
    npts = 4 * 3 * 18  # K = 0 and K = 1 (z = 0, 400 m) are not above the hilltop
    assert e["points"] == npts
    assert math.isclose(e["L1"], 12 / npts) and math.isclose(e["L2"], math.sqrt(12 / npts))


def test_lee_wavelength_of_a_damped_wave():
    dx = 100.0
    x = np.arange(640) * dx
    x0 = 32000.0
    lam = 6500.0
    w = np.where(x > x0, np.exp(-(x - x0) / 20000.0) * np.sin(2 * np.pi * (x - x0) / lam), 0.0)
    r = S.lee_wavelength(w, dx, x0, 2000.0, 30000.0)
    assert abs(r["wavelength_m"] - lam) < 0.01 * lam
    assert len(r["maxima_m"]) >= 3


def test_lee_wavelength_ignores_ripples_on_a_crest():
    dx = 100.0
    x = np.arange(640) * dx
    x0 = 32000.0
    lam = 6300.0
    w = np.where(x > x0, np.sin(2 * np.pi * (x - x0) / lam), 0.0)
    w = w + np.where((x > x0 + 24000.0) & (x < x0 + 26000.0), 0.05 * np.sin(2 * np.pi * x / 500.0), 0.0)
    r = S.lee_wavelength(w, dx, x0, 2000.0, 30000.0)
    assert all(s > 2000.0 for s in r["spacings_m"])
    assert abs(r["wavelength_m"] - lam) < 0.05 * lam
