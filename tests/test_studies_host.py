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


# ---- the refined-grid experiment of Sec. 3.2 ----

from paper_1509_02572_amd import workloads as W


def test_cbcm_cube_counts_of_the_paper():
    # Sec. 3.2: 64, 148 and 232 cubes of 20^3 cells for refinement levels 0, 1 and 2; 4096 for the
    # uniform 100 m mesh over the same 64 x 32 x 16 km domain
    assert [len(W.cbcm_hemisphere(L).blocks) for L in (1, 2, 3)] == [64, 148, 232]
    assert (640 * 320 * 160) // W.CBCM_CUBE ** 3 == 4096
    lay = W.cbcm_hemisphere(3)
    b = lay.base
    assert (b.nx * b.dx, b.ny * b.dy, b.nz * b.dz) == (S.LX, S.LY, S.LZ)
    assert all(bl.size == (20, 20, 20) for bl in lay.blocks)
    # spacings 400 / 200 / 100 m, time steps delta / 800 s
    for lev in range(3):
        bl = next(x for x in lay.blocks if x.level == lev)
        c = lay.block_config(bl)
        assert c.dx == 400.0 / (1 << lev) and c.dt == c.dx / 800.0


def _level_map(lay):
    """Covering level of every level-2 cell of the domain (-1: not covered; -2: covered twice)."""
    b = lay.base
    f = 1 << (lay.levels - 1)
    occ = np.full((b.nx * f, b.ny * f, b.nz * f), -1, dtype=np.int8)
    for bl in lay.blocks:
        s = f >> bl.level
        sl = tuple(slice(o * s, (o + n) * s) for o, n in zip(bl.org, bl.size))
        occ[sl] = np.where(occ[sl] == -1, bl.level, -2)
    return occ


def test_cbcm_cubes_tile_the_domain_with_two_to_one_balance():
    for L in (2, 3):
        lay = W.cbcm_hemisphere(L)
        occ = _level_map(lay)
        assert occ.min() >= 0  # every cell covered exactly once
        # 2:1 balance across faces, edges and corners, at the finest cube size (periodic in x, y)
        n = W.CBCM_CUBE
        lev = occ[::n, ::n, ::n].astype(np.int64)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    sh = np.roll(np.roll(lev, dx, axis=0), dy, axis=1)
                    a = lev[:, :, max(dz, 0): lev.shape[2] + min(dz, 0)]
                    c = sh[:, :, max(-dz, 0): lev.shape[2] + min(-dz, 0)]
                    assert np.abs(a - c).max() <= 1
        # the finest cubes enclose the hill (radius 1 km at (32, 16) km) with room to spare
        f = 1 << (L - 1)
        d = 400.0 / f
        i, j = int(32000 / d), int(16000 / d)
        r = int(np.ceil(1000 / d)) + 2
        assert (occ[i - r:i + r, j - r:j + r, : r] == L - 1).all()


def test_block_sampling_is_exact_for_linear_fields():
    # every block box holds the values of one linear function at its lattice points (positions
    # unwrapped beyond the domain edge); sampling the comparison points through the finest own
    # block reproduces the function exactly
    lay = W.cbcm_hemisphere(3)
    fn = lambda x, y, z: 0.5 + 1e-4 * x - 2e-4 * y + 3e-4 * z
    blocks = []
    for bl in lay.blocks:
        org, size, gb, gt = lay.box(bl)
        d = 400.0 / (1 << bl.level)
        X, Y, Z = np.meshgrid(*(d * (o + np.arange(n)) for o, n in zip(org, size)), indexing="ij")
        blocks.append((bl.level, bl.org, tuple(o + s for o, s in zip(bl.org, bl.size)), org, fn(X, Y, Z)))
    tg = S.refined_targets()
    for k, v in tg.items():
        pts = v[::37]
        got = S.sample_blocks(blocks, pts, 400.0)
        assert np.isfinite(got).all()
        np.testing.assert_allclose(got, fn(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=0, atol=1e-9)


def test_uniform_grid_sampling_wraps_periodically():
    n = (8, 4, 5)
    arr = np.arange(np.prod(n), dtype=np.float64).reshape(n)
    blk = [S.uniform_as_block(arr)]
    # lattice points themselves, including the last index in x and y
    pts = np.array([[7 * 100.0, 3 * 100.0, 2 * 100.0], [0.0, 0.0, 100.0], [3 * 100.0, 1 * 100.0, 3 * 100.0]])
    got = S.sample_blocks(blk, pts, 100.0)
    assert got[0] == arr[7, 3, 2] and got[1] == arr[0, 0, 1] and got[2] == arr[3, 1, 3]
    # half-way between the last point in x and its periodic image at x = 0
    mid = S.sample_blocks(blk, np.array([[750.0, 0.0, 0.0]]), 100.0)
    assert mid[0] == 0.5 * (arr[7, 0, 0] + arr[0, 0, 0])


def test_regions_of_the_level_two_layout():
    pts = np.array([[32000.0, 16000.0, 500.0],    # above the hill: level 2
                    [38000.0, 13000.0, 7000.0],   # level 2 reaches 28-40 km, 12-20 km, 0-8 km
                    [41000.0, 16000.0, 500.0],    # downstream beyond it: level 1
                    [26000.0, 10000.0, 15000.0],  # level 1 reaches 24-48 km, 8-24 km, 0-16 km
                    [20000.0, 16000.0, 500.0],    # upstream: level 0
                    [50000.0, 5000.0, 1000.0]])
    assert S.region_of(pts).tolist() == [2, 2, 1, 1, 0, 0]
    n = S.diff_norms(np.array([1.0, 2.0, 3.0]), np.array([1.0, 1.0, 1.0]), np.array([0, 2, 2]))
    assert n["L0"]["rms"] == 0.0 and n["L2"]["max"] == 2.0 and "L1" not in n
    assert math.isclose(n["all"]["rms"], math.sqrt(5.0 / 3.0))


def test_block_boxes_stop_at_ground_and_lid():
    # with 12 ghost layers a 20-cell cube above the ground has 12 below it, the bottom cubes none, and
    # no box reaches above the lid; laterally the ghost layers wrap periodically
    lay = W.cbcm_hemisphere(3, ghost=12)
    for b in lay.blocks:
        org, size, gb, gt = lay.box(b)
        nzl = lay.base.nz << b.level
        assert gb == min(12, b.org[2]) and gt == min(12, nzl - b.org[2] - b.size[2])
        assert org[2] >= 0 and org[2] + size[2] <= nzl
        assert org[0] == b.org[0] - 12 and size[0] == b.size[0] + 24
        c = lay.block_config(b)
        assert c.z0 == org[2] * c.dz and c.ztop == lay.base.nz * lay.base.dz
