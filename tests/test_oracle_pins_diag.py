"""More pins of the FP64 CPU oracle (no GPU): the corner normal, the velocity diagnostics, the
closure of the cut cells' face-area vectors, the hill volume against its analytic value, and the
refined grid's ghost refills between levels.

Each test checks the oracle against something other than itself: the exact normal of a planar
surface, the exact result of the diagnostics for a uniform flow (the nearest-plane interpolation of
a constant reproduces it; eq. 33 removes its normal component; the merged-face rule interpolates
linearly along the vertical), mirror symmetry of the diagnostics for a random flow, the divergence
theorem applied to each cut cell, the closed-form integral of the bell and hemisphere, and linear
fields, which the eight-point mean and the injection between levels must carry exactly.
"""
import math

import numpy as np
import pytest

from oracle import amr_oracle as A
from oracle import oracle as O
from paper_1509_02572_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def _steep_random_cfg():
    """A 6x6x6 grid of random corner heights with horizontal merges and no unmergeable cell."""
    for seed in range(1, 200):
        H = W.random_corners(6, 6, 6, 100.0, seed, 0.05, 0.6)
        cfg = W.Config("rand", 6, 6, 6, 100.0, 100.0, 100.0, W.Hill("flat"), H=H, u0=3.0, v0=-2.0, dt=0.02)
        o = O.Oracle(cfg).merge()
        d = np.bincount(o.dir.ravel(), minlength=6)
        if o.counts[0] == 0 and d[2:].sum() > 0:
            return cfg
    raise RuntimeError("no suitable random terrain")


# ---------------------------------------------------------------------------------------------
# Corner normal (Sec. 2.4): centred gradients of the four surrounding column-centre heights
# ---------------------------------------------------------------------------------------------

def test_corner_normal_on_planar_patch():
    """Where the four columns around a corner lie on one plane h = c + alpha x + beta y, the normal
    is the plane's upward unit normal (-alpha, -beta, 1)/sqrt(alpha^2 + beta^2 + 1)."""
    nx, ny, nz, dx, dy, dz = 16, 12, 20, 50.0, 40.0, 50.0
    alpha, beta = 0.7, -0.4
    I = np.arange(nx)[:, None] * dx
    J = np.arange(ny)[None, :] * dy
    # a plane over corners 2..12 x 2..9; outside it the heights are arbitrary (a ridge)
    H = 300.0 + 100.0 * np.cos(2 * np.pi * I / (nx * dx)) + 0 * J
    plane = 200.0 + alpha * I + beta * J
    H[2:13, 2:10] = plane[2:13, 2:10]
    cfg = W.Config("plane", nx, ny, nz, dx, dy, dz, W.Hill("flat"), H=np.ascontiguousarray(H))
    o = O.Oracle(cfg).geometry()
    want = np.array([-alpha, -beta, 1.0]) / math.sqrt(alpha * alpha + beta * beta + 1.0)
    n = 0
    for a in range(3, 12):  # corners whose four surrounding columns lie inside the plane
        for b in range(3, 9):
            assert np.abs(o.nrm[:, a, b] - want).max() <= 1e-14, (a, b, o.nrm[:, a, b])
            n += 1
    assert n == 54
    # everywhere: unit length and pointing up, away from the ground
    assert np.abs((o.nrm ** 2).sum(axis=0) - 1.0).max() <= 1e-14
    assert (o.nrm[2] > 0).all()


# ---------------------------------------------------------------------------------------------
# Velocity diagnostics (Sec. 2.4: nearest plane, eq. 33, merged-face interpolation)
# ---------------------------------------------------------------------------------------------

def _corner_density(o, K):
    """Mean of the eight total densities around lattice level K when rho' = 0, in the oracle's
    summation order (four cells of level K-1, then four of level K)."""
    a, b = o.rhob[K - 1], o.rhob[K]
    return 0.125 * (((a + a) + (a + a)) + ((b + b) + (b + b)))


def _state_with_velocity(o, vel):
    """State with rho' = (rho theta)' = 0 and momentum rho_c * vel at predicted points (vel: array
    (3, nx, ny, nz) or a constant 3-vector)."""
    nx, ny, nz = o.shape
    q = O.State(o.shape)
    pred = o.vcls == O.PRED
    K = np.broadcast_to(np.arange(nz)[None, None, :], o.shape)
    rc = np.zeros(o.shape)
    rc[pred] = np.array([_corner_density(o, k) if k >= 1 else 0.0 for k in range(nz)])[K[pred]]
    vel = np.asarray(vel, dtype=float)
    if vel.ndim == 1:
        vel = np.broadcast_to(vel[:, None, None, None], (3, nx, ny, nz))
    for c, f in enumerate(("mu", "mv", "mw")):
        q.a[f][pred] = rc[pred] * vel[c][pred]
    return q


@pytest.mark.parametrize("which", ["hemi_tiny", "steep_random"])
def test_diagnostics_of_a_uniform_flow(which):
    """A uniform velocity U (with w != 0) at every predicted point.  Then at every column corner the
    nearest-plane mean is U (bilinear interpolation of a constant), and eq. 33 gives
    u_B = U - (U.n) n, tangent to the terrain; points on or below the terrain carry u_B; a merged-face
    point at level K takes gamma U + (1 - gamma) u_B with gamma = (K dz - H)/(K_p dz - H), K_p the
    lowest predicted level above it (u_B when there is none within 8 levels)."""
    cfg = W.get("hemi_tiny") if which == "hemi_tiny" else _steep_random_cfg()
    o = O.Oracle(cfg).merge()
    U = np.array([3.0, -2.0, 1.5])
    q = _state_with_velocity(o, U)
    ub, flag = o.boundary_velocity(q)
    assert not flag.any()
    n = np.moveaxis(o.nrm, 0, -1)  # (nx, ny, 3)
    want = U[None, None, :] - (n @ U)[:, :, None] * n
    scale = np.abs(U).max()
    assert np.abs(ub - want).max() <= 1e-14 * scale
    assert np.abs((ub * n).sum(axis=-1)).max() <= 1e-14 * scale  # free slip: no normal component
    o.diagnose(q)
    assert o.counts[1] == 0
    nx, ny, nz = o.shape
    got = np.stack([q.a["mu"], q.a["mv"], q.a["mw"]], axis=-1)
    pred = o.vcls == O.PRED
    checked = {"ground": 0, "mface": 0}
    for I in range(nx):
        for J in range(ny):
            h = o.H[I, J]
            for K in range(nz):
                if pred[I, J, K]:
                    continue
                if K * cfg.dz <= h:
                    exp = ub[I, J]
                    checked["ground"] += 1
                else:
                    above = [k for k in range(K + 1, min(K + 9, nz)) if pred[I, J, k]]
                    if above:
                        gam = (K * cfg.dz - h) / (above[0] * cfg.dz - h)
                        exp = U * gam + ub[I, J] * (1.0 - gam)
                    else:
                        exp = ub[I, J]
                    checked["mface"] += 1
                assert np.abs(got[I, J, K] - exp).max() <= 1e-14 * scale, (I, J, K, got[I, J, K], exp)
    assert checked["ground"] > 0 and checked["mface"] > 0
    # predicted points keep their momentum
    for c, f in enumerate(("mu", "mv", "mw")):
        rc = np.array([_corner_density(o, k) if k >= 1 else 0.0 for k in range(nz)])
        assert np.array_equal(q.a[f][pred], (rc[None, None, :] * U[c] * np.ones(o.shape))[pred])


@pytest.mark.parametrize("axis", [0, 1])
def test_diagnostics_mirror_symmetry(axis):
    """On a hill symmetric about the corner line I = nx/2 (J = ny/2), a random velocity field and its
    mirror image (the field at the mirrored point, with the normal component reversed) give mirrored
    diagnosed velocities: the nearest-plane walk, its weights and eq. 33 commute with the mirror."""
    cfg = W.get("hemi_tiny")
    o = O.Oracle(cfg).merge()
    nx, ny, nz = o.shape
    rng = np.random.Generator(np.random.PCG64(21))
    vel = rng.normal(0.0, 1.0, size=(3, nx, ny, nz))
    # the lattice mirror maps corner I to (n - I) mod n
    idx = [np.arange(nx), np.arange(ny)]
    idx[axis] = (-idx[axis]) % (nx, ny)[axis]
    mir = vel[:, idx[0][:, None], idx[1][None, :], :].copy()
    mir[axis] *= -1.0
    assert np.array_equal(o.vcls, o.vcls[idx[0][:, None], idx[1][None, :], :])  # the grid is symmetric
    qa, qb = _state_with_velocity(o, vel), _state_with_velocity(o, mir)
    o.diagnose(qa)
    o.diagnose(qb)
    ga = np.stack([qa.a["mu"], qa.a["mv"], qa.a["mw"]])
    gb = np.stack([qb.a["mu"], qb.a["mv"], qb.a["mw"]])
    back = gb[:, idx[0][:, None], idx[1][None, :], :].copy()
    back[axis] *= -1.0
    diag = o.vcls != O.PRED
    assert diag.sum() > 0
    assert np.abs(back[:, diag] - ga[:, diag]).max() <= 1e-13 * np.abs(ga[:, diag]).max()


# ---------------------------------------------------------------------------------------------
# P5: closure of each cut cell's face-area vector (divergence theorem for a constant field)
# ---------------------------------------------------------------------------------------------

def _bilin(h, xi, eta):
    h00, h10, h01, h11 = h
    return h00 + xi * (h10 - h00) + eta * (h01 - h00) + (xi * eta) * ((h00 - h01) + (h11 - h10))


def _terrain_surface_vector(cfg, h, k, nsub):
    """Integral of the terrain's outward (downward) surface element (h_x, h_y, -1) dx dy over the
    part of column footprint whose surface lies in the layer of cell k, by strips and sub-columns:
    along each strip the integral of h_x over the layer part is the difference of the clamped end
    heights (fundamental theorem); the z part counts the sub-columns whose centre lies in the layer."""
    zb, zt = k * cfg.dz, (k + 1) * cfg.dz
    t = (np.arange(nsub) + 0.5) / nsub
    clamp = lambda z: np.minimum(np.maximum(z, zb), zt)
    sx = (cfg.dy / nsub) * (clamp(_bilin(h, 1.0, t)) - clamp(_bilin(h, 0.0, t))).sum()
    sy = (cfg.dx / nsub) * (clamp(_bilin(h, t, 1.0)) - clamp(_bilin(h, t, 0.0))).sum()
    hab = _bilin(h, t[:, None], t[None, :])
    sz = -(cfg.dx * cfg.dy / nsub ** 2) * ((hab >= zb) & (hab < zt)).sum()
    return np.array([sx, sy, sz])


def _cut_cells(o):
    return np.argwhere((o.V > 0) & (o.V < 1))


@pytest.mark.parametrize("which", ["bell32", "hemi_small", "steep_random"])
def test_face_area_vectors_close(which):
    """Sum over the six faces of +-A S n plus the terrain surface vector S_b is zero for every cut
    cell (to 1e-12 dx dy), apart from faces the solid-neighbour rule closed (counted)."""
    cfg = W.get(which) if which != "steep_random" else _steep_random_cfg()
    o = O.Oracle(cfg).merge()
    nx, ny, nz = o.shape
    Sx, Sy, Sz = cfg.dy * cfg.dz, cfg.dz * cfg.dx, cfg.dx * cfg.dy
    closed, n = 0, 0
    for i, j, k in _cut_cells(o):
        H = o.H
        h = (H[i, j], H[(i + 1) % nx, j], H[i, (j + 1) % ny], H[(i + 1) % nx, (j + 1) % ny])
        sb = _terrain_surface_vector(cfg, h, k, cfg.nsub)
        ip, jp = (i + 1) % nx, (j + 1) % ny
        azt = o.Az[i, j, k + 1] if k + 1 < nz else 1.0
        area = np.array([(o.Ax[ip, j, k] - o.Ax[i, j, k]) * Sx, (o.Ay[i, jp, k] - o.Ay[i, j, k]) * Sy,
                         (azt - (o.Az[i, j, k] if k > 0 else 0.0)) * Sz])
        if k == 0:  # the ground closes the bottom face: the layer starts at z = 0 with nothing below
            area[2] = azt * Sz
        neighbours_solid = (o.V[(i - 1) % nx, j, k] == 0 or o.V[ip, j, k] == 0 or o.V[i, (j - 1) % ny, k] == 0
                            or o.V[i, jp, k] == 0 or (k > 0 and o.V[i, j, k - 1] == 0) or
                            (k + 1 < nz and o.V[i, j, k + 1] == 0))
        res = np.abs(area + sb).max()
        if neighbours_solid and res > 1e-12 * Sz:
            closed += 1
            continue
        assert res <= 1e-12 * Sz, (i, j, k, area, sb)
        n += 1
    assert n > 0
    print(f"{which}: {n} cut cells closed, {closed} with a face closed by the solid rule")


def test_face_area_closure_converges_with_subcolumns():
    """Against a fine (1024-strip, 1024^2 sub-column) evaluation of the terrain surface vector, the
    closure residual of the apertures shrinks as the sub-column count grows 8 -> 16 -> 32."""
    base = _steep_random_cfg()
    res = []
    for ns in (8, 16, 32):
        cfg = base.replace(nsub=ns)
        o = O.Oracle(cfg).merge()
        nx, ny, nz = o.shape
        Sx, Sy, Sz = cfg.dy * cfg.dz, cfg.dz * cfg.dx, cfg.dx * cfg.dy
        worst = 0.0
        for i, j, k in _cut_cells(o)[:40]:
            H = o.H
            h = (H[i, j], H[(i + 1) % nx, j], H[i, (j + 1) % ny], H[(i + 1) % nx, (j + 1) % ny])
            fine = _terrain_surface_vector(cfg, h, k, 1024)
            ip, jp = (i + 1) % nx, (j + 1) % ny
            if min(o.V[(i - 1) % nx, j, k], o.V[ip, j, k], o.V[i, (j - 1) % ny, k], o.V[i, jp, k]) == 0:
                continue
            ax = (o.Ax[ip, j, k] - o.Ax[i, j, k]) * Sx
            ay = (o.Ay[i, jp, k] - o.Ay[i, j, k]) * Sy
            worst = max(worst, abs(ax + fine[0]), abs(ay + fine[1]))
        res.append(worst / Sz)
    assert res[0] > res[1] > res[2], res
    assert res[2] < 0.02, res


# ---------------------------------------------------------------------------------------------
# P4: cut-cell volumes against the analytic volume of the hill (Sec. 2.3, Sec. 3.1)
# ---------------------------------------------------------------------------------------------

def _terrain_volume(cfg):
    o = O.Oracle(cfg).geometry()
    dv = cfg.dx * cfg.dy * cfg.dz
    return cfg.nx * cfg.ny * cfg.nz * dv - o.V.sum() * dv


def test_bell_volume_converges_to_analytic_integral():
    """The bell h0/(1 + r^2/a^2)^(3/2) integrates to 2 pi a^2 h0 over the plane; over the square
    domain [-L/2, L/2]^2 to 4 h0 a^2 atan(L^2/4 / (a sqrt(a^2 + L^2/2))) (solid-angle integral of a
    rectangle).  The volume below the cut-cell terrain converges to it at second order in dx."""
    h0, a, L = 400.0, 2000.0, 25600.0
    square = lambda L: 4.0 * h0 * a * a * math.atan((L * L / 4.0) / (a * math.sqrt(a * a + L * L / 2.0)))
    exact = square(L)
    # the square integral tends to the plane's 2 pi a^2 h0 (the bell's 1/r^3 tail leaves 16 % of it
    # outside this domain)
    assert abs(square(1e12) - 2 * math.pi * a * a * h0) <= 1e-6 * exact and exact < 2 * math.pi * a * a * h0
    errs = []
    for n in (32, 64, 128):
        d = L / n
        cfg = W.Config("bellvol", n, n, 10, d, d, 50.0, W.Hill("bell", h0, a))
        errs.append(abs(_terrain_volume(cfg) - exact) / exact)
    assert errs[2] <= 1e-3, errs
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 <= e0 / e1 <= 4.5, errs  # second order


def test_hemisphere_volume_against_analytic():
    """The hemisphere of radius R holds (2/3) pi R^3; at the 50 m and 100 m spacings the cut-cell
    terrain volume is within 1e-2 of it, and closer at the finer spacing."""
    R = 1000.0
    exact = 2.0 / 3.0 * math.pi * R ** 3
    errs = []
    for d, n in ((100.0, 40), (50.0, 80)):
        cfg = W.Config("hemivol", n, n, 24, d, d, 50.0, W.Hill("hemisphere", 0.0, R))
        errs.append(abs(_terrain_volume(cfg) - exact) / exact)
    assert errs[1] < errs[0] and errs[1] <= 1e-2, errs


# ---------------------------------------------------------------------------------------------
# Refined grid (Sec. 2.2): restriction (eight-point mean) and injection between levels
# ---------------------------------------------------------------------------------------------

def _amr_small():
    base = W.Config("amr_test", 16, 16, 24, 200.0, 200.0, 200.0, W.Hill("hemisphere", 0.0, 600.0), dt=0.2)
    return W.amr_layout(base, levels=3, brick=8, ghost=6, d_fine=300.0, band=400.0, seed=1)


def test_refills_between_levels_carry_linear_fields():
    """Fill every block (own and ghost cells) with fields linear in the global position: scalars at
    cell centres, momenta at lattice points, each with distinct slopes in x, y and z.  Ghost cells of
    level l covered by level l+1 then take the eight-point mean of their children, which for a
    linear field is the value at the coarse centre; ghost cells of level l+1 covered by level l take
    the coarse field interpolated linearly to their own centre (momenta: the value at the coincident
    fine lattice point, or the coarse lattice points interpolated to the fine one), which reproduces
    a linear field exactly; where the coarse stencil reaches terrain, the ground or the lid the
    fine ghost keeps the parent's value, so away from the hill (above 1.2 km, below the lid) every
    injected value must be the field at the fine point itself.  At predicted
    points the momentum holds its level's reference flow rhobar_c(K) U on top of the linear part
    (rhobar_c of the box's own base state, which differs between levels at the same height): what
    moves is the linear part, the perturbation from each level's reference, so the destination
    holds the source's linear value plus its own reference flow."""
    lay = _amr_small()
    a = A.AmrOracle(lay)
    coef = {"rho": (1e-3, 2e-7, -3e-7, 5e-7), "rth": (0.2, -1e-5, 4e-5, 2e-5),
            "mu": (10.0, 1e-3, 2e-3, -4e-3), "mv": (-1.0, 3e-3, -1e-3, 2e-3), "mw": (0.5, -2e-3, 1e-3, 3e-3)}

    def lin(f, x, y, z):
        c = coef[f]
        return c[0] + c[1] * x + c[2] * y + c[3] * z

    def positions(m, centre):
        """Global positions [m] of the box points of block m (x, y wrapped into the domain)."""
        b = lay.blocks[m]
        o = a.boxes[m]
        l = b.level
        N = a.N[l]
        d = (lay.base.dx / (1 << l), lay.base.dy / (1 << l), lay.base.dz / (1 << l))
        ox, oy, oz = a.org[m]
        nx, ny, nz = o.shape
        off = 0.5 if centre else 0.0
        gx = np.mod(ox + np.arange(nx), N[0])
        gy = np.mod(oy + np.arange(ny), N[1])
        gz = oz + np.arange(nz)
        return ((gx + off) * d[0])[:, None, None], ((gy + off) * d[1])[None, :, None], ((gz + off) * d[2])[None, None, :]

    U = {"mu": lay.base.u0, "mv": lay.base.v0, "mw": 0.0}
    assert U["mu"] != 0.0

    def ref_flow(o, f):
        """rhobar_c(K) U of box o at its predicted lattice points, 0 elsewhere."""
        rbc = np.zeros(o.shape[2])
        rbc[1:] = 0.5 * (o.rhob[:-1] + o.rhob[1:])
        return np.where(o.vcls == O.PRED, rbc[None, None, :] * U[f], 0.0)

    for m, o in enumerate(a.boxes):
        xc, yc, zc = positions(m, True)
        xl, yl, zl = positions(m, False)
        for f in ("rho", "rth"):
            a.q[m].a[f][...] = lin(f, xc, yc, zc)
        for f in ("mu", "mv", "mw"):
            a.q[m].a[f][...] = lin(f, xl, yl, zl) + ref_flow(o, f)
    # refill targets start as NaN so that every one is seen written
    targets = {}
    for m, b in enumerate(lay.blocks):
        for (kind, sm), (di, si) in a.maps[m].items():
            if kind in ("fine", "coarse"):
                for f in O.FIELDS:
                    a.q[m].a[f].ravel()[di] = np.nan
                targets.setdefault(m, []).append((kind, sm, di, si))
    assert any(k == "fine" for v in targets.values() for k, _, _, _ in v)
    assert any(k == "coarse" for v in targets.values() for k, _, _, _ in v)
    for l in range(lay.levels):
        a._fill(l, a.q, ("fine", "coarse"))
    n = n_far = 0
    for m, lst in targets.items():
        b = lay.blocks[m]
        o = a.boxes[m]
        xc, yc, zc = positions(m, True)
        xl, yl, zl = positions(m, False)
        shape = o.shape
        for kind, sm, di, si in lst:
            i, j, k = np.unravel_index(di, shape)
            if kind == "fine":  # restriction: the coarse ghost's own centre / lattice point
                px, py, pz = xc[i, 0, 0], yc[0, j, 0], zc[0, 0, k]
                lx, ly, lz = xl[i, 0, 0], yl[0, j, 0], zl[0, 0, k]
            else:  # injection: the fine cell's own centre and lattice point
                px, py, pz = xc[i, 0, 0], yc[0, j, 0], zc[0, 0, k]
                lx, ly, lz = xl[i, 0, 0], yl[0, j, 0], zl[0, 0, k]
                dc = (lay.base.dx / (1 << (b.level - 1)), lay.base.dy / (1 << (b.level - 1)),
                      lay.base.dz / (1 << (b.level - 1)))
                gx = np.mod(a.org[m][0] + i, a.N[b.level][0])
                gy = np.mod(a.org[m][1] + j, a.N[b.level][1])
                gz = a.org[m][2] + k
                # parent centre and halved lattice index: where the stencil fails
                ppx, ppy, ppz = ((gx // 2 + 0.5) * dc[0], (gy // 2 + 0.5) * dc[1], (gz // 2 + 0.5) * dc[2])
                plx, ply, plz = ((gx // 2) * dc[0], (gy // 2) * dc[1], (gz // 2) * dc[2])
                # the linear field is not periodic: leave out stencils that wrap round the domain
                Lx, Ly = lay.base.nx * lay.base.dx, lay.base.ny * lay.base.dy
                inner = ((gx + 0.5) * dc[0] / 2 > dc[0]) & ((gx + 0.5) * dc[0] / 2 < Lx - dc[0]) \
                    & ((gy + 0.5) * dc[1] / 2 > dc[1]) & ((gy + 0.5) * dc[1] / 2 < Ly - dc[1])
                far = inner & (zc[0, 0, k] > 1200.0) & (zc[0, 0, k] < lay.base.nz * lay.base.dz - 2 * dc[2])
                n_far += int(far.sum())
            close = lambda g, w: np.abs(g - w) <= 1e-13 * (np.abs(w) + 1.0)  # fields of order 1-10
            for f in ("rho", "rth"):
                want = lin(f, px, py, pz)
                got = a.q[m].a[f][i, j, k]
                if kind == "fine":
                    assert np.all(close(got, want)), (kind, m, f)
                else:
                    assert np.all(close(got, want)[far]), (kind, m, f)
                    assert np.all((close(got, want) | close(got, lin(f, ppx, ppy, ppz)))[inner]), (kind, m, f)
            # both ends predicted: the linear part moves, the destination adds its own reference
            # flow; otherwise the stored value moves as it is
            both = (o.vcls.ravel()[di] == O.PRED) & (a.boxes[sm].vcls.ravel()[si] == O.PRED)
            for f in ("mu", "mv", "mw"):
                src_ref = ref_flow(a.boxes[sm], f).ravel()[si]
                extra = np.where(both, ref_flow(o, f).ravel()[di], src_ref)
                want = lin(f, lx, ly, lz) + extra
                got = a.q[m].a[f][i, j, k]
                if kind == "fine":
                    assert np.all(close(got, want)), (kind, m, f)
                else:
                    assert np.all(close(got, want)[far & both]), (kind, m, f)
                    # (an odd fine level under the source box's top level interpolates in x and y only)
                    snz = a.boxes[sm].shape[2]
                    zok = ~(((gz & 1) == 1) & (si % snz + 1 >= snz))
                    assert np.all((close(got, want) | close(got, lin(f, plx, ply, plz) + extra))[inner & zok]), \
                        (kind, m, f)
            if kind == "coarse":
                assert both.any()
            n += len(di)
    assert n > 100 and n_far > 1000, (n, n_far)
