"""Seeded synthetic inputs for the cut-cell stage: terrain heights, noise and run configurations.

This module holds no arithmetic of the method itself (no geometry, merging, base state, equation of
state or fluxes).  It only produces the *data* that both the HIP path and the CPU oracle consume:

* terrain heights ``H[I, J]`` sampled at lattice corners ``(I*dx, J*dy)`` from an analytic hill whose
  centre sits on a lattice corner (paper, Sec. 3: hills centred on the lower boundary; the bell of
  Sec. 3.1.1 and the hemisphere of Sec. 3.1.2; the cosine hill of Appendix A);
* per-cell potential-temperature noise ``theta'`` drawn with numpy's PCG64 from a seed;
* the run parameters (grid, physical constants, inflow, stratification, time step, step count).

The paper runs no public dataset: its workloads are analytic hills, so these generators stand in for
them exactly.  The sizes below are the configurations the benchmark and the parity tests use.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

# Physical constants handed to both implementations as parameters (the paper does not print them;
# these are the conventional dry-air values).
G = 9.81
RD = 287.0
CP = 1004.5
P0 = 1.0e5


@dataclasses.dataclass
class Hill:
    """Analytic terrain shape h(x, y) with the centre at the origin."""

    kind: str  # "bell", "hemisphere", "cosine", "gauss", "flat", "table"
    h0: float = 0.0  # peak height [m]
    a: float = 1.0  # half-width (bell, cosine), radius (hemisphere), sigma (gauss) [m]
    extra: Optional[list] = None  # gauss: list of (h, sigma, xc, yc); table: explicit heights

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        if self.kind == "flat":
            return np.zeros(np.broadcast(x, y).shape)
        if self.kind == "bell":  # Sec. 3.1.1: h = h_m / (1 + r^2/a^2)^(3/2)
            return self.h0 / (1.0 + (x * x + y * y) / (self.a * self.a)) ** 1.5
        if self.kind == "hemisphere":  # Sec. 3.1.2: radius r = a
            r2 = x * x + y * y
            return np.sqrt(np.maximum(self.a * self.a - r2, 0.0))
        if self.kind == "cosine":  # Appendix A: h_m/2 (1 + cos(pi r / a)) for r < a
            r = np.sqrt(x * x + y * y)
            return np.where(r < self.a, 0.5 * self.h0 * (1.0 + np.cos(np.pi * r / self.a)), 0.0)
        raise ValueError(self.kind)


@dataclasses.dataclass
class Config:
    """One uniform-grid domain: grid, terrain, atmosphere and time stepping."""

    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    hill: Hill
    bvn: float = 0.01  # Brunt-Vaisala frequency N [1/s]
    theta0: float = 300.0  # sea-level potential temperature [K]
    u0: float = 10.0  # inflow along x [m/s]
    v0: float = 0.0
    dt: float = 0.05
    nsteps: int = 100
    noise_sigma: float = 0.0  # std of theta' noise [K]; 0 = none
    seed: int = 0
    nsub: int = 16  # sub-columns per cell edge for volumes and apertures
    g: float = G
    rd: float = RD
    cp: float = CP
    p0: float = P0
    H: Optional[np.ndarray] = None  # explicit corner heights (overrides ``hill``)
    z0: float = 0.0  # height of the grid's bottom face (blocks of a refined grid); H is then relative to it
    kdh: float = 0.0  # rate of the fourth-order artificial diffusion in x and y [1/s] (0: none)
    kdv: float = 0.0  # the same in z
    redraws: int = 0  # ensemble members: hill sets redrawn before this one was accepted
    zsp: float = 0.0  # bottom height of the sponge layer below the lid [m]
    rsp: float = 0.0  # damping rate of the sponge at the lid [1/s] (0: none)
    ztop: float = 0.0  # height of the domain's lid for the sponge [m] (0: the grid's own top)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


def terrain(cfg: Config) -> np.ndarray:
    """Corner heights ``H[I, J]`` (shape ``(nx, ny)``, float64, laterally periodic).

    The hill centre is placed on the lattice corner ``(nx/2 * dx, ny/2 * dy)`` and sampled at the
    corners, as the paper defines the bilinear columns from corner heights (Sec. 2.3, eq. bilin).
    """
    if cfg.H is not None:
        H = np.ascontiguousarray(cfg.H, dtype=np.float64)
        assert H.shape == (cfg.nx, cfg.ny)
        return H
    I = np.arange(cfg.nx, dtype=np.float64)[:, None]
    J = np.arange(cfg.ny, dtype=np.float64)[None, :]
    x = I * cfg.dx - (cfg.nx // 2) * cfg.dx
    y = J * cfg.dy - (cfg.ny // 2) * cfg.dy
    if cfg.hill.kind == "gauss":
        return _gauss_sum(cfg, I, J)
    return np.ascontiguousarray(cfg.hill(x, y), dtype=np.float64)


def _gauss_sum(cfg: Config, I: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Sum of Gaussian hills with their periodic images (ensemble terrain)."""
    Lx, Ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    x = I * cfg.dx
    y = J * cfg.dy
    H = np.zeros((cfg.nx, cfg.ny))
    for (hh, sig, xc, yc) in cfg.hill.extra:
        nim = int(math.ceil(6.0 * sig / min(Lx, Ly))) + 1
        for ix in range(-nim, nim + 1):
            for iy in range(-nim, nim + 1):
                dxv = x - xc + ix * Lx
                dyv = y - yc + iy * Ly
                H += hh * np.exp(-(dxv * dxv + dyv * dyv) / (2.0 * sig * sig))
    return np.ascontiguousarray(H)


def theta_noise(cfg: Config) -> Optional[np.ndarray]:
    """Per-cell potential-temperature noise (shape ``(nx, ny, nz)``, k fastest) or ``None``.

    Drawn for every cell in linear order with ``numpy.random.Generator(PCG64(seed))``; each
    implementation uses the value at a group's representative cell only.
    """
    if cfg.noise_sigma <= 0.0:
        return None
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    return np.ascontiguousarray(rng.normal(0.0, cfg.noise_sigma, size=(cfg.nx, cfg.ny, cfg.nz)))


def random_corners(nx: int, ny: int, nz: int, dz: float, seed: int, lo=0.05, hi=0.85) -> np.ndarray:
    """Random corner heights in ``[lo, hi] * nz*dz`` for brute-force tests on tiny grids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.uniform(lo, hi, size=(nx, ny)) * nz * dz)


def random_state(cfg: Config, seed: int, amp=(1e-3, 0.3, 1.0)) -> dict:
    """Random perturbation fields (rho', rho*theta', and three momentum/velocity fields).

    Used to feed a tendency evaluation with a state that exercises every term.  The arrays are
    returned on the unpadded ``(nx, ny, nz)`` layout, k fastest.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sh = (cfg.nx, cfg.ny, cfg.nz)
    return {
        "rho": rng.normal(0.0, amp[0], size=sh),
        "rth": rng.normal(0.0, amp[1], size=sh),
        "mu": cfg.u0 + rng.normal(0.0, amp[2], size=sh),
        "mv": cfg.v0 + rng.normal(0.0, amp[2], size=sh),
        "mw": rng.normal(0.0, amp[2], size=sh),
    }


# --------------------------------------------------------------------------------------------
# Named configurations.
#
# bell32    : 32^3, 250 m, bell h0=400 m a=1 km, 10 steps.  The written time step of 1 s violates the
#             explicit acoustic limit (c_s*dt/dx = 1.39), so it runs at 0.25 s.
# bell256   : 256x256x128, dx=dy=100 m, dz=50 m, bell h0=400 m a=2 km, 100 steps, theta' noise.
# hemi512   : 512x512x160 at 50 m, hemisphere R=1 km, 100 steps.
# The *_small variants keep each hill's shape and spacing on grids the oracle finishes in seconds.
# --------------------------------------------------------------------------------------------

def _bell32() -> Config:
    return Config("bell32", 32, 32, 32, 250.0, 250.0, 250.0, Hill("bell", 400.0, 1000.0),
                  dt=0.25, nsteps=10)


def _bell256(seed: int = 0) -> Config:
    return Config("bell256", 256, 256, 128, 100.0, 100.0, 50.0, Hill("bell", 400.0, 2000.0),
                  dt=0.05, nsteps=100, noise_sigma=0.01, seed=seed)


def _hemi512() -> Config:
    return Config("hemi512", 512, 512, 160, 50.0, 50.0, 50.0, Hill("hemisphere", 0.0, 1000.0),
                  dt=0.05, nsteps=100)


def _bell_small(seed: int = 0) -> Config:
    return Config("bell_small", 64, 48, 40, 100.0, 100.0, 50.0, Hill("bell", 400.0, 800.0),
                  dt=0.05, nsteps=100, noise_sigma=0.01, seed=seed)


def _hemi_small() -> Config:
    return Config("hemi_small", 64, 64, 40, 50.0, 50.0, 50.0, Hill("hemisphere", 0.0, 1000.0),
                  dt=0.05, nsteps=100)


def _hemi_tiny() -> Config:
    return Config("hemi_tiny", 40, 40, 28, 50.0, 50.0, 50.0, Hill("hemisphere", 0.0, 800.0),
                  dt=0.05, nsteps=100)


CONFIGS: dict = {
    "hemi_tiny": _hemi_tiny,
    "bell32": _bell32,
    "bell256": _bell256,
    "hemi512": _hemi512,
    "bell_small": _bell_small,
    "hemi_small": _hemi_small,
}


def get(name: str, **kw) -> Config:
    cfg = CONFIGS[name]()
    return cfg.replace(**kw) if kw else cfg


def paper_grid(hill: str) -> Config:
    """The paper's uniform 200 m grid of Sec. 3.1 (64 x 32 km, 16 km top)."""
    h = Hill("bell", 400.0, 1000.0) if hill == "bell" else Hill("hemisphere", 0.0, 1000.0)
    return Config("paper_" + hill, 320, 160, 80, 200.0, 200.0, 200.0, h)


# --------------------------------------------------------------------------------------------
# Ensemble of independent domains (uneven sizes, random Gaussian terrain).
# --------------------------------------------------------------------------------------------

TAN60 = math.tan(math.radians(60.0))


def _column_slope(H: np.ndarray, dx: float, dy: float) -> float:
    """Largest resolved slope of the terrain: max over columns of max(|gx|, |gy|), a column's
    gradient being the mean of the height differences along its two edges in that direction (the
    slope a grid of this spacing resolves, not the steeper corner-to-corner one)."""
    Hx = np.roll(H, -1, 0)
    gx = ((Hx + np.roll(Hx, -1, 1)) - (H + np.roll(H, -1, 1))) / (2.0 * dx)
    Hy = np.roll(H, -1, 1)
    gy = ((Hy + np.roll(Hy, -1, 0)) - (H + np.roll(H, -1, 0))) / (2.0 * dy)
    return float(max(np.abs(gx).max(), np.abs(gy).max()))


def ensemble(count: int = 64, seed: int = 0, nx_range=(48, 96), nz_range=(48, 64),
             delta: float = 100.0, dt: float = 0.09, nsteps: int = 50) -> List[Config]:
    """Draw ``count`` independent periodic domains with 1-5 Gaussian hills each.

    Per domain: ``nx, ny ~ U{48..96}``, ``nz ~ U{48..64}``, spacing ``delta`` in all directions,
    ``n ~ U{1..5}`` hills with heights ``U[100, 800]`` m, widths ``U[300, 3000]`` m and uniform
    centres, inflow ``U ~ U[5, 20]`` m/s along x and ``N ~ U[0.008, 0.02]`` 1/s.  A domain's hill set
    is redrawn (sub-seed + 1) while its largest resolved column slope exceeds 60 degrees or its
    highest point exceeds half the domain height; the number of redraws is kept in
    ``Config.redraws``.  An unmergeable cell is not redrawn here (finding one takes the merge
    rule, which this module does not hold): the merge map counts such cells and the callers treat a
    non-zero count as an error.
    """
    out = []
    master = np.random.Generator(np.random.PCG64(seed))
    for d in range(count):
        nx = int(master.integers(nx_range[0], nx_range[1] + 1))
        ny = int(master.integers(nx_range[0], nx_range[1] + 1))
        nz = int(master.integers(nz_range[0], nz_range[1] + 1))
        u0 = float(master.uniform(5.0, 20.0))
        bvn = float(master.uniform(0.008, 0.02))
        sub = int(master.integers(0, 2**31 - 1))
        redraws = 0
        while True:
            rng = np.random.Generator(np.random.PCG64(sub + redraws))
            nh = int(rng.integers(1, 6))
            hills = []
            for _ in range(nh):
                hills.append((float(rng.uniform(100.0, 800.0)), float(rng.uniform(300.0, 3000.0)),
                              float(rng.uniform(0.0, nx * delta)), float(rng.uniform(0.0, ny * delta))))
            cfg = Config(f"ens{d}", nx, ny, nz, delta, delta, delta, Hill("gauss", extra=hills),
                         bvn=bvn, u0=u0, dt=dt, nsteps=nsteps, seed=sub + redraws)
            H = terrain(cfg)
            if _column_slope(H, delta, delta) <= TAN60 and H.max() <= 0.5 * nz * delta:
                break
            redraws += 1
        cfg.H = H
        cfg.redraws = redraws
        out.append(cfg)
    return out


# --------------------------------------------------------------------------------------------
# Refined grid: cubes ("bricks") of equal cell count per level, refined near the terrain with 2:1
# balance, fully buried bricks removed, then grouped into blocks of uneven size (Sec. 2.2).
# --------------------------------------------------------------------------------------------

def terrain_at(cfg: Config, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Height of ``cfg``'s analytic hill at positions (x, y), laterally periodic with the hill centre
    on the lattice corner ``(nx/2 dx, ny/2 dy)`` of ``cfg`` (the same placement as ``terrain``)."""
    Lx, Ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    rx = np.mod(np.asarray(x, dtype=np.float64) - (cfg.nx // 2) * cfg.dx + 0.5 * Lx, Lx) - 0.5 * Lx
    ry = np.mod(np.asarray(y, dtype=np.float64) - (cfg.ny // 2) * cfg.dy + 0.5 * Ly, Ly) - 0.5 * Ly
    return np.asarray(cfg.hill(rx, ry), dtype=np.float64)


@dataclasses.dataclass
class AmrBlock:
    level: int
    org: tuple  # interior origin in level-l global cells (x, y, z)
    size: tuple  # interior size in cells


@dataclasses.dataclass
class AmrLayout:
    base: Config  # level-0 grid, hill, physics and time step dt(0)
    levels: int  # number of refinement levels (0 .. levels-1)
    brick: int  # brick edge in cells (the same at every level)
    ghost: int  # ghost cells beyond each block side (integrated on, Sec. 2.2)
    dist: list  # refinement distances d_l [m]
    blocks: List[AmrBlock]

    def cells(self, level: Optional[int] = None) -> int:
        return sum(int(np.prod(b.size)) for b in self.blocks if level is None or b.level == level)

    def box(self, b: AmrBlock):
        """Padded box of block b: (origin in level-l global cells, size, ghost below, ghost above)."""
        nzl = self.base.nz << b.level
        gb = min(self.ghost, b.org[2])  # the box stops at the ground and at the lid
        gt = min(self.ghost, nzl - (b.org[2] + b.size[2]))
        org = (b.org[0] - self.ghost, b.org[1] - self.ghost, b.org[2] - gb)
        size = (b.size[0] + 2 * self.ghost, b.size[1] + 2 * self.ghost, b.size[2] + gb + gt)
        return org, size, gb, gt

    def block_config(self, b: AmrBlock) -> Config:
        """Uniform-grid configuration of block b's padded box: spacing of its level, corner heights of
        the hill relative to the box bottom z0 (negative where the terrain lies below the box)."""
        c = self.base
        f = 1 << b.level
        dx, dy, dz = c.dx / f, c.dy / f, c.dz / f
        org, size, gb, gt = self.box(b)
        I = np.mod(org[0] + np.arange(size[0]), c.nx * f).astype(np.float64)[:, None]
        J = np.mod(org[1] + np.arange(size[1]), c.ny * f).astype(np.float64)[None, :]
        z0 = org[2] * dz
        H = terrain_at(c, I * dx, J * dy) - z0
        return c.replace(name=f"{c.name}-L{b.level}-{b.org}", nx=size[0], ny=size[1], nz=size[2], dx=dx, dy=dy,
                         dz=dz, H=np.ascontiguousarray(H), z0=z0, dt=c.dt / f, ztop=c.ztop or c.nz * c.dz)


def _leaf_of(leaves, lev, p, nb):
    """Level of the leaf brick covering brick position p of level lev (x, y periodic), or -1."""
    x, y, z = p
    for m in range(lev, -1, -1):
        sh = lev - m
        key = ((x % (nb[0] << lev)) >> sh, (y % (nb[1] << lev)) >> sh, z >> sh)
        if key in leaves[m]:
            return m
    for m in range(lev + 1, len(leaves)):
        sh = m - lev
        key = ((x % (nb[0] << lev)) << sh, (y % (nb[1] << lev)) << sh, z << sh)
        if key in leaves[m]:
            return m
    return -1


def amr_layout(base: Config, levels: int = 3, brick: int = 8, ghost: int = 6, d_fine: float = 0.0,
               band: float = 1600.0, seed: int = 0, shapes=((2, 2, 2), (4, 4, 2), (3, 3, 3))) -> AmrLayout:
    """Bricks of ``brick``^3 cells per level over the level-0 grid of ``base``.

    A brick of level l < levels-1 is refined when its bottom lies within d_l of the highest terrain
    point of its footprint (d_{levels-2} = d_fine, each coarser level adds ``band``); 2:1 balance is
    enforced across faces, edges and corners; bricks whose every cell is below the terrain are
    removed.  Each level's bricks are then grouped in lexicographic order: at every unclaimed brick a
    shape is drawn from ``shapes`` (PCG64(seed)) and the largest box of at most that shape made of
    unclaimed bricks of the level is claimed as one block.
    """
    nb0 = (base.nx // brick, base.ny // brick, base.nz // brick)
    assert all(n * brick == m for n, m in zip(nb0, (base.nx, base.ny, base.nz))), "grid must hold whole bricks"
    L = levels - 1
    dist = [d_fine + band * (L - 1 - l) for l in range(L)]
    fL = 1 << L
    # terrain at the finest corners: per-level footprint max / min from it
    hx = np.arange(base.nx * fL + 1) * (base.dx / fL)
    hy = np.arange(base.ny * fL + 1) * (base.dy / fL)
    hf = terrain_at(base, hx[:, None], hy[None, :])

    def foot(lev, bx, by):
        s = brick << (L - lev)
        return hf[bx * s:(bx + 1) * s + 1, by * s:(by + 1) * s + 1]

    leaves = [set() for _ in range(levels)]
    for bx in range(nb0[0]):
        for by in range(nb0[1]):
            for bz in range(nb0[2]):
                leaves[0].add((bx, by, bz))
    for lev in range(L):
        dz = base.dz / (1 << lev)
        for key in sorted(leaves[lev]):
            bx, by, bz = key
            if bz * brick * dz - foot(lev, bx, by).max() <= dist[lev]:
                leaves[lev].remove(key)
                for c in range(8):
                    leaves[lev + 1].add((2 * bx + (c >> 2), 2 * by + ((c >> 1) & 1), 2 * bz + (c & 1)))
    # 2:1 balance over the 26 neighbours
    changed = True
    while changed:
        changed = False
        for lev in range(L, 1, -1):
            nbl = (nb0[0] << lev, nb0[1] << lev, nb0[2] << lev)
            for (bx, by, bz) in sorted(leaves[lev]):
                for ddx in (-1, 0, 1):
                    for ddy in (-1, 0, 1):
                        for ddz in (-1, 0, 1):
                            z = bz + ddz
                            if (ddx, ddy, ddz) == (0, 0, 0) or z < 0 or z >= nbl[2]:
                                continue
                            p = ((bx + ddx) % nbl[0], (by + ddy) % nbl[1], z)
                            m = _leaf_of(leaves, lev, p, nb0)
                            if 0 <= m < lev - 1:
                                sh = lev - m
                                key = (p[0] >> sh, p[1] >> sh, p[2] >> sh)
                                leaves[m].remove(key)
                                for c in range(8):
                                    leaves[m + 1].add((2 * key[0] + (c >> 2), 2 * key[1] + ((c >> 1) & 1),
                                                       2 * key[2] + (c & 1)))
                                changed = True
    # fully buried bricks: top at or below the lowest corner height of the footprint at their level
    for lev in range(levels):
        dz = base.dz / (1 << lev)
        step = 1 << (L - lev)
        for key in sorted(leaves[lev]):
            bx, by, bz = key
            if (bz + 1) * brick * dz <= foot(lev, bx, by)[::step, ::step].min():
                leaves[lev].remove(key)
    # group into blocks
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = []
    for lev in range(levels):
        nbl = (nb0[0] << lev, nb0[1] << lev, nb0[2] << lev)
        free = set(leaves[lev])
        for key in sorted(leaves[lev]):
            if key not in free:
                continue
            sx, sy, sz = shapes[int(rng.integers(len(shapes)))]
            best, bv = (1, 1, 1), 0
            for ax in range(1, sx + 1):
                for ay in range(1, sy + 1):
                    for az in range(1, sz + 1):
                        if key[0] + ax > nbl[0] or key[1] + ay > nbl[1] or key[2] + az > nbl[2]:
                            continue
                        if ax * ay * az <= bv:
                            continue
                        if all((key[0] + a, key[1] + b, key[2] + c) in free
                               for a in range(ax) for b in range(ay) for c in range(az)):
                            best, bv = (ax, ay, az), ax * ay * az
            ax, ay, az = best
            for a in range(ax):
                for b in range(ay):
                    for c in range(az):
                        free.discard((key[0] + a, key[1] + b, key[2] + c))
            blocks.append(AmrBlock(lev, (key[0] * brick, key[1] * brick, key[2] * brick),
                                   (ax * brick, ay * brick, az * brick)))
    return AmrLayout(base, levels, brick, ghost, dist, blocks)


def amr_hemisphere(target_blocks: int = 2000, seed: int = 0) -> AmrLayout:
    """The refined hemisphere workload: level-0 grid 128x128x64 at 200 m (25.6 x 25.6 x 12.8 km),
    hemisphere of radius 1 km, levels 1 (100 m) and 2 (50 m), dt(0) = 0.2 s, 25 level-0 steps; the
    level-2 distance is chosen by bisection so that the block count is closest to ``target_blocks``."""
    base = Config("amr_hemi", 128, 128, 64, 200.0, 200.0, 200.0, Hill("hemisphere", 0.0, 1000.0),
                  dt=0.2, nsteps=25)
    lo, hi = 0.0, 6400.0
    best = None
    for _ in range(14):
        mid = 0.5 * (lo + hi)
        lay = amr_layout(base, d_fine=mid, seed=seed)
        n = len(lay.blocks)
        if best is None or abs(n - target_blocks) < abs(len(best.blocks) - target_blocks):
            best = lay
        if n < target_blocks:
            lo = mid
        else:
            hi = mid
    return best


# --------------------------------------------------------------------------------------------
# The refined-grid experiment of Sec. 3.2: cubes of 20^3 cells over the 64 x 32 x 16 km domain.
# --------------------------------------------------------------------------------------------

CBCM_CUBE = 20  # cells per cube edge at every level (Sec. 3.2)


def cbcm_regions(levels: int):
    """Cubes each level refines in the Sec. 3.2 layouts, as index ranges of that level's cubes
    ((x0, x1), (y0, y1), (z0, z1)), half-open.  The paper gives the cube counts (64, 148, 232) and
    the spacings, not the criterion; the counts fix 12 refined cubes per level, read here as the
    3 x 2 x 2 cubes around the hill and one cube downstream of it: level 0 (8 x 4 x 2 cubes of
    8 km) refines x 24-48 km, y 8-24 km, z 0-16 km; level 1 (4 km cubes) refines x 28-40 km,
    y 12-20 km, z 0-8 km."""
    return [((3, 6), (1, 3), (0, 2)), ((7, 10), (3, 5), (0, 2))][: levels - 1]


def cbcm_hemisphere(levels: int = 3, ghost: int = 6) -> AmrLayout:
    """The grids of Sec. 3.2 over the hemisphere of Sec. 3.1.2 (radius 1 km at (32, 16) km, U = 10 m/s,
    N = 0.01 1/s, theta_0 = 300 K): level 0 is 160 x 80 x 40 cells at 400 m (8 x 4 x 2 cubes of
    20^3 cells); ``levels`` = 2 and 3 add the 200 m and 100 m cubes of ``cbcm_regions`` (148 and 232
    cubes in all; the uniform 100 m grid holds 4096).  Every cube is one block; dt(0) = 0.5 s
    (dt = delta / 800 s at every level)."""
    base = Config("cbcm_hemi", 160, 80, 40, 400.0, 400.0, 400.0, Hill("hemisphere", 0.0, 1000.0), u0=10.0,
                  v0=0.0, bvn=0.01, theta0=300.0, dt=0.5, nsteps=7200)
    n = CBCM_CUBE
    regions = cbcm_regions(levels)
    cubes = {(x, y, z) for x in range(base.nx // n) for y in range(base.ny // n) for z in range(base.nz // n)}
    blocks = []
    for lev in range(levels):
        nxt = set()
        if lev < len(regions):
            (x0, x1), (y0, y1), (z0, z1) = regions[lev]
            for x in range(x0, x1):
                for y in range(y0, y1):
                    for z in range(z0, z1):
                        cubes.discard((x, y, z))
                        nxt.update((2 * x + a, 2 * y + b, 2 * z + c) for a in (0, 1) for b in (0, 1) for c in (0, 1))
        blocks += [AmrBlock(lev, (x * n, y * n, z * n), (n, n, n)) for (x, y, z) in sorted(cubes)]
        cubes = nxt
    return AmrLayout(base, levels, n, ghost, [], blocks)
