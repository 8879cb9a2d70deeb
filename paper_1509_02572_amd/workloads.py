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


def _edge_slope(H: np.ndarray, dx: float, dy: float) -> float:
    """Largest corner-to-corner height difference per unit length (terrain-only check)."""
    sx = np.abs(np.roll(H, -1, 0) - H).max() / dx
    sy = np.abs(np.roll(H, -1, 1) - H).max() / dy
    return float(max(sx, sy))


def ensemble(count: int = 64, seed: int = 0, nx_range=(48, 96), nz_range=(48, 64),
             delta: float = 100.0, dt: float = 0.09, nsteps: int = 50) -> List[Config]:
    """Draw ``count`` independent periodic domains with 1-5 Gaussian hills each.

    Per domain: ``nx, ny ~ U{48..96}``, ``nz ~ U{48..64}``, spacing ``delta`` in all directions,
    ``n ~ U{1..5}`` hills with heights ``U[100, 800]`` m, widths ``U[300, 3000]`` m and uniform
    centres, inflow ``U ~ U[5, 20]`` m/s along x and ``N ~ U[0.008, 0.02]`` 1/s.  A domain's hill set
    is redrawn (sub-seed + 1) while its steepest corner-to-corner slope exceeds 60 degrees or its
    highest point exceeds half the domain height.
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
            if _edge_slope(H, delta, delta) <= TAN60 and H.max() <= 0.5 * nz * delta:
                break
            redraws += 1
        cfg.H = H
        out.append(cfg)
    return out
