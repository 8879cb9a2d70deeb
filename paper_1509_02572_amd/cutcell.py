"""Python binding of libcutcell.so (C ABI in include/cutcell.h).

Argument marshalling only: every step of the cut-cell stage runs in the library's HIP kernels.
PyTorch provides device memory and the stream.  The functions below carry the same names as the C
entry points and take torch tensors; ``Domain`` allocates the arrays of one uniform grid and chains
the calls of a Runge-Kutta step.  Importing this module on a machine without the built library, or
calling it without a HIP device, raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libcutcell.so")

CC_OK, CC_EINVAL, CC_EDEVICE, CC_EUNMERGEABLE, CC_ENOPLANE, CC_ENONFINITE, CC_ETERRAIN = range(7)
CC_F64, CC_F32_PERT = 0, 1
CC_NSTATUS = 8
SOLID, OPEN, ABSORBED, ORPHAN = 0, 1, 2, 3
GROUND, PRED, MFACE = 0, 1, 2
STATUS_NAMES = ("unmergeable", "noplane", "nonfinite", "terrain", "groupsize")


class cc_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nzs", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("nsub", C.c_int32), ("tile", C.c_int32), ("z0", C.c_double)]


class cc_phys(C.Structure):
    _fields_ = [(n, C.c_double)
                for n in ("g", "rd", "cp", "p0", "theta0", "bvn", "u0", "v0", "kdh", "kdv", "zsp", "rsp", "ztop")]


class cc_geom(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("H", "V", "Ax", "Ay", "Az", "col", "nrm", "cls", "dir",
                                           "vcls", "master", "gnext", "Vgroup", "colk", "stage_ws")] + \
               [("kband", C.c_int32), ("nband_tiles", C.c_int32), ("side", C.c_void_p)]


class cc_state(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("rho", "rth", "mu", "mv", "mw", "rho_lo", "rth_lo")]


class cc_block(C.Structure):
    _fields_ = [("grid", cc_grid), ("phys", cc_phys), ("geom", cc_geom), ("base", C.c_void_p),
                ("q", cc_state * 3), ("level", C.c_int32), ("org", C.c_int32 * 3), ("ilo", C.c_int32 * 3),
                ("ihi", C.c_int32 * 3)]


_lib = None


def lib():
    """Load libcutcell.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"libcutcell.so not built at {LIBPATH}; run __graft_entry__.build()")
        L = C.CDLL(LIBPATH)
        G, P, GM, S = C.POINTER(cc_grid), C.POINTER(cc_phys), C.POINTER(cc_geom), C.POINTER(cc_state)
        vp, i64p = C.c_void_p, C.c_void_p
        L.cutcell_version.restype = C.c_char_p
        L.cutcell_last_error.restype = C.c_char_p
        L.cutcell_base_state.argtypes = [G, P, vp, vp]
        L.cutcell_geometry.argtypes = [G, GM, i64p, vp]
        L.cutcell_merge_map.argtypes = [G, GM, i64p, vp]
        L.cutcell_band_setup.argtypes = [G, GM, vp]
        L.cutcell_stage_ctx_create.argtypes = [C.POINTER(C.c_void_p)]
        L.cutcell_stage_ctx_destroy.argtypes = [vp]
        L.cutcell_init_state.argtypes = [G, P, GM, vp, C.c_int, vp, S, i64p, vp]
        L.cutcell_diagnose.argtypes = [G, P, GM, vp, C.c_int, S, i64p, vp]
        L.cutcell_tendency.argtypes = [G, P, GM, vp, C.c_int, S, S, vp]
        L.cutcell_rk_stage.argtypes = [G, P, GM, vp, C.c_int, S, S, S, C.c_double, C.c_int32, i64p, vp]
        L.cutcell_rk_update.argtypes = [G, P, GM, vp, C.c_int, S, S, S, C.c_double, C.c_int32, i64p, vp]
        L.cutcell_lf_workspace_bytes.argtypes = [G, C.c_int]
        L.cutcell_lf_workspace_bytes.restype = C.c_size_t
        L.cutcell_pform.argtypes = [G, P, GM, vp, C.c_int, S, C.c_int32, vp]
        L.cutcell_lf_step.argtypes = [G, P, GM, vp, C.c_int, S, S, S, vp, C.c_double, C.c_double, C.c_int32, i64p,
                                      vp]
        L.cutcell_stage_workspace_bytes.argtypes = [G, C.c_int]
        L.cutcell_stage_workspace_bytes.restype = C.c_size_t
        L.cutcell_reduce_workspace.argtypes = [G]
        L.cutcell_reduce_workspace.restype = C.c_size_t
        L.cutcell_reduce.argtypes = [G, P, GM, vp, C.c_int, S, vp, vp, vp]
        L.cutcell_reduce_noalloc.argtypes = [G, P, GM, vp, C.c_int, S, vp, vp]
        L.cutcell_check_status.argtypes = [vp, vp, vp]
        L.amr_batch_workspace_bytes.argtypes = [C.c_int32, C.c_int]
        L.amr_batch_workspace_bytes.restype = C.c_size_t
        L.amr_batch_create.argtypes = [C.POINTER(cc_block), C.c_int32, C.c_int, C.c_int32, vp,
                                       C.POINTER(C.c_void_p), vp]
        L.amr_block_step.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, i64p, vp]
        L.amr_batch_current.argtypes = [vp, C.c_int32]
        L.amr_batch_current.restype = C.c_int32
        L.amr_batch_levels.argtypes = [vp]
        L.amr_batch_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
        L.amr_batch_info.restype = C.c_int
        L.amr_batch_levels.restype = C.c_int32
        i3 = C.c_int32 * 3
        L.amr_hierarchy_workspace_bytes.argtypes = [C.POINTER(cc_block), C.c_int32, C.c_int, i3,
                                                    C.POINTER(C.c_size_t)]
        L.amr_hierarchy_create.argtypes = [C.POINTER(cc_block), C.c_int32, C.c_int, C.c_int32, i3, vp, C.c_size_t,
                                           C.POINTER(C.c_void_p), vp]
        L.amr_hierarchy_sync.argtypes = [vp, vp]
        L.amr_batch_destroy.argtypes = [vp]
        for name in ("cutcell_base_state", "cutcell_geometry", "cutcell_merge_map", "cutcell_init_state",
                     "cutcell_diagnose", "cutcell_tendency", "cutcell_rk_stage", "cutcell_rk_update", "cutcell_reduce",
                     "cutcell_reduce_noalloc", "cutcell_band_setup", "cutcell_stage_ctx_create", "cutcell_pform",
                     "cutcell_lf_step",
                     "cutcell_stage_ctx_destroy",
                     "cutcell_check_status", "amr_batch_create", "amr_block_step", "amr_batch_destroy",
                     "amr_hierarchy_workspace_bytes", "amr_hierarchy_create", "amr_hierarchy_sync"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(rc: int, what: str):
    if rc != CC_OK:
        raise RuntimeError(f"{what} failed ({rc}): {lib().cutcell_last_error().decode()}")


def version() -> str:
    return lib().cutcell_version().decode()


# ------------------------------------------------------------------------------------------------
# entry points with the C names (torch tensors in, status checked)
# ------------------------------------------------------------------------------------------------

def cutcell_base_state(grid: cc_grid, phys: cc_phys, base: torch.Tensor, stream=None):
    _check(lib().cutcell_base_state(C.byref(grid), C.byref(phys), _ptr(base), _stream(stream)),
           "cutcell_base_state")


def cutcell_geometry(grid: cc_grid, geom: cc_geom, status: torch.Tensor, stream=None):
    _check(lib().cutcell_geometry(C.byref(grid), C.byref(geom), _ptr(status), _stream(stream)),
           "cutcell_geometry")


def cutcell_merge_map(grid: cc_grid, geom: cc_geom, status: torch.Tensor, stream=None):
    _check(lib().cutcell_merge_map(C.byref(grid), C.byref(geom), _ptr(status), _stream(stream)),
           "cutcell_merge_map")


def cutcell_band_setup(grid: cc_grid, geom: cc_geom, stream=None):
    _check(lib().cutcell_band_setup(C.byref(grid), C.byref(geom), _stream(stream)), "cutcell_band_setup")


def cutcell_stage_ctx_create() -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().cutcell_stage_ctx_create(C.byref(out)), "cutcell_stage_ctx_create")
    return out


def cutcell_stage_ctx_destroy(ctx):
    _check(lib().cutcell_stage_ctx_destroy(ctx), "cutcell_stage_ctx_destroy")


def cutcell_init_state(grid, phys, geom, base, prec, noise, q: cc_state, status, stream=None):
    _check(lib().cutcell_init_state(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                    _ptr(noise), C.byref(q), _ptr(status), _stream(stream)),
           "cutcell_init_state")


def cutcell_diagnose(grid, phys, geom, base, prec, q: cc_state, status, stream=None):
    _check(lib().cutcell_diagnose(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                  C.byref(q), _ptr(status), _stream(stream)), "cutcell_diagnose")


def cutcell_tendency(grid, phys, geom, base, prec, q: cc_state, dq: cc_state, stream=None):
    _check(lib().cutcell_tendency(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                  C.byref(q), C.byref(dq), _stream(stream)), "cutcell_tendency")


def cutcell_pform(grid, phys, geom, base, prec, q: cc_state, to_p: bool, stream=None):
    _check(lib().cutcell_pform(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec, C.byref(q),
                               1 if to_p else 0, _stream(stream)), "cutcell_pform")


def cutcell_lf_step(grid, phys, geom, base, prec, qm: Optional[cc_state], q0: cc_state, qp: cc_state, work, dt: float,
                    nu: float, first: bool, status, stream=None):
    _check(lib().cutcell_lf_step(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                 C.byref(qm) if qm is not None else None, C.byref(q0), C.byref(qp), _ptr(work), dt,
                                 nu, 1 if first else 0, _ptr(status), _stream(stream)), "cutcell_lf_step")


def cutcell_rk_stage(grid, phys, geom, base, prec, qn: cc_state, qs: cc_state, qo: cc_state,
                     stage_dt: float, final_stage: bool, status, stream=None):
    _check(lib().cutcell_rk_stage(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                  C.byref(qn), C.byref(qs), C.byref(qo), stage_dt, int(final_stage),
                                  _ptr(status), _stream(stream)), "cutcell_rk_stage")


def cutcell_rk_update(grid, phys, geom, base, prec, qn: cc_state, qs: cc_state, qo: cc_state,
                      stage_dt: float, final_stage: bool, status, stream=None):
    _check(lib().cutcell_rk_update(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                   C.byref(qn), C.byref(qs), C.byref(qo), stage_dt, int(final_stage),
                                   _ptr(status), _stream(stream)), "cutcell_rk_update")


def cutcell_reduce(grid, phys, geom, base, prec, q: cc_state, workspace, out, stream=None):
    _check(lib().cutcell_reduce(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                C.byref(q), _ptr(workspace), _ptr(out), _stream(stream)), "cutcell_reduce")


def cutcell_reduce_noalloc(grid, phys, geom, base, prec, q: cc_state, out, stream=None):
    _check(lib().cutcell_reduce_noalloc(C.byref(grid), C.byref(phys), C.byref(geom), _ptr(base), prec,
                                        C.byref(q), _ptr(out), _stream(stream)), "cutcell_reduce_noalloc")


def cutcell_check_status(status: torch.Tensor, stream=None) -> (int, np.ndarray):
    host = np.zeros(CC_NSTATUS, np.int64)
    rc = lib().cutcell_check_status(_ptr(status), host.ctypes.data_as(C.c_void_p), _stream(stream))
    return rc, host


def amr_batch_workspace_bytes(nblocks: int, prec: int) -> int:
    return int(lib().amr_batch_workspace_bytes(nblocks, prec))


def amr_batch_create(blocks, prec: int, tile: int, workspace: torch.Tensor, stream=None) -> C.c_void_p:
    arr = (cc_block * len(blocks))(*blocks)
    h = C.c_void_p()
    _check(lib().amr_batch_create(arr, len(blocks), prec, tile, _ptr(workspace), C.byref(h), _stream(stream)),
           "amr_batch_create")
    return h


def amr_block_step(batch: C.c_void_p, dt: float, nsteps: int, use_graph: bool, status: torch.Tensor,
                   stream=None):
    _check(lib().amr_block_step(batch, dt, nsteps, int(use_graph), _ptr(status), _stream(stream)),
           "amr_block_step")


def amr_batch_current(batch: C.c_void_p, level: int = 0) -> int:
    return int(lib().amr_batch_current(batch, level))


def amr_batch_info(batch: C.c_void_p, level: int) -> Dict[str, int]:
    out = (C.c_int64 * 8)()
    _check(lib().amr_batch_info(batch, level, out), "amr_batch_info")
    keys = ("blocks", "regular_tiles", "band_tiles", "diag_columns", "same_refill", "same_refill_near",
            "inject", "restrict")
    return {k: int(v) for k, v in zip(keys, out)}


def amr_batch_levels(batch: C.c_void_p) -> int:
    return int(lib().amr_batch_levels(batch))


def amr_hierarchy_workspace_bytes(blocks, prec: int, domain0) -> int:
    arr = (cc_block * len(blocks))(*blocks)
    n = C.c_size_t()
    _check(lib().amr_hierarchy_workspace_bytes(arr, len(blocks), prec, (C.c_int32 * 3)(*domain0), C.byref(n)),
           "amr_hierarchy_workspace_bytes")
    return int(n.value)


def amr_hierarchy_create(blocks, prec: int, tile: int, domain0, workspace: torch.Tensor, stream=None) -> C.c_void_p:
    arr = (cc_block * len(blocks))(*blocks)
    h = C.c_void_p()
    _check(lib().amr_hierarchy_create(arr, len(blocks), prec, tile, (C.c_int32 * 3)(*domain0), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), C.byref(h), _stream(stream)),
           "amr_hierarchy_create")
    return h


def amr_hierarchy_sync(batch: C.c_void_p, stream=None):
    _check(lib().amr_hierarchy_sync(batch, _stream(stream)), "amr_hierarchy_sync")


def amr_batch_destroy(batch: C.c_void_p):
    _check(lib().amr_batch_destroy(batch), "amr_batch_destroy")


# ------------------------------------------------------------------------------------------------
# Domain: the arrays of one uniform grid on one device
# ------------------------------------------------------------------------------------------------
FIELDS = ("rho", "rth", "mu", "mv", "mw")


def default_nzs(nz: int) -> int:
    return (nz + 15) // 16 * 16


class State:
    """Device arrays of one state (double: paper variables; float: perturbation form with the
    low-order parts of rho' and (rho theta)')."""

    def __init__(self, n: int, dtype, device):
        self.t = {f: torch.zeros(n, dtype=dtype, device=device) for f in FIELDS}
        if dtype == torch.float32:
            self.t["rho_lo"] = torch.zeros(n, dtype=dtype, device=device)
            self.t["rth_lo"] = torch.zeros(n, dtype=dtype, device=device)
        self.c = cc_state(*[_ptr(self.t[f]) for f in FIELDS], _ptr(self.t.get("rho_lo")),
                          _ptr(self.t.get("rth_lo")))

    def __getitem__(self, f):
        return self.t[f]


class Domain:
    """Grid, geometry, merge map and base state of one configuration on ``device``.

    ``prec`` is ``"f64"`` (paper variables in double) or ``"f32"`` (float perturbation form).
    ``side_stream``: give the geometry a stage context, so that the band points of an update run on
    its side stream beside the regular points (members of a batch do not need one)."""

    def __init__(self, cfg, prec: str = "f64", device: str = "cuda:0", nzs: Optional[int] = None,
                 H: Optional[np.ndarray] = None, tile: int = 0, stage_ws: bool = True, side_stream: bool = True):
        from . import workloads
        if not torch.cuda.is_available():
            raise RuntimeError("libcutcell needs a HIP device")
        self.cfg = cfg
        self.dev = torch.device(device)
        self.prec = CC_F64 if prec == "f64" else CC_F32_PERT
        self.dtype = torch.float64 if self.prec == CC_F64 else torch.float32
        nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
        self.nzs = nzs or default_nzs(nz)
        self.n = nx * ny * self.nzs
        self.grid = cc_grid(nx, ny, nz, self.nzs, cfg.dx, cfg.dy, cfg.dz, cfg.nsub, tile, cfg.z0)
        self.phys = cc_phys(cfg.g, cfg.rd, cfg.cp, cfg.p0, cfg.theta0, cfg.bvn, cfg.u0, cfg.v0, cfg.kdh, cfg.kdv,
                            cfg.zsp, cfg.rsp, cfg.ztop)
        Hn = workloads.terrain(cfg) if H is None else H
        d, f64, i8, i32 = self.dev, torch.float64, torch.int8, torch.int32
        nc = nx * ny
        self.g: Dict[str, torch.Tensor] = {
            "H": torch.from_numpy(np.ascontiguousarray(Hn, dtype=np.float64).ravel()).to(d),
            "V": torch.zeros(self.n, dtype=f64, device=d), "Ax": torch.zeros(self.n, dtype=f64, device=d),
            "Ay": torch.zeros(self.n, dtype=f64, device=d), "Az": torch.zeros(self.n, dtype=f64, device=d),
            "col": torch.zeros(3 * nc, dtype=f64, device=d), "nrm": torch.zeros(3 * nc, dtype=f64, device=d),
            "cls": torch.zeros(self.n, dtype=i8, device=d), "dir": torch.zeros(self.n, dtype=i8, device=d),
            "vcls": torch.zeros(self.n, dtype=i8, device=d), "master": torch.zeros(self.n, dtype=i32, device=d),
            "gnext": torch.zeros(self.n, dtype=i32, device=d), "Vgroup": torch.zeros(self.n, dtype=f64, device=d),
            "colk": torch.zeros(3 * nc, dtype=i32, device=d),
        }
        # workspace of the two-pass update (p' and lattice velocities), bytes rounded up to 8
        wsb = lib().cutcell_stage_workspace_bytes(C.byref(self.grid), self.prec) if stage_ws else 0
        self.g["stage_ws"] = torch.empty(max(wsb // 8, 1), dtype=torch.float64, device=d) if stage_ws else None
        self.geom = cc_geom(*[_ptr(self.g[k]) for k in ("H", "V", "Ax", "Ay", "Az", "col", "nrm", "cls",
                                                         "dir", "vcls", "master", "gnext", "Vgroup", "colk",
                                                         "stage_ws")])
        self.base = torch.zeros(6 * nz, dtype=f64, device=d)
        self.status = torch.zeros(CC_NSTATUS, dtype=torch.int64, device=d)
        self.ws = torch.zeros(lib().cutcell_reduce_workspace(C.byref(self.grid)) // 8 + 1, dtype=f64, device=d)
        self.red = torch.zeros(4, dtype=f64, device=d)
        cutcell_base_state(self.grid, self.phys, self.base)
        cutcell_geometry(self.grid, self.geom, self.status)
        cutcell_merge_map(self.grid, self.geom, self.status)
        cutcell_band_setup(self.grid, self.geom)
        self.ctx = None
        if side_stream:
            self.ctx = cutcell_stage_ctx_create()
            self.geom.side = self.ctx

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and _lib is not None:
            self.geom.side = None
            cutcell_stage_ctx_destroy(ctx)
            self.ctx = None

    # -- states -------------------------------------------------------------------------------
    def new_state(self) -> State:
        return State(self.n, self.dtype, self.dev)

    def pad(self, a: np.ndarray) -> torch.Tensor:
        """(nx, ny, nz) host array -> padded device vector of the state layout (double)."""
        cfg = self.cfg
        out = np.zeros((cfg.nx, cfg.ny, self.nzs))
        out[:, :, :cfg.nz] = a
        return torch.from_numpy(out.ravel()).to(self.dev)

    def unpad(self, t: torch.Tensor) -> np.ndarray:
        cfg = self.cfg
        return t.detach().cpu().numpy().reshape(cfg.nx, cfg.ny, self.nzs)[:, :, :cfg.nz].copy()

    def init_state(self, noise: Optional[np.ndarray] = None) -> State:
        q = self.new_state()
        nt = self.pad(noise) if noise is not None else None
        cutcell_init_state(self.grid, self.phys, self.geom, self.base, self.prec, nt, q.c, self.status)
        return q

    # -- hot path -----------------------------------------------------------------------------
    def diagnose(self, q: State):
        cutcell_diagnose(self.grid, self.phys, self.geom, self.base, self.prec, q.c, self.status)

    def tendency(self, q: State) -> State:
        dq = self.new_state()
        cutcell_tendency(self.grid, self.phys, self.geom, self.base, self.prec, q.c, dq.c)
        return dq

    def rk_stage(self, qn: State, qs: State, qo: State, stage_dt: float, final_stage: bool = False):
        cutcell_rk_stage(self.grid, self.phys, self.geom, self.base, self.prec, qn.c, qs.c, qo.c,
                         stage_dt, final_stage, self.status)

    def rk_update(self, qn: State, qs: State, qo: State, stage_dt: float, final_stage: bool = False):
        cutcell_rk_update(self.grid, self.phys, self.geom, self.base, self.prec, qn.c, qs.c, qo.c,
                          stage_dt, final_stage, self.status)

    def step(self, q: State, s1: State, s2: State, dt: float):
        """One three-stage step; the new state is left in ``s1`` (returns (s1, q, s2) rotated so
        that the first element is the new state)."""
        self.rk_stage(q, q, s1, dt / 3.0)
        self.rk_stage(q, s1, s2, dt / 2.0)
        self.rk_stage(q, s2, s1, dt, final_stage=True)
        return s1, q, s2

    def run(self, q: State, dt: float, nsteps: int) -> State:
        a, b, c = q, self.new_state(), self.new_state()
        for _ in range(nsteps):
            a, b, c = self.step(a, b, c, dt)
        return a

    # -- leap-frog with the Robert-Asselin filter, p' form -------------------------------------
    def pform(self, q: State, to_p: bool = True) -> State:
        """Convert q's thermodynamic slot in place: (rho theta)' -> p' (to_p) or back; returns q."""
        cutcell_pform(self.grid, self.phys, self.geom, self.base, self.prec, q.c, to_p)
        return q

    def lf_step(self, qm: Optional[State], q0: State, qp: State, dt: float, nu: float, first: bool = False):
        """One leap-frog step in p' form into qp; q0 is filtered in place unless `first`."""
        if getattr(self, "_lfws", None) is None:
            nb = lib().cutcell_lf_workspace_bytes(C.byref(self.grid), self.prec)
            self._lfws = torch.empty(nb // 8 + 1, dtype=torch.float64, device=self.dev)
        cutcell_lf_step(self.grid, self.phys, self.geom, self.base, self.prec, qm.c if qm is not None else None,
                        q0.c, qp.c, self._lfws, dt, nu, first, self.status)

    def run_lf(self, q: State, dt: float, nsteps: int, nu: float):
        """nsteps leap-frog steps from q (p' form, left untouched; the first a forward step):
        returns (q^N, filtered q^{N-1})."""
        qm, q0, qp = self.new_state(), self.new_state(), self.new_state()
        for f in q.t:
            q0.t[f].copy_(q.t[f])
        self.lf_step(None, q0, qp, dt, nu, first=True)
        qm, q0, qp = q0, qp, qm
        for _ in range(nsteps - 1):
            self.lf_step(qm, q0, qp, dt, nu)
            qm, q0, qp = q0, qp, qm
        return q0, qm

    def reduce(self, q: State) -> np.ndarray:
        cutcell_reduce(self.grid, self.phys, self.geom, self.base, self.prec, q.c, self.ws, self.red)
        return self.red.cpu().numpy().copy()

    def check(self) -> np.ndarray:
        rc, host = cutcell_check_status(self.status)
        return host

    # -- host views ---------------------------------------------------------------------------
    def geometry_numpy(self) -> Dict[str, np.ndarray]:
        cfg = self.cfg
        out = {}
        for k in ("V", "Ax", "Ay", "Az", "cls", "dir", "vcls", "master", "gnext", "Vgroup"):
            out[k] = self.unpad(self.g[k])
        nc = cfg.nx * cfg.ny
        col = self.g["col"].cpu().numpy().reshape(3, cfg.nx, cfg.ny)
        out["hc"], out["gx"], out["gy"] = col[0].copy(), col[1].copy(), col[2].copy()
        out["nrm"] = self.g["nrm"].cpu().numpy().reshape(3, cfg.nx, cfg.ny).copy()
        out["colk"] = self.g["colk"].cpu().numpy().reshape(3, cfg.nx, cfg.ny).copy()
        m = out["master"].astype(np.int64)
        ok = m >= 0  # padded linear index -> unpadded linear index
        mm = m[ok]
        k = mm % self.nzs
        col_ = mm // self.nzs
        m[ok] = col_ * cfg.nz + k
        out["master"] = m.astype(np.int32)
        return out

    def state_numpy(self, q: State) -> Dict[str, np.ndarray]:
        """Host copy in double; the float form's low-order parts are added to rho', (rho theta)'."""
        out = {f: self.unpad(q.t[f]).astype(np.float64) for f in FIELDS}
        if "rho_lo" in q.t:
            out["rho"] += self.unpad(q.t["rho_lo"]).astype(np.float64)
            out["rth"] += self.unpad(q.t["rth_lo"]).astype(np.float64)
        return out


# ------------------------------------------------------------------------------------------------
# Batch: independent domains stepped together (one update and one diagnostic launch per stage)
# ------------------------------------------------------------------------------------------------
class Batch:
    """Level-0 blocks (each a ``Domain`` with three state buffers) stepped by ``amr_block_step``.

    ``states[m]`` is the initial state of member m; it is copied into the member's first buffer."""

    def __init__(self, domains, states, tile: int = 0):
        if not domains or len(domains) != len(states):
            raise ValueError("one initial state per domain expected")
        prec = domains[0].prec
        if any(d.prec != prec for d in domains):
            raise ValueError("all members of a batch share one precision")
        self.domains = list(domains)
        self.prec = prec
        self.bufs = []
        blocks = []
        for d, q in zip(domains, states):
            b = [d.new_state(), d.new_state(), d.new_state()]
            for f in q.t:
                b[0].t[f].copy_(q.t[f])
            self.bufs.append(b)
            blocks.append(cc_block(d.grid, d.phys, d.geom, C.c_void_p(d.base.data_ptr()),
                                   (cc_state * 3)(b[0].c, b[1].c, b[2].c), 0, (C.c_int32 * 3)(0, 0, 0),
                                   (C.c_int32 * 3)(0, 0, 0), (C.c_int32 * 3)(d.cfg.nx, d.cfg.ny, d.cfg.nz)))
        dev = domains[0].dev
        self.status = torch.zeros(CC_NSTATUS, dtype=torch.int64, device=dev)
        nbytes = amr_batch_workspace_bytes(len(domains), prec)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.h = amr_batch_create(blocks, prec, tile, self.ws)
        self.cells = sum(d.cfg.nx * d.cfg.ny * d.cfg.nz for d in domains)

    def step(self, dt: float, nsteps: int = 1, use_graph: bool = False, stream=None):
        amr_block_step(self.h, dt, nsteps, use_graph, self.status, stream)

    def current(self):
        """Current state of every member."""
        c = amr_batch_current(self.h, 0)
        return [b[c] for b in self.bufs]

    def check(self) -> np.ndarray:
        rc, host = cutcell_check_status(self.status)
        return host

    def close(self):
        if self.h:
            amr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# Hierarchy: a refined grid (blocks of several levels, each a padded box) stepped by amr_block_step
# ------------------------------------------------------------------------------------------------
class Hierarchy:
    """Blocks of a ``workloads.AmrLayout`` on ``device``: one ``Domain`` per block (its padded box,
    terrain heights relative to the box bottom), three state buffers each, initial state of uniform
    inflow, all ghost cells synchronised."""

    def __init__(self, layout, prec: str = "f64", device: str = "cuda:0", tile: int = 0):
        self.layout = layout
        self.doms = []
        self.bufs = []
        self.own = []  # (ilo, ihi) of each block's own cells in its box
        blocks = []
        for b in layout.blocks:
            cfg = layout.block_config(b)
            d = Domain(cfg, prec, device, stage_ws=False, side_stream=False)
            org, size, gb, gt = layout.box(b)
            ilo = (layout.ghost, layout.ghost, gb)
            ihi = (ilo[0] + b.size[0], ilo[1] + b.size[1], ilo[2] + b.size[2])
            q = [d.init_state(), d.new_state(), d.new_state()]
            self.doms.append(d)
            self.bufs.append(q)
            self.own.append((ilo, ihi))
            blocks.append(cc_block(d.grid, d.phys, d.geom, C.c_void_p(d.base.data_ptr()),
                                   (cc_state * 3)(q[0].c, q[1].c, q[2].c), b.level, (C.c_int32 * 3)(*org),
                                   (C.c_int32 * 3)(*ilo), (C.c_int32 * 3)(*ihi)))
        self.prec = self.doms[0].prec
        dev = self.doms[0].dev
        self.domain0 = (layout.base.nx, layout.base.ny, layout.base.nz)
        nbytes = amr_hierarchy_workspace_bytes(blocks, self.prec, self.domain0)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.status = torch.zeros(CC_NSTATUS, dtype=torch.int64, device=dev)
        self.h = amr_hierarchy_create(blocks, self.prec, tile, self.domain0, self.ws)
        amr_hierarchy_sync(self.h)

    def sync(self):
        amr_hierarchy_sync(self.h)

    def step(self, nsteps: int = 1, use_graph: bool = False, dt: Optional[float] = None, stream=None):
        amr_block_step(self.h, self.layout.base.dt if dt is None else dt, nsteps, use_graph, self.status, stream)

    def current(self):
        cur = [amr_batch_current(self.h, l) for l in range(amr_batch_levels(self.h))]
        return [q[cur[b.level]] for q, b in zip(self.bufs, self.layout.blocks)]

    def own_cells(self, m: int, q: State) -> Dict[str, np.ndarray]:
        """Host copy (double, low-order parts added) of block m's own cells."""
        (i0, j0, k0), (i1, j1, k1) = self.own[m]
        full = self.doms[m].state_numpy(q)
        return {f: v[i0:i1, j0:j1, k0:k1] for f, v in full.items()}

    def check(self) -> np.ndarray:
        rc, host = cutcell_check_status(self.status)
        return host

    def close(self):
        if getattr(self, "h", None):
            amr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
