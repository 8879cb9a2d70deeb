"""Plain reference of the refined-grid step (Sec. 2.2 of the paper) on top of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the library's refined-grid batches.  It
shares nothing with the HIP path: owners of ghost cells are found by searching the blocks, the
coarse-fine faces by walking every face of every coarse cell, and each block's box is stepped by
the uniform-grid oracle (a box is a grid of its own: laterally periodic, ground at its bottom, lid
at its top; those box boundaries only ever touch ghost layers that are refilled or go stale).

The step, in the paper's order:
  * levels advance finest first: a level-l step of dt(l) follows two level-(l+1) steps of dt(l)/2;
  * every step of a level is the three-stage Runge-Kutta step q_out = q_n + c dt L(q_s),
    c = 1/3, 1/2, 1, on every block of the level; after each stage the block's ghost cells that
    belong to another block of the same level take that block's values;
  * flux matching: for every face between a coarse cell and fine cells, the fine fluxes of the
    final stage of each fine step (x its dt) are summed over the four sub-faces and the two fine
    steps; in the coarse final stage that sum replaces dt x the coarse flux through the face;
  * after the level-l step, ghost cells of level l covered by level l+1 take the mean of the eight
    fine cells (momentum: the coincident fine lattice point), and ghost cells of level l+1 covered
    by level l take the coarse field at their own position: linear interpolation between the coarse
    cell centres (weights 3/4 and 1/4 along each axis) and between the coarse lattice points (1/2 and
    1/2 along each axis where the fine lattice index is odd); where the coarse stencil holds a solid
    cell, a lattice point that is not predicted, or would reach below the ground or above the lid,
    the fine ghost takes the coarse cell's own values (the coarse lattice point at the halved index;
    for an odd fine lattice level over a coarse level that is not predicted, as at the ground, the
    coarse level above it, so that a predicted fine point never takes a diagnosed ground value).
Readings (the paper leaves them open): the coarse-to-fine transfer interpolates linearly (the paper
gives the coarse value; a piecewise-constant field in the fine ghosts forces the fine level at its
grid scale at every coarse step).  The values moved between levels are perturbations, each from
the level's own reference: rho' and (rho theta)' from the level's base state, and at predicted
lattice points the momentum rho u - rhobar_c(K) (u0, v0, 0) from the level's reference flow (the
base density of a lattice level depends on the level's spacing, so moving the total rho u would put
a vertical staircase of size d rhobar_c/dz dz U into the fine ghost cells at every transfer).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from oracle import oracle as O

FIELDS = O.FIELDS


class AmrOracle:
    """``match_fluxes=False`` skips the flux matching (for tests that show it is needed)."""

    def __init__(self, layout, match_fluxes: bool = True):
        self.match_fluxes = match_fluxes
        self.lay = layout
        self.blocks = layout.blocks
        self.nl = layout.levels
        self.boxes: List[O.Oracle] = []
        self.own: List[Tuple[tuple, tuple]] = []
        self.org: List[tuple] = []
        for b in self.blocks:
            cfg = layout.block_config(b)
            o = O.Oracle(cfg).merge()
            org, size, gb, gt = layout.box(b)
            lo = (layout.ghost, layout.ghost, gb)
            self.boxes.append(o)
            self.own.append((lo, (lo[0] + b.size[0], lo[1] + b.size[1], lo[2] + b.size[2])))
            self.org.append(org)
        self.q = [o.init_state() for o in self.boxes]
        base = layout.base
        self.N = [(base.nx << l, base.ny << l, base.nz << l) for l in range(self.nl)]
        # owner of every own cell: level -> {(x, y, z): (block, (i, j, k) in the box)}
        self.owner: List[Dict[tuple, tuple]] = [dict() for _ in range(self.nl)]
        for m, b in enumerate(self.blocks):
            (i0, j0, k0), (i1, j1, k1) = self.own[m]
            ox, oy, oz = self.org[m]
            d = self.owner[b.level]
            for i in range(i0, i1):
                for j in range(j0, j1):
                    for k in range(k0, k1):
                        d[(ox + i, oy + j, oz + k)] = (m, (i, j, k))
        self.faces = self._coarse_fine_faces()
        self.maps = self._ghost_maps()
        self.reg = {key: np.zeros(2) for key in self.faces}
        self.sync()  # every ghost cell starts from its owner's initial values

    # -- lookups ---------------------------------------------------------------------------------
    def _find(self, level, g):
        if level < 0 or level >= self.nl:
            return None
        N = self.N[level]
        if g[2] < 0 or g[2] >= N[2]:
            return None
        return self.owner[level].get((g[0] % N[0], g[1] % N[1], g[2]))

    def _coarse_fine_faces(self):
        """{(coarse block, cell, face): (fine block, [+side cell of each of the 4 sub-faces])}"""
        out = {}
        for m, b in enumerate(self.blocks):
            l = b.level
            if l + 1 >= self.nl:
                continue
            (i0, j0, k0), (i1, j1, k1) = self.own[m]
            ox, oy, oz = self.org[m]
            for i in range(i0, i1):
                for j in range(j0, j1):
                    for k in range(k0, k1):
                        g = (ox + i, oy + j, oz + k)
                        for f in range(6):
                            a, sg = f // 2, (1 if f % 2 else -1)
                            gn = list(g)
                            gn[a] += sg
                            if a == 2 and not (0 <= gn[2] < self.N[l][2]):
                                continue
                            if self._find(l, gn) is not None:
                                continue
                            kids = []
                            fb = None
                            others = [x for x in range(3) if x != a]
                            for s in range(4):
                                c = [0, 0, 0]
                                c[a] = 2 * gn[a] + (0 if sg > 0 else 1)
                                c[others[0]] = 2 * gn[others[0]] + (s & 1)
                                c[others[1]] = 2 * gn[others[1]] + (s >> 1)
                                hit = self._find(l + 1, c)
                                if hit is None:
                                    break
                                fm, cell = hit
                                assert fb is None or fb == fm
                                fb = fm
                                cell = list(cell)
                                if sg < 0:
                                    cell[a] += 1  # the face is at the fine cell's upper side
                                kids.append(tuple(cell))
                            if len(kids) == 4:
                                out[(m, (i, j, k), f)] = (fb, kids)
        return out

    # -- ghost refills ---------------------------------------------------------------------------
    def _ghost_maps(self):
        """For every block: ghost cells grouped by (kind, source block) as flat index arrays
        (destination box index, source box index); found by looking every ghost cell up."""
        maps = []
        for m, b in enumerate(self.blocks):
            l = b.level
            o = self.boxes[m]
            (i0, j0, k0), (i1, j1, k1) = self.own[m]
            nx, ny, nz = o.shape
            ox, oy, oz = self.org[m]
            groups: Dict[tuple, tuple] = {}
            for i in range(nx):
                for j in range(ny):
                    for k in range(nz):
                        if i0 <= i < i1 and j0 <= j < j1 and k0 <= k < k1:
                            continue
                        g = (ox + i, oy + j, oz + k)
                        if not (0 <= g[2] < self.N[l][2]):
                            continue
                        dst = (i * ny + j) * nz + k
                        hit = self._find(l, g)
                        kind = "same"
                        if hit is None:
                            hit = self._find(l - 1, (g[0] // 2, g[1] // 2, g[2] // 2))
                            kind = "coarse"
                        if hit is None:
                            hit = self._find(l + 1, (2 * g[0], 2 * g[1], 2 * g[2]))
                            kind = "fine"
                        if hit is None:
                            continue
                        sm, (a, bb, c) = hit
                        sny, snz = self.boxes[sm].shape[1], self.boxes[sm].shape[2]
                        src = (a * sny + bb) * snz + c
                        groups.setdefault((kind, sm), ([], []))
                        groups[(kind, sm)][0].append(dst)
                        groups[(kind, sm)][1].append(src)
            maps.append({key: (np.array(d, np.int64), np.array(s_, np.int64)) for key, (d, s_) in groups.items()})
        return maps

    def _fill(self, level, states, kinds):
        """Refill the ghost cells of the level's blocks (in `states`) of the given kinds: 'same'
        (copy within the level, from `states`), 'coarse' (the level-1 cell's values) and 'fine' (the
        mean of the eight level+1 cells; momentum of the coincident fine lattice point)."""
        for m, b in enumerate(self.blocks):
            if b.level != level:
                continue
            dst = states[m]
            for (kind, sm), (di, si) in self.maps[m].items():
                if kind not in kinds:
                    continue
                src = states[sm] if kind == "same" else self.q[sm]
                if kind == "fine":
                    sh = self.boxes[sm].shape
                    sx, sy = sh[1] * sh[2], sh[2]
                    for f in ("rho", "rth"):
                        a = src.a[f].ravel()
                        v = [a[si + off] for off in (0, sx, sy, sx + sy, 1, sx + 1, sy + 1, sx + sy + 1)]
                        dst.a[f].ravel()[di] = (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * 0.125
                    fields = ("mu", "mv", "mw")
                else:
                    fields = FIELDS
                for f in fields:
                    dst.a[f].ravel()[di] = src.a[f].ravel()[si]
                if kind != "same":
                    self._momentum_reference(m, sm, dst, di, si)
                if kind == "coarse":
                    self._prolong(m, sm, dst, src, di, si)

    def _momentum_reference(self, m, sm, dst, di, si):
        """Moved momenta at predicted lattice points keep their perturbation from the reference flow
        rhobar_c(K) (u0, v0): add (rhobar_c of the destination level - that of the source) U."""
        od, os_ = self.boxes[m], self.boxes[sm]
        pred = (od.vcls.ravel()[di] == O.PRED) & (os_.vcls.ravel()[si] == O.PRED)
        if not pred.any():
            return
        kd, ks = di[pred] % od.shape[2], si[pred] % os_.shape[2]

        def rbc(o, k):  # mean base density of the levels k-1 and k (k >= 1 at predicted points)
            return 0.5 * (o.rhob[k - 1] + o.rhob[k])

        dr = rbc(od, kd) - rbc(os_, ks)
        for f, u in (("mu", od.cfg.u0), ("mv", od.cfg.v0)):
            dst.a[f].ravel()[di[pred]] += dr * u

    def _prolong(self, m, sm, dst, src, di, si):
        """Linear interpolation of the coarse fields to the fine ghost cells (centres) and lattice
        points di of block m from the coarse box sm (parents at si); entries whose stencil fails keep
        the parent's values already written."""
        od, os_ = self.boxes[m], self.boxes[sm]
        nx, ny, nz = od.shape
        i, j, k = np.unravel_index(di, od.shape)
        ox, oy, oz = self.org[m]
        N = self.N[self.blocks[m].level]
        par = [np.mod(ox + i, N[0]) & 1, np.mod(oy + j, N[1]) & 1, (oz + k) & 1]
        sny, snz = os_.shape[1], os_.shape[2]
        st = (sny * snz, snz, 1)
        ks = si % snz
        # scalars: the fine centre lies a quarter of a coarse cell from the parent's centre, towards
        # the neighbour on the child's side (upper for an odd fine index)
        sg = [np.where(p == 1, 1, -1) for p in par]
        zin = (ks + sg[2] >= 0) & (ks + sg[2] < snz)
        ok = np.ones(len(di), dtype=bool)
        acc = {f: np.zeros(len(di)) for f in ("rho", "rth")}
        V = os_.V.ravel()
        for c in range(8):
            a, b, e = c >> 2, (c >> 1) & 1, c & 1
            p = si + a * sg[0] * st[0] + b * sg[1] * st[1] + e * np.where(zin, sg[2], 0)
            w = (0.75 if a == 0 else 0.25) * (0.75 if b == 0 else 0.25) * np.where(zin, 0.75 if e == 0 else 0.25, 0.5)
            ok &= V[p] > 0.0
            for f in acc:
                acc[f] += w * src.a[f].ravel()[p]
        for f in acc:
            dst.a[f].ravel()[di[ok]] = acc[f][ok]
        # momentum: average of the coarse lattice points around the fine one (odd fine index: the
        # point at the halved index and the next one), as perturbations from each level's reference
        zup = (par[2] == 1) & (ks + 1 < snz)
        pred_s = os_.vcls.ravel() == O.PRED
        pred_d = od.vcls.ravel()[di] == O.PRED
        # an odd fine level above a coarse level whose point is not predicted (the ground) takes the
        # coarse level above it alone
        shift = zup & ~pred_s[si] & pred_s[np.minimum(si + 1, len(pred_s) - 1)]
        base = si + shift
        odd = [par[0] == 1, par[1] == 1, zup & ~shift]

        def rbc(o, kk):
            return 0.5 * (o.rhob[np.maximum(kk - 1, 0)] + o.rhob[kk])

        kd = di % nz
        if shift.any():  # the fallback of a shifted point: the coarse point above, as a perturbation
            sh = shift & pred_d
            for f, u in (("mu", od.cfg.u0), ("mv", od.cfg.v0), ("mw", 0.0)):
                v = src.a[f].ravel()[base] - rbc(os_, base % snz) * u + rbc(od, kd) * u
                dst.a[f].ravel()[di[sh]] = v[sh]
        okm = pred_d.copy()
        pts = []
        for c in range(8):
            a, b, e = c >> 2, (c >> 1) & 1, c & 1
            use = (odd[0] | (a == 0)) & (odd[1] | (b == 0)) & (odd[2] | (e == 0))
            p = base + a * st[0] + b * st[1] + e
            p = np.where(use, p, base)
            okm &= ~use | pred_s[p]
            pts.append((use, p))
        n = (1 + odd[0]) * (1 + odd[1]) * (1 + odd[2])
        for f, u in (("mu", od.cfg.u0), ("mv", od.cfg.v0), ("mw", 0.0)):
            s = np.zeros(len(di))
            for use, p in pts:
                s += np.where(use, src.a[f].ravel()[p] - rbc(os_, p % snz) * u, 0.0)
            val = s / n + rbc(od, kd) * u
            dst.a[f].ravel()[di[okm]] = val[okm]

    def sync(self):
        for l in range(self.nl):
            self._fill(l, self.q, ("same", "coarse", "fine"))

    # -- stepping --------------------------------------------------------------------------------
    def _level_step(self, l, dt):
        if l + 1 < self.nl:
            self._level_step(l + 1, 0.5 * dt)
            self._level_step(l + 1, 0.5 * dt)
        ms = [m for m, b in enumerate(self.blocks) if b.level == l]
        qn = {m: self.q[m] for m in ms}
        qs = dict(qn)
        for s, c in enumerate((1.0 / 3.0, 0.5, 1.0)):
            out = {m: self.boxes[m].rk_update(qn[m], qs[m], c * dt) for m in ms}
            if s == 2 and self.match_fluxes:
                # fine side: accumulate dt x the final-stage fluxes of this level's interface faces
                for key, (fb, kids) in self.faces.items():
                    if self.blocks[fb].level != l:
                        continue
                    a = key[2] // 2
                    for cell in kids:
                        self.reg[key] += dt * self.boxes[fb].face_flux(qs[fb], a, *cell)
                # coarse side: replace dt x the coarse flux by the accumulated fine fluxes
                for key, (fb, kids) in self.faces.items():
                    m, (i, j, k), f = key
                    if self.blocks[m].level != l:
                        continue
                    a, plus = f // 2, f % 2
                    cell = [i, j, k]
                    if plus:
                        cell[a] += 1
                    Fc = self.boxes[m].face_flux(qs[m], a, *cell)
                    sg = 1.0 if plus else -1.0
                    o = self.boxes[m]
                    vol = o.Vgroup[i, j, k] * o.cfg.dx * o.cfg.dy * o.cfg.dz
                    corr = sg * (dt * Fc - self.reg[key])
                    out[m].a["rho"][i, j, k] += corr[0] / vol
                    out[m].a["rth"][i, j, k] += corr[1] / vol
                    self.reg[key] = np.zeros(2)
            for m in ms:
                self.boxes[m].diagnose(out[m])
            states = list(self.q)
            for m in ms:
                states[m] = out[m]
            self._fill(l, states, ("same",))
            qs = out
        for m in ms:
            self.q[m] = qs[m]
        if l + 1 < self.nl:
            self._fill(l, self.q, ("fine",))
            self._fill(l + 1, self.q, ("coarse",))

    def step(self, nsteps: int = 1, dt: float = None):
        dt = self.lay.base.dt if dt is None else dt
        for _ in range(nsteps):
            self._level_step(0, dt)

    # -- diagnostics -----------------------------------------------------------------------------
    def own_cells(self, m):
        (i0, j0, k0), (i1, j1, k1) = self.own[m]
        return {f: self.q[m].a[f][i0:i1, j0:j1, k0:k1] for f in FIELDS}

    def mass(self):
        """(sum of V dV rho' over own cells, the same for (rho theta)', total mass)."""
        mp = tp = mt = 0.0
        for m, o in enumerate(self.boxes):
            (i0, j0, k0), (i1, j1, k1) = self.own[m]
            dv = o.cfg.dx * o.cfg.dy * o.cfg.dz
            V = o.V[i0:i1, j0:j1, k0:k1]
            r = self.q[m].a["rho"][i0:i1, j0:j1, k0:k1]
            t = self.q[m].a["rth"][i0:i1, j0:j1, k0:k1]
            mp += float((V * r).sum()) * dv
            tp += float((V * t).sum()) * dv
            mt += float((V * (r + o.rhob[None, None, k0:k1])).sum()) * dv
        return mp, tp, mt
