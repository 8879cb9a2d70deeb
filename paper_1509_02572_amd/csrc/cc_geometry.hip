// Base state, cut-cell geometry and the cell-merging map (setup kernels, run once per terrain).
//
// Every floating-point expression here is evaluated in the written order with no FMA contraction,
// so that volumes, apertures, gradients and normals -- and the integer decisions taken from them
// (classification, merge direction, masters, lattice classes) -- are reproducible bit for bit by
// any IEEE-754 double implementation that follows the same order.
#pragma clang fp contract(off)

#include <algorithm>
#include <vector>

#include "cc_internal.hpp"

namespace cc {

// ------------------------------------------------------------------------------------------------
// Base state (Sec. 2.1): constant N, theta0 at z = 0, surface pressure p0.
// theta = theta0 exp(N^2 z / g); Exner pi solves d pi/dz = -g/(cp theta); (rho theta) from the
// equation of state; pbar through the same equation of state, so (rho theta)' = 0 <=> p' = 0.
// ------------------------------------------------------------------------------------------------
__global__ void k_base_state(int nz, double dz, double z0, cc_phys ph, double *base)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    double cv = ph.cp - ph.rd;
    double n2 = ph.bvn * ph.bvn;
    double z = z0 + ((double)k + 0.5) * dz;
    double th, pi;
    if (n2 > 0.0) {
        th = ph.theta0 * exp(n2 * z / ph.g);
        pi = 1.0 + ph.g * ph.g / (ph.cp * ph.theta0 * n2) * (exp(-n2 * z / ph.g) - 1.0);
    } else {
        th = ph.theta0;
        pi = 1.0 - ph.g * z / (ph.cp * ph.theta0);
    }
    double rth = ph.p0 / ph.rd * pow(pi, cv / ph.rd);
    base[k] = rth / th;                                          // rhobar
    base[nz + k] = rth;                                          // (rho theta)bar
    base[2 * nz + k] = ph.p0 * pow(ph.rd * rth / ph.p0, ph.cp / cv);  // pbar
    base[3 * nz + k] = th;                                       // thetabar
    base[4 * nz + k] = 1.0 / rth;                                // 1 / (rho theta)bar
}

// mean base density of the two cell levels around lattice level K (K = 0: the lowest level)
__global__ void k_base_lattice(int nz, double *base)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    base[5 * nz + k] = k > 0 ? 0.5 * (base[k - 1] + base[k]) : base[0];
}

// ------------------------------------------------------------------------------------------------
// Geometry (Sec. 2.3)
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }

// wetted height of one sub-column of the layer [zb, zt] above terrain height h
__device__ __forceinline__ double wet_height(double h, double zb, double zt, double dz)
{
    double top = h > zb ? h : zb;
    double w = zt - top;
    if (w < 0.0) w = 0.0;
    if (w > dz) w = dz;
    return w;
}

// bilinear surface of eq. bilin in local coordinates (xi, eta) of a column with corners
// h00 (origin), h10 (+x), h01 (+y), h11
__device__ __forceinline__ double bilin(double h00, double h10, double h01, double h11, double xi,
                                        double eta)
{
    return h00 + xi * (h10 - h00) + eta * (h01 - h00) + (xi * eta) * ((h00 - h01) + (h11 - h10));
}

// column centre height and the column gradients of eqs. xgrad / ygrad
__global__ void k_columns(Dims d, const double *__restrict__ H, double *__restrict__ col)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nc = (int64_t)d.nx * d.ny;
    if (t >= nc) return;
    int i = (int)(t / d.ny), j = (int)(t % d.ny);
    double h00 = H[hidx(d, i, j)], h10 = H[hidx(d, i + 1, j)];
    double h01 = H[hidx(d, i, j + 1)], h11 = H[hidx(d, i + 1, j + 1)];
    col[t] = ((h00 + h10) + (h01 + h11)) / 4.0;
    col[nc + t] = ((h10 + h11) - (h00 + h01)) / (2.0 * d.dx);
    col[2 * nc + t] = ((h01 + h11) - (h00 + h10)) / (2.0 * d.dy);
}

// terrain must stay inside [0, (nz-2) dz] so the two top layers are regular
__global__ void k_terrain_check(Dims d, const double *__restrict__ H, int64_t *st)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny) return;
    double h = H[t];
    // a grid on the ground holds its terrain below the lid; a raised block of a refined grid may
    // have the terrain below or above it
    bool ok = d.z0 > 0.0 ? (h == h) : (h >= 0.0 && h <= (double)(d.nz - 2) * d.dz);
    if (!ok) count_status(st, ST_TERRAIN);
}

// volume fraction and raw apertures of cell (i,j,k); one thread per cell, k fastest
__global__ void k_cells(Dims d, const double *__restrict__ H, double *__restrict__ V,
                        double *__restrict__ Ax, double *__restrict__ Ay, double *__restrict__ Az)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int k = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int j = (int)(colI % d.ny), i = (int)(colI / d.ny);
    int64_t c = cidx(d, i, j, k);
    double h00 = H[hidx(d, i, j)], h10 = H[hidx(d, i + 1, j)];
    double h01 = H[hidx(d, i, j + 1)], h11 = H[hidx(d, i + 1, j + 1)];
    double zb = (double)k * d.dz, zt = (double)(k + 1) * d.dz;
    double hmax = dmax(dmax(dmax(h00, h10), h01), h11);
    double hmin = dmin(dmin(dmin(h00, h10), h01), h11);
    const int ns = d.nsub;
    const double rns = (double)ns;
    // volume: mean wetted height of ns x ns sub-columns at their midpoints
    double v;
    if (hmax <= zb) v = 1.0;
    else if (hmin >= zt) v = 0.0;
    else {
        double s = 0.0;
        for (int b = 0; b < ns; ++b) {
            double eta = ((double)b + 0.5) / rns;
            for (int a = 0; a < ns; ++a) {
                double xi = ((double)a + 0.5) / rns;
                s += wet_height(bilin(h00, h10, h01, h11, xi, eta), zb, zt, d.dz);
            }
        }
        v = s / ((double)(ns * ns) * d.dz);
    }
    V[c] = v;
    // x-face x = i dx: its bottom edge runs from corner (i,j) to (i,j+1); y-face from (i,j) to (i+1,j)
    for (int axis = 0; axis < 2; ++axis) {
        double e0 = h00, e1 = axis == 0 ? h01 : h10;
        double emax = e0 > e1 ? e0 : e1, emin = e0 < e1 ? e0 : e1;
        double a;
        if (emax <= zb) a = 1.0;
        else if (emin >= zt) a = 0.0;
        else {
            double s = 0.0;
            for (int b = 0; b < ns; ++b) {
                double tt = ((double)b + 0.5) / rns;
                s += wet_height(e0 + tt * (e1 - e0), zb, zt, d.dz);
            }
            a = s / (rns * d.dz);
        }
        (axis == 0 ? Ax : Ay)[c] = a;
    }
    // z-face z = k dz: share of sub-columns whose terrain lies below it
    double az = 0.0;
    if (k > 0) {
        if (hmax < zb) az = 1.0;
        else if (hmin >= zb) az = 0.0;
        else {
            int cnt = 0;
            for (int b = 0; b < ns; ++b) {
                double eta = ((double)b + 0.5) / rns;
                for (int a = 0; a < ns; ++a) {
                    double xi = ((double)a + 0.5) / rns;
                    if (bilin(h00, h10, h01, h11, xi, eta) < zb) ++cnt;
                }
            }
            az = (double)cnt / (double)(ns * ns);
        }
    }
    Az[c] = az;
}

// a face that touches a fully buried cell is closed
__global__ void k_solid_rule(Dims d, const double *__restrict__ V, double *__restrict__ Ax,
                             double *__restrict__ Ay, double *__restrict__ Az)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int k = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int j = (int)(colI % d.ny), i = (int)(colI / d.ny);
    int64_t c = cidx(d, i, j, k);
    bool self = V[c] == 0.0;
    if (self || V[cidx(d, i - 1, j, k)] == 0.0) Ax[c] = 0.0;
    if (self || V[cidx(d, i, j - 1, k)] == 0.0) Ay[c] = 0.0;
    if (k > 0 && (self || V[c - 1] == 0.0)) Az[c] = 0.0;
}

// unit terrain normal at corner (I,J) from the centred gradients of the four surrounding column
// centre heights (Sec. 2.4: the normal of the boundary velocity point)
__global__ void k_normals(Dims d, const double *__restrict__ col, double *__restrict__ nrm)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nc = (int64_t)d.nx * d.ny;
    if (t >= nc) return;
    int I = (int)(t / d.ny), J = (int)(t % d.ny);
    const double *hc = col;
    double gxc = ((hc[hidx(d, I, J - 1)] + hc[hidx(d, I, J)]) -
                  (hc[hidx(d, I - 1, J - 1)] + hc[hidx(d, I - 1, J)])) / (2.0 * d.dx);
    double gyc = ((hc[hidx(d, I - 1, J)] + hc[hidx(d, I, J)]) -
                  (hc[hidx(d, I - 1, J - 1)] + hc[hidx(d, I, J - 1)])) / (2.0 * d.dy);
    double den = sqrt(gxc * gxc + gyc * gyc + 1.0);
    nrm[t] = -gxc / den;
    nrm[nc + t] = -gyc / den;
    nrm[2 * nc + t] = 1.0 / den;
}

// ------------------------------------------------------------------------------------------------
// Cell merging (Sec. 2.3, Figs. 5 and 6)
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ bool needs_merge(double v, double hc, int k, double dz)
{
    double zc = ((double)k + 0.5) * dz;
    return v > 0.0 && (hc > zc || v < 0.5);
}

// Sec. 2.3, Fig. 5: where both column gradients are at most 1 in magnitude the cell merges upward;
// otherwise it merges along the axis of the steeper gradient (x when the two are equal), towards
// the lower terrain (a positive gradient means lower ground on the minus side)
__device__ __forceinline__ int merge_direction(double gx, double gy)
{
    const double ax = fabs(gx), ay = fabs(gy);
    if (ax <= 1.0 && ay <= 1.0) return CC_DIR_ZP;
    if (ax >= ay) return gx > 0.0 ? CC_DIR_XM : CC_DIR_XP;
    return gy > 0.0 ? CC_DIR_YM : CC_DIR_YP;
}

// target cell of direction dir; false if it lies above the domain
__device__ __forceinline__ bool merge_target(const Dims &d, int i, int j, int k, int dir, int &ti,
                                             int &tj, int &tk)
{
    ti = i; tj = j; tk = k;
    switch (dir) {
    case CC_DIR_ZP: tk = k + 1; break;
    case CC_DIR_XM: ti = wrap(i - 1, d.nx); break;
    case CC_DIR_XP: ti = wrap(i + 1, d.nx); break;
    case CC_DIR_YM: tj = wrap(j - 1, d.ny); break;
    case CC_DIR_YP: tj = wrap(j + 1, d.ny); break;
    default: return false;
    }
    return tk < d.nz;
}

// pass 1: solid / needs merging (provisionally CC_ABSORBED) / available, and the direction
__global__ void k_merge_classify(Dims d, const double *__restrict__ V, const double *__restrict__ col,
                                 int8_t *cls, int8_t *dir, int32_t *gnext, double *Vgroup)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int k = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int j = (int)(colI % d.ny), i = (int)(colI / d.ny);
    int64_t c = cidx(d, i, j, k);
    int64_t nc = (int64_t)d.nx * d.ny;
    double v = V[c];
    int8_t cl, dr = CC_DIR_NONE;
    if (v == 0.0) cl = CC_SOLID;
    else if (needs_merge(v, col[colI], k, d.dz)) {
        cl = CC_ABSORBED;
        dr = (int8_t)merge_direction(col[nc + colI], col[2 * nc + colI]);
    } else cl = CC_OPEN;
    cls[c] = cl;
    dir[c] = dr;
    gnext[c] = -1;
    Vgroup[c] = 0.0;
}

// pass 2: follow the targets while the target itself needs merging, at most 8 hops
__global__ void k_merge_master(Dims d, const double *__restrict__ V, const int8_t *__restrict__ cls,
                               const int8_t *__restrict__ dir, int32_t *master, int64_t *st)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int k = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int j = (int)(colI % d.ny), i = (int)(colI / d.ny);
    int64_t c = cidx(d, i, j, k);
    int8_t cl = cls[c];
    if (cl == CC_SOLID) { master[c] = -1; return; }
    if (cl == CC_OPEN) { master[c] = (int32_t)c; return; }
    int ci = i, cj = j, ck = k;
    int64_t m = c;
    bool ok = false;
    for (int hop = 0; hop < 8; ++hop) {
        int ti, tj, tk;
        if (!merge_target(d, ci, cj, ck, dir[cidx(d, ci, cj, ck)], ti, tj, tk)) break;
        int64_t tt = cidx(d, ti, tj, tk);
        if (V[tt] == 0.0) break;
        if (cls[tt] == CC_OPEN) { m = tt; ok = true; break; }
        ci = ti; cj = tj; ck = tk;
    }
    if (ok) master[c] = (int32_t)m;
    else {
        master[c] = (int32_t)c;
        count_status(st, ST_UNMERGEABLE);
    }
}

// pass 3: unmergeable cells become their own master; every master collects its members (the donor
// tree of cells whose target is a group cell), sorts them by linear index, sums the group volume
// (master first, then members in increasing index) and threads them into the gnext list.
__global__ void k_merge_groups(Dims d, const double *__restrict__ V, int8_t *cls,
                               const int8_t *__restrict__ dir, const int32_t *__restrict__ master,
                               int32_t *gnext, double *Vgroup, int64_t *st)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int k = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int j = (int)(colI % d.ny), i = (int)(colI / d.ny);
    int64_t c = cidx(d, i, j, k);
    int8_t cl = cls[c];
    if (cl == CC_SOLID) return;
    if (cl == CC_ABSORBED) {
        if (master[c] == (int32_t)c) {
            cls[c] = CC_ORPHAN;
            Vgroup[c] = V[c];
        }
        return;
    }
    // an available cell: the master of its group
    int64_t mem[CC_MAX_GROUP];
    int64_t stack[CC_MAX_GROUP];
    int nm = 0, sp = 0;
    bool overflow = false;
    stack[sp++] = c;
    while (sp > 0) {
        int64_t node = stack[--sp];
        int ni, nj, nk;
        unidx(d, node, ni, nj, nk);
        // cells whose merge target is `node`
        const int di[5] = {0, 1, -1, 0, 0}, dj[5] = {0, 0, 0, 1, -1}, dk[5] = {-1, 0, 0, 0, 0};
        const int8_t need[5] = {CC_DIR_ZP, CC_DIR_XM, CC_DIR_XP, CC_DIR_YM, CC_DIR_YP};
        for (int q = 0; q < 5; ++q) {
            int kk = nk + dk[q];
            if (kk < 0) continue;
            int64_t dn = cidx(d, ni + di[q], nj + dj[q], kk);
            if (dn == c || dir[dn] != need[q] || master[dn] != (int32_t)c) continue;
            if (nm < CC_MAX_GROUP && sp < CC_MAX_GROUP) {
                mem[nm++] = dn;
                stack[sp++] = dn;
            } else overflow = true;
        }
    }
    if (overflow) count_status(st, ST_GROUPSIZE);
    for (int a = 1; a < nm; ++a) {  // insertion sort by linear index
        int64_t x = mem[a];
        int b = a - 1;
        while (b >= 0 && mem[b] > x) { mem[b + 1] = mem[b]; --b; }
        mem[b + 1] = x;
    }
    double vg = V[c];
    for (int a = 0; a < nm; ++a) vg += V[mem[a]];
    Vgroup[c] = vg;
    gnext[c] = nm > 0 ? (int32_t)mem[0] : -1;
    for (int a = 0; a < nm; ++a) gnext[mem[a]] = a + 1 < nm ? (int32_t)mem[a + 1] : -1;
}

// lattice points: on/below the terrain -> ground; all eight surrounding cells available ->
// predicted; otherwise a merged-face point (Sec. 2.4)
__global__ void k_lattice_class(Dims d, const double *__restrict__ H, const int8_t *__restrict__ cls,
                                int8_t *vcls)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int K = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int J = (int)(colI % d.ny), I = (int)(colI / d.ny);
    int64_t p = cidx(d, I, J, K);
    if ((double)K * d.dz <= H[colI]) { vcls[p] = CC_GROUND; return; }
    bool all = K >= 1;
    for (int q = 0; q < 8 && all; ++q)
        all = cls[cidx(d, I - 1 + (q & 1), J - 1 + ((q >> 1) & 1), K - 1 + (q >> 2))] == CC_OPEN;
    vcls[p] = all ? CC_PRED : CC_MFACE;
}

// Per-column thresholds used by the stage kernels to skip geometry and class reads away from the
// terrain:
//   colk[0] (cell band): from this k up every cell is a single-cell available group with V = 1,
//           six open faces (k >= 1) and available neighbours;
//   colk[1] (lattice band): 1 + the top level K < nz of a lattice point that is not predicted;
//   colk[2] (diagnostic top): max(colk[1], 1 + top k of an absorbed or solid cell).
__global__ void k_column_bands(Dims d, const double *__restrict__ V, const double *__restrict__ Ax,
                               const double *__restrict__ Ay, const double *__restrict__ Az,
                               const int8_t *__restrict__ cls, const int32_t *__restrict__ gnext,
                               const int8_t *__restrict__ vcls, int32_t *colk)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nc = (int64_t)d.nx * d.ny;
    if (t >= nc) return;
    int i = (int)(t / d.ny), j = (int)(t % d.ny);
    int kcell = 0, klat = 0, kdiag = 0;
    for (int k = 0; k < d.nz; ++k) {
        int64_t c = cidx(d, i, j, k);
        int8_t cl = cls[c];
        if (vcls[c] != CC_PRED) klat = k + 1;
        if (cl == CC_ABSORBED || cl == CC_SOLID) kdiag = k + 1;
        // a regular cell: full, open, unmerged, every face fully open and every neighbour open; the
        // ground (below k = 0) and the lid (above nz-1) are closed faces the regular update skips
        bool sp = cl != CC_OPEN || gnext[c] != -1 || V[c] != 1.0;
        sp = sp || Ax[c] != 1.0 || Ax[cidx(d, i + 1, j, k)] != 1.0 || Ay[c] != 1.0 ||
             Ay[cidx(d, i, j + 1, k)] != 1.0 || (k > 0 && Az[c] != 1.0) || (k + 1 < d.nz && Az[c + 1] != 1.0);
        sp = sp || cls[cidx(d, i - 1, j, k)] != CC_OPEN || cls[cidx(d, i + 1, j, k)] != CC_OPEN ||
             cls[cidx(d, i, j - 1, k)] != CC_OPEN || cls[cidx(d, i, j + 1, k)] != CC_OPEN ||
             (k > 0 && cls[c - 1] != CC_OPEN) || (k + 1 < d.nz && cls[c + 1] != CC_OPEN);
        if (sp) kcell = k + 1;
    }
    colk[t] = kcell;
    colk[nc + t] = klat;
    colk[2 * nc + t] = kdiag > klat ? kdiag : klat;
}

}  // namespace cc

using namespace cc;

extern "C" cc_status cutcell_base_state(const cc_grid *grid, const cc_phys *phys, double *base,
                                        cc_stream_t stream)
{
    if (!check_grid(grid)) return CC_EINVAL;
    CC_REQUIRE(phys && base, "cutcell_base_state: null argument");
    hipLaunchKernelGGL(k_base_state, dim3(blocks_for(grid->nz, 64)), dim3(64), 0, (hipStream_t)stream,
                       grid->nz, grid->dz, grid->z0, *phys, base);
    hipLaunchKernelGGL(k_base_lattice, dim3(blocks_for(grid->nz, 64)), dim3(64), 0, (hipStream_t)stream,
                       grid->nz, base);
    return launch_status("cutcell_base_state");
}

extern "C" cc_status cutcell_geometry(const cc_grid *grid, cc_geom *g, int64_t *st, cc_stream_t stream)
{
    if (!check_grid(grid)) return CC_EINVAL;
    CC_REQUIRE(g, "cutcell_geometry: null geometry");
    const void *p[] = {g->H, g->V, g->Ax, g->Ay, g->Az, g->col, g->nrm};
    if (!check_ptrs("cutcell_geometry", 7, p)) return CC_EINVAL;
    Dims d = dims_of(grid);
    hipStream_t s = (hipStream_t)stream;
    int64_t nc = (int64_t)d.nx * d.ny, n = nc * d.nz;
    hipLaunchKernelGGL(k_terrain_check, dim3(blocks_for(nc, 256)), dim3(256), 0, s, d, g->H, st);
    hipLaunchKernelGGL(k_columns, dim3(blocks_for(nc, 256)), dim3(256), 0, s, d, g->H, g->col);
    hipLaunchKernelGGL(k_cells, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, g->H, g->V, g->Ax, g->Ay, g->Az);
    hipLaunchKernelGGL(k_solid_rule, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, g->V, g->Ax, g->Ay, g->Az);
    hipLaunchKernelGGL(k_normals, dim3(blocks_for(nc, 256)), dim3(256), 0, s, d, g->col, g->nrm);
    return launch_status("cutcell_geometry");
}

extern "C" cc_status cutcell_merge_map(const cc_grid *grid, cc_geom *g, int64_t *st, cc_stream_t stream)
{
    if (!check_grid(grid)) return CC_EINVAL;
    CC_REQUIRE(g, "cutcell_merge_map: null geometry");
    const void *p[] = {g->H, g->V, g->Ax, g->Ay, g->Az, g->col, g->cls, g->dir, g->vcls, g->master,
                       g->gnext, g->Vgroup, g->colk};
    if (!check_ptrs("cutcell_merge_map", 13, p)) return CC_EINVAL;
    Dims d = dims_of(grid);
    CC_REQUIRE((int64_t)d.nx * d.ny * d.nzs < ((int64_t)1 << 31),
               "cutcell_merge_map: grid too large for 32-bit master indices");
    hipStream_t s = (hipStream_t)stream;
    int64_t nc = (int64_t)d.nx * d.ny, n = nc * d.nz;
    dim3 gb(blocks_for(n, 256)), tb(256);
    hipLaunchKernelGGL(k_merge_classify, gb, tb, 0, s, d, g->V, g->col, g->cls, g->dir, g->gnext, g->Vgroup);
    hipLaunchKernelGGL(k_merge_master, gb, tb, 0, s, d, g->V, g->cls, g->dir, g->master, st);
    hipLaunchKernelGGL(k_merge_groups, gb, tb, 0, s, d, g->V, g->cls, g->dir, g->master, g->gnext, g->Vgroup, st);
    hipLaunchKernelGGL(k_lattice_class, gb, tb, 0, s, d, g->H, g->cls, g->vcls);
    hipLaunchKernelGGL(k_column_bands, dim3(blocks_for(nc, 256)), tb, 0, s, d, g->V, g->Ax, g->Ay, g->Az,
                       g->cls, g->gnext, g->vcls, g->colk);
    g->kband = 0;  // unknown until cutcell_band_setup
    g->nband_tiles = -1;
    return launch_status("cutcell_merge_map");
}

extern "C" cc_status cutcell_band_setup(const cc_grid *grid, cc_geom *g, cc_stream_t stream)
{
    if (!check_grid(grid)) return CC_EINVAL;
    CC_REQUIRE(g && g->colk, "cutcell_band_setup: null geometry or column bands");
    Dims d = dims_of(grid);
    hipStream_t s = (hipStream_t)stream;
    int64_t nc = (int64_t)d.nx * d.ny;
    // band height: the highest cell band or lattice band top over all columns
    std::vector<int32_t> bands((size_t)(2 * nc));
    hipError_t e = hipMemcpyAsync(bands.data(), g->colk, sizeof(int32_t) * 2 * nc, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("cutcell_band_setup: %s", hipGetErrorString(e));
        return CC_EDEVICE;
    }
    int32_t top = 1;
    for (int64_t c = 0; c < nc; ++c) {
        int32_t b = band_top(bands[(size_t)c], bands[(size_t)(nc + c)]);
        top = b > top ? b : top;
    }
    g->kband = top < d.nz ? top : d.nz;
    // the band-point launch's one-wave tiles that hold band points, each listed as
    // (bk nbx + bi) nby + bj in (bi, bj, bk) order, at the start of the stage workspace
    g->nband_tiles = -1;
    if (g->stage_ws) {
        const BandTile bt = band_tile_of(d.nx, d.ny, d.nz);
        std::vector<int32_t> list;
        for (int bi = 0; bi < bt.nbx; ++bi)
            for (int bj = 0; bj < bt.nby; ++bj) {
                int deep = 0;
                for (int i = bi * bt.bx; i < std::min(d.nx, (bi + 1) * bt.bx); ++i)
                    for (int j = bj * bt.by; j < std::min(d.ny, (bj + 1) * bt.by); ++j) {
                        const int64_t c = (int64_t)i * d.ny + j;
                        deep = std::max(deep, band_top(bands[(size_t)c], bands[(size_t)(nc + c)]));
                    }
                for (int bk = 0; bk * bt.bz < std::min(deep, d.nz); ++bk)
                    list.push_back((bk * bt.nbx + bi) * bt.nby + bj);
            }
        if (!list.empty()) {
            e = hipMemcpyAsync(g->stage_ws, list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host list is freed on return
            if (e != hipSuccess) {
                set_error("cutcell_band_setup: %s", hipGetErrorString(e));
                return CC_EDEVICE;
            }
        }
        g->nband_tiles = (int32_t)list.size();
    }
    return CC_OK;
}
