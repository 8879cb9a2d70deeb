/*
 * cutcell_oracle.c -- plain, slow, FP64 CPU reference of the cut-cell stage.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the CPU-baseline leg
 * of the benchmark load this library.  It shares no code, header, table or constant with the HIP
 * path: it is written from the paper (Yamazaki, Satomura & Nikiforakis, "3D cut-cell modelling for
 * high-resolution atmospheric simulations") and from the readings listed in the design notes.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no FMA contraction, no fast-math), so
 * every floating-point expression is evaluated exactly in the order written here.
 *
 * Layout: every 3-D array is indexed ((i*ny + j)*nz + k), k fastest, without padding.  Cell (i,j,k)
 * spans [i dx,(i+1)dx] x [j dy,(j+1)dy] x [k dz,(k+1)dz].  Lattice point (I,J,K) sits at the cell
 * corner (I dx, J dy, K dz) and shares the index of cell (I,J,K); K = nz (the lid) is not stored.
 * x and y are periodic.  Terrain heights H[I*ny+J] are given at the column corners.
 *
 * Pins (tests): the 18.1 and 71 degree slopes of Sec. 3.1, the merge directions of Sec. 3.1.1/3.1.2,
 * the volume closed form and the analytic hill volumes, face-area closure of every cut cell, brute
 * force on 4^3 grids, the exact normal of a planar patch, the diagnostics of a uniform flow (eq. 33
 * and the merged-face interpolation in closed form) and their mirror symmetry, rest stays at rest,
 * the flat terrain finite-difference reduction of Sec. 2.4, mass conservation, a face-list scatter
 * form of the flux divergence, symmetry and translation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t nx, ny, nz, nsub; double dx, dy, dz, z0; } or_grid;  /* z0: bottom height */
/* kdh, kdv: rates [1/s] of the fourth-order artificial diffusion in the horizontal and the vertical
 * (0: none); zsp, rsp: bottom height [m] of the sponge layer and its damping rate [1/s] at the lid
 * (rsp = 0: none) */
typedef struct { double g, rd, cp, p0, theta0, bvn, u0, v0, kdh, kdv, zsp, rsp, ztop; } or_phys;

/* cell classes, merge directions and lattice-point classes (numeric codes are an interface) */
enum { OR_SOLID = 0, OR_OPEN = 1, OR_ABSORBED = 2, OR_ORPHAN = 3 };
enum { OR_NONE = 0, OR_ZP = 1, OR_XM = 2, OR_XP = 3, OR_YM = 4, OR_YP = 5 };
enum { OR_GROUND = 0, OR_PRED = 1, OR_MFACE = 2 };

#define OR_MAXHOPS 8

typedef struct {
    const double *H;                   /* [nx*ny] corner heights */
    double *V, *Ax, *Ay, *Az;          /* [nx*ny*nz] */
    double *hc, *gx, *gy;              /* [nx*ny] column centre height and gradients */
    double *nrm;                       /* [3][nx*ny] unit terrain normal at corners */
    int8_t *cls, *dir, *vcls;          /* [nx*ny*nz] */
    int32_t *master;                   /* [nx*ny*nz], -1 for solid cells */
    double *Vgroup;                    /* [nx*ny*nz], valid at masters */
} or_geom;

typedef struct { double *rho, *rth, *mu, *mv, *mw; } or_state;

static inline int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }
static inline size_t cidx(const or_grid *g, int i, int j, int k)
{
    return ((size_t)wrapi(i, g->nx) * g->ny + wrapi(j, g->ny)) * g->nz + k;
}
static inline size_t hidx(const or_grid *g, int i, int j)
{
    return (size_t)wrapi(i, g->nx) * g->ny + wrapi(j, g->ny);
}

/* ------------------------------------------------------------------------------------------ */
/* Base state: constant N, theta0 at z = 0, surface pressure p0 (Sec. 2.1, Sec. 3).             */
/* theta(z) = theta0 exp(N^2 z/g); Exner pi from d pi/dz = -g/(cp theta); rho*theta from the     */
/* equation of state; pbar through the same equation of state so that (rho theta)' = 0 <=> p'=0. */
/* ------------------------------------------------------------------------------------------ */
void or_base_state(const or_phys *ph, int nz, double dz, double z0, double *rhob, double *rthb, double *pb,
                   double *thb)
{
    double cv = ph->cp - ph->rd;
    double n2 = ph->bvn * ph->bvn;
    for (int k = 0; k < nz; ++k) {
        double z = z0 + ((double)k + 0.5) * dz;
        double th, pi;
        if (n2 > 0.0) {
            th = ph->theta0 * exp(n2 * z / ph->g);
            pi = 1.0 + ph->g * ph->g / (ph->cp * ph->theta0 * n2) * (exp(-n2 * z / ph->g) - 1.0);
        } else {
            th = ph->theta0;
            pi = 1.0 - ph->g * z / (ph->cp * ph->theta0);
        }
        double rth = ph->p0 / ph->rd * pow(pi, cv / ph->rd);
        rthb[k] = rth;
        pb[k] = ph->p0 * pow(ph->rd * rth / ph->p0, ph->cp / cv);
        rhob[k] = rth / th;
        thb[k] = th;
    }
}

/* Perturbation pressure from (rho theta)' via the ideal-gas equation of state (Sec. 2.1):
 * p = p0 (R rho theta / p0)^(cp/cv), so p' = pbar ((1 + rth'/rthbar)^(cp/cv) - 1). */
static double eos_pprime(double rthp, double rthbar, double pbar, double gam)
{
    return pbar * expm1(gam * log1p(rthp / rthbar));
}

/* ------------------------------------------------------------------------------------------ */
/* Geometry (Sec. 2.3): bilinear terrain per column (eq. bilin), volumes and apertures from      */
/* nsub x nsub narrow rectangular sub-columns, column gradients (eqs. xgrad/ygrad) and the unit  */
/* terrain normal at column corners from the centred gradients of column-centre heights.        */
/* ------------------------------------------------------------------------------------------ */

/* wetted height of one sub-column of the layer [zb, zt] above terrain height h */
static double wet_height(double h, double zb, double zt, double dz)
{
    double top = h > zb ? h : zb;
    double w = zt - top;
    if (w < 0.0) w = 0.0;
    if (w > dz) w = dz;
    return w;
}

static double max4(double a, double b, double c, double d)
{
    double m = a > b ? a : b;
    m = m > c ? m : c;
    return m > d ? m : d;
}
static double min4(double a, double b, double c, double d)
{
    double m = a < b ? a : b;
    m = m < c ? m : c;
    return m < d ? m : d;
}

/* height of the bilinear surface at local coordinates (xi, eta) in [0,1]^2 of a column with corner
 * heights h00 (origin), h10 (+x), h01 (+y), h11: h = c + m1 x + m3 y + m2 x y of eq. bilin */
static double bilinear(double h00, double h10, double h01, double h11, double xi, double eta)
{
    return h00 + xi * (h10 - h00) + eta * (h01 - h00) + (xi * eta) * ((h00 - h01) + (h11 - h10));
}

static double cell_volume(const or_grid *g, double h00, double h10, double h01, double h11, int k)
{
    double zb = (double)k * g->dz, zt = (double)(k + 1) * g->dz;
    if (max4(h00, h10, h01, h11) <= zb) return 1.0;
    if (min4(h00, h10, h01, h11) >= zt) return 0.0;
    int ns = g->nsub;
    double s = 0.0;
    for (int b = 0; b < ns; ++b) {
        double eta = ((double)b + 0.5) / (double)ns;
        for (int a = 0; a < ns; ++a) {
            double xi = ((double)a + 0.5) / (double)ns;
            s += wet_height(bilinear(h00, h10, h01, h11, xi, eta), zb, zt, g->dz);
        }
    }
    return s / ((double)(ns * ns) * g->dz);
}

/* open fraction of a vertical face whose bottom edge runs linearly from e0 to e1 */
static double side_aperture(const or_grid *g, double e0, double e1, int k)
{
    double zb = (double)k * g->dz, zt = (double)(k + 1) * g->dz;
    double emax = e0 > e1 ? e0 : e1, emin = e0 < e1 ? e0 : e1;
    if (emax <= zb) return 1.0;
    if (emin >= zt) return 0.0;
    int ns = g->nsub;
    double s = 0.0;
    for (int b = 0; b < ns; ++b) {
        double t = ((double)b + 0.5) / (double)ns;
        s += wet_height(e0 + t * (e1 - e0), zb, zt, g->dz);
    }
    return s / ((double)ns * g->dz);
}

/* open fraction of the horizontal face z = K dz of a column: share of sub-columns below it */
static double bottom_aperture(const or_grid *g, double h00, double h10, double h01, double h11, int K)
{
    double zl = (double)K * g->dz;
    if (max4(h00, h10, h01, h11) < zl) return 1.0;
    if (min4(h00, h10, h01, h11) >= zl) return 0.0;
    int ns = g->nsub, cnt = 0;
    for (int b = 0; b < ns; ++b) {
        double eta = ((double)b + 0.5) / (double)ns;
        for (int a = 0; a < ns; ++a) {
            double xi = ((double)a + 0.5) / (double)ns;
            if (bilinear(h00, h10, h01, h11, xi, eta) < zl) ++cnt;
        }
    }
    return (double)cnt / (double)(ns * ns);
}

void or_geometry(const or_grid *g, or_geom *G)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    const double *H = G->H;
    /* columns: centre height and the gradients of eqs. xgrad / ygrad */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double h00 = H[hidx(g, i, j)], h10 = H[hidx(g, i + 1, j)];
            double h01 = H[hidx(g, i, j + 1)], h11 = H[hidx(g, i + 1, j + 1)];
            size_t c = hidx(g, i, j);
            G->hc[c] = ((h00 + h10) + (h01 + h11)) / 4.0;
            G->gx[c] = ((h10 + h11) - (h00 + h01)) / (2.0 * g->dx);
            G->gy[c] = ((h01 + h11) - (h00 + h10)) / (2.0 * g->dy);
        }
    /* volumes */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double h00 = H[hidx(g, i, j)], h10 = H[hidx(g, i + 1, j)];
            double h01 = H[hidx(g, i, j + 1)], h11 = H[hidx(g, i + 1, j + 1)];
            for (int k = 0; k < nz; ++k) G->V[cidx(g, i, j, k)] = cell_volume(g, h00, h10, h01, h11, k);
        }
    /* apertures, then the rule that a face touching a fully buried cell is closed */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double h00 = H[hidx(g, i, j)], h10 = H[hidx(g, i + 1, j)];
            double h01 = H[hidx(g, i, j + 1)], h11 = H[hidx(g, i + 1, j + 1)];
            for (int k = 0; k < nz; ++k) {
                size_t c = cidx(g, i, j, k);
                /* x-face at x = i dx: bottom edge from corner (i,j) to (i,j+1) */
                double ax = side_aperture(g, h00, h01, k);
                if (G->V[cidx(g, i - 1, j, k)] == 0.0 || G->V[c] == 0.0) ax = 0.0;
                G->Ax[c] = ax;
                /* y-face at y = j dy: bottom edge from corner (i,j) to (i+1,j) */
                double ay = side_aperture(g, h00, h10, k);
                if (G->V[cidx(g, i, j - 1, k)] == 0.0 || G->V[c] == 0.0) ay = 0.0;
                G->Ay[c] = ay;
                /* z-face at z = k dz */
                double az = 0.0;
                if (k > 0) {
                    az = bottom_aperture(g, h00, h10, h01, h11, k);
                    if (G->V[cidx(g, i, j, k - 1)] == 0.0 || G->V[c] == 0.0) az = 0.0;
                }
                G->Az[c] = az;
            }
        }
    /* unit normal at corner (I,J) from the four surrounding column-centre heights (Sec. 2.4) */
    size_t nc = (size_t)nx * ny;
    for (int I = 0; I < nx; ++I)
        for (int J = 0; J < ny; ++J) {
            double gxc = ((G->hc[hidx(g, I, J - 1)] + G->hc[hidx(g, I, J)]) -
                          (G->hc[hidx(g, I - 1, J - 1)] + G->hc[hidx(g, I - 1, J)])) / (2.0 * g->dx);
            double gyc = ((G->hc[hidx(g, I - 1, J)] + G->hc[hidx(g, I, J)]) -
                          (G->hc[hidx(g, I - 1, J - 1)] + G->hc[hidx(g, I, J - 1)])) / (2.0 * g->dy);
            double den = sqrt(gxc * gxc + gyc * gyc + 1.0);
            size_t c = hidx(g, I, J);
            G->nrm[c] = -gxc / den;
            G->nrm[nc + c] = -gyc / den;
            G->nrm[2 * nc + c] = 1.0 / den;
        }
}

/* ------------------------------------------------------------------------------------------ */
/* Cell merging (Sec. 2.3, Fig. 6): which cells merge, in which direction, and with whom.        */
/* ------------------------------------------------------------------------------------------ */

/* the paper's rule: merge a cut cell whose centre is underground or whose volume is below half */
static int needs_merge(const or_grid *g, const or_geom *G, size_t c, int k)
{
    double zc = ((double)k + 0.5) * g->dz;
    double v = G->V[c];
    double hc = G->hc[c / g->nz];
    return v > 0.0 && (hc > zc || v < 0.5);
}

/* merge direction from the column gradients (Sec. 2.3, Fig. 5): upward where neither gradient
 * exceeds 1 in magnitude; otherwise along the steeper axis (x when both are equally steep), to the
 * neighbour on the lower side of the slope */
int or_merge_direction(double gx, double gy)
{
    double ax = fabs(gx), ay = fabs(gy);
    if (ax <= 1.0 && ay <= 1.0) return OR_ZP;
    if (ax >= ay) return gx > 0.0 ? OR_XM : OR_XP;
    return gy > 0.0 ? OR_YM : OR_YP;
}

/* the cell a cut cell merges into; returns 0 if it lies outside the domain */
static int merge_target(const or_grid *g, int i, int j, int k, int d, int *ti, int *tj, int *tk)
{
    *ti = i; *tj = j; *tk = k;
    switch (d) {
    case OR_ZP: *tk = k + 1; break;
    case OR_XM: *ti = wrapi(i - 1, g->nx); break;
    case OR_XP: *ti = wrapi(i + 1, g->nx); break;
    case OR_YM: *tj = wrapi(j - 1, g->ny); break;
    case OR_YP: *tj = wrapi(j + 1, g->ny); break;
    default: return 0;
    }
    return *tk < g->nz;
}

/* counts[0] += unmergeable cells.  Writes cls, dir, master, Vgroup and vcls. */
void or_merge(const or_grid *g, or_geom *G, int64_t *counts)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t n = (size_t)nx * ny * nz;
    int64_t bad = 0;
    /* classification and direction */
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                size_t c = cidx(g, i, j, k);
                if (G->V[c] == 0.0) { G->cls[c] = OR_SOLID; G->dir[c] = OR_NONE; continue; }
                if (needs_merge(g, G, c, k)) {
                    G->cls[c] = OR_ABSORBED; /* provisional */
                    G->dir[c] = (int8_t)or_merge_direction(G->gx[hidx(g, i, j)], G->gy[hidx(g, i, j)]);
                } else {
                    G->cls[c] = OR_OPEN;
                    G->dir[c] = OR_NONE;
                }
            }
    /* masters: follow targets while the target itself has to merge, at most OR_MAXHOPS hops */
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                size_t c = cidx(g, i, j, k);
                if (G->cls[c] == OR_SOLID) { G->master[c] = -1; continue; }
                if (G->cls[c] == OR_OPEN) { G->master[c] = (int32_t)c; continue; }
                int ci = i, cj = j, ck = k, ok = 0;
                size_t m = c;
                for (int hop = 0; hop < OR_MAXHOPS; ++hop) {
                    int ti, tj, tk;
                    size_t cc = cidx(g, ci, cj, ck);
                    if (!merge_target(g, ci, cj, ck, G->dir[cc], &ti, &tj, &tk)) break;
                    size_t t = cidx(g, ti, tj, tk);
                    if (G->V[t] == 0.0) break;
                    if (!needs_merge(g, G, t, tk)) { m = t; ok = 1; break; }
                    ci = ti; cj = tj; ck = tk;
                }
                if (ok) {
                    G->master[c] = (int32_t)m;
                } else {
                    G->master[c] = (int32_t)c;
                    G->cls[c] = OR_ORPHAN;
                    ++bad;
                }
            }
    /* group volumes: the master's own volume, then members in increasing linear index */
    for (size_t c = 0; c < n; ++c)
        G->Vgroup[c] = (G->cls[c] == OR_OPEN || G->cls[c] == OR_ORPHAN) ? G->V[c] : 0.0;
    for (size_t c = 0; c < n; ++c)
        if (G->cls[c] == OR_ABSORBED) G->Vgroup[G->master[c]] += G->V[c];
    /* lattice points (Sec. 2.3 variable arrangement, Sec. 2.4 predicted points):
     * on or below the terrain -> diagnosed boundary point; all eight surrounding cells available ->
     * predicted; otherwise a point on a merged face, diagnosed by interpolation. */
    for (int I = 0; I < nx; ++I)
        for (int J = 0; J < ny; ++J)
            for (int K = 0; K < nz; ++K) {
                size_t p = cidx(g, I, J, K);
                double h = G->H[hidx(g, I, J)];
                if ((double)K * g->dz <= h) { G->vcls[p] = OR_GROUND; continue; }
                int all = K >= 1;
                for (int di = -1; di <= 0 && all; ++di)
                    for (int dj = -1; dj <= 0 && all; ++dj)
                        for (int dk = -1; dk <= 0 && all; ++dk)
                            if (G->cls[cidx(g, I + di, J + dj, K + dk)] != OR_OPEN) all = 0;
                G->vcls[p] = all ? OR_PRED : OR_MFACE;
            }
    if (counts) counts[0] += bad;
}

/* ------------------------------------------------------------------------------------------ */
/* Field access                                                                                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const or_grid *g;
    const or_phys *ph;
    const or_geom *G;
    const double *rhob, *rthb, *pb; /* base state at cell centres */
    const or_state *q;
} or_ctx;

/* total density of an available (own-master) cell */
static double rho_tot(const or_ctx *x, int i, int j, int k)
{
    return x->rhob[k] + x->q->rho[cidx(x->g, i, j, k)];
}
static double pprime(const or_ctx *x, int i, int j, int k)
{
    double gam = x->ph->cp / (x->ph->cp - x->ph->rd);
    return eos_pprime(x->q->rth[cidx(x->g, i, j, k)], x->rthb[k], x->pb[k], gam);
}
/* density at a velocity point: mean of the eight surrounding cell densities */
static double rho_corner(const or_ctx *x, int I, int J, int K)
{
    double s0 = (rho_tot(x, I - 1, J - 1, K - 1) + rho_tot(x, I, J - 1, K - 1)) +
                (rho_tot(x, I - 1, J, K - 1) + rho_tot(x, I, J, K - 1));
    double s1 = (rho_tot(x, I - 1, J - 1, K) + rho_tot(x, I, J - 1, K)) +
                (rho_tot(x, I - 1, J, K) + rho_tot(x, I, J, K));
    return 0.125 * (s0 + s1);
}
/* velocity component c (0=u,1=v,2=w) at lattice point (I,J,K): predicted points divide momentum by
 * the corner density, diagnosed points store the velocity itself, the lid has w = 0 and copies
 * the horizontal velocity of the level below (rigid top). */
static double lat_vel(const or_ctx *x, int I, int J, int K, int c)
{
    const or_grid *g = x->g;
    if (K >= g->nz) {
        if (c == 2) return 0.0;
        K = g->nz - 1;
    }
    size_t p = cidx(g, I, J, K);
    const double *m = c == 0 ? x->q->mu : (c == 1 ? x->q->mv : x->q->mw);
    if (x->G->vcls[p] == OR_PRED) return m[p] / rho_corner(x, I, J, K);
    return m[p];
}

/* ------------------------------------------------------------------------------------------ */
/* Velocity diagnostics (Sec. 2.4): boundary velocity by the nearest plane and the free-slip     */
/* projection (eq. 33), merged-face points by linear interpolation, absorbed cells mirror their  */
/* master, fully buried cells hold zero.                                                        */
/* ------------------------------------------------------------------------------------------ */
static int is_pred(const or_ctx *x, int I, int J, int K)
{
    if (K < 0 || K >= x->g->nz) return 0;
    return x->G->vcls[cidx(x->g, I, J, K)] == OR_PRED;
}

/* bilinear weights of the four face corners (lower-index corner first) */
static void face_weights(double a, double b, double w[4])
{
    w[0] = (1.0 - a) * (1.0 - b);
    w[1] = a * (1.0 - b);
    w[2] = (1.0 - a) * b;
    w[3] = a * b;
}

/* Try the first three lattice planes of one family (0: x = const, 1: y = const, 2: z = const)
 * beyond the terrain point B along the normal line.  On each plane the line's intersection falls in
 * a face of four lattice points (located with floor); the first plane whose weighted corners are
 * all predicted gives the bilinear mean velocity (the paper's u_N, weights measured from the face's
 * lower-index corner; a corner whose weight is exactly zero is not required). */
static int plane_family(const or_ctx *x, int fam, int I, int J, double ut[3])
{
    const or_grid *g = x->g;
    size_t nc = (size_t)g->nx * g->ny, hc = hidx(g, I, J);
    double n0 = x->G->nrm[hc], n1 = x->G->nrm[nc + hc], n2 = x->G->nrm[2 * nc + hc];
    double h = x->G->H[hc];
    if (!(h >= 0.0 && h < (double)g->nz * g->dz)) return 0; /* terrain outside the column */
    /* horizontal positions are measured from the corner (I,J) in cell units, so the located face
     * and weights do not depend on where the grid's origin lies */
    for (int m = 0; m < 3; ++m) {
        int P[4][3], ia, ib;
        double a, b;
        if (fam == 2) {
            int K0 = (int)floor(h / g->dz) + 1;
            while (K0 > 0 && (double)(K0 - 1) * g->dz > h) --K0;
            while ((double)K0 * g->dz <= h) ++K0;
            int K = K0 + m;
            if (K > g->nz - 1) return 0;
            double t = ((double)K * g->dz - h) / n2;
            double fx = (t * n0) / g->dx, fy = (t * n1) / g->dy;
            int sx = (int)floor(fx), sy = (int)floor(fy);
            a = fx - (double)sx; b = fy - (double)sy;
            ia = I + sx; ib = J + sy;
            int Q[4][3] = {{ia, ib, K}, {ia + 1, ib, K}, {ia, ib + 1, K}, {ia + 1, ib + 1, K}};
            memcpy(P, Q, sizeof(P));
        } else {
            double nn = fam == 0 ? n0 : n1;
            if (nn == 0.0) return 0;
            int step = (m + 1) * (nn > 0.0 ? 1 : -1);
            double t = fam == 0 ? ((double)step * g->dx) / nn : ((double)step * g->dy) / nn;
            double fa = fam == 0 ? (t * n1) / g->dy : (t * n0) / g->dx;
            double fz = (h + t * n2) / g->dz;
            int sa = (int)floor(fa);
            ib = (int)floor(fz);
            a = fa - (double)sa; b = fz - (double)ib;
            ia = (fam == 0 ? J : I) + sa;
            if (ib < 0 || ib + 1 > g->nz - 1) continue;
            if (fam == 0) {
                int X = I + step;
                int Q[4][3] = {{X, ia, ib}, {X, ia + 1, ib}, {X, ia, ib + 1}, {X, ia + 1, ib + 1}};
                memcpy(P, Q, sizeof(P));
            } else {
                int Y = J + step;
                int Q[4][3] = {{ia, Y, ib}, {ia + 1, Y, ib}, {ia, Y, ib + 1}, {ia + 1, Y, ib + 1}};
                memcpy(P, Q, sizeof(P));
            }
        }
        /* every corner that carries weight must be a predicted point */
        double w[4];
        face_weights(a, b, w);
        int ok = 1;
        for (int t = 0; t < 4 && ok; ++t)
            if (w[t] != 0.0) ok = is_pred(x, P[t][0], P[t][1], P[t][2]);
        if (!ok) continue;
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int t = 0; t < 4; ++t)
                if (w[t] != 0.0) s += w[t] * lat_vel(x, P[t][0], P[t][1], P[t][2], c);
            ut[c] = s;
        }
        return 1;
    }
    return 0;
}

/* mean velocity near the boundary point of corner (I,J): the plane family normal to the dominant
 * component of the terrain normal first (ties: z, x, y), then the other two families in the order
 * z, x, y. */
static int nearest_plane_velocity(const or_ctx *x, int I, int J, double ut[3])
{
    const or_grid *g = x->g;
    size_t nc = (size_t)g->nx * g->ny, hc = hidx(g, I, J);
    double an0 = fabs(x->G->nrm[hc]), an1 = fabs(x->G->nrm[nc + hc]), an2 = fabs(x->G->nrm[2 * nc + hc]);
    int dom = (an2 >= an0 && an2 >= an1) ? 2 : (an0 >= an1 ? 0 : 1);
    if (plane_family(x, dom, I, J, ut)) return 1;
    static const int order[3] = {2, 0, 1};
    for (int f = 0; f < 3; ++f)
        if (order[f] != dom && plane_family(x, order[f], I, J, ut)) return 1;
    return 0;
}

/* boundary velocity at every column corner: nearest-plane mean velocity followed by the free-slip
 * projection u_B = u~ - (u~ . n) n of eq. 33; corners without a usable plane take u~ = 0 and are
 * flagged.  Returns the number of flagged corners. */
int64_t or_boundary_velocity(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                             const double *rthb, const double *pb, const or_state *q, double *ub,
                             int8_t *flag)
{
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
    size_t nc = (size_t)g->nx * g->ny;
    int64_t noplane = 0;
    for (int I = 0; I < g->nx; ++I)
        for (int J = 0; J < g->ny; ++J) {
            size_t hc = hidx(g, I, J);
            double ut[3] = {0.0, 0.0, 0.0};
            int ok = nearest_plane_velocity(&x, I, J, ut);
            /* counted when the terrain point lies in the grid's height range (a raised block of a
             * refined grid has its ground elsewhere) */
            double h = G->H[hc];
            if (!ok && h >= 0.0 && h < (double)g->nz * g->dz) ++noplane;
            if (flag) flag[hc] = (int8_t)!ok;
            double n0 = G->nrm[hc], n1 = G->nrm[nc + hc], n2 = G->nrm[2 * nc + hc];
            double d = ut[0] * n0 + ut[1] * n1 + ut[2] * n2;
            ub[3 * hc + 0] = ut[0] - d * n0;
            ub[3 * hc + 1] = ut[1] - d * n1;
            ub[3 * hc + 2] = ut[2] - d * n2;
        }
    return noplane;
}

/* counts[1] += corners without a usable nearest plane */
void or_diagnose(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                 const double *rthb, const double *pb, or_state *q, int64_t *counts)
{
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t nc = (size_t)nx * ny;
    double *ub = (double *)malloc(sizeof(double) * 3 * nc);
    /* step 2 of the three-step procedure: boundary velocities from predicted ones */
    int64_t noplane = or_boundary_velocity(g, ph, G, rhob, rthb, pb, q, ub, NULL);
    /* step 3: points on or below the terrain carry the boundary velocity; merged-face points
     * interpolate linearly between the boundary point and the lowest predicted point above. */
    for (int I = 0; I < nx; ++I)
        for (int J = 0; J < ny; ++J) {
            size_t hc = hidx(g, I, J);
            double h = G->H[hc];
            for (int K = 0; K < nz; ++K) {
                size_t p = cidx(g, I, J, K);
                int vc = G->vcls[p];
                if (vc == OR_PRED) continue;
                double u[3] = {ub[3 * hc], ub[3 * hc + 1], ub[3 * hc + 2]};
                if (vc == OR_MFACE) {
                    int kp = -1;
                    for (int kk = K + 1; kk <= K + OR_MAXHOPS && kk < nz; ++kk)
                        if (G->vcls[cidx(g, I, J, kk)] == OR_PRED) { kp = kk; break; }
                    if (kp >= 0) {
                        double gam = ((double)K * g->dz - h) / ((double)kp * g->dz - h);
                        for (int c = 0; c < 3; ++c)
                            u[c] = lat_vel(&x, I, J, kp, c) * gam + ub[3 * hc + c] * (1.0 - gam);
                    }
                }
                q->mu[p] = u[0];
                q->mv[p] = u[1];
                q->mw[p] = u[2];
            }
        }
    /* scalars: absorbed cells mirror their master, buried cells hold zero (Sec. 2.5) */
    size_t n = (size_t)nx * ny * nz;
    for (size_t c = 0; c < n; ++c) {
        if (G->cls[c] == OR_SOLID) { q->rho[c] = 0.0; q->rth[c] = 0.0; }
        else if (G->cls[c] == OR_ABSORBED) { q->rho[c] = q->rho[G->master[c]]; q->rth[c] = q->rth[G->master[c]]; }
    }
    free(ub);
    if (counts) counts[1] += noplane;
}

/* ------------------------------------------------------------------------------------------ */
/* Initial state: theta' noise applied at constant pressure ((rho theta)' = 0), uniform inflow    */
/* (U0, V0, 0) as momentum rho_c U0 at predicted points, then one diagnostic pass.              */
/* ------------------------------------------------------------------------------------------ */
void or_init_state(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                   const double *rthb, const double *pb, const double *thb, const double *noise,
                   or_state *q, int64_t *counts)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                size_t c = cidx(g, i, j, k);
                q->rth[c] = 0.0;
                q->rho[c] = 0.0;
                if (G->cls[c] == OR_OPEN || G->cls[c] == OR_ORPHAN) {
                    /* rho' = (rho theta)bar/(thetabar + theta') - rhobar, written without the
                     * cancellation: rhobar = (rho theta)bar / thetabar */
                    double thp = noise ? noise[c] : 0.0;
                    q->rho[c] = thp != 0.0 ? -(rhob[k] * thp) / (thb[k] + thp) : 0.0;
                }
                q->mu[c] = 0.0; q->mv[c] = 0.0; q->mw[c] = 0.0;
            }
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
    for (int I = 0; I < nx; ++I)
        for (int J = 0; J < ny; ++J)
            for (int K = 0; K < nz; ++K) {
                size_t p = cidx(g, I, J, K);
                if (G->vcls[p] != OR_PRED) continue;
                double rc = rho_corner(&x, I, J, K);
                q->mu[p] = rc * ph->u0;
                q->mv[p] = rc * ph->v0;
                q->mw[p] = 0.0;
            }
    or_diagnose(g, ph, G, rhob, rthb, pb, q, counts);
}

/* ------------------------------------------------------------------------------------------ */
/* Tendencies (Sec. 2.4).                                                                       */
/* ------------------------------------------------------------------------------------------ */

/* total value of a scalar for the group that owns cell (i,j,k), at the master's level */
static double group_scalar(const or_ctx *x, size_t c, int which)
{
    int32_t m = x->G->master[c];
    int km = (int)(m % x->g->nz);
    return which == 0 ? x->rhob[km] + x->q->rho[m] : x->rthb[km] + x->q->rth[m];
}

/* Fluxes of rho (F[0]) and rho*theta (F[1]) through a face, positive along +axis.
 * axis 0: x-face at x = I dx between cells (I-1,j,k) and (I,j,k); similarly for y and z.
 * Scalar: mean of the two exchanging groups' values (first-order, conservative).
 * Normal velocity: mean of the four corner values (eqs. ux1-ux3).  Area: aperture x full area. */
static void face_flux(const or_ctx *x, int axis, int I, int J, int K, double F[2])
{
    const or_grid *g = x->g;
    size_t up = cidx(g, I, J, K), lo;
    double A, S, un;
    if (axis == 0) {
        lo = cidx(g, I - 1, J, K);
        A = x->G->Ax[up];
        S = g->dy * g->dz;
        un = 0.25 * ((lat_vel(x, I, J, K, 0) + lat_vel(x, I, J + 1, K, 0)) +
                     (lat_vel(x, I, J, K + 1, 0) + lat_vel(x, I, J + 1, K + 1, 0)));
    } else if (axis == 1) {
        lo = cidx(g, I, J - 1, K);
        A = x->G->Ay[up];
        S = g->dz * g->dx;
        un = 0.25 * ((lat_vel(x, I, J, K, 1) + lat_vel(x, I + 1, J, K, 1)) +
                     (lat_vel(x, I, J, K + 1, 1) + lat_vel(x, I + 1, J, K + 1, 1)));
    } else {
        lo = cidx(g, I, J, K - 1);
        A = x->G->Az[up];
        S = g->dx * g->dy;
        un = 0.25 * ((lat_vel(x, I, J, K, 2) + lat_vel(x, I + 1, J, K, 2)) +
                     (lat_vel(x, I, J + 1, K, 2) + lat_vel(x, I + 1, J + 1, K, 2)));
    }
    for (int w = 0; w < 2; ++w) {
        double phi = 0.5 * (group_scalar(x, lo, w) + group_scalar(x, up, w));
        F[w] = phi * un * A * S;
    }
}

/* net outward flux of a merged group with master m (members in increasing linear index, faces in
 * the order -x,+x,-y,+y,-z,+z; faces between members of the same group are internal) */
static void group_divergence(const or_ctx *x, size_t m, const size_t *mem, int nmem, double R[2])
{
    const or_grid *g = x->g;
    R[0] = 0.0; R[1] = 0.0;
    for (int t = 0; t < nmem; ++t) {
        size_t c = mem[t];
        int k = (int)(c % g->nz);
        int j = (int)((c / g->nz) % g->ny);
        int i = (int)(c / ((size_t)g->nz * g->ny));
        for (int f = 0; f < 6; ++f) {
            int axis = f / 2, plus = f & 1;
            int fi = i, fj = j, fk = k;      /* the "upper" cell of the face */
            int ni = i, nj = j, nk = k;      /* the neighbour across the face */
            if (axis == 0) { if (plus) { fi = i + 1; ni = i + 1; } else { ni = i - 1; } }
            if (axis == 1) { if (plus) { fj = j + 1; nj = j + 1; } else { nj = j - 1; } }
            if (axis == 2) {
                if (plus) { fk = k + 1; nk = k + 1; } else { nk = k - 1; }
                if (nk < 0 || nk >= g->nz) continue; /* ground and rigid lid carry no flux */
            }
            size_t fu = cidx(g, fi, fj, fk);
            double A = axis == 0 ? x->G->Ax[fu] : (axis == 1 ? x->G->Ay[fu] : x->G->Az[fu]);
            if (A == 0.0) continue; /* closed face, incl. the terrain and buried neighbours */
            size_t nb = cidx(g, ni, nj, nk);
            if ((size_t)x->G->master[nb] == m) continue;
            double F[2];
            face_flux(x, axis, fi, fj, fk, F);
            if (plus) { R[0] += F[0]; R[1] += F[1]; }
            else { R[0] -= F[0]; R[1] -= F[1]; }
        }
    }
}

/* momentum tendency at a predicted point: quasi-flux-form advection through the faces of the
 * rectangular velocity cell, second-order pressure gradient and buoyancy (eqs. momentum_u_d ...) */
static void momentum_tendency(const or_ctx *x, int I, int J, int K, double out[3])
{
    const or_grid *g = x->g;
    double u[7][3]; /* p, p-x, p+x, p-y, p+y, p-z, p+z */
    static const int off[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    for (int s = 0; s < 7; ++s)
        for (int c = 0; c < 3; ++c) u[s][c] = lat_vel(x, I + off[s][0], J + off[s][1], K + off[s][2], c);
    /* face densities: mean of the four cell densities on each face of the velocity cell */
    double Rxm = 0.25 * ((rho_tot(x, I - 1, J - 1, K - 1) + rho_tot(x, I - 1, J, K - 1)) +
                         (rho_tot(x, I - 1, J - 1, K) + rho_tot(x, I - 1, J, K)));
    double Rxp = 0.25 * ((rho_tot(x, I, J - 1, K - 1) + rho_tot(x, I, J, K - 1)) +
                         (rho_tot(x, I, J - 1, K) + rho_tot(x, I, J, K)));
    double Rym = 0.25 * ((rho_tot(x, I - 1, J - 1, K - 1) + rho_tot(x, I, J - 1, K - 1)) +
                         (rho_tot(x, I - 1, J - 1, K) + rho_tot(x, I, J - 1, K)));
    double Ryp = 0.25 * ((rho_tot(x, I - 1, J, K - 1) + rho_tot(x, I, J, K - 1)) +
                         (rho_tot(x, I - 1, J, K) + rho_tot(x, I, J, K)));
    double Rzm = 0.25 * ((rho_tot(x, I - 1, J - 1, K - 1) + rho_tot(x, I, J - 1, K - 1)) +
                         (rho_tot(x, I - 1, J, K - 1) + rho_tot(x, I, J, K - 1)));
    double Rzp = 0.25 * ((rho_tot(x, I - 1, J - 1, K) + rho_tot(x, I, J - 1, K)) +
                         (rho_tot(x, I - 1, J, K) + rho_tot(x, I, J, K)));
    /* pressure perturbation means on the same faces */
    double Pxm = 0.25 * ((pprime(x, I - 1, J - 1, K - 1) + pprime(x, I - 1, J, K - 1)) +
                         (pprime(x, I - 1, J - 1, K) + pprime(x, I - 1, J, K)));
    double Pxp = 0.25 * ((pprime(x, I, J - 1, K - 1) + pprime(x, I, J, K - 1)) +
                         (pprime(x, I, J - 1, K) + pprime(x, I, J, K)));
    double Pym = 0.25 * ((pprime(x, I - 1, J - 1, K - 1) + pprime(x, I, J - 1, K - 1)) +
                         (pprime(x, I - 1, J - 1, K) + pprime(x, I, J - 1, K)));
    double Pyp = 0.25 * ((pprime(x, I - 1, J, K - 1) + pprime(x, I, J, K - 1)) +
                         (pprime(x, I - 1, J, K) + pprime(x, I, J, K)));
    double Pzm = 0.25 * ((pprime(x, I - 1, J - 1, K - 1) + pprime(x, I, J - 1, K - 1)) +
                         (pprime(x, I - 1, J, K - 1) + pprime(x, I, J, K - 1)));
    double Pzp = 0.25 * ((pprime(x, I - 1, J - 1, K) + pprime(x, I, J - 1, K)) +
                         (pprime(x, I - 1, J, K) + pprime(x, I, J, K)));
    double rp8 = 0.0;
    for (int dk = -1; dk <= 0; ++dk)
        for (int dj = -1; dj <= 0; ++dj)
            for (int di = -1; di <= 0; ++di) rp8 += x->q->rho[cidx(g, I + di, J + dj, K + dk)];
    rp8 *= 0.125;
    for (int c = 0; c < 3; ++c) {
        double fxp = Rxp * (0.5 * (u[0][0] + u[2][0])) * (0.5 * (u[0][c] + u[2][c]));
        double fxm = Rxm * (0.5 * (u[1][0] + u[0][0])) * (0.5 * (u[1][c] + u[0][c]));
        double fyp = Ryp * (0.5 * (u[0][1] + u[4][1])) * (0.5 * (u[0][c] + u[4][c]));
        double fym = Rym * (0.5 * (u[3][1] + u[0][1])) * (0.5 * (u[3][c] + u[0][c]));
        double fzp = Rzp * (0.5 * (u[0][2] + u[6][2])) * (0.5 * (u[0][c] + u[6][c]));
        double fzm = Rzm * (0.5 * (u[5][2] + u[0][2])) * (0.5 * (u[5][c] + u[0][c]));
        double adv = (fxp - fxm) / g->dx + (fyp - fym) / g->dy + (fzp - fzm) / g->dz;
        double pgf = c == 0 ? (Pxp - Pxm) / g->dx : (c == 1 ? (Pyp - Pym) / g->dy : (Pzp - Pzm) / g->dz);
        double buoy = c == 2 ? x->ph->g * rp8 : 0.0;
        out[c] = -adv - pgf - buoy;
    }
}

/* member lists of every group in increasing linear index (head/next linked list) */
static void build_groups(const or_grid *g, const or_geom *G, int64_t *head, int64_t *next)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    for (size_t c = 0; c < n; ++c) { head[c] = -1; next[c] = -1; }
    int64_t *tail = (int64_t *)malloc(sizeof(int64_t) * n);
    for (size_t c = 0; c < n; ++c) tail[c] = -1;
    for (size_t c = 0; c < n; ++c) {
        if (G->cls[c] == OR_SOLID) continue;
        size_t m = (size_t)G->master[c];
        if (head[m] < 0) head[m] = (int64_t)c;
        else next[tail[m]] = (int64_t)c;
        tail[m] = (int64_t)c;
    }
    free(tail);
}

/* ------------------------------------------------------------------------------------------ */
/* Fourth-order artificial diffusion (Sec. 2.1: source terms D of every prognostic equation; a  */
/* 5-point stencil per direction, Sec. 2.2; a second-order term where the fourth-order stencil  */
/* lacks fluid neighbours, with the terrain as boundary, Sec. 2.4).  Written in flux form: the   */
/* flux through a face is the third difference of the four values straddling it, or -4 x their  */
/* first difference when one of the outer two is missing, and zero through a closed face, so    */
/* D = -k x (flux out - flux in) reduces to -k (phi_{i-2} - 4 phi_{i-1} + 6 phi_i - 4 phi_{i+1} + */
/* phi_{i+2}) in the interior and conserves the scalars.  Scalars: the group values of rho' and  */
/* (rho theta)', apertures and group volume as for the advective fluxes; momentum: the           */
/* perturbation rho u - rhobar_c (u0, v0, 0) at predicted points, the others act as boundary.    */
/* ------------------------------------------------------------------------------------------ */

/* group value of scalar w (0: rho', 1: (rho theta)') of non-solid cell c */
static double group_pert(const or_ctx *x, size_t c, int w)
{
    int32_t m = x->G->master[c];
    return w == 0 ? x->q->rho[m] : x->q->rth[m];
}

/* diffusive flux of both scalars through the face between L = (i,j,k) - e_a and U = (i,j,k) along
 * axis a, positive along +a (without the rate): F[w] */
static void diffusion_face(const or_ctx *x, int a, int i, int j, int k, double F[2])
{
    const or_grid *g = x->g;
    int dl[3] = {0, 0, 0};
    dl[a] = 1;
    size_t U = cidx(g, i, j, k), L = cidx(g, i - dl[0], j - dl[1], k - dl[2]);
    double A = a == 0 ? x->G->Ax[U] : (a == 1 ? x->G->Ay[U] : x->G->Az[U]);
    F[0] = F[1] = 0.0;
    if (a == 2 && (k - 1 < 0 || k >= g->nz)) return; /* ground and lid */
    if (A == 0.0 || x->G->master[L] == x->G->master[U]) return; /* closed or internal face */
    int k2l = k - 2 * dl[2], k2u = k + dl[2];
    int outer = k2l >= 0 && k2u < g->nz;
    size_t L2 = 0, U2 = 0;
    if (outer) {
        L2 = cidx(g, i - 2 * dl[0], j - 2 * dl[1], k2l);
        U2 = cidx(g, i + dl[0], j + dl[1], k2u);
        outer = x->G->V[L2] > 0.0 && x->G->V[U2] > 0.0;
    }
    for (int w = 0; w < 2; ++w) {
        double pl = group_pert(x, L, w), pu = group_pert(x, U, w);
        if (outer)
            F[w] = ((group_pert(x, U2, w) - 3.0 * pu) + 3.0 * pl) - group_pert(x, L2, w);
        else
            F[w] = -4.0 * (pu - pl);
    }
}

/* D of the two scalars at master m (members in increasing linear index, faces -x,+x,-y,+y,-z,+z) */
static void diffusion_group(const or_ctx *x, size_t m, const size_t *mem, int nmem, double D[2])
{
    const or_grid *g = x->g;
    double acc[2] = {0.0, 0.0};
    for (int t = 0; t < nmem; ++t) {
        size_t c = mem[t];
        int k = (int)(c % g->nz), j = (int)((c / g->nz) % g->ny), i = (int)(c / ((size_t)g->nz * g->ny));
        for (int f = 0; f < 6; ++f) {
            int a = f / 2, plus = f & 1;
            int fi = i + (a == 0 && plus), fj = j + (a == 1 && plus), fk = k + (a == 2 && plus);
            if (a == 2 && (fk <= 0 || fk >= g->nz)) continue;
            size_t fu = cidx(g, fi, fj, fk);
            double A = a == 0 ? x->G->Ax[fu] : (a == 1 ? x->G->Ay[fu] : x->G->Az[fu]);
            double kr = a == 2 ? x->ph->kdv : x->ph->kdh;
            double F[2];
            diffusion_face(x, a, fi, fj, fk, F);
            for (int w = 0; w < 2; ++w) {
                double term = (kr * A) * F[w];
                acc[w] = plus ? acc[w] + term : acc[w] - term;
            }
        }
    }
    double vg = x->G->Vgroup[m];
    D[0] = -acc[0] / vg;
    D[1] = -acc[1] / vg;
}

/* momentum perturbation component c at lattice point p (level K) */
static double mom_pert(const or_ctx *x, size_t p, int K, int c)
{
    double rbc = 0.5 * (x->rhob[K - 1] + x->rhob[K]);
    if (c == 0) return x->q->mu[p] - rbc * x->ph->u0;
    if (c == 1) return x->q->mv[p] - rbc * x->ph->v0;
    return x->q->mw[p];
}

/* diffusive flux of the momentum perturbation through the face between lattice points P = (I,J,K)
 * and Q = P + e_a, positive along +a: F[3] */
static void diffusion_lattice_face(const or_ctx *x, int a, int I, int J, int K, double F[3])
{
    int d[3] = {0, 0, 0};
    d[a] = 1;
    F[0] = F[1] = F[2] = 0.0;
    if (!is_pred(x, I, J, K) || !is_pred(x, I + d[0], J + d[1], K + d[2])) return;
    const or_grid *g = x->g;
    size_t P = cidx(g, I, J, K), Q = cidx(g, I + d[0], J + d[1], K + d[2]);
    int outer = is_pred(x, I - d[0], J - d[1], K - d[2]) && is_pred(x, I + 2 * d[0], J + 2 * d[1], K + 2 * d[2]);
    size_t P2 = outer ? cidx(g, I - d[0], J - d[1], K - d[2]) : 0;
    size_t Q2 = outer ? cidx(g, I + 2 * d[0], J + 2 * d[1], K + 2 * d[2]) : 0;
    for (int c = 0; c < 3; ++c) {
        double mp = mom_pert(x, P, K, c), mq = mom_pert(x, Q, K + d[2], c);
        if (outer)
            F[c] = ((mom_pert(x, Q2, K + 2 * d[2], c) - 3.0 * mq) + 3.0 * mp) - mom_pert(x, P2, K - d[2], c);
        else
            F[c] = -4.0 * (mq - mp);
    }
}

/* D of the momentum perturbation at predicted point (I,J,K): axes x, y, z */
static void diffusion_point(const or_ctx *x, int I, int J, int K, double D[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
        int d[3] = {0, 0, 0};
        d[a] = 1;
        double kr = a == 2 ? x->ph->kdv : x->ph->kdh;
        double Fp[3], Fm[3];
        diffusion_lattice_face(x, a, I, J, K, Fp);
        diffusion_lattice_face(x, a, I - d[0], J - d[1], K - d[2], Fm);
        for (int c = 0; c < 3; ++c) acc[c] += kr * (Fp[c] - Fm[c]);
    }
    for (int c = 0; c < 3; ++c) D[c] = -acc[c];
}

/* ------------------------------------------------------------------------------------------ */
/* Sponge layer below the rigid lid (Sec. 3: absorbing layer above 10 km after Klemp & Lilly).   */
/* The paper names the layer but not its form.  Reading: Rayleigh damping towards the initial    */
/* state, -tau(z) (q - q_ref), with tau rising from 0 at z = zsp to rsp at the lid as             */
/* sin^2(pi/2 (z - zsp)/(ztop - zsp)).  It acts on (rho theta)' at group masters (cell centre     */
/* height) and on the momentum perturbation rho u - rhobar_c (u0, v0, 0) at predicted points      */
/* (lattice height); rho' is left alone, so the total mass stays conserved.                       */
/* ------------------------------------------------------------------------------------------ */
static double sponge_rate(const or_grid *g, const or_phys *ph, double z)
{
    double ztop = ph->ztop != 0.0 ? ph->ztop : g->z0 + g->nz * g->dz;  /* the domain's lid */
    if (ph->rsp == 0.0 || z <= ph->zsp || ph->zsp >= ztop) return 0.0;
    double s = sin(0.5 * 3.14159265358979323846 * (z - ph->zsp) / (ztop - ph->zsp));
    return ph->rsp * (s * s);
}

static void tendency_cell(const or_ctx *x, size_t c, const int64_t *head, const int64_t *next,
                          double dq[5], int *has_scalar, int *has_mom)
{
    const or_grid *g = x->g;
    const or_geom *G = x->G;
    int k = (int)(c % g->nz), j = (int)((c / g->nz) % g->ny), i = (int)(c / ((size_t)g->nz * g->ny));
    *has_scalar = 0; *has_mom = 0;
    for (int t = 0; t < 5; ++t) dq[t] = 0.0;
    if (G->cls[c] == OR_OPEN || G->cls[c] == OR_ORPHAN) {
        size_t mem[64];
        int nm = 0;
        for (int64_t t = head[c]; t >= 0 && nm < 64; t = next[t]) mem[nm++] = (size_t)t;
        double R[2];
        group_divergence(x, c, mem, nm, R);
        double vol = G->Vgroup[c] * (g->dx * g->dy * g->dz);
        dq[0] = -R[0] / vol;
        dq[1] = -R[1] / vol;
        if (x->ph->kdh != 0.0 || x->ph->kdv != 0.0) {
            double D[2];
            diffusion_group(x, c, mem, nm, D);
            dq[0] += D[0];
            dq[1] += D[1];
        }
        double tau = sponge_rate(g, x->ph, g->z0 + (k + 0.5) * g->dz);
        if (tau != 0.0) dq[1] += -tau * x->q->rth[c];
        *has_scalar = 1;
    }
    if (G->vcls[c] == OR_PRED) {
        double m3[3];
        momentum_tendency(x, i, j, k, m3);
        dq[2] = m3[0]; dq[3] = m3[1]; dq[4] = m3[2];
        if (x->ph->kdh != 0.0 || x->ph->kdv != 0.0) {
            double D[3];
            diffusion_point(x, i, j, k, D);
            dq[2] += D[0]; dq[3] += D[1]; dq[4] += D[2];
        }
        double tau = sponge_rate(g, x->ph, g->z0 + k * g->dz);
        if (tau != 0.0) {
            dq[2] += -tau * mom_pert(x, c, k, 0);
            dq[3] += -tau * mom_pert(x, c, k, 1);
            dq[4] += -tau * mom_pert(x, c, k, 2);
        }
        *has_mom = 1;
    }
}

/* full tendency field: scalars at group masters, momentum at predicted points, zero elsewhere */
void or_tendency(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                 const double *rthb, const double *pb, const or_state *q, or_state *dq)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * n), *next = (int64_t *)malloc(sizeof(int64_t) * n);
    build_groups(g, G, head, next);
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
#pragma omp parallel for schedule(static)
    for (long long cc = 0; cc < (long long)n; ++cc) {
        double d[5];
        int hs, hm;
        tendency_cell(&x, (size_t)cc, head, next, d, &hs, &hm);
        dq->rho[cc] = d[0]; dq->rth[cc] = d[1]; dq->mu[cc] = d[2]; dq->mv[cc] = d[3]; dq->mw[cc] = d[4];
    }
    free(head); free(next);
}

/* tendency at a list of cells only (for sampled comparison on large grids) */
void or_tendency_points(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                        const double *rthb, const double *pb, const or_state *q, const int64_t *pts,
                        int64_t npts, double *out /* [npts][5] */)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * n), *next = (int64_t *)malloc(sizeof(int64_t) * n);
    build_groups(g, G, head, next);
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
#pragma omp parallel for schedule(static)
    for (long long t = 0; t < (long long)npts; ++t) {
        int hs, hm;
        tendency_cell(&x, (size_t)pts[t], head, next, out + 5 * t, &hs, &hm);
    }
    free(head); free(next);
}

/* ------------------------------------------------------------------------------------------ */
/* Explicit three-stage Runge-Kutta (Wicker & Skamarock 2002): q_out = q_n + cdt * L(q_s),       */
/* applied to group masters and predicted points, followed by the diagnostic pass.              */
/* ------------------------------------------------------------------------------------------ */
/* the update alone (group masters and predicted points) with the group member lists given */
static void rk_update_groups(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                             const double *rthb, const double *pb, const or_state *qn, const or_state *qs,
                             or_state *qout, double cdt, const int64_t *head, const int64_t *next)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    or_ctx x = {g, ph, G, rhob, rthb, pb, qs};
#pragma omp parallel for schedule(static)
    for (long long cc = 0; cc < (long long)n; ++cc) {
        double d[5];
        int hs, hm;
        tendency_cell(&x, (size_t)cc, head, next, d, &hs, &hm);
        if (hs) {
            qout->rho[cc] = qn->rho[cc] + cdt * d[0];
            qout->rth[cc] = qn->rth[cc] + cdt * d[1];
        }
        if (hm) {
            qout->mu[cc] = qn->mu[cc] + cdt * d[2];
            qout->mv[cc] = qn->mv[cc] + cdt * d[3];
            qout->mw[cc] = qn->mw[cc] + cdt * d[4];
        }
    }
}

/* the update alone (group masters and predicted points), without the diagnostic pass */
void or_rk_update(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                  const double *rthb, const double *pb, const or_state *qn, const or_state *qs,
                  or_state *qout, double cdt)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * n), *next = (int64_t *)malloc(sizeof(int64_t) * n);
    build_groups(g, G, head, next);
    rk_update_groups(g, ph, G, rhob, rthb, pb, qn, qs, qout, cdt, head, next);
    free(head); free(next);
}

void or_rk_stage(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                 const double *rthb, const double *pb, const or_state *qn, const or_state *qs,
                 or_state *qout, double cdt, int64_t *counts)
{
    or_rk_update(g, ph, G, rhob, rthb, pb, qn, qs, qout, cdt);
    or_diagnose(g, ph, G, rhob, rthb, pb, qout, counts);
}

/* total fluxes of rho and rho*theta through the face at the lower side of cell (I,J,K) along
 * `axis` (positive along +axis), as the tendency uses them */
void or_face_flux(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                  const double *rthb, const double *pb, const or_state *q, int axis, int I, int J, int K,
                  double *F)
{
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
    face_flux(&x, axis, I, J, K, F);
}

/* ------------------------------------------------------------------------------------------ */
/* Conservation diagnostics: out = {M', Theta', M_total, E}                                    */
/* M' = sum over groups of Vgroup dV rho'_m (conserved), Theta' likewise for (rho theta)',      */
/* M_total adds the base density at the master's level, E = internal + potential energy of the  */
/* groups + kinetic energy of predicted points (not conserved by the scheme).  Summed in linear */
/* index order.                                                                                 */
/* ------------------------------------------------------------------------------------------ */
/* compensated (Neumaier) running sum: the sums below run over every cell of a grid (tens of
 * millions of terms of one sign), where a plain running sum loses accuracy in proportion to the
 * number of terms; with the correction term the result is within a few rounding errors of the
 * exact sum whatever the count */
typedef struct { double s, c; } or_ksum;
static inline void ksum_add(or_ksum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

void or_reduce(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
               const double *rthb, const double *pb, const or_state *q, double out[4])
{
    or_ctx x = {g, ph, G, rhob, rthb, pb, q};
    size_t n = (size_t)g->nx * g->ny * g->nz;
    double dV = g->dx * g->dy * g->dz;
    double gam = ph->cp / (ph->cp - ph->rd);
    or_ksum mp = {0.0, 0.0}, tp = {0.0, 0.0}, mt = {0.0, 0.0}, e = {0.0, 0.0};
    for (size_t c = 0; c < n; ++c) {
        int k = (int)(c % g->nz);
        int j = (int)((c / g->nz) % g->ny);
        int i = (int)(c / ((size_t)g->nz * g->ny));
        if (G->cls[c] == OR_OPEN || G->cls[c] == OR_ORPHAN) {
            double vg = G->Vgroup[c] * dV;
            double rho = rhob[k] + q->rho[c];
            double p = pb[k] + eos_pprime(q->rth[c], rthb[k], pb[k], gam);
            double z = g->z0 + ((double)k + 0.5) * g->dz;
            ksum_add(&mp, vg * q->rho[c]);
            ksum_add(&tp, vg * q->rth[c]);
            ksum_add(&mt, vg * rho);
            ksum_add(&e, vg * (p / (gam - 1.0) + rho * ph->g * z));
        }
        if (G->vcls[c] == OR_PRED) {
            double rc = rho_corner(&x, i, j, k);
            double u = q->mu[c] / rc, v = q->mv[c] / rc, w = q->mw[c] / rc;
            ksum_add(&e, dV * 0.5 * rc * (u * u + v * v + w * w));
        }
    }
    out[0] = mp.s + mp.c; out[1] = tp.s + tp.c; out[2] = mt.s + mt.c; out[3] = e.s + e.c;
}

/* nsteps full WS-RK3 steps; q is advanced in place using two scratch states (the group member
 * lists depend only on the geometry and are built once) */
void or_run(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
            const double *rthb, const double *pb, or_state *q, or_state *s1, or_state *s2,
            double dt, int nsteps, int64_t *counts)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * n), *next = (int64_t *)malloc(sizeof(int64_t) * n);
    build_groups(g, G, head, next);
    for (int st = 0; st < nsteps; ++st) {
        rk_update_groups(g, ph, G, rhob, rthb, pb, q, q, s1, dt / 3.0, head, next);
        or_diagnose(g, ph, G, rhob, rthb, pb, s1, counts);
        rk_update_groups(g, ph, G, rhob, rthb, pb, q, s1, s2, dt / 2.0, head, next);
        or_diagnose(g, ph, G, rhob, rthb, pb, s2, counts);
        rk_update_groups(g, ph, G, rhob, rthb, pb, q, s2, s1, dt, head, next);
        or_diagnose(g, ph, G, rhob, rthb, pb, s1, counts);
        memcpy(q->rho, s1->rho, n * sizeof(double));
        memcpy(q->rth, s1->rth, n * sizeof(double));
        memcpy(q->mu, s1->mu, n * sizeof(double));
        memcpy(q->mv, s1->mv, n * sizeof(double));
        memcpy(q->mw, s1->mw, n * sizeof(double));
    }
    free(head); free(next);
}

/* ------------------------------------------------------------------------------------------ */
/* The paper's own time stepping (Sec. 2.2): leap-frog with the Robert-Asselin filter, with the   */
/* perturbation pressure p' as the prognostic thermodynamic variable (Sec. 2.1, eq. heat).  A     */
/* state "in p' form" holds p' where the (rho theta)' form holds (rho theta)'.                   */
/*                                                                                               */
/* Readings: the coefficient of eq. heat is taken as (cp/cv) R (p/p0)^(R/cp), the factor that     */
/* makes it the chain rule of p = p0 (R rho theta / p0)^(cp/cv) (the printed 1/p0 does not fit    */
/* the units); rho theta in the flux follows from p through that equation of state; D_theta is    */
/* the diffusion and sponge term of (rho theta)'.  The first step is a forward step; the filter   */
/* weight nu is a parameter (the paper gives none).                                             */
/* ------------------------------------------------------------------------------------------ */
/* (rho theta)' from p' through the equation of state: rho theta = rthbar (1 + p'/pbar)^(cv/cp) */
static double eos_rthprime(double pp, double rthbar, double pbar, double gam)
{
    return rthbar * expm1(log1p(pp / pbar) / gam);
}

/* convert the thermodynamic slot of q in place at every non-solid cell: to_p != 0: (rho theta)' ->
 * p'; else p' -> (rho theta)'.  A merged group's value belongs to its master, so the base state of
 * the master's level applies to every member (absorbed cells keep mirroring the master). */
void or_pform(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rthb, const double *pb,
              or_state *q, int to_p)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    double gam = ph->cp / (ph->cp - ph->rd);
    for (size_t c = 0; c < n; ++c) {
        if (G->cls[c] == OR_SOLID) continue;
        int k = (int)((size_t)G->master[c] % g->nz);
        q->rth[c] = to_p ? eos_pprime(q->rth[c], rthb[k], pb[k], gam) : eos_rthprime(q->rth[c], rthb[k], pb[k], gam);
    }
}

/* one leap-frog step in p' form.  first != 0: forward step qp = q0 + dt L(q0) (qm unused, q0 not
 * filtered).  Else qp = qm + 2 dt L(q0), with qm the filtered state of the previous time level,
 * then q0 is filtered in place: q0 += nu (qm - 2 q0 + qp).  L of p' at a group master is
 * (cp/cv) R (p/p0)^(R/cp) times the (rho theta)' tendency of the merged-cell scheme, p and rho
 * theta of the master's level at time n.  Updates and the filter act at group masters (scalars)
 * and predicted points (momentum); qp then takes the diagnostic pass. */
void or_lf_step(const or_grid *g, const or_phys *ph, const or_geom *G, const double *rhob,
                const double *rthb, const double *pb, const or_state *qm, or_state *q0, or_state *qp,
                double dt, double nu, int first, int64_t *counts)
{
    size_t n = (size_t)g->nx * g->ny * g->nz;
    double gam = ph->cp / (ph->cp - ph->rd);
    double kappa = ph->rd / ph->cp;
    /* the tendency of the (rho theta)' form at time n */
    or_state t = {(double *)malloc(n * sizeof(double)), (double *)malloc(n * sizeof(double)), q0->mu, q0->mv,
                  q0->mw};
    memcpy(t.rho, q0->rho, n * sizeof(double));
    memcpy(t.rth, q0->rth, n * sizeof(double));
    or_pform(g, ph, G, rthb, pb, &t, 0);
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * n), *next = (int64_t *)malloc(sizeof(int64_t) * n);
    build_groups(g, G, head, next);
    or_ctx x = {g, ph, G, rhob, rthb, pb, &t};
    const or_state *base = first ? q0 : qm;
    double h = first ? dt : 2.0 * dt;
#pragma omp parallel for schedule(static)
    for (long long cc = 0; cc < (long long)n; ++cc) {
        size_t c = (size_t)cc;
        double d[5];
        int hs, hm;
        tendency_cell(&x, c, head, next, d, &hs, &hm);
        if (hs) {
            int k = (int)(c % g->nz);
            double p = pb[k] + q0->rth[c];
            double coef = gam * ph->rd * pow(p / ph->p0, kappa);
            qp->rho[c] = base->rho[c] + h * d[0];
            qp->rth[c] = base->rth[c] + h * (coef * d[1]);
        }
        if (hm) {
            qp->mu[c] = base->mu[c] + h * d[2];
            qp->mv[c] = base->mv[c] + h * d[3];
            qp->mw[c] = base->mw[c] + h * d[4];
        }
    }
    /* the filter, once every tendency (which reads q0's momentum) has been taken */
    if (!first) {
#pragma omp parallel for schedule(static)
        for (long long cc = 0; cc < (long long)n; ++cc) {
            size_t c = (size_t)cc;
            int hs = G->cls[c] == OR_OPEN || G->cls[c] == OR_ORPHAN, hm = G->vcls[c] == OR_PRED;
            if (hs) {
                q0->rho[c] += nu * ((qm->rho[c] - 2.0 * q0->rho[c]) + qp->rho[c]);
                q0->rth[c] += nu * ((qm->rth[c] - 2.0 * q0->rth[c]) + qp->rth[c]);
            }
            if (hm) {
                q0->mu[c] += nu * ((qm->mu[c] - 2.0 * q0->mu[c]) + qp->mu[c]);
                q0->mv[c] += nu * ((qm->mv[c] - 2.0 * q0->mv[c]) + qp->mv[c]);
                q0->mw[c] += nu * ((qm->mw[c] - 2.0 * q0->mw[c]) + qp->mw[c]);
            }
        }
    }
    /* solid cells of qp hold zero, as after a Runge-Kutta update */
    for (size_t c = 0; c < n; ++c)
        if (G->cls[c] == OR_SOLID) { qp->rho[c] = 0.0; qp->rth[c] = 0.0; }
    free(head); free(next);
    free(t.rho); free(t.rth);
    or_diagnose(g, ph, G, rhob, rthb, pb, qp, counts);
}

/* thread count for the OpenMP loops (results are independent of it: every output element is
 * written by one thread and every sum runs in a fixed order) */
#ifdef _OPENMP
#include <omp.h>
#endif
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
