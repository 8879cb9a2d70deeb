// Streaming form of the regular-point update (Sec. 2.4 tendencies with the Runge-Kutta stage).
//
// A workgroup owns TY x TZ columns-by-levels of a j-k cross-section (k fastest across the threads,
// so every wave reads contiguous k) and marches along x through a chunk of CH planes.  The planes it
// needs are kept in rolling LDS rings: rho' and (rho theta)' of the cell planes i-1, i, i+1 (with a
// halo of two cells in j and k), p' of the cell planes i-1 and i, and the lattice velocities of the
// planes i-1, i and i+1.  Each new plane is loaded once, its p' and velocities evaluated once, and
// the flux through the x face between planes i and i+1 (scalars and the three momentum components)
// is computed once and carried in registers to the next plane, where it is the x face on the other
// side.  Compared with a three-dimensional tile this removes the halo re-evaluation in x and half of
// the x-face work.
//
// Every value is formed by the same expression, with the same operands in the same order, as in the
// tiled kernel's regular path (stage_point with REG), so the results are bitwise the same as those of
// every other tile shape; only points at or above their column's band top are written (the band
// points are the band-point launch's).
#pragma clang fp contract(off)

#include "cc_kernels.hpp"
#include "cc_stream.hpp"

namespace cc {

// element at a 32-bit byte offset from a workgroup-uniform base (scalar base + vector offset form)
template <typename T>
__device__ __forceinline__ T ld_at(const T *base, unsigned boff)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void st_at(T *base, unsigned boff, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff) = v;
}

// NBAR: barriers per plane.  2: rings of 4 cell planes and 3 lattice planes, the new plane's cells
// stored, a barrier, its velocities, a barrier, then the update.  1: rings of 5 and 4 planes, the cells
// of plane s+2 stored, one barrier, then the velocities of plane s+2 and the update of plane s (a
// plane's velocities are formed one step before they are read).
// The streaming update of one workgroup: logical block lb of a grid with nby x nbz (j, k) tiles per
// chunk of CH planes (k tile fastest, then j tile, then chunk).
template <typename T, int TY, int TZ, int CH, int NBAR>
__device__ __forceinline__ void stream_body(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &qs,
                                            const SIn<T> &qn, const SOut<T> &qo, double cdt, int final_stage,
                                            int nby, int nbz, int lb, int64_t *st)
{
    using R = typename Compute<T>::R;
    constexpr int NT = TY * TZ;
    // cell planes of rho': rows j0-2 .. j0+TY, columns k0-2 .. k0+TZ
    constexpr int CW = TZ + 3, CR = TY + 3, NC = CR * CW;
    // (rho theta)' and lattice velocities: rows j0-1 .. j0+TY, columns k0-1 .. k0+TZ
    constexpr int HW = TZ + 2, HR = TY + 2, NH = HR * HW;
    // p': rows j0-1 .. j0+TY-1, columns k0-1 .. k0+TZ-1
    constexpr int PW = TZ + 1, NPP = (TY + 1) * PW;
    constexpr int NB = TZ + 4;  // staged base levels k0-2 .. k0+TZ+1
    constexpr int IC = (NC + NT - 1) / NT, IH = (NH + NT - 1) / NT;
    constexpr int RC = NBAR == 1 ? 5 : 4, RV = NBAR == 1 ? 4 : 3;  // ring slots: cell planes, lattice planes
    // one spare element at the end of each box takes the stores of staging entries outside it, so that
    // the stores need no per-lane conditions
    __shared__ R s_rho[RC][NC + 1], s_rth[RC][NH + 1], s_pp[RC][NPP + 1];
    __shared__ R s_u[RV][NH + 1], s_v[RV][NH + 1], s_w[RV][NH + 1];
    __shared__ R s_b[6][NB];

    const int nx = d.nx, ny = d.ny, nz = d.nz, nzs = d.nzs;
    const unsigned ncol = (unsigned)(nx * ny);
    const unsigned pstride = (unsigned)ny * (unsigned)nzs;  // elements per x plane
    // every global access below is the array's base plus a 32-bit byte offset (the launchers take this
    // form only for grids whose arrays stay below 4 GiB), so that no per-plane 64-bit addresses are formed
    const unsigned pbytes = pstride * (unsigned)sizeof(T);
    const R Ux = (R)P.ux, Vy = (R)P.vy;

    // this workgroup's chunk, j-tile and k-tile
    const int kt = lb % nbz, jt = (lb / nbz) % nby, ct = lb / (nbz * nby);
    const int i_s = ct * CH, i_e = min(i_s + CH, nx);
    const int j0 = jt * TY, k0 = kt * TZ;
    const int tid = threadIdx.x;
    const int tz = tid % TZ, ty = tid / TZ;
    const int j = j0 + ty, k = k0 + tz;
    const bool inside = j < ny && k < nz;

    // ---- per-thread staging descriptors (the same for every plane) ----
    // cell elements: offset within an x plane, LDS slots of rho' / (rho theta)' / p' (-1: not in the box)
    unsigned c_off[IC];
    int c_rth[IC], c_pp[IC], c_lev[IC];
    bool c_ok[IC];
#pragma unroll
    for (int it = 0; it < IC; ++it) {
        const int e = tid + it * NT;
        const int r = e / CW, cc = e - r * CW;
        const int jj = wrap(j0 - 2 + r, ny), kk = k0 - 2 + cc;
        c_ok[it] = e < NC && kk >= 0 && kk < nz;
        c_off[it] = c_ok[it] ? ((unsigned)jj * (unsigned)nzs + (unsigned)kk) * (unsigned)sizeof(T) : 0u;
        c_lev[it] = cc;  // staged base level of the cell
        const bool in_h = e < NC && r >= 1 && r <= TY + 2 && cc >= 1 && cc <= TZ + 2;
        c_rth[it] = in_h ? (r - 1) * HW + (cc - 1) : NH;
        const bool in_p = e < NC && r >= 1 && r <= TY + 1 && cc >= 1 && cc <= TZ + 1;
        c_pp[it] = in_p ? (r - 1) * PW + (cc - 1) : NPP;
    }
    // lattice elements: offset of the (clamped) lattice level within a plane, column index within a
    // plane, rho' slot of the cell (J-1, Kc-1) in the cell box, lid flag
    unsigned l_off[IH], l_col[IH];
    int l_rho[IH], l_kc[IH];
    bool l_ok[IH], l_lid[IH];
#pragma unroll
    for (int it = 0; it < IH; ++it) {
        const int e = tid + it * NT;
        const int rv = e / HW, cv = e - rv * HW;
        const int JJ = wrap(j0 - 1 + rv, ny), K = k0 - 1 + cv;
        l_ok[it] = e < NH && K >= 0 && K <= nz;
        const int Kc = K < nz ? K : nz - 1;  // the rigid lid copies the level below
        l_lid[it] = K == nz;
        l_kc[it] = Kc;
        l_col[it] = (unsigned)JJ * (unsigned)sizeof(int);
        l_off[it] = l_ok[it] ? ((unsigned)JJ * (unsigned)nzs + (unsigned)Kc) * (unsigned)sizeof(T) : 0u;
        l_rho[it] = rv * CW + (Kc - k0 + 1);  // cell (J-1, Kc-1) of the rho' box
    }

    // ---- base profiles in the compute precision ----
    for (int e = tid; e < 6 * NB; e += NT) {
        int pr = e / NB, kk = k0 - 2 + (e - pr * NB);
        kk = kk < 0 ? 0 : (kk >= nz ? nz - 1 : kk);
        double v;
        switch (pr) {
        case 0: v = P.rhob[kk]; break;
        case 1: v = P.rthb[kk]; break;
        case 2: v = P.pb[kk]; break;
        case 3: v = P.irthb[kk]; break;
        case 4: v = P.rhobc[kk]; break;
        default: v = kk > 0 ? 0.5 * (P.rthb[kk - 1] + P.rthb[kk]) : P.rthb[0]; break;
        }
        s_b[pr][e - pr * NB] = (R)v;
    }

    // ---- plane loads (registers) and their LDS stores ----
    R p_rho[IC], p_rth[IC], p_m0[IH], p_m1[IH], p_m2[IH];
    int p_kb[IH];
    auto load_plane = [&](int ip) {
        const unsigned ib = (unsigned)wrap(ip, nx);
        const unsigned pb = ib * pbytes;
#pragma unroll
        for (int it = 0; it < IC; ++it) {
            const unsigned o = pb + c_off[it];
            p_rho[it] = c_ok[it] ? (R)ld_at(qs.rho, o) : (R)0;
            p_rth[it] = c_ok[it] ? (R)ld_at(qs.rth, o) : (R)0;
        }
        const unsigned kbo = (ncol + ib * (unsigned)ny) * (unsigned)sizeof(int);
#pragma unroll
        for (int it = 0; it < IH; ++it) {
            const unsigned o = pb + l_off[it];
            p_m0[it] = l_ok[it] ? (R)ld_at(qs.mu, o) : (R)0;
            p_m1[it] = l_ok[it] ? (R)ld_at(qs.mv, o) : (R)0;
            p_m2[it] = l_ok[it] ? (R)ld_at(qs.mw, o) : (R)0;
            p_kb[it] = l_ok[it] ? ld_at(G.colk, kbo + l_col[it]) : 0;
        }
    };
    // rho', (rho theta)' and p' of the loaded plane into ring slot sl
    auto store_cells = [&](int sl) {
#pragma unroll
        for (int it = 0; it < IC; ++it) {
            const int e = tid + it * NT;
            s_rho[sl][e < NC ? e : NC] = p_rho[it];
            s_rth[sl][c_rth[it]] = p_rth[it];
            R pp = (R)0;  // zero outside the grid in k
            if (c_ok[it]) pp = eos_staged<R>(p_rth[it], s_b[3][c_lev[it]], s_b[2][c_lev[it]], P);
            s_pp[sl][c_pp[it]] = pp;
        }
    };
    // velocities of lattice plane ip (cells of the old plane ring slot so and the new one sn) into
    // velocity slot sv; the momentum of the plane is in the load registers
    auto store_vel = [&](int ip, int so, int sn, int sv) {
        const unsigned base = (unsigned)wrap(ip, nx) * pstride;  // vcls holds one byte per cell
#pragma unroll
        for (int it = 0; it < IH; ++it) {
            const int e = tid + it * NT;
            R u0 = (R)0, u1 = (R)0, u2 = (R)0;
            if (l_ok[it]) {
                const int Kc = l_kc[it];
                const bool pred = Kc >= p_kb[it] || ld_at(G.vcls, base + l_off[it] / (unsigned)sizeof(T)) == CC_PRED;
                if (pred) {
                    const R *ro = s_rho[so] + l_rho[it], *rn = s_rho[sn] + l_rho[it];
                    R sm = ((ro[0] + rn[0]) + (ro[CW] + rn[CW])) + ((ro[1] + rn[1]) + (ro[CW + 1] + rn[CW + 1]));
                    R rpc = sm * (R)0.125;
                    R ri = recip(s_b[4][Kc - k0 + 2] + rpc);
                    u0 = fmaR(-rpc, Ux, p_m0[it]) * ri;
                    u1 = fmaR(-rpc, Vy, p_m1[it]) * ri;
                    u2 = p_m2[it] * ri;
                } else {
                    u0 = p_m0[it];
                    u1 = p_m1[it];
                    u2 = p_m2[it];
                }
                if (l_lid[it]) u2 = (R)0;
            }
            const int eh = e < NH ? e : NH;
            s_u[sv][eh] = u0;
            s_v[sv][eh] = u1;
            s_w[sv][eh] = u2;
        }
    };

    // ring slots of cell plane p and lattice plane p (p >= i_s - 2); inside the loop the slots advance
    // by one per plane
    auto cslot = [&](int p) { return (p - i_s + 2 * RC) % RC; };
    auto vslot = [&](int p) { return (p - i_s + 2 * RV) % RV; };
    auto cnext = [](int x) { return x + 1 == RC ? 0 : x + 1; };
    auto vnext = [](int x) { return x + 1 == RV ? 0 : x + 1; };
    // ---- prologue: cell planes i_s-2 .. i_s (i_s+1 with one barrier per plane), their lattice planes
    // from i_s-1, and the loads of the next plane in flight ----
    load_plane(i_s - 2);
    __syncthreads();  // base profiles staged
    store_cells(cslot(i_s - 2));
    constexpr int PRO = NBAR == 1 ? 1 : 0;  // the last plane stored before the loop: i_s + PRO
    for (int p = i_s - 1; p <= i_s + PRO; ++p) {
        load_plane(p);
        store_cells(cslot(p));
        __syncthreads();
        store_vel(p, cslot(p - 1), cslot(p), vslot(p));
    }
    load_plane(i_s + PRO + 1);  // in flight through the first plane

    // offsets of this thread's point in the boxes
    const int oc = (ty + 2) * CW + (tz + 2);  // cell (j, k) in the rho' box
    const int oh = (ty + 1) * HW + (tz + 1);  // cell (j, k) in the (rho theta)' box; lattice (j, k)
    const int op = ty * PW + tz;              // cell (j-1, k-1) in the p' box
    const int kb = tz + 2;                    // base level k
    const R ASx = (R)(0.25 * 1.0 * (d.dy * d.dz)), ASy = (R)(0.25 * 1.0 * (d.dz * d.dx));
    const R ASz = (R)(0.25 * 1.0 * (d.dx * d.dy));
    const R UASx = (R)(P.ux * 1.0 * (d.dy * d.dz)), UASy = (R)(P.vy * 1.0 * (d.dz * d.dx));
    const R h = (R)0.5, q4 = (R)0.25;
    const R ix = (R)P.idx, iy = (R)P.idy, iz = (R)P.idz;
    // x-face fluxes carried from the previous plane: scalars (rho', (rho theta)') and momentum
    R cm0 = (R)0, cm1 = (R)0, cmx[3] = {(R)0, (R)0, (R)0};
    int c_first = cslot(i_s - 1), v_first = vslot(i_s - 1);  // slots of plane s-1

    for (int s = i_s; s < i_e; ++s) {
        const int sm1 = c_first, s0 = cnext(sm1), sp1 = cnext(s0), sp2 = cnext(sp1);
        const int vm1 = v_first, v0 = vnext(vm1), vp1 = vnext(v0), vp2 = vnext(vp1);
        c_first = s0;
        v_first = v0;
        // q_n at this thread's point of plane s and its column's band tops: loaded first, so that they
        // arrive while the rings are filled
        const int i = s;  // s < i_e <= nx
        // byte offset of this thread's point (i, j, k)
        const unsigned c = (unsigned)i * pbytes + (j * (unsigned)nzs + (unsigned)k) * (unsigned)sizeof(T);
        T n_rho = (T)0, n_rth = (T)0, n_rlo = (T)0, n_tlo = (T)0, n_mu = (T)0, n_mv = (T)0, n_mw = (T)0;
        int kcell = 0, klat = 0;
        if (inside) {
            const unsigned co = ((unsigned)i * (unsigned)ny + (unsigned)j) * (unsigned)sizeof(int);
            kcell = ld_at(G.colk, co);
            klat = ld_at(G.colk, co + ncol * (unsigned)sizeof(int));
            n_rho = ld_at(qn.rho, c);
            n_rth = ld_at(qn.rth, c);
            if (final_stage && qo.rho_lo && qn.rho_lo) {
                n_rlo = ld_at(qn.rho_lo, c);
                n_tlo = ld_at(qn.rth_lo, c);
            }
            n_mu = ld_at(qn.mu, c);
            n_mv = ld_at(qn.mv, c);
            n_mw = ld_at(qn.mw, c);
        }
        if constexpr (NBAR == 2) {
            // the loaded plane s+1 into the rings, a barrier, its lattice velocities, a barrier
            store_cells(sp1);
            __syncthreads();
            store_vel(s + 1, s0, sp1, vp1);
            __syncthreads();
            // the next plane's loads go out, then the update of plane s
            if (s + 2 <= i_e) load_plane(s + 2);
        } else {
            // the loaded plane s+2 into the rings, a barrier, its lattice velocities (read from the next
            // step on), the loads of plane s+3, then the update of plane s
            if (s + 2 <= i_e) store_cells(sp2);
            __syncthreads();
            if (s + 2 <= i_e) store_vel(s + 2, sp1, sp2, vp2);
            if (s + 3 <= i_e) load_plane(s + 3);
        }
        const bool mine = inside && k >= band_top(kcell, klat);
        const bool first = s == i_s;
        // ---- scalars ----
        const R *rm = s_rho[sm1] + oc, *r0p = s_rho[s0] + oc, *rp = s_rho[sp1] + oc;
        const R *tm = s_rth[sm1] + oh, *t0 = s_rth[s0] + oh, *tp = s_rth[sp1] + oh;
        const R *um = s_u[vm1] + oh, *u0p = s_u[v0] + oh, *upp = s_u[vp1] + oh;
        const R *vm = s_v[vm1] + oh, *v0p = s_v[v0] + oh, *vpp = s_v[vp1] + oh;
        const R *wm = s_w[vm1] + oh, *w0p = s_w[v0] + oh, *wpp = s_w[vp1] + oh;
        const R rc0 = r0p[0], rc1 = t0[0];
        const R b0 = s_b[0][kb], b1 = s_b[1][kb];
        R fm0 = cm0, fm1 = cm1, fp0, fp1;
        double r0, r1;
        {  // x faces: the -x face is the previous plane's +x face
            if (first) {
                R sm = (u0p[0] + u0p[HW]) + (u0p[1] + u0p[HW + 1]);
                scalar_face_flux<R>(sm, ASx, UASx, b0, b1, rm[0], rc0, tm[0], rc1, fm0, fm1);
            }
            R sp = (upp[0] + upp[HW]) + (upp[1] + upp[HW + 1]);
            scalar_face_flux<R>(sp, ASx, UASx, b0, b1, rc0, rp[0], rc1, tp[0], fp0, fp1);
            r0 = (double)fp0 - (double)fm0;
            r1 = (double)fp1 - (double)fm1;
            cm0 = fp0;
            cm1 = fp1;
        }
        {  // y faces
            R fa0, fa1, fb0, fb1;
            R sm = (v0p[0] + vpp[0]) + (v0p[1] + vpp[1]);
            R sp = (v0p[HW] + vpp[HW]) + (v0p[HW + 1] + vpp[HW + 1]);
            scalar_face_flux<R>(sm, ASy, UASy, b0, b1, r0p[-CW], rc0, t0[-HW], rc1, fa0, fa1);
            scalar_face_flux<R>(sp, ASy, UASy, b0, b1, rc0, r0p[CW], rc1, t0[HW], fb0, fb1);
            r0 += (double)fb0 - (double)fa0;
            r1 += (double)fb1 - (double)fa1;
        }
        {  // z faces (the ground closes the bottom of k = 0, the rigid lid the top of nz-1)
            R fa0, fa1;
            if (k > 0) {
                R sm = (w0p[0] + wpp[0]) + (w0p[HW] + wpp[HW]);
                scalar_face_flux<R>(sm, ASz, (R)0, s_b[4][kb], s_b[5][kb], r0p[-1], rc0, t0[-1], rc1, fa0, fa1);
                r0 -= (double)fa0;
                r1 -= (double)fa1;
            }
            if (k + 1 < nz) {
                R sp = (w0p[1] + wpp[1]) + (w0p[HW + 1] + wpp[HW + 1]);
                scalar_face_flux<R>(sp, ASz, (R)0, s_b[4][kb + 1], s_b[5][kb + 1], rc0, r0p[1], rc1, t0[1], fa0, fa1);
                r0 += (double)fa0;
                r1 += (double)fa1;
            }
        }
        const double L0 = -r0 * P.idV, L1 = -r1 * P.idV;

        // ---- momentum at the lattice point (every lattice point above the ground row is predicted) ----
        R u[7][3];
        u[0][0] = u0p[0]; u[0][1] = v0p[0]; u[0][2] = w0p[0];
        u[1][0] = um[0]; u[1][1] = vm[0]; u[1][2] = wm[0];
        u[2][0] = upp[0]; u[2][1] = vpp[0]; u[2][2] = wpp[0];
        u[3][0] = u0p[-HW]; u[3][1] = v0p[-HW]; u[3][2] = w0p[-HW];
        u[4][0] = u0p[HW]; u[4][1] = v0p[HW]; u[4][2] = w0p[HW];
        u[5][0] = u0p[-1]; u[5][1] = v0p[-1]; u[5][2] = w0p[-1];
        u[6][0] = u0p[1]; u[6][1] = v0p[1]; u[6][2] = w0p[1];
        R rq[8], pq[8];  // bit0: i-1/i, bit1: j-1/j, bit2: k-1/k
        {
            const R *ra = s_rho[sm1] + oc - CW - 1, *rb = s_rho[s0] + oc - CW - 1;
            const R *pa = s_pp[sm1] + op, *pb = s_pp[s0] + op;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int o = ((b >> 1) & 1) * CW + (b >> 2);
                const int q = ((b >> 1) & 1) * PW + (b >> 2);
                rq[b] = (b & 1) ? rb[o] : ra[o];
                pq[b] = (b & 1) ? pb[q] : pa[q];
            }
        }
        const R rxp = q4 * ((rq[1] + rq[3]) + (rq[5] + rq[7]));
        const R rym = q4 * ((rq[0] + rq[1]) + (rq[4] + rq[5])), ryp = q4 * ((rq[2] + rq[3]) + (rq[6] + rq[7]));
        const R rzm = q4 * ((rq[0] + rq[1]) + (rq[2] + rq[3])), rzp = q4 * ((rq[4] + rq[5]) + (rq[6] + rq[7]));
        const R pgx = (((pq[1] + pq[3]) + (pq[5] + pq[7])) - ((pq[0] + pq[2]) + (pq[4] + pq[6]))) * (q4 * ix);
        const R pgy = (((pq[2] + pq[3]) + (pq[6] + pq[7])) - ((pq[0] + pq[1]) + (pq[4] + pq[5]))) * (q4 * iy);
        const R pgz = (((pq[4] + pq[5]) + (pq[6] + pq[7])) - ((pq[0] + pq[1]) + (pq[2] + pq[3]))) * (q4 * iz);
        const R r8 = (R)0.125 * (((rq[0] + rq[1]) + (rq[2] + rq[3])) + ((rq[4] + rq[5]) + (rq[6] + rq[7])));
        const R rbc = s_b[4][kb];
        const R rbzm = s_b[0][kb - 1], rbzp = s_b[0][kb];
        const R uxp = h * (u[0][0] + u[2][0]);
        const R vyp = h * (u[0][1] + u[4][1]), vym = h * (u[3][1] + u[0][1]);
        const R wzp = h * (u[0][2] + u[6][2]), wzm = h * (u[5][2] + u[0][2]);
        const R Czp = (rbzp + rzp) * wzp, Czm = (rbzm + rzm) * wzm;
        R Lm[3];
        if (first) {  // the -x face of the first plane of the chunk
            const R rxm = q4 * ((rq[0] + rq[2]) + (rq[4] + rq[6]));
            const R uxm = h * (u[1][0] + u[0][0]);
            if constexpr (sizeof(T) == 4) {
                const R Axf = rbc * Ux, Bxm = fmaR(rxm, Ux + uxm, rbc * uxm);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const R M0 = c == 0 ? Ux : (c == 1 ? Vy : (R)0);
                    const R mb = h * (u[1][c] + u[0][c]);
                    cmx[c] = fmaR(Axf, mb, Bxm * (M0 + mb));
                }
            } else {
                const R Bxm = (rbc + rxm) * uxm;
#pragma unroll
                for (int c = 0; c < 3; ++c) cmx[c] = Bxm * (h * (u[1][c] + u[0][c]));
            }
        }
        if constexpr (sizeof(T) == 4) {  // perturbation form
            const R Axf = rbc * Ux, Ayf = rbc * Vy;
            const R Bxp = fmaR(rxp, Ux + uxp, rbc * uxp);
            const R Byp = fmaR(ryp, Vy + vyp, rbc * vyp), Bym = fmaR(rym, Vy + vym, rbc * vym);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R M0 = c == 0 ? Ux : (c == 1 ? Vy : (R)0);
                R mb;
                mb = h * (u[0][c] + u[2][c]);
                const R fxp = fmaR(Axf, mb, Bxp * (M0 + mb));
                const R fxm = cmx[c];
                mb = h * (u[0][c] + u[4][c]);
                const R fyp = fmaR(Ayf, mb, Byp * (M0 + mb));
                mb = h * (u[3][c] + u[0][c]);
                const R fym = fmaR(Ayf, mb, Bym * (M0 + mb));
                mb = h * (u[0][c] + u[6][c]);
                const R fzp = Czp * (M0 + mb);
                mb = h * (u[5][c] + u[0][c]);
                const R fzm = Czm * (M0 + mb);
                const R adv = fmaR(fzp - fzm, iz, fmaR(fyp - fym, iy, (fxp - fxm) * ix));
                const R src = c == 0 ? pgx : (c == 1 ? pgy : fmaR((R)P.g, r8, pgz));
                Lm[c] = -(adv + src);
                cmx[c] = fxp;
            }
        } else {  // paper variables
            const R Bxp = (rbc + rxp) * uxp;
            const R Byp = (rbc + ryp) * vyp, Bym = (rbc + rym) * vym;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R fxp = Bxp * (h * (u[0][c] + u[2][c])), fxm = cmx[c];
                const R fyp = Byp * (h * (u[0][c] + u[4][c])), fym = Bym * (h * (u[3][c] + u[0][c]));
                const R fzp = Czp * (h * (u[0][c] + u[6][c])), fzm = Czm * (h * (u[5][c] + u[0][c]));
                const R adv = fmaR(fzp - fzm, iz, fmaR(fyp - fym, iy, (fxp - fxm) * ix));
                const R src = c == 0 ? pgx : (c == 1 ? pgy : fmaR((R)P.g, r8, pgz));
                Lm[c] = -(adv + src);
                cmx[c] = fxp;
            }
        }

        // ---- the stage update of cell (i,j,k) and lattice point (i,j,k) ----
        if (mine) {
            bool bad;
            {
                double x0 = (double)n_rho, x1 = (double)n_rth;
                if (final_stage && qo.rho_lo) {
                    x0 += (double)n_rlo;
                    x1 += (double)n_tlo;
                }
                x0 = fmaR(cdt, L0, x0);
                x1 = fmaR(cdt, L1, x1);
                const T a = (T)x0, bb = (T)x1;
                bad = !isfinite(a) || !isfinite(bb);
                st_at(qo.rho, c, a);
                st_at(qo.rth, c, bb);
                if (final_stage && qo.rho_lo) {
                    st_at(qo.rho_lo, c, (T)(x0 - (double)a));
                    st_at(qo.rth_lo, c, (T)(x1 - (double)bb));
                }
            }
            if (k >= 1) {
                const R cd = (R)cdt;
                const T a = (T)fmaR(cd, Lm[0], (R)n_mu);
                const T bb = (T)fmaR(cd, Lm[1], (R)n_mv);
                const T e = (T)fmaR(cd, Lm[2], (R)n_mw);
                bad = bad || !isfinite(a) || !isfinite(bb) || !isfinite(e);
                st_at(qo.mu, c, a);
                st_at(qo.mv, c, bb);
                st_at(qo.mw, c, e);
            }
            if (bad) count_status(st, ST_NONFINITE);
        }
    }
}

// one grid: workgroups dealt to the XCDs in contiguous ranges of logical blocks
template <typename T, int TY, int TZ, int CH, int MINW, int NBAR>
__global__ void __launch_bounds__(TY * TZ, MINW)
    k_stage_stream(Dims d, Geo G, Phy P, SIn<T> qs, SIn<T> qn, SOut<T> qo, double cdt, int final_stage, int nby,
                   int nbz, int64_t *st)
{
    const int b = blockIdx.x, n = gridDim.x;
    const int xcd = b & 7, idx = b >> 3, per = n >> 3, rem = n & 7;
    stream_body<T, TY, TZ, CH, NBAR>(d, G, P, qs, qn, qo, cdt, final_stage, nby, nbz,
                                     xcd * per + (xcd < rem ? xcd : rem) + idx, st);
}

// a batch of independent grids (ensemble members): the logical blocks of all members in one launch,
// XCD-aware over the whole batch; each workgroup finds its member by binary search over the members'
// first logical blocks (tile0r, counted in the streaming decomposition)
template <typename T, int TY, int TZ, int CH, int MINW, int NBAR>
__global__ void __launch_bounds__(TY * TZ, MINW)
    k_stage_stream_batch(const BlockDesc<T> *__restrict__ desc, int nblk, int ntiles, int rn, int rs, int ro,
                         double cdt, int final_stage, int64_t *st)
{
    const int b = blockIdx.x;
    const int xcd = b & 7, idx = b >> 3, per = ntiles >> 3, rem = ntiles & 7;
    const int lb = xcd * per + (xcd < rem ? xcd : rem) + idx;
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].tile0r <= lb) lo = mid;
        else hi = mid - 1;
    }
    const BlockDesc<T> &D = desc[lo];
    stream_body<T, TY, TZ, CH, NBAR>(D.d, D.G, D.P, as_in(D.q[rs]), as_in(D.q[rn]), D.q[ro], cdt, final_stage,
                                     D.nby, D.nbz, lb - D.tile0r, st);
}

// the streaming kernels address every array with 32-bit byte offsets
bool stream_offsets_fit(int nx, int ny, int nzs, int prec_bytes)
{
    return (uint64_t)nx * (uint64_t)ny * (uint64_t)nzs * (uint64_t)prec_bytes <= (uint64_t)UINT32_MAX;
}

// the number of workgroups of a launch over the grid
static inline unsigned stream_blocks(const Dims &d, int TY, int TZ, int CH)
{
    const unsigned nch = (d.nx + CH - 1) / CH, nby = (d.ny + TY - 1) / TY, nbz = (d.nz + TZ - 1) / TZ;
    return nch * nby * nbz;
}

// LDS bytes of the rings and base profiles of a streaming form
template <typename R, int TY, int TZ, int NBAR>
constexpr size_t stream_lds_bytes()
{
    constexpr size_t RC = NBAR == 1 ? 5 : 4, RV = NBAR == 1 ? 4 : 3;
    return sizeof(R) * (RC * ((size_t)(TY + 3) * (TZ + 3) + 1) + RC * ((size_t)(TY + 2) * (TZ + 2) + 1) +
                        RC * ((size_t)(TY + 1) * (TZ + 1) + 1) + 3 * RV * ((size_t)(TY + 2) * (TZ + 2) + 1) +
                        6 * (size_t)(TZ + 4));
}

template <typename T, int TY, int TZ, int CH, int MINW, int NBAR>
static bool launch_stream_t(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                            cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s)
{
    if constexpr (stream_lds_bytes<typename Compute<T>::R, TY, TZ, NBAR>() > 65536) {
        return false;
    } else {
        if (!stream_offsets_fit(d.nx, d.ny, d.nzs, (int)sizeof(T))) return false;
        const int nby = (d.ny + TY - 1) / TY, nbz = (d.nz + TZ - 1) / TZ;
        hipLaunchKernelGGL((k_stage_stream<T, TY, TZ, CH, MINW, NBAR>), dim3(stream_blocks(d, TY, TZ, CH)), dim3(TY * TZ), 0,
                           s, d, G, P, sin_of<T>(qs), sin_of<T>(qn), sout_of<T>(qo), cdt, final_stage, nby, nbz, st);
        return true;
    }
}

template <typename T>
bool launch_stream(int id, const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                   cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s)
{
    // float: registers capped for 4 waves per SIMD
    constexpr int W = sizeof(T) == 4 ? 4 : 1;
    switch (id) {
    case 21: return launch_stream_t<T, 8, 32, 32, W, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 22: return launch_stream_t<T, 8, 32, 32, W, 1>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 23: return launch_stream_t<T, 8, 16, 32, W, 1>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 24: return launch_stream_t<T, 8, 32, 64, W, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 25: return launch_stream_t<T, 8, 32, 64, W, 1>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 26: return launch_stream_t<T, 8, 16, 32, W, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 27: return launch_stream_t<T, 16, 16, 32, W, 1>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 28: return launch_stream_t<T, 16, 16, 32, W, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    case 29: return launch_stream_t<T, 16, 32, 32, W, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
    default: return false;
    }
}

bool stream_shape(int id, int prec_bytes, int &TY, int &TZ, int &CH)
{
    int ty, tz, ch;
    switch (id) {
    case 21: case 22: ty = 8; tz = 32; ch = 32; break;
    case 23: case 26: ty = 8; tz = 16; ch = 32; break;
    case 24: case 25: ty = 8; tz = 32; ch = 64; break;
    case 27: case 28: ty = 16; tz = 16; ch = 32; break;
    case 29: ty = 16; tz = 32; ch = 32; break;
    default: return false;
    }
    const int nbar = (id == 22 || id == 23 || id == 25 || id == 27) ? 1 : 2;
    const size_t RC = nbar == 1 ? 5 : 4, RV = nbar == 1 ? 4 : 3;
    const size_t lds = (size_t)prec_bytes * (RC * ((ty + 3) * (tz + 3) + 1) + RC * ((ty + 2) * (tz + 2) + 1) +
                                             RC * ((ty + 1) * (tz + 1) + 1) + 3 * RV * ((ty + 2) * (tz + 2) + 1) +
                                             6 * (tz + 4));
    if (lds > 65536) return false;
    TY = ty; TZ = tz; CH = ch;
    return true;
}

template <typename T, int TY, int TZ, int CH, int MINW, int NBAR>
static void launch_stream_batch_t(const void *desc, int nblk, int ntiles, int rn, int rs, int ro, double cdt,
                                  int final_stage, int64_t *st, hipStream_t s)
{
    if constexpr (stream_lds_bytes<typename Compute<T>::R, TY, TZ, NBAR>() <= 65536)
        hipLaunchKernelGGL((k_stage_stream_batch<T, TY, TZ, CH, MINW, NBAR>), dim3(ntiles), dim3(TY * TZ), 0, s,
                           (const BlockDesc<T> *)desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st);
}

template <typename T>
void launch_stream_batch(int id, const void *desc, int nblk, int ntiles, int rn, int rs, int ro, double cdt,
                         int final_stage, int64_t *st, hipStream_t s)
{
    constexpr int W = sizeof(T) == 4 ? 4 : 1;
    switch (id) {
    case 21: launch_stream_batch_t<T, 8, 32, 32, W, 2>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 22: launch_stream_batch_t<T, 8, 32, 32, W, 1>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 23: launch_stream_batch_t<T, 8, 16, 32, W, 1>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 24: launch_stream_batch_t<T, 8, 32, 64, W, 2>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 25: launch_stream_batch_t<T, 8, 32, 64, W, 1>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 26: launch_stream_batch_t<T, 8, 16, 32, W, 2>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 27: launch_stream_batch_t<T, 16, 16, 32, W, 1>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 28: launch_stream_batch_t<T, 16, 16, 32, W, 2>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    case 29: launch_stream_batch_t<T, 16, 32, 32, W, 2>(desc, nblk, ntiles, rn, rs, ro, cdt, final_stage, st, s); break;
    default: break;
    }
}

template void launch_stream_batch<float>(int, const void *, int, int, int, int, int, double, int, int64_t *,
                                         hipStream_t);
template void launch_stream_batch<double>(int, const void *, int, int, int, int, int, double, int, int64_t *,
                                          hipStream_t);

template bool launch_stream<float>(int, const Dims &, const Geo &, const Phy &, const cc_state *, const cc_state *,
                                   cc_state *, double, int, int64_t *, hipStream_t);
template bool launch_stream<double>(int, const Dims &, const Geo &, const Phy &, const cc_state *, const cc_state *,
                                    cc_state *, double, int, int64_t *, hipStream_t);

}  // namespace cc
