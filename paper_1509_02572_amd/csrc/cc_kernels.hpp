// Device code of the cut-cell stage shared by the uniform-grid and the batched entry points:
// state views, the equation of state, face fluxes, the tiled update kernel (single grid and
// batched blocks) and the velocity diagnostics.  Host helpers at the end turn the C-ABI structs
// into kernel views.
//
// Precision forms
//   double : the paper's variables; reference velocity (ux, vy) = 0.
//   float  : perturbation form.  Momentum is stored as m' = rho u - rhobar_c(K) (ux, vy, 0) and
//            diagnosed velocities as u - (ux, vy, 0).  Fluxes are split into the part carried by
//            the base state and the uniform reference flow, which is evaluated in double (it is a
//            static quantity that cancels exactly on regular cells), and the perturbation part,
//            evaluated in float (momentum fluxes also accumulated in float; the few scalar face
//            fluxes of a cell are summed in double so that their cancellation between neighbours
//            is exact).  Base state, group volumes and global sums stay double.
//
// Floating-point expressions are evaluated as written (no FMA contraction): a face flux is then
// bitwise the same whichever of its two cells, and whichever code path, evaluates it, so the flux
// divergence telescopes exactly and mass is conserved to rounding of the per-cell sums.
#pragma once
#pragma clang fp contract(off)

#include "cc_internal.hpp"

namespace cc {


template <typename T>
struct SIn {
    const T *rho, *rth, *mu, *mv, *mw;
    const T *rho_lo, *rth_lo;  // low-order parts (float form, nullable)
};
template <typename T>
struct SOut {
    T *rho, *rth, *mu, *mv, *mw;
    T *rho_lo, *rth_lo;
};

struct Geo {
    const double *H, *V, *Ax, *Ay, *Az, *nrm, *Vgroup;
    const int8_t *cls, *vcls;
    const int32_t *master, *gnext, *colk;
    void *ws;   // optional stage workspace (band-tile list, two-pass update), may be null
    int kband;  // highest column band top: every point at k >= kband is regular (0: unknown)
    int nband;  // tiles in the band-tile list at the start of ws (-1: no list)
    cc_stage_ctx side;  // host only: stage context of the band-point launch (may be null)
};

constexpr int EOS_TERMS = 11;  // binomial series terms of (1+x)^gamma - 1 (double; float uses 6)
constexpr double EOS_XMAX = 0.03;  // |x| above which the exact form is used

struct Phy {
    const double *rhob, *rthb, *pb, *thb;  // base state at cell centres [nz]
    const double *irthb;                   // 1 / (rho theta)bar [nz]
    const double *rhobc;                   // mean base density of levels K-1, K at lattice level K [nz]
    double g, gam, ux, vy, dV, idV, idx, idy, idz;
    double u0, v0, kdh, kdv;               // inflow and diffusion rates (always the caller's values)
    double zsp, rsp, ztop;                 // sponge: bottom height, rate at the lid, lid height
    double binom[EOS_TERMS];               // (1+x)^gamma - 1 = sum_n binom[n-1] x^n
    float binomf[EOS_TERMS];
};

template <typename T>
struct Compute;
template <>
struct Compute<double> {
    using R = double;
};
template <>
struct Compute<float> {
    using R = float;
};

__device__ __forceinline__ double expm1_r(double x) { return expm1(x); }
__device__ __forceinline__ float expm1_r(float x) { return expm1f(x); }
__device__ __forceinline__ double log1p_r(double x) { return log1p(x); }
__device__ __forceinline__ float log1p_r(float x) { return log1pf(x); }

// p' from (rho theta)' through the ideal-gas equation of state (Sec. 2.1):
// p = p0 (R rho theta / p0)^(cp/cv)  =>  p' = pbar ((1 + rth'/rthbar)^gamma - 1)
template <typename R>
__device__ __forceinline__ R eos_pprime(R rthp, double rthb, double pb, double gam)
{
    return (R)pb * expm1_r((R)gam * log1p_r(rthp / (R)rthb));
}

// the same p' for cell level k, evaluated with the binomial series of (1+x)^gamma when
// |x| = |rth'/rthbar| <= EOS_XMAX (truncation below the storage precision: 6 terms in float, 11 in
// double), otherwise with the exact form
template <typename R>
__device__ __forceinline__ R eos_pprime_k(R rthp, int k, const Phy &P)
{
    R x = rthp * (R)P.irthb[k];
    R ax = x < (R)0 ? -x : x;
    if (ax > (R)EOS_XMAX) return (R)P.pb[k] * expm1_r((R)P.gam * log1p_r(x));
    constexpr int NTERM = sizeof(R) == 4 ? 6 : EOS_TERMS;
    R acc = (R)P.binom[NTERM - 1];
#pragma unroll
    for (int n = NTERM - 2; n >= 0; --n) acc = (R)P.binom[n] + x * acc;
    return (R)P.pb[k] * (x * acc);
}

// reciprocal used for velocities: hardware reciprocal in float (deterministic, 1 ulp), IEEE in double
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

__device__ __forceinline__ int wrap1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Fluxes of rho' and (rho theta)' (perturbation part) through one face.  Every code path calls
// this with the same operands, so both cells of a face obtain bitwise the same value.
//   s4   sum of the four corner normal velocities, ((a + b) + (c + d)) in canonical corner order
//   AS4  aperture x area / 4, UAS = reference normal velocity x aperture x area
//   b0,b1 base values on the face, lo*/up* perturbations of the lower / upper exchanging group
// flux = bar (un A S) + (lo + up)/2 ((un + Un) A S) with un = s4 / 4.
template <typename R>
__device__ __forceinline__ void scalar_face_flux(R s4, R AS4, R UAS, R b0, R b1, R lo0, R up0, R lo1,
                                                 R up1, R &f0, R &f1)
{
    R unS = s4 * AS4;
    R htS = (R)0.5 * fmaR(s4, AS4, UAS);
    f0 = fmaR(b0, unS, (lo0 + up0) * htS);
    f1 = fmaR(b1, unS, (lo1 + up1) * htS);
}

// Velocity of a predicted lattice point (1 <= K <= nz-1): momentum over the mean of the eight
// surrounding cell densities, as in lat_vel
template <typename T, typename R = typename Compute<T>::R>
__device__ __forceinline__ void lat_vel_pred(const Dims &d, const Phy &P, const SIn<T> &q, int I, int J, int K, R u[3])
{
    int64_t p = cidx(d, I, J, K);
    int64_t c00 = cidx(d, I - 1, J - 1, K - 1), c10 = cidx(d, I, J - 1, K - 1);
    int64_t c01 = cidx(d, I - 1, J, K - 1), c11 = cidx(d, I, J, K - 1);
    R s = (((R)q.rho[c00] + (R)q.rho[c10]) + ((R)q.rho[c01] + (R)q.rho[c11])) +
          (((R)q.rho[c00 + 1] + (R)q.rho[c10 + 1]) + ((R)q.rho[c01 + 1] + (R)q.rho[c11 + 1]));
    R rpc = s * (R)0.125;
    R ri = recip((R)P.rhobc[K] + rpc);
    u[0] = fmaR(-rpc, (R)P.ux, (R)q.mu[p]) * ri;
    u[1] = fmaR(-rpc, (R)P.vy, (R)q.mv[p]) * ri;
    u[2] = (R)q.mw[p] * ri;
}

// Velocity (perturbation from the reference flow) at lattice point (I,J,K).
// Predicted points divide the momentum by the mean of the eight surrounding cell densities;
// diagnosed points store the velocity; the rigid lid (K = nz) has w = 0 and copies (u, v) of the
// level below.
template <typename T, typename R = typename Compute<T>::R>
__device__ __forceinline__ void lat_vel(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &q,
                                        int I, int J, int K, R u[3])
{
    bool lid = K >= d.nz;
    if (lid) K = d.nz - 1;
    int64_t p = cidx(d, I, J, K);
    if (G.vcls[p] == CC_PRED) {
        int64_t c00 = cidx(d, I - 1, J - 1, K - 1), c10 = cidx(d, I, J - 1, K - 1);
        int64_t c01 = cidx(d, I - 1, J, K - 1), c11 = cidx(d, I, J, K - 1);
        R s = (((R)q.rho[c00] + (R)q.rho[c10]) + ((R)q.rho[c01] + (R)q.rho[c11])) +
              (((R)q.rho[c00 + 1] + (R)q.rho[c10 + 1]) + ((R)q.rho[c01 + 1] + (R)q.rho[c11 + 1]));
        R rpc = s * (R)0.125;
        R ri = recip((R)P.rhobc[K] + rpc);
        u[0] = fmaR(-rpc, (R)P.ux, (R)q.mu[p]) * ri;
        u[1] = fmaR(-rpc, (R)P.vy, (R)q.mv[p]) * ri;
        u[2] = (R)q.mw[p] * ri;
    } else {
        u[0] = (R)q.mu[p];
        u[1] = (R)q.mv[p];
        u[2] = (R)q.mw[p];
    }
    if (lid) u[2] = (R)0;
}

// ------------------------------------------------------------------------------------------------
// Scalar tendency of a merged group (Sec. 2.4): the surface integral over every external face of
// every member (a face split among several neighbours contributes one sub-face per neighbour, with
// its own aperture), face scalar = mean of the two exchanging groups, face normal velocity = mean
// of the four corner velocities (eqs. ux1-ux3), zero flux through closed faces (terrain, ground,
// rigid lid).  Returns d(rho')/dt and d(rho theta)'/dt of master c.
// ------------------------------------------------------------------------------------------------
// Offset b - a on a periodic axis of n points, in (-n/2, n/2].
__device__ __forceinline__ int periodic_offset(int b, int a, int n)
{
    int r = b - a;
    if (2 * r > n) r -= n;
    else if (2 * r <= -n) r += n;
    return r;
}

// The master (i,j,k) = c reads the staged neighbourhood V where a member's corner or neighbour lies in
// it (the staged values are the ones lat_vel and the state hold) and global memory elsewhere.  The
// apertures and neighbour masters of a member's six faces are read together.
template <typename T, typename VW, typename R = typename Compute<T>::R>
__device__ void group_scalar_tendency(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &q, int64_t c,
                                      const VW &V, int i, int j, int k, double L[2])
{
    double rb0 = 0.0, rb1 = 0.0;  // base-state / reference-flow part
    // perturbation part: each face flux is evaluated in R; the per-group sum of those fluxes is
    // formed in double, where a sum of a few floats is exact, so a face contributes exactly
    // opposite amounts to its two groups and mass is conserved to FP64 rounding
    double rp0 = 0.0, rp1 = 0.0;
    const int kc = k;
    const R rc0 = V.rho[V.C(0, 0, 0)], rc1 = V.rth[V.Ct(0, 0, 0)];
    // normal velocity component ax of lattice point (I,J,K)
    auto vel = [&](int I, int J, int K, int ax) -> R {
        const int di = periodic_offset(I, i, d.nx), dj = periodic_offset(J, j, d.ny), dk = K - k;
        if (V.has_lat(di, dj, dk)) {
            const int e = V.Lg(di, dj, dk);
            return ax == 0 ? V.u[e] : (ax == 1 ? V.v[e] : V.w[e]);
        }
        R u[3];
        lat_vel<T>(d, G, P, q, I, J, K, u);
        return u[ax];
    };
    int64_t mem = c;
    for (int guard = 0; mem >= 0 && guard <= CC_MAX_GROUP; ++guard) {
        int mi, mj, mk;
        unidx(d, mem, mi, mj, mk);
        double Af[6];
        int32_t mnf[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int axis = f >> 1, plus = f & 1;
            const int dc = axis == 2 ? (plus ? 1 : -1) : 0;
            Af[f] = 0.0;
            mnf[f] = -1;
            if (axis == 2 && (mk + dc < 0 || mk + dc >= d.nz)) continue;  // ground and rigid lid
            const int fi = mi + (axis == 0 && plus), fj = mj + (axis == 1 && plus), fk = mk + (axis == 2 && plus);
            const int64_t fu = cidx(d, fi, fj, fk);
            Af[f] = axis == 0 ? G.Ax[fu] : (axis == 1 ? G.Ay[fu] : G.Az[fu]);
            const int ni = mi + (axis == 0 ? (plus ? 1 : -1) : 0), nj = mj + (axis == 1 ? (plus ? 1 : -1) : 0);
            mnf[f] = G.master[cidx(d, ni, nj, mk + dc)];
        }
        const int64_t next = G.gnext[mem];
        for (int f = 0; f < 6; ++f) {
            const int axis = f >> 1, plus = f & 1;
            const double A = Af[f];
            if (A == 0.0) continue;
            const int32_t mn = mnf[f];
            if (mn == (int32_t)c || mn < 0) continue;  // internal face of the group
            const int fi = mi + (axis == 0 && plus), fj = mj + (axis == 1 && plus), fk = mk + (axis == 2 && plus);
            R s4;
            double S, Un;
            if (axis == 0) {
                s4 = (vel(fi, fj, fk, 0) + vel(fi, fj + 1, fk, 0)) + (vel(fi, fj, fk + 1, 0) + vel(fi, fj + 1, fk + 1, 0));
                S = d.dy * d.dz; Un = P.ux;
            } else if (axis == 1) {
                s4 = (vel(fi, fj, fk, 1) + vel(fi + 1, fj, fk, 1)) + (vel(fi, fj, fk + 1, 1) + vel(fi + 1, fj, fk + 1, 1));
                S = d.dz * d.dx; Un = P.vy;
            } else {
                s4 = (vel(fi, fj, fk, 2) + vel(fi + 1, fj, fk, 2)) + (vel(fi, fj + 1, fk, 2) + vel(fi + 1, fj + 1, fk, 2));
                S = d.dx * d.dy; Un = 0.0;
            }
            // scalars of the neighbouring master
            int ni, nj, nk;
            unidx(d, mn, ni, nj, nk);
            const int ei = periodic_offset(ni, i, d.nx), ej = periodic_offset(nj, j, d.ny), ek = nk - k;
            R rn0, rn1;
            rn0 = V.has_cell(ei, ej, ek) ? V.rho[V.Cg(ei, ej, ek)] : (R)q.rho[mn];
            rn1 = V.has_rth(ei, ej, ek) ? V.rth[V.Ct(ei, ej, ek)] : (R)q.rth[mn];
            const int klo = plus ? kc : nk, kup = plus ? nk : kc;
            double pb0 = 0.5 * (P.rhob[klo] + P.rhob[kup]);
            double pb1 = 0.5 * (P.rthb[klo] + P.rthb[kup]);
            R f0, f1;
            if (plus)
                scalar_face_flux<R>(s4, (R)(0.25 * A * S), (R)(Un * A * S), (R)pb0, (R)pb1, rc0, rn0, rc1, rn1, f0, f1);
            else
                scalar_face_flux<R>(s4, (R)(0.25 * A * S), (R)(Un * A * S), (R)pb0, (R)pb1, rn0, rc0, rn1, rc1, f0, f1);
            double g0 = pb0 * Un * A * S, g1 = pb1 * Un * A * S;
            if (plus) { rp0 += (double)f0; rp1 += (double)f1; rb0 += g0; rb1 += g1; }
            else { rp0 -= (double)f0; rp1 -= (double)f1; rb0 -= g0; rb1 -= g1; }
        }
        mem = next;
    }
    double vol = G.Vgroup[c] * P.dV;
    L[0] = -(rb0 + rp0) / vol;
    L[1] = -(rb1 + rp1) / vol;
}

// ------------------------------------------------------------------------------------------------
// Tiled update kernel.  A block owns TX x TY columns x TZ levels.  It stages rho', (rho theta)' and
// p' of the cells around the tile, and the velocities of the lattice points around it, in LDS once,
// then every thread updates one cell (scalars) and one lattice point (momentum).  Above the
// per-column bands (colk) cells and lattice points are regular and no geometry or class array is
// read; inside the bands single-cell groups read their apertures, group volume and neighbour
// masters, and masters of multi-cell groups take the general gather path.
// ------------------------------------------------------------------------------------------------
template <int TX, int TY, int TZ>
struct Tile {
    static constexpr int NT = TX * TY * TZ;
    static constexpr int CX = TX + 3, CY = TY + 3, CZ = TZ + 3, NC = CX * CY * CZ;  // cells from (i0-2, j0-2, k0-2)
    static constexpr int LX = TX + 2, LY = TY + 2, LZ = TZ + 2, NL = LX * LY * LZ;  // lattice from (i0-1, j0-1, k0-1)
    // (rho theta)' is read one cell around the tile, p' at the cells i0-1.. i0+TX-1 (and so in y, z)
    static constexpr int RX = TX + 2, RY = TY + 2, RZ = TZ + 2, NR = RX * RY * RZ;  // from (i0-1, j0-1, k0-1)
    static constexpr int PX = TX + 1, PY = TY + 1, PZ = TZ + 1, NP = PX * PY * PZ;  // from (i0-1, j0-1, k0-1)
    __device__ static constexpr int cs(int a, int b, int c) { return (a * CY + b) * CZ + c; }
    __device__ static constexpr int ls(int a, int b, int c) { return (a * LY + b) * LZ + c; }
    __device__ static constexpr int rs(int a, int b, int c) { return (a * RY + b) * RZ + c; }
    __device__ static constexpr int ps(int a, int b, int c) { return (a * PY + b) * PZ + c; }
};

// Tile lb of an nbx x nby x nbz grid of tiles: the tiles run through strips of SJ tile columns in j,
// and inside a strip k fastest, then j, then i, so a tile's neighbours in i and j follow it within a
// few strip rows, while their halos are still in L2.
// tile_of_block: the tile of this block with an XCD-aware order: blocks are dealt round-robin to the
// 8 XCDs, so each XCD is given a contiguous range of tiles and shares halos in its own L2.
__device__ __forceinline__ void strip_tile(int lb, int nbx, int nby, int nbz, int &bi, int &bj, int &bk)
{
    constexpr int SJ = 4;
    const int nfull = nby / SJ, full = nfull * SJ * nbx * nbz;
    int s, w, r;
    if (lb < full) {
        s = lb / (SJ * nbx * nbz);
        r = lb - s * (SJ * nbx * nbz);
        w = SJ;
    } else {  // the last, narrower strip
        s = nfull;
        r = lb - full;
        w = nby - nfull * SJ;
    }
    bk = r % nbz;
    r /= nbz;
    bj = s * SJ + r % w;
    bi = r / w;
}

__device__ __forceinline__ void tile_of_block(int nbx, int nby, int nbz, int &bi, int &bj, int &bk)
{
    const int nb = nbx * nby * nbz;
    const int b = blockIdx.x;
    const int xcd = b & 7, idx = b >> 3, per = nb >> 3, rem = nb & 7;
    strip_tile(xcd * per + (xcd < rem ? xcd : rem) + idx, nbx, nby, nbz, bi, bj, bk);
}

// p' of a cell from its (rho theta)' with base values staged in the compute precision: binomial
// series of (1+x)^gamma when |x| <= EOS_XMAX, exact form otherwise
template <typename R>
__device__ __forceinline__ R eos_staged(R rthp, R irthb, R pb, const Phy &P)
{
    R x = rthp * irthb;
    R ax = x < (R)0 ? -x : x;
    if (ax > (R)EOS_XMAX) return pb * expm1_r((R)P.gam * log1p_r(x));
    constexpr int NTERM = sizeof(R) == 4 ? 6 : EOS_TERMS;
    R acc = sizeof(R) == 4 ? (R)P.binomf[NTERM - 1] : (R)P.binom[NTERM - 1];
#pragma unroll
    for (int n = NTERM - 2; n >= 0; --n) acc = fmaR(x, acc, sizeof(R) == 4 ? (R)P.binomf[n] : (R)P.binom[n]);
    return pb * (x * acc);
}

// LDS view of the staged neighbourhood of one output point (i,j,k): cells at (i+di, j+dj, k+dk)
// and lattice points at (i+di, j+dj, k+dk) for di in {-1,0,1}, addressed through the index of the
// i-1 / i / i+1 plane entry plus dj * stride + dk; staged base profiles b[6][nb] at level kb.
template <typename R>
struct LView {
    const R *rho, *rth, *pp, *u, *v, *w, *b;
    int cb[3], lb[3];
    int csj, lsj, nb, kb;
    // the point's position in the tile (lattice box from (i0-1, j0-1, k0-1), cell box from
    // (i0-2, j0-2, k0-2)) and the boxes' extents and x strides, for reads at any offset
    int px, py, pz, lx, ly, lz, cx, cy, cz, lsi, csi;
    // (rho theta)' box (cells one around the tile) and p' box: index of the point's own cell, strides
    int rb, rsi, rsj, rx, ry, rz, pb, psi, psj;
    __device__ __forceinline__ int C(int di, int dj, int dk) const { return cb[di + 1] + dj * csj + dk; }
    __device__ __forceinline__ int Ct(int di, int dj, int dk) const { return rb + di * rsi + dj * rsj + dk; }
    __device__ __forceinline__ int Pp(int di, int dj, int dk) const { return pb + di * psi + dj * psj + dk; }
    __device__ __forceinline__ bool has_rth(int di, int dj, int dk) const
    {
        const int a = px + 1 + di, b_ = py + 1 + dj, c = pz + 1 + dk;
        return a >= 0 && a < rx && b_ >= 0 && b_ < ry && c >= 0 && c < rz;
    }
    __device__ __forceinline__ int L(int di, int dj, int dk) const { return lb[di + 1] + dj * lsj + dk; }
    __device__ __forceinline__ R B(int prof, int dk) const { return b[prof * nb + kb + dk]; }
    __device__ __forceinline__ bool has_lat(int di, int dj, int dk) const
    {
        const int a = px + 1 + di, b_ = py + 1 + dj, c = pz + 1 + dk;
        return a >= 0 && a < lx && b_ >= 0 && b_ < ly && c >= 0 && c < lz;
    }
    __device__ __forceinline__ int Lg(int di, int dj, int dk) const { return lb[1] + di * lsi + dj * lsj + dk; }
    __device__ __forceinline__ bool has_cell(int di, int dj, int dk) const
    {
        const int a = px + 2 + di, b_ = py + 2 + dj, c = pz + 2 + dk;
        return a >= 0 && a < cx && b_ >= 0 && b_ < cy && c >= 0 && c < cz;
    }
    __device__ __forceinline__ int Cg(int di, int dj, int dk) const { return cb[1] + di * csi + dj * csj + dk; }
};

// The same neighbourhood read from global memory: q_s scalars, and p' and lattice velocities from
// the prepare pass (p' at cells with the cells' stride, velocities at lattice levels 0..nz with a
// stride of nzs + 16 so that the lid row is stored); base profiles converted on the fly exactly as
// they are staged.
template <typename R>
struct GView {
    const R *rho, *rth, *pp, *u, *v, *w;
    const double *rhob, *rthb, *pb, *irthb, *rhobc;
    int cb[3], cj[3], lb[3], lj[3];
    int k, nz;
    __device__ __forceinline__ int C(int di, int dj, int dk) const { return cb[di + 1] + cj[dj + 1] + dk; }
    __device__ __forceinline__ int L(int di, int dj, int dk) const { return lb[di + 1] + lj[dj + 1] + dk; }
    __device__ __forceinline__ int Ct(int di, int dj, int dk) const { return C(di, dj, dk); }
    __device__ __forceinline__ int Pp(int di, int dj, int dk) const { return C(di, dj, dk); }
    __device__ __forceinline__ bool has_rth(int, int, int) const { return false; }
    // reads beyond the immediate neighbours go to the state and lat_vel
    __device__ __forceinline__ bool has_lat(int, int, int) const { return false; }
    __device__ __forceinline__ int Lg(int, int, int) const { return 0; }
    __device__ __forceinline__ bool has_cell(int, int, int) const { return false; }
    __device__ __forceinline__ int Cg(int, int, int) const { return 0; }
    __device__ __forceinline__ R B(int prof, int dk) const
    {
        int kk = k + dk;
        kk = kk < 0 ? 0 : (kk >= nz ? nz - 1 : kk);
        double v;
        switch (prof) {
        case 0: v = rhob[kk]; break;
        case 1: v = rthb[kk]; break;
        case 2: v = pb[kk]; break;
        case 3: v = irthb[kk]; break;
        case 4: v = rhobc[kk]; break;
        default: v = kk > 0 ? 0.5 * (rthb[kk - 1] + rthb[kk]) : rthb[0]; break;
        }
        return (R)v;
    }
};

// Update (MODE 0) or tendency (MODE 1) of cell (i,j,k) and lattice point (i,j,k) from the staged
// neighbourhood.  Above the per-column bands cells and lattice points are regular and no geometry
// or class array is read; inside the bands single-cell groups read their apertures, group volume
// and neighbour masters, and masters of multi-cell groups take the general gather path.
// values of q_n at the output point and its column thresholds, loaded ahead of the staging phases
template <typename T>
struct PointIn {
    T rho, rth, rho_lo, rth_lo, mu, mv, mw;
    int kcell, klat;
};

template <typename T, int MODE>
__device__ __forceinline__ void load_point(const Dims &d, const Geo &G, const SIn<T> &qn, int i, int j, int k,
                                           int final_stage, PointIn<T> &pi)
{
    const unsigned hc = __umul24(i, d.ny) + j;
    const unsigned c = __umul24(hc, d.nzs) + k;
    pi.kcell = G.colk[hc];
    pi.klat = G.colk[(unsigned)(d.nx * d.ny) + hc];
    if (MODE == 0) {
        pi.rho = qn.rho[c]; pi.rth = qn.rth[c];
        pi.mu = qn.mu[c]; pi.mv = qn.mv[c]; pi.mw = qn.mw[c];
        if (final_stage && qn.rho_lo) { pi.rho_lo = qn.rho_lo[c]; pi.rth_lo = qn.rth_lo[c]; }
        else { pi.rho_lo = (T)0; pi.rth_lo = (T)0; }
    }
}

// REG: the point lies at or above the band height (regular cell, predicted lattice point), so the
// band and gather paths are not compiled in
template <typename T, int MODE, typename VW, bool REG = false>
__device__ __forceinline__ void stage_point(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &qs,
                                            const PointIn<T> &pin, const SOut<T> &qo, double cdt, int final_stage,
                                            int i, int j, int k, const VW &V,
                                            int64_t *st, bool ghost)
{
    using R = typename Compute<T>::R;
    const int nx = d.nx, ny = d.ny, nz = d.nz, nzs = d.nzs;
    const R Ux = (R)P.ux, Vy = (R)P.vy;
    const unsigned hc = __umul24(i, ny) + j;
    const unsigned c = __umul24(hc, nzs) + k;
    bool bad = false;

    // ---- scalars ----
    const bool band = !REG && k < pin.kcell;
    const int8_t cl = band ? G.cls[c] : (int8_t)CC_OPEN;
    if (cl == CC_OPEN || cl == CC_ORPHAN) {
        double L0, L1;
        const R rc0 = V.rho[V.C(0, 0, 0)], rc1 = V.rth[V.Ct(0, 0, 0)];
        if (!band) {
            // regular cell: V = 1, open faces, neighbours at their own level; the base-state and
            // reference-flow fluxes of opposite faces cancel exactly
            const R ASx = (R)(0.25 * 1.0 * (d.dy * d.dz)), ASy = (R)(0.25 * 1.0 * (d.dz * d.dx));
            const R ASz = (R)(0.25 * 1.0 * (d.dx * d.dy));
            const R UASx = (R)(P.ux * 1.0 * (d.dy * d.dz)), UASy = (R)(P.vy * 1.0 * (d.dz * d.dx));
            const R b0 = V.B(0, 0), b1 = V.B(1, 0);
            R fm0, fm1, fp0, fp1;
            double r0, r1;
            {  // x faces
                R sm = (V.u[V.L(0, 0, 0)] + V.u[V.L(0, 1, 0)]) + (V.u[V.L(0, 0, 1)] + V.u[V.L(0, 1, 1)]);
                R sp = (V.u[V.L(1, 0, 0)] + V.u[V.L(1, 1, 0)]) + (V.u[V.L(1, 0, 1)] + V.u[V.L(1, 1, 1)]);
                scalar_face_flux<R>(sm, ASx, UASx, b0, b1, V.rho[V.C(-1, 0, 0)], rc0, V.rth[V.Ct(-1, 0, 0)], rc1, fm0, fm1);
                scalar_face_flux<R>(sp, ASx, UASx, b0, b1, rc0, V.rho[V.C(1, 0, 0)], rc1, V.rth[V.Ct(1, 0, 0)], fp0, fp1);
                r0 = (double)fp0 - (double)fm0;
                r1 = (double)fp1 - (double)fm1;
            }
            {  // y faces
                R sm = (V.v[V.L(0, 0, 0)] + V.v[V.L(1, 0, 0)]) + (V.v[V.L(0, 0, 1)] + V.v[V.L(1, 0, 1)]);
                R sp = (V.v[V.L(0, 1, 0)] + V.v[V.L(1, 1, 0)]) + (V.v[V.L(0, 1, 1)] + V.v[V.L(1, 1, 1)]);
                scalar_face_flux<R>(sm, ASy, UASy, b0, b1, V.rho[V.C(0, -1, 0)], rc0, V.rth[V.Ct(0, -1, 0)], rc1, fm0, fm1);
                scalar_face_flux<R>(sp, ASy, UASy, b0, b1, rc0, V.rho[V.C(0, 1, 0)], rc1, V.rth[V.Ct(0, 1, 0)], fp0, fp1);
                r0 += (double)fp0 - (double)fm0;
                r1 += (double)fp1 - (double)fm1;
            }
            {  // z faces (the ground closes the bottom of k = 0, the rigid lid the top of nz-1)
                if (k > 0) {
                    R sm = (V.w[V.L(0, 0, 0)] + V.w[V.L(1, 0, 0)]) + (V.w[V.L(0, 1, 0)] + V.w[V.L(1, 1, 0)]);
                    scalar_face_flux<R>(sm, ASz, (R)0, V.B(4, 0), V.B(5, 0), V.rho[V.C(0, 0, -1)], rc0,
                                        V.rth[V.Ct(0, 0, -1)], rc1, fm0, fm1);
                    r0 -= (double)fm0;
                    r1 -= (double)fm1;
                }
                if (k + 1 < nz) {
                    R sp = (V.w[V.L(0, 0, 1)] + V.w[V.L(1, 0, 1)]) + (V.w[V.L(0, 1, 1)] + V.w[V.L(1, 1, 1)]);
                    scalar_face_flux<R>(sp, ASz, (R)0, V.B(4, 1), V.B(5, 1), rc0, V.rho[V.C(0, 0, 1)], rc1,
                                        V.rth[V.Ct(0, 0, 1)], fp0, fp1);
                    r0 += (double)fp0;
                    r1 += (double)fp1;
                }
            }
            L0 = -r0 * P.idV;
            L1 = -r1 * P.idV;
        } else if (G.gnext[c] != -1) {  // master of a multi-cell group: general gather
            double L[2];
            group_scalar_tendency<T>(d, G, P, qs, c, V, i, j, k, L);
            L0 = L[0]; L1 = L[1];
        } else {
            // single-cell group in the band: apertures, group volume and neighbour masters.  The
            // apertures and neighbour masters of the six faces are read together first.
            double Af[6];
            int32_t mnf[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                int axis = f >> 1, plus = f & 1;
                int da = axis == 0 ? (plus ? 1 : -1) : 0, db = axis == 1 ? (plus ? 1 : -1) : 0;
                int dc = axis == 2 ? (plus ? 1 : -1) : 0;
                Af[f] = 0.0;
                mnf[f] = -1;
                if (axis == 2 && (k + dc < 0 || k + dc >= nz)) continue;  // ground and rigid lid
                int ip = wrap1(i + (axis == 0 && plus), nx), jp = wrap1(j + (axis == 1 && plus), ny);
                unsigned fu = __umul24(__umul24(ip, ny) + jp, nzs) + k + (axis == 2 && plus);
                Af[f] = axis == 0 ? G.Ax[fu] : (axis == 1 ? G.Ay[fu] : G.Az[fu]);
                int in = wrap1(i + da, nx), jn = wrap1(j + db, ny);
                mnf[f] = G.master[__umul24(__umul24(in, ny) + jn, nzs) + k + dc];
            }
            const double vgroup = G.Vgroup[c];
            double r0 = 0.0, r1 = 0.0, g0 = 0.0, g1 = 0.0;
            for (int f = 0; f < 6; ++f) {
                int axis = f >> 1, plus = f & 1;
                int da = 0, db = 0, dc = 0;
                if (axis == 0) da = plus ? 1 : -1;
                else if (axis == 1) db = plus ? 1 : -1;
                else dc = plus ? 1 : -1;
                const double A = Af[f];
                if (A == 0.0) continue;  // closed face (terrain, solid neighbour, ground, lid)
                const int32_t mn = mnf[f];
                if (mn < 0) continue;
                int kn = mn % nzs;
                int fa = axis == 0 && plus, fb = axis == 1 && plus, fc = axis == 2 && plus;
                R s4;
                double S, Un;
                if (axis == 0) {
                    s4 = (V.u[V.L(fa, fb, fc)] + V.u[V.L(fa, fb + 1, fc)]) + (V.u[V.L(fa, fb, fc + 1)] + V.u[V.L(fa, fb + 1, fc + 1)]);
                    S = d.dy * d.dz; Un = P.ux;
                } else if (axis == 1) {
                    s4 = (V.v[V.L(fa, fb, fc)] + V.v[V.L(fa + 1, fb, fc)]) + (V.v[V.L(fa, fb, fc + 1)] + V.v[V.L(fa + 1, fb, fc + 1)]);
                    S = d.dz * d.dx; Un = P.vy;
                } else {
                    s4 = (V.w[V.L(fa, fb, fc)] + V.w[V.L(fa + 1, fb, fc)]) + (V.w[V.L(fa, fb + 1, fc)] + V.w[V.L(fa + 1, fb + 1, fc)]);
                    S = d.dx * d.dy; Un = 0.0;
                }
                const R rn0 = V.rho[V.C(da, db, dc)], rn1 = V.rth[V.Ct(da, db, dc)];
                int klo = plus ? k : kn, kup = plus ? kn : k;
                double pb0 = 0.5 * (P.rhob[klo] + P.rhob[kup]);
                double pb1 = 0.5 * (P.rthb[klo] + P.rthb[kup]);
                R f0, f1;
                if (plus)
                    scalar_face_flux<R>(s4, (R)(0.25 * A * S), (R)(Un * A * S), (R)pb0, (R)pb1, rc0, rn0, rc1, rn1, f0, f1);
                else
                    scalar_face_flux<R>(s4, (R)(0.25 * A * S), (R)(Un * A * S), (R)pb0, (R)pb1, rn0, rc0, rn1, rc1, f0, f1);
                double h0 = pb0 * Un * A * S, h1 = pb1 * Un * A * S;
                if (plus) { r0 += (double)f0; r1 += (double)f1; g0 += h0; g1 += h1; }
                else { r0 -= (double)f0; r1 -= (double)f1; g0 -= h0; g1 -= h1; }
            }
            double vol = vgroup * P.dV;
            L0 = -(g0 + r0) / vol;
            L1 = -(g1 + r1) / vol;
        }
        if (MODE == 0) {
            double x0 = (double)pin.rho, x1 = (double)pin.rth;
            if (final_stage && qo.rho_lo) { x0 += (double)pin.rho_lo; x1 += (double)pin.rth_lo; }
            x0 = fmaR(cdt, L0, x0);
            x1 = fmaR(cdt, L1, x1);
            T a = (T)x0, b = (T)x1;
            bad = !isfinite(a) || !isfinite(b);
            qo.rho[c] = a;
            qo.rth[c] = b;
            if (final_stage && qo.rho_lo) {
                qo.rho_lo[c] = (T)(x0 - (double)a);
                qo.rth_lo[c] = (T)(x1 - (double)b);
            }
        } else {
            qo.rho[c] = (T)L0;
            qo.rth[c] = (T)L1;
        }
    } else if (cl == CC_SOLID || MODE == 1) {
        qo.rho[c] = (T)0;
        qo.rth[c] = (T)0;
        if (MODE == 0 && final_stage && qo.rho_lo) { qo.rho_lo[c] = (T)0; qo.rth_lo[c] = (T)0; }
    }

    // ---- momentum at the lattice point (i,j,k) ----
    // (REG: every lattice point of the tile above the ground row is predicted)
    const bool pred = REG ? k >= 1 : (k >= pin.klat || G.vcls[c] == CC_PRED);
    if (pred) {
        const R h = (R)0.5, q4 = (R)0.25;
        R u[7][3];
        const int off[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            int e = V.L(off[s][0], off[s][1], off[s][2]);
            u[s][0] = V.u[e]; u[s][1] = V.v[e]; u[s][2] = V.w[e];
        }
        R rp[8], pp[8];  // bit0: i-1/i, bit1: j-1/j, bit2: k-1/k
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            rp[s] = V.rho[V.C((s & 1) - 1, ((s >> 1) & 1) - 1, (s >> 2) - 1)];
            pp[s] = V.pp[V.Pp((s & 1) - 1, ((s >> 1) & 1) - 1, (s >> 2) - 1)];
        }
        // density perturbation on the six faces of the velocity cell, pressure gradient, buoyancy
        const R rxm = q4 * ((rp[0] + rp[2]) + (rp[4] + rp[6])), rxp = q4 * ((rp[1] + rp[3]) + (rp[5] + rp[7]));
        const R rym = q4 * ((rp[0] + rp[1]) + (rp[4] + rp[5])), ryp = q4 * ((rp[2] + rp[3]) + (rp[6] + rp[7]));
        const R rzm = q4 * ((rp[0] + rp[1]) + (rp[2] + rp[3])), rzp = q4 * ((rp[4] + rp[5]) + (rp[6] + rp[7]));
        const R ix = (R)P.idx, iy = (R)P.idy, iz = (R)P.idz;
        const R pgx = (((pp[1] + pp[3]) + (pp[5] + pp[7])) - ((pp[0] + pp[2]) + (pp[4] + pp[6]))) * (q4 * ix);
        const R pgy = (((pp[2] + pp[3]) + (pp[6] + pp[7])) - ((pp[0] + pp[1]) + (pp[4] + pp[5]))) * (q4 * iy);
        const R pgz = (((pp[4] + pp[5]) + (pp[6] + pp[7])) - ((pp[0] + pp[1]) + (pp[2] + pp[3]))) * (q4 * iz);
        const R r8 = (R)0.125 * (((rp[0] + rp[1]) + (rp[2] + rp[3])) + ((rp[4] + rp[5]) + (rp[6] + rp[7])));
        const R rbc = V.B(4, 0);                         // base density on x and y faces
        const R rbzm = V.B(0, -1), rbzp = V.B(0, 0);     // base density on the z faces
        // Face flux of component m (perturbation form; the base product rbc U M0 cancels between
        // opposite faces):  F = rbc U mb + (rbc ub + r'(U + ub)) (M0 + mb) on x/y faces with
        // ub, mb the face means of the normal and m velocity perturbations; F = (rbz + r') wb (M0 + mb)
        // on z faces.  The factor in front of (M0 + mb) is shared by the three components.
        const R uxp = h * (u[0][0] + u[2][0]), uxm = h * (u[1][0] + u[0][0]);
        const R vyp = h * (u[0][1] + u[4][1]), vym = h * (u[3][1] + u[0][1]);
        const R wzp = h * (u[0][2] + u[6][2]), wzm = h * (u[5][2] + u[0][2]);
        const R Czp = (rbzp + rzp) * wzp, Czm = (rbzm + rzm) * wzm;
        R Lm[3];
        if constexpr (sizeof(T) == 4) {  // perturbation form
            const R Axf = rbc * Ux, Ayf = rbc * Vy;
            const R Bxp = fmaR(rxp, Ux + uxp, rbc * uxp), Bxm = fmaR(rxm, Ux + uxm, rbc * uxm);
            const R Byp = fmaR(ryp, Vy + vyp, rbc * vyp), Bym = fmaR(rym, Vy + vym, rbc * vym);
#pragma unroll
            for (int cm = 0; cm < 3; ++cm) {
                const R M0 = cm == 0 ? Ux : (cm == 1 ? Vy : (R)0);
                R mb;
                mb = h * (u[0][cm] + u[2][cm]);
                R fxp = fmaR(Axf, mb, Bxp * (M0 + mb));
                mb = h * (u[1][cm] + u[0][cm]);
                R fxm = fmaR(Axf, mb, Bxm * (M0 + mb));
                mb = h * (u[0][cm] + u[4][cm]);
                R fyp = fmaR(Ayf, mb, Byp * (M0 + mb));
                mb = h * (u[3][cm] + u[0][cm]);
                R fym = fmaR(Ayf, mb, Bym * (M0 + mb));
                mb = h * (u[0][cm] + u[6][cm]);
                R fzp = Czp * (M0 + mb);
                mb = h * (u[5][cm] + u[0][cm]);
                R fzm = Czm * (M0 + mb);
                R adv = fmaR(fzp - fzm, iz, fmaR(fyp - fym, iy, (fxp - fxm) * ix));
                R src = cm == 0 ? pgx : (cm == 1 ? pgy : fmaR((R)P.g, r8, pgz));
                Lm[cm] = -(adv + src);
            }
        } else {  // paper variables: F = (rbar + r') ub mb on every face
            const R Bxp = (rbc + rxp) * uxp, Bxm = (rbc + rxm) * uxm;
            const R Byp = (rbc + ryp) * vyp, Bym = (rbc + rym) * vym;
#pragma unroll
            for (int cm = 0; cm < 3; ++cm) {
                R fxp = Bxp * (h * (u[0][cm] + u[2][cm])), fxm = Bxm * (h * (u[1][cm] + u[0][cm]));
                R fyp = Byp * (h * (u[0][cm] + u[4][cm])), fym = Bym * (h * (u[3][cm] + u[0][cm]));
                R fzp = Czp * (h * (u[0][cm] + u[6][cm])), fzm = Czm * (h * (u[5][cm] + u[0][cm]));
                R adv = fmaR(fzp - fzm, iz, fmaR(fyp - fym, iy, (fxp - fxm) * ix));
                R src = cm == 0 ? pgx : (cm == 1 ? pgy : fmaR((R)P.g, r8, pgz));
                Lm[cm] = -(adv + src);
            }
        }
        if (MODE == 0) {
            const R cd = (R)cdt;
            T a = (T)fmaR(cd, Lm[0], (R)pin.mu);
            T b = (T)fmaR(cd, Lm[1], (R)pin.mv);
            T e = (T)fmaR(cd, Lm[2], (R)pin.mw);
            bad = bad || !isfinite(a) || !isfinite(b) || !isfinite(e);
            qo.mu[c] = a; qo.mv[c] = b; qo.mw[c] = e;
        } else {
            qo.mu[c] = (T)Lm[0]; qo.mv[c] = (T)Lm[1]; qo.mw[c] = (T)Lm[2];
        }
    } else if (MODE == 1) {
        qo.mu[c] = (T)0; qo.mv[c] = (T)0; qo.mw[c] = (T)0;
    }
    // ghost cells of a refined-grid block go stale between refills and are counted apart
    if (bad) count_status(st, ghost ? ST_STALE : ST_NONFINITE);
}

// the cells a grid owns (a block of a refined grid: its own cells; any other grid: all of it)
struct OwnRange { int lo[3], hi[3]; };

// TX x TY x TZ threads; each thread updates KP points spaced TZ apart in k, so the tile spans
// TX x TY x (TZ KP) cells
// REG: every point the tile updates takes the regular update
// SEL: 0 updates every point of the tile, 1 only the points at or above their column's band top, 2
// only the points below it
template <typename T, int TX, int TY, int TZ, int MODE, int KP = 1, bool REG = false, int SEL = 0>
__device__ __forceinline__ void tile_body(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &qs,
                                          const SIn<T> &qn, const SOut<T> &qo, double cdt, int final_stage,
                                          const int i0, const int j0, const int k0, int64_t *st, const OwnRange &ownr)
{
    using R = typename Compute<T>::R;
    using TL = Tile<TX, TY, TZ * KP>;
    constexpr int NT = TX * TY * TZ;
    constexpr int IT1 = (TL::NC + NT - 1) / NT, IT2 = (TL::NL + NT - 1) / NT;
    constexpr int NB = TZ * KP + 4;  // staged base levels k0-2 .. k0+TZ KP+1
    __shared__ R s_rho[TL::NC], s_rth[TL::NR], s_pp[TL::NP];
    __shared__ R s_u[TL::NL], s_v[TL::NL], s_w[TL::NL];
    // base profiles in the compute precision: rhobar, (rho theta)bar, pbar, 1/(rho theta)bar, and
    // the means of rhobar and (rho theta)bar over levels k-1, k (z faces / lattice level k)
    __shared__ R s_b[6][NB];
    const int tid = threadIdx.x;
    const int nx = d.nx, ny = d.ny, nz = d.nz, nzs = d.nzs;
    const unsigned ncol = (unsigned)(nx * ny);
    const R Ux = (R)P.ux, Vy = (R)P.vy;

    // the output points of this thread; their q_n values and column thresholds are loaded first
    const int tx = tid / (TY * TZ), ty = (tid / TZ) % TY, tz = tid % TZ;
    const int i = i0 + tx, j = j0 + ty;
    PointIn<T> pin[KP];
#pragma unroll
    for (int p = 0; p < KP; ++p)
        if (i < nx && j < ny && k0 + tz + p * TZ < nz)
            load_point<T, MODE>(d, G, qn, i, j, k0 + tz + p * TZ, final_stage, pin[p]);
    // tiles whose halo lies inside the grid in x, y and k need no periodic wrap and no range check
    const bool inner = i0 >= 2 && i0 + TX < nx && j0 >= 2 && j0 + TY < ny && k0 >= 2 && k0 + TZ * KP < nz;
    // ---- issue the global loads of the staging phases first ----
    R c_rho[IT1], c_rth[IT1];
    if (inner) {
        const unsigned tbase = __umul24(__umul24(i0 - 2, ny) + (j0 - 2), nzs) + (k0 - 2);
#pragma unroll
        for (int it = 0; it < IT1; ++it) {
            int e = tid + it * NT;
            c_rho[it] = (R)0;
            c_rth[it] = (R)0;
            if (e < TL::NC) {
                int a = e / (TL::CY * TL::CZ), r = e - a * (TL::CY * TL::CZ), b = r / TL::CZ, c = r - b * TL::CZ;
                unsigned ci = tbase + __umul24(__umul24(a, ny) + b, nzs) + c;
                c_rho[it] = (R)qs.rho[ci];
                c_rth[it] = (R)qs.rth[ci];
            }
        }
    } else {
#pragma unroll
        for (int it = 0; it < IT1; ++it) {
            int e = tid + it * NT;
            c_rho[it] = (R)0;
            c_rth[it] = (R)0;
            if (e < TL::NC) {
                int a = e / (TL::CY * TL::CZ), r = e - a * (TL::CY * TL::CZ), b = r / TL::CZ, c = r - b * TL::CZ;
                int k = k0 - 2 + c;
                if (k >= 0 && k < nz) {
                    unsigned col = __umul24(wrap1(i0 - 2 + a, nx), ny) + wrap1(j0 - 2 + b, ny);
                    unsigned ci = __umul24(col, nzs) + k;
                    c_rho[it] = (R)qs.rho[ci];
                    c_rth[it] = (R)qs.rth[ci];
                }
            }
        }
    }
    R l_m0[IT2], l_m1[IT2], l_m2[IT2];
    int l_kb[IT2];
    unsigned l_p[IT2];
    if (inner) {
        const unsigned tcol = __umul24(i0 - 1, ny) + (j0 - 1);
#pragma unroll
        for (int it = 0; it < IT2; ++it) {
            int e = tid + it * NT;
            l_m0[it] = l_m1[it] = l_m2[it] = (R)0;
            l_kb[it] = 0;
            l_p[it] = 0;
            if (e < TL::NL) {
                int a = e / (TL::LY * TL::LZ), r = e - a * (TL::LY * TL::LZ), b = r / TL::LZ, c = r - b * TL::LZ;
                unsigned col = tcol + __umul24(a, ny) + b;
                unsigned p = __umul24(col, nzs) + (k0 - 1 + c);
                l_p[it] = p;
                l_m0[it] = (R)qs.mu[p];
                l_m1[it] = (R)qs.mv[p];
                l_m2[it] = (R)qs.mw[p];
                l_kb[it] = G.colk[ncol + col];
            }
        }
    } else {
#pragma unroll
        for (int it = 0; it < IT2; ++it) {
            int e = tid + it * NT;
            l_m0[it] = l_m1[it] = l_m2[it] = (R)0;
            l_kb[it] = 0;
            l_p[it] = 0;
            if (e < TL::NL) {
                int a = e / (TL::LY * TL::LZ), r = e - a * (TL::LY * TL::LZ), b = r / TL::LZ, c = r - b * TL::LZ;
                int K = k0 - 1 + c;
                if (K >= 0 && K <= nz) {
                    int Kc = K < nz ? K : nz - 1;
                    unsigned col = __umul24(wrap1(i0 - 1 + a, nx), ny) + wrap1(j0 - 1 + b, ny);
                    unsigned p = __umul24(col, nzs) + Kc;
                    l_p[it] = p;
                    l_m0[it] = (R)qs.mu[p];
                    l_m1[it] = (R)qs.mv[p];
                    l_m2[it] = (R)qs.mw[p];
                    l_kb[it] = G.colk[ncol + col];
                }
            }
        }
    }
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
    __syncthreads();
    // ---- phase 1: cell scalars and p' (p' for the cells i0-1..i0+TX-1 x ... used by the momentum
    // stencils of the tile) ----
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
        int e = tid + it * NT;
        if (e < TL::NC) {
            int a = e / (TL::CY * TL::CZ), r = e - a * (TL::CY * TL::CZ), b = r / TL::CZ, c = r - b * TL::CZ;
            int k = k0 - 2 + c;
            s_rho[e] = c_rho[it];
            if (a >= 1 && a <= TX + 2 && b >= 1 && b <= TY + 2 && c >= 1 && c <= TZ * KP + 2)
                s_rth[TL::rs(a - 1, b - 1, c - 1)] = c_rth[it];
            if (a >= 1 && a <= TX + 1 && b >= 1 && b <= TY + 1 && c >= 1 && c <= TZ * KP + 1) {
                R pp = (R)0;
                if (k >= 0 && k < nz) pp = eos_staged<R>(c_rth[it], s_b[3][c], s_b[2][c], P);
                s_pp[TL::ps(a - 1, b - 1, c - 1)] = pp;
            }
        }
    }
    __syncthreads();
    // ---- phase 2: lattice velocities (perturbations from the reference flow) ----
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
        int e = tid + it * NT;
        if (e < TL::NL) {
            int a = e / (TL::LY * TL::LZ), r = e - a * (TL::LY * TL::LZ), b = r / TL::LZ, c = r - b * TL::LZ;
            int K = k0 - 1 + c;
            R u0 = (R)0, u1 = (R)0, u2 = (R)0;
            if (K >= 0 && K <= nz) {
                int Kc = K < nz ? K : nz - 1;  // the rigid lid copies the level below
                bool pred = Kc >= l_kb[it] || G.vcls[l_p[it]] == CC_PRED;
                if (pred) {
                    int cz = Kc - k0 + 1;  // LDS level of cell level Kc-1
                    R sm = ((s_rho[TL::cs(a, b, cz)] + s_rho[TL::cs(a + 1, b, cz)]) +
                            (s_rho[TL::cs(a, b + 1, cz)] + s_rho[TL::cs(a + 1, b + 1, cz)])) +
                           ((s_rho[TL::cs(a, b, cz + 1)] + s_rho[TL::cs(a + 1, b, cz + 1)]) +
                            (s_rho[TL::cs(a, b + 1, cz + 1)] + s_rho[TL::cs(a + 1, b + 1, cz + 1)]));
                    R rpc = sm * (R)0.125;
                    R ri = recip(s_b[4][Kc - k0 + 2] + rpc);
                    u0 = fmaR(-rpc, Ux, l_m0[it]) * ri;
                    u1 = fmaR(-rpc, Vy, l_m1[it]) * ri;
                    u2 = l_m2[it] * ri;
                } else {
                    u0 = l_m0[it];
                    u1 = l_m1[it];
                    u2 = l_m2[it];
                }
                if (K == nz) u2 = (R)0;
            }
            s_u[e] = u0;
            s_v[e] = u1;
            s_w[e] = u2;
        }
    }
    __syncthreads();

    // ---- phase 3: KP cells and lattice points per thread ----
#pragma unroll
    for (int p = 0; p < KP; ++p) {
        const int tzp = tz + p * TZ, k = k0 + tzp;
        bool mine = i < nx && j < ny && k < nz;
        if (SEL != 0 && mine) mine = (k >= band_top(pin[p].kcell, pin[p].klat)) == (SEL == 1);
        if (mine) {
            LView<R> V;
            V.rho = s_rho; V.rth = s_rth; V.pp = s_pp; V.u = s_u; V.v = s_v; V.w = s_w; V.b = &s_b[0][0];
            for (int m = 0; m < 3; ++m) {
                V.cb[m] = TL::cs(tx + 1 + m, ty + 2, tzp + 2);
                V.lb[m] = TL::ls(tx + m, ty + 1, tzp + 1);
            }
            V.csj = TL::CZ; V.lsj = TL::LZ; V.nb = NB; V.kb = tzp + 2;
            V.px = tx; V.py = ty; V.pz = tzp;
            V.lx = TL::LX; V.ly = TL::LY; V.lz = TL::LZ; V.cx = TL::CX; V.cy = TL::CY; V.cz = TL::CZ;
            V.lsi = TL::LY * TL::LZ; V.csi = TL::CY * TL::CZ;
            V.rb = TL::rs(tx + 1, ty + 1, tzp + 1); V.rsi = TL::RY * TL::RZ; V.rsj = TL::RZ;
            V.rx = TL::RX; V.ry = TL::RY; V.rz = TL::RZ;
            V.pb = TL::ps(tx + 1, ty + 1, tzp + 1); V.psi = TL::PY * TL::PZ; V.psj = TL::PZ;
            const bool ghost = i < ownr.lo[0] || i >= ownr.hi[0] || j < ownr.lo[1] || j >= ownr.hi[1] ||
                               k < ownr.lo[2] || k >= ownr.hi[2];
            stage_point<T, MODE, LView<R>, REG>(d, G, P, qs, pin[p], qo, cdt, final_stage, i, j, k, V, st, ghost);
        }
    }
}

// whether a tile holds a point below its column's band top (block-uniform; every thread calls it)
template <int TX, int TY, int TZ>
__device__ __forceinline__ bool band_tile_busy(const Dims &d, const Geo &G, int i0, int j0, int k0)
{
    const int t = threadIdx.x;
    const int i = i0 + t / (TY * TZ), j = j0 + (t / TZ) % TY, k = k0 + t % TZ;
    bool any = false;
    if (i < d.nx && j < d.ny && k < d.nz) {
        const unsigned hc = __umul24(i, d.ny) + j;
        any = k < band_top(G.colk[hc], G.colk[(unsigned)(d.nx * d.ny) + hc]);
    }
    return __syncthreads_or(any);
}

// the launch covers the k-tiles [bk0, bk0 + nbz); REG: every point the launch updates takes the
// regular update; SEL as in tile_body (SEL 2: a tile with no point below its column's band top ends
// at once)
template <typename T, int TX, int TY, int TZ, int MODE, int MINW, int KP = 1, bool REG = false, int SEL = 0>
__global__ void __launch_bounds__(TX * TY * TZ, MINW)
    k_stage_tiled(Dims d, Geo G, Phy P, SIn<T> qs, SIn<T> qn, SOut<T> qo, double cdt, int final_stage,
                  int nbx, int nby, int nbz, int bk0, int64_t *st)
{
    static_assert(SEL != 2 || KP == 1, "band tiles hold one point per thread");
    int bi, bj, bk;
    if (SEL == 2 && G.nband >= 0) {  // the listed band tiles (each holds band points), XCD-aware order
        const int b = blockIdx.x, n = G.nband;
        const int xcd = b & 7, idx = b >> 3, per = n >> 3, rem = n & 7;
        const int t = ((const int32_t *)G.ws)[xcd * per + (xcd < rem ? xcd : rem) + idx];
        if (t < 0 || t >= nbx * nby * nbz) return;  // not a tile of this grid (a stale list)
        const int r = t % (nbx * nby);
        bk = t / (nbx * nby);
        bi = r / nby;
        bj = r % nby;
    } else {
        tile_of_block(nbx, nby, nbz, bi, bj, bk);
    }
    const int k0 = (bk0 + bk) * TZ * KP;
    if (SEL == 2 && G.nband < 0 && !band_tile_busy<TX, TY, TZ>(d, G, bi * TX, bj * TY, k0)) return;
    const OwnRange all{{0, 0, 0}, {d.nx, d.ny, d.nz}};
    tile_body<T, TX, TY, TZ, MODE, KP, REG, SEL>(d, G, P, qs, qn, qo, cdt, final_stage, bi * TX, bj * TY, k0, st,
                                                 all);
}

// ------------------------------------------------------------------------------------------------
// Two-pass form.  Pass 1 evaluates p' at every cell and the velocity at every lattice point (the
// lid row included) once, into a workspace; pass 2 updates one point per thread, reading its
// neighbourhood through the caches.  Both passes use the staging arithmetic of the tiled kernel,
// so the results are bitwise the same.
// ------------------------------------------------------------------------------------------------
__host__ __device__ constexpr int lattice_stride(int nzs) { return nzs + 16; }

template <typename T>
__global__ void __launch_bounds__(256) k_prepare(Dims d, Geo G, Phy P, SIn<T> qs, typename Compute<T>::R *ws)
{
    using R = typename Compute<T>::R;
    const int nzl = lattice_stride(d.nzs);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncol = (int64_t)d.nx * d.ny;
    if (t >= ncol * nzl) return;
    const int K = (int)(t % nzl);
    const int64_t col = t / nzl;
    if (K > d.nz) return;
    const int I = (int)(col / d.ny), J = (int)(col % d.ny);
    const int nz = d.nz, nzs = d.nzs;
    R *pp = ws, *uu = ws + ncol * nzs, *vv = uu + ncol * nzl, *ww = vv + ncol * nzl;
    if (K < nz) {
        const int64_t c = col * nzs + K;
        pp[c] = eos_staged<R>((R)qs.rth[c], (R)P.irthb[K], (R)P.pb[K], P);
    }
    const int Kc = K < nz ? K : nz - 1;  // the rigid lid copies the level below
    const int64_t p = col * nzs + Kc;
    const R m0 = (R)qs.mu[p], m1 = (R)qs.mv[p], m2 = (R)qs.mw[p];
    R u0, u1, u2;
    const bool pred = Kc >= G.colk[ncol + col] || G.vcls[p] == CC_PRED;
    if (pred) {
        const int64_t c00 = cidx(d, I - 1, J - 1, Kc - 1), c10 = cidx(d, I, J - 1, Kc - 1);
        const int64_t c01 = cidx(d, I - 1, J, Kc - 1), c11 = cidx(d, I, J, Kc - 1);
        R sm = (((R)qs.rho[c00] + (R)qs.rho[c10]) + ((R)qs.rho[c01] + (R)qs.rho[c11])) +
               (((R)qs.rho[c00 + 1] + (R)qs.rho[c10 + 1]) + ((R)qs.rho[c01 + 1] + (R)qs.rho[c11 + 1]));
        R rpc = sm * (R)0.125;
        R ri = recip((R)P.rhobc[Kc] + rpc);
        u0 = fmaR(-rpc, (R)P.ux, m0) * ri;
        u1 = fmaR(-rpc, (R)P.vy, m1) * ri;
        u2 = m2 * ri;
    } else {
        u0 = m0; u1 = m1; u2 = m2;
    }
    if (K == nz) u2 = (R)0;
    const int64_t l = col * nzl + K;
    uu[l] = u0; vv[l] = u1; ww[l] = u2;
}

// one point (cell and lattice point) per thread, k fastest across the wave
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_stage_points(Dims d, Geo G, Phy P, SIn<T> qs, SIn<T> qn, SOut<T> qo,
                                                      const typename Compute<T>::R *ws, double cdt, int final_stage,
                                                      int64_t *st)
{
    using R = typename Compute<T>::R;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncol = (int64_t)d.nx * d.ny;
    if (t >= ncol * d.nz) return;
    const int k = (int)(t % d.nz);
    const int64_t col = t / d.nz;
    const int i = (int)(col / d.ny), j = (int)(col % d.ny);
    const int nzs = d.nzs, nzl = lattice_stride(nzs), ny = d.ny;
    PointIn<T> pin;
    load_point<T, MODE>(d, G, qn, i, j, k, final_stage, pin);
    GView<R> V;
    V.rho = qs.rho; V.rth = qs.rth;
    V.pp = ws;
    V.u = ws + ncol * nzs; V.v = V.u + ncol * nzl; V.w = V.v + ncol * nzl;
    V.rhob = P.rhob; V.rthb = P.rthb; V.pb = P.pb; V.irthb = P.irthb; V.rhobc = P.rhobc;
    const int jm = wrap1(j - 1, ny), jp = wrap1(j + 1, ny);
    for (int m = 0; m < 3; ++m) {
        const int col_m = wrap1(i - 1 + m, d.nx) * ny + j;
        V.cb[m] = col_m * nzs + k;
        V.lb[m] = col_m * nzl + k;
    }
    V.cj[0] = (jm - j) * nzs; V.cj[1] = 0; V.cj[2] = (jp - j) * nzs;
    V.lj[0] = (jm - j) * nzl; V.lj[1] = 0; V.lj[2] = (jp - j) * nzl;
    V.k = k; V.nz = d.nz;
    stage_point<T, MODE, GView<R>>(d, G, P, qs, pin, qo, cdt, final_stage, i, j, k, V, st, false);
}

// ------------------------------------------------------------------------------------------------
// Batched form: many independent blocks (ensemble members, refined blocks) in one launch.  Each
// block is described on the device; the grid enumerates the tiles of all blocks (prefix table
// tile0), each workgroup finds its block by binary search and runs the same tile body.
// ------------------------------------------------------------------------------------------------
template <typename T>
struct BlockDesc {
    Dims d;
    Geo G;
    Phy P;
    SOut<T> q[3];       // the block's three state buffers
    int nbx, nby, nbz;     // tiles of the regular-point launch (the batch's tile shape) over the range
    int nbxb, nbyb, nbzb;  // tiles of the band-point launch (one-wave tiles) over the range below kband
    int blist;             // 1: the band-point launch takes the block's listed band tiles (G.nband of
                           // them, at the start of G.ws) instead of all nbxb nbyb nbzb
    int tile0;             // first tile of the block in the batched band-point grid
    int tile0r;            // first tile of the block in the batched regular-point grid
    int col0;           // first column of the block in the batched diagnostic grid
    int ilo[3], ihi[3];  // the block's own cells (the rest of the grid is ghost cells)
    int rlo[3], rhi[3];  // cells the batch updates: own cells and the ghost cells no same-level block
                         // refills (the tiles start at rlo; the diagnostics cover columns [rlo, rhi))
};

template <typename T>
__device__ __forceinline__ SIn<T> as_in(const SOut<T> &q)
{
    return SIn<T>{q.rho, q.rth, q.mu, q.mv, q.mw, q.rho_lo, q.rth_lo};
}

// SEL = 1 (REG): the points at or above their column's band top, in the batch's tiles over every
// block's range; SEL = 2: the points below it, in one-wave tiles over the range below kband
template <typename T, int TX, int TY, int TZ, int MODE, int MINW, int SEL>
__global__ void __launch_bounds__(TX * TY * TZ, MINW)
    k_stage_batch(const BlockDesc<T> *__restrict__ desc, int nblk, int ntiles, int rn, int rs, int ro,
                  double cdt, int final_stage, int64_t *st)
{
    static_assert(SEL == 1 || SEL == 2, "regular or band points");
    // XCD-aware order over the whole batch, then the block that owns this tile
    int b = blockIdx.x;
    int xcd = b & 7, idx = b >> 3, per = ntiles >> 3, rem = ntiles & 7;
    int lb = xcd * per + (xcd < rem ? xcd : rem) + idx;
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((SEL == 1 ? desc[mid].tile0r : desc[mid].tile0) <= lb) lo = mid;
        else hi = mid - 1;
    }
    const BlockDesc<T> &D = desc[lo];
    const int nk = SEL == 1 ? D.nbz : D.nbzb, ny = SEL == 1 ? D.nby : D.nbyb;
    int bi, bj, bk;
    if (SEL == 2 && D.blist) {  // the block's listed band tiles (each holds band points)
        const int t = ((const int32_t *)D.G.ws)[lb - D.tile0];
        if (t < 0 || t >= D.nbxb * D.nbyb * D.nbzb) return;  // not a tile of this block (a stale list)
        const int r = t % (D.nbxb * D.nbyb);
        bk = t / (D.nbxb * D.nbyb);
        bi = r / D.nbyb;
        bj = r % D.nbyb;
    } else {
        strip_tile(lb - (SEL == 1 ? D.tile0r : D.tile0), SEL == 1 ? D.nbx : D.nbxb, ny, nk, bi, bj, bk);
    }
    const int i0 = D.rlo[0] + bi * TX, j0 = D.rlo[1] + bj * TY, k0 = D.rlo[2] + bk * TZ;
    if (SEL == 2 && !D.blist && !band_tile_busy<TX, TY, TZ>(D.d, D.G, i0, j0, k0)) return;
    tile_body<T, TX, TY, TZ, MODE, 1, SEL == 1, SEL>(D.d, D.G, D.P, as_in(D.q[rs]), as_in(D.q[rn]), D.q[ro], cdt,
                                                     final_stage, i0, j0, k0, st,
                                                     OwnRange{{D.ilo[0], D.ilo[1], D.ilo[2]},
                                                              {D.ihi[0], D.ihi[1], D.ihi[2]}});
}

// ------------------------------------------------------------------------------------------------
// Velocity diagnostics (Sec. 2.4).  The plane search takes integer decisions (which plane, which
// face, which corners carry weight) from floating-point positions, so it is evaluated without FMA
// contraction in the written order.
// ------------------------------------------------------------------------------------------------

// Try the first three lattice planes of one family (0: x = const, 1: y = const, 2: z = const) beyond
// the terrain point B along the normal line; on each plane the intersection falls in a face of four
// lattice points (located with floor); the first plane whose corners with non-zero bilinear weight
// are all predicted gives the interpolated velocity (the paper's u_N).  The faces and weights of the
// three planes are formed first and the classes of their corners read together; then the velocities
// of the chosen face's corners are read together (a corner that is not predicted is read at a level
// of at least 1, which keeps the read in range, and takes no part).
template <typename T, typename R = typename Compute<T>::R>
__device__ bool plane_family(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &q, int fam,
                             int I, int J, R ut[3])
{
#pragma clang fp contract(off)
    int64_t nc = (int64_t)d.nx * d.ny, hc = hidx(d, I, J);
    double n0 = G.nrm[hc], n1 = G.nrm[nc + hc], n2 = G.nrm[2 * nc + hc];
    double hh = G.H[hc];
    if (!(hh >= 0.0 && hh < (double)d.nz * d.dz)) return false;  // terrain outside the column
    if (fam != 2 && (fam == 0 ? n0 : n1) == 0.0) return false;
    // horizontal positions are measured from the corner (I,J) in cell units, so the located face
    // and weights do not depend on where the grid's origin lies
    int P4[3][4][3];
    double w[3][4];
    bool valid[3];
    int K0 = 0;
    if (fam == 2) {
        K0 = (int)floor(hh / d.dz) + 1;
        while (K0 > 0 && (double)(K0 - 1) * d.dz > hh) --K0;
        while ((double)K0 * d.dz <= hh) ++K0;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        int ia, ib;
        double a, b;
        valid[m] = true;
        if (fam == 2) {
            int K = K0 + m;
            valid[m] = K <= d.nz - 1;  // (a plane above the lid ends the search)
            double t = ((double)K * d.dz - hh) / n2;
            double fx = (t * n0) / d.dx, fy = (t * n1) / d.dy;
            int sx = (int)floor(fx), sy = (int)floor(fy);
            a = fx - (double)sx; b = fy - (double)sy;
            ia = I + sx; ib = J + sy;
            P4[m][0][0] = ia; P4[m][0][1] = ib; P4[m][0][2] = K;
            P4[m][1][0] = ia + 1; P4[m][1][1] = ib; P4[m][1][2] = K;
            P4[m][2][0] = ia; P4[m][2][1] = ib + 1; P4[m][2][2] = K;
            P4[m][3][0] = ia + 1; P4[m][3][1] = ib + 1; P4[m][3][2] = K;
        } else {
            double nn = fam == 0 ? n0 : n1;
            int step = (m + 1) * (nn > 0.0 ? 1 : -1);
            double t = fam == 0 ? ((double)step * d.dx) / nn : ((double)step * d.dy) / nn;
            double fa = fam == 0 ? (t * n1) / d.dy : (t * n0) / d.dx;
            double fz = (hh + t * n2) / d.dz;
            int sa = (int)floor(fa);
            ib = (int)floor(fz);
            a = fa - (double)sa; b = fz - (double)ib;
            ia = (fam == 0 ? J : I) + sa;
            valid[m] = !(ib < 0 || ib + 1 > d.nz - 1);
            for (int s = 0; s < 4; ++s) {
                int pa = ia + (s & 1), pz = ib + (s >> 1);
                if (fam == 0) { P4[m][s][0] = I + step; P4[m][s][1] = pa; }
                else { P4[m][s][0] = pa; P4[m][s][1] = J + step; }
                P4[m][s][2] = pz;
            }
        }
        w[m][0] = (1.0 - a) * (1.0 - b); w[m][1] = a * (1.0 - b); w[m][2] = (1.0 - a) * b; w[m][3] = a * b;
    }
    // classes of the valid planes' corners of nonzero weight (every corner index of a valid plane is
    // in range; a corner of zero weight does not enter the mean, whatever its class)
    int8_t vc[3][4];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int s = 0; s < 4; ++s)
            vc[m][s] = valid[m] && w[m][s] != 0.0 ? G.vcls[cidx(d, P4[m][s][0], P4[m][s][1], P4[m][s][2])]
                                                  : (int8_t)CC_GROUND;
    int pick = -1;
    for (int m = 0; m < 3 && pick < 0; ++m) {
        if (!valid[m]) {
            if (fam == 2) return false;  // planes further up lie above the lid too
            continue;
        }
        bool ok = true;
        for (int s = 0; s < 4; ++s)
            if (w[m][s] != 0.0 && vc[m][s] != CC_PRED) ok = false;
        if (ok) pick = m;
    }
    if (pick < 0) return false;
    int C4[4][3];
    double wp[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        for (int e = 0; e < 3; ++e) C4[s][e] = pick == 0 ? P4[0][s][e] : (pick == 1 ? P4[1][s][e] : P4[2][s][e]);
        wp[s] = pick == 0 ? w[0][s] : (pick == 1 ? w[1][s] : w[2][s]);
    }
    R acc[3] = {(R)0, (R)0, (R)0};
    for (int s = 0; s < 4; ++s) {
        if (wp[s] == 0.0) continue;  // only corners of nonzero weight are read
        R v[3];
        lat_vel_pred<T>(d, P, q, C4[s][0], C4[s][1], C4[s][2] > 1 ? C4[s][2] : 1, v);
        for (int cc = 0; cc < 3; ++cc) acc[cc] += (R)wp[s] * v[cc];
    }
    ut[0] = acc[0]; ut[1] = acc[1]; ut[2] = acc[2];
    return true;
}

// boundary velocity of the column corner t = (I,J): free-slip projection of the nearest-plane mean
// (eq. 33).  Corners whose terrain point lies in [zlo, zhi) count a missing nearest plane (for a
// block of a refined grid: its own columns and levels; elsewhere the block's ghost layers, which go
// stale).
template <typename T, typename R = typename Compute<T>::R>
__device__ __forceinline__ void boundary_velocity(const Dims &d, const Geo &G, const Phy &P, const SOut<T> &qw,
                                                  int64_t t, int64_t *st, double zlo, double zhi, R ub[3])
{
    int64_t nc = (int64_t)d.nx * d.ny;
    int I = (int)(t / d.ny), J = (int)(t % d.ny);
    SIn<T> q{qw.rho, qw.rth, qw.mu, qw.mv, qw.mw, qw.rho_lo, qw.rth_lo};
    double n0 = G.nrm[t], n1 = G.nrm[nc + t], n2 = G.nrm[2 * nc + t];
    int dom = (fabs(n2) >= fabs(n0) && fabs(n2) >= fabs(n1)) ? 2 : (fabs(n0) >= fabs(n1) ? 0 : 1);
    R ut[3];
    bool ok = plane_family<T>(d, G, P, q, dom, I, J, ut);
    const int order[3] = {2, 0, 1};
    for (int f = 0; f < 3 && !ok; ++f)
        if (order[f] != dom) ok = plane_family<T>(d, G, P, q, order[f], I, J, ut);
    if (!ok) {  // no usable plane: u~ = 0 (as a perturbation: minus the reference flow)
        ut[0] = -(R)P.ux; ut[1] = -(R)P.vy; ut[2] = (R)0;
        double h0 = G.H[t];
        if (h0 >= zlo && h0 < zhi) count_status(st, ST_NOPLANE);
    }
    R dn = (ut[0] + (R)P.ux) * (R)n0 + (ut[1] + (R)P.vy) * (R)n1 + ut[2] * (R)n2;
    ub[0] = ut[0] - dn * (R)n0;
    ub[1] = ut[1] - dn * (R)n1;
    ub[2] = ut[2] - dn * (R)n2;
}

// Level K of column corner t (K below the column's diagnostic top), in two parts.  The first reads
// the classes, writes the scalars of an absorbed cell (its master's) or a solid cell (zero), and for a
// diagnosed lattice point forms what does not need u_B: a ground point takes u_B itself; a merged-face
// point the interpolation v gm + u_B (1 - gm) between u_B and the lowest predicted point above (v),
// whose first product and weight are formed here.  The second writes the lattice velocity.  Every
// level reads only predicted points and masters, which no level writes, so levels are independent.
template <typename R>
struct DiagLevel {
    R a[3], b;  // interpolation: u = a + u_B b
    int mode;   // 0: nothing to write, 1: u = u_B, 2: interpolation
};

template <typename T, typename R = typename Compute<T>::R>
__device__ __forceinline__ void diagnose_level_pre(const Dims &d, const Geo &G, const Phy &P, const SOut<T> &qw,
                                                   int64_t t, int K, DiagLevel<R> &o)
{
    int I = (int)(t / d.ny), J = (int)(t % d.ny);
    SIn<T> q{qw.rho, qw.rth, qw.mu, qw.mv, qw.mw, qw.rho_lo, qw.rth_lo};
    const int64_t base = cidx(d, I, J, 0), p = base + K;
    const int8_t vc = G.vcls[p], cl = G.cls[p];
    o.mode = 0;
    if (vc != CC_PRED) {
        o.mode = 1;
        if (vc == CC_MFACE) {
            // the lowest predicted point within 8 levels above (classes read together)
            int8_t cv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) cv[s] = K + 1 + s < d.nz ? G.vcls[base + K + 1 + s] : (int8_t)-1;
            int kp = -1;
            for (int s = 0; s < 8; ++s)
                if (cv[s] == CC_PRED) { kp = K + 1 + s; break; }
            if (kp >= 0) {
                double hh = G.H[t];
                double gm = ((double)K * d.dz - hh) / ((double)kp * d.dz - hh);
                R v[3];
                lat_vel_pred<T>(d, P, q, I, J, kp, v);
                for (int cc = 0; cc < 3; ++cc) o.a[cc] = v[cc] * (R)gm;
                o.b = (R)(1.0 - gm);
                o.mode = 2;
            }
        }
    }
    if (cl == CC_SOLID) {
        qw.rho[p] = (T)0; qw.rth[p] = (T)0;
        if (qw.rho_lo) { qw.rho_lo[p] = (T)0; qw.rth_lo[p] = (T)0; }
    } else if (cl == CC_ABSORBED) {
        int64_t m = G.master[p];
        T r0 = qw.rho[m], r1 = qw.rth[m];
        if (qw.rho_lo) {
            T l0 = qw.rho_lo[m], l1 = qw.rth_lo[m];
            qw.rho_lo[p] = l0; qw.rth_lo[p] = l1;
        }
        qw.rho[p] = r0; qw.rth[p] = r1;
    }
}

template <typename T, typename R = typename Compute<T>::R>
__device__ __forceinline__ void diagnose_level_post(const Dims &d, const SOut<T> &qw, int64_t t, int K,
                                                    const DiagLevel<R> &o, const R ub[3])
{
    if (o.mode == 0) return;
    const int64_t p = t * d.nzs + K;
    R u[3];
    for (int cc = 0; cc < 3; ++cc) u[cc] = o.mode == 2 ? o.a[cc] + ub[cc] * o.b : ub[cc];
    qw.mu[p] = (T)u[0]; qw.mv[p] = (T)u[1]; qw.mw[p] = (T)u[2];
}

// Diagnostics in blocks of DIAG_COLS column corners and DIAG_THREADS threads.  The first DIAG_COLS
// threads find the corners' boundary velocities while the others take levels 0 .. DIAG_EARLY-1 of the
// corners (one each) up to the point where u_B is needed; after a barrier those levels are finished
// and all threads take the levels above, level by level, so a deep column is spread over many threads.
constexpr int DIAG_COLS = 64, DIAG_THREADS = 256, DIAG_EARLY = DIAG_THREADS / DIAG_COLS - 1;

// the column of a slot: its grid (b: block of a batch), corner index and the terrain range that
// counts a missing plane
struct DiagCol {
    bool valid;
    int b;
    int64_t t;
    double zlo, zhi;
};

// Run f(b) for the member b of each lane: with the wave-uniform member (read through scalar loads)
// when every lane of the wave has the same one, as is the case away from the members' boundaries.
template <typename VIEWS, typename F>
__device__ __forceinline__ void with_member(int b, F &&f)
{
    if constexpr (VIEWS::MULTI) {
        const int bu = __builtin_amdgcn_readfirstlane(b);
        if (__all(b == bu)) f(bu);
        else f(b);
    } else {
        f(b);
    }
}

template <typename T, typename VIEWS>
__device__ __forceinline__ void diagnose_block(const VIEWS &views, int64_t *st)
{
    using R = typename Compute<T>::R;
    __shared__ R s_ub[3][DIAG_COLS];
    __shared__ int s_top[DIAG_COLS], s_b[DIAG_COLS];
    __shared__ int64_t s_t[DIAG_COLS];
    __shared__ int s_kmax;
    const int tid = threadIdx.x, slot = tid % DIAG_COLS, grp = tid / DIAG_COLS;
    if (tid == 0) s_kmax = 0;
    __syncthreads();
    const DiagCol col = views.column(slot);
    DiagLevel<R> early;
    early.mode = 0;
    int top = 0;
    with_member<VIEWS>(col.b, [&](int b) {
        const Dims &d = views.dims(b);
        const Geo &G = views.geo(b);
        const Phy &P = views.phy(b);
        const SOut<T> &qw = views.state(b);
        top = col.valid ? G.colk[2 * (int64_t)d.nx * d.ny + col.t] : 0;
        if (grp == 0) {
            if (col.valid) {
                R ub[3];
                boundary_velocity<T>(d, G, P, qw, col.t, st, col.zlo, col.zhi, ub);
                s_ub[0][slot] = ub[0]; s_ub[1][slot] = ub[1]; s_ub[2][slot] = ub[2];
            }
        } else if (grp - 1 < top) {
            diagnose_level_pre<T>(d, G, P, qw, col.t, grp - 1, early);
        }
    });
    if (grp == 0) {
        s_top[slot] = top;
        s_b[slot] = col.b;
        s_t[slot] = col.t;
        atomicMax(&s_kmax, top);
    }
    __syncthreads();
    if (early.mode != 0) {
        const R ub[3] = {s_ub[0][slot], s_ub[1][slot], s_ub[2][slot]};
        with_member<VIEWS>(col.b, [&](int b) { diagnose_level_post<T>(views.dims(b), views.state(b), col.t, grp - 1, early, ub); });
    }
    const int n = (s_kmax - DIAG_EARLY) * DIAG_COLS;
    for (int it = tid; it < n; it += DIAG_THREADS) {
        const int sl = it % DIAG_COLS, K = DIAG_EARLY + it / DIAG_COLS;
        if (K >= s_top[sl]) continue;
        const int64_t t = s_t[sl];
        const R ub[3] = {s_ub[0][sl], s_ub[1][sl], s_ub[2][sl]};
        with_member<VIEWS>(s_b[sl], [&](int b) {
            const Dims &d2 = views.dims(b);
            const SOut<T> &q2 = views.state(b);
            DiagLevel<R> o;
            diagnose_level_pre<T>(d2, views.geo(b), views.phy(b), q2, t, K, o);
            diagnose_level_post<T>(d2, q2, t, K, o, ub);
        });
    }
}

// views of a single grid: slot s of block b is corner b DIAG_COLS + s
template <typename T>
struct GridDiagViews {
    static constexpr bool MULTI = false;
    const Dims &d;
    const Geo &G;
    const Phy &P;
    const SOut<T> &q;
    __device__ DiagCol column(int slot) const
    {
        const int64_t t = (int64_t)blockIdx.x * DIAG_COLS + slot;
        return DiagCol{t < (int64_t)d.nx * d.ny, 0, t, 0.0, (double)d.nz * d.dz};
    }
    __device__ const Dims &dims(int) const { return d; }
    __device__ const Geo &geo(int) const { return G; }
    __device__ const Phy &phy(int) const { return P; }
    __device__ const SOut<T> &state(int) const { return q; }
};

template <typename T>
__global__ void __launch_bounds__(DIAG_THREADS) k_diagnose(Dims d, Geo G, Phy P, SOut<T> qw, int64_t *st)
{
    diagnose_block<T>(GridDiagViews<T>{d, G, P, qw}, st);
}

// views of a batch: column indices follow the blocks' col0 offsets; each block maps its columns over
// [rlo, rhi) in x and y; corners of a block's own columns count a missing plane for terrain in its
// own levels, the others (ghost layers, which go stale) never
template <typename T>
struct BatchDiagViews {
    static constexpr bool MULTI = true;
    const BlockDesc<T> *desc;
    int nblk, ncols, ro;
    // the block holding column t (the last whose first column is at or before t)
    __device__ int block_of(int t) const
    {
        int lo = 0, hi = nblk - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (desc[mid].col0 <= t) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
    __device__ DiagCol column(int slot) const
    {
        // one search for the workgroup's first column (uniform), then forward to each lane's block
        const int t0 = blockIdx.x * DIAG_COLS;
        const int t = t0 + slot;
        if (t >= ncols) return DiagCol{false, 0, 0, 0.0, 0.0};
        int b = block_of(t0);
        while (b + 1 < nblk && desc[b + 1].col0 <= t) ++b;
        const BlockDesc<T> &D = desc[b];
        const int wy = D.rhi[1] - D.rlo[1];
        const int r = t - D.col0;
        const int I = D.rlo[0] + r / wy, J = D.rlo[1] + r % wy;
        const bool own = I >= D.ilo[0] && I < D.ihi[0] && J >= D.ilo[1] && J < D.ihi[1];
        return DiagCol{true, b, (int64_t)I * D.d.ny + J, own ? (double)D.ilo[2] * D.d.dz : 0.0,
                       own ? (double)D.ihi[2] * D.d.dz : 0.0};
    }
    __device__ const Dims &dims(int b) const { return desc[b].d; }
    __device__ const Geo &geo(int b) const { return desc[b].G; }
    __device__ const Phy &phy(int b) const { return desc[b].P; }
    __device__ const SOut<T> &state(int b) const { return desc[b].q[ro]; }
};

template <typename T>
__global__ void __launch_bounds__(DIAG_THREADS) k_diagnose_batch(const BlockDesc<T> *__restrict__ desc, int nblk,
                                                                 int ncols, int ro, int64_t *st)
{
    diagnose_block<T>(BatchDiagViews<T>{desc, nblk, ncols, ro}, st);
}

// ------------------------------------------------------------------------------------------------
// host helpers: C-ABI structs -> kernel views
// ------------------------------------------------------------------------------------------------
inline bool make_views(const char *what, const cc_grid *grid, const cc_phys *phys, const cc_geom *g,
                       const double *base, cc_prec prec, Dims &d, Geo &G, Phy &P)
{
    if (!check_grid(grid)) return false;
    if (!phys || !g || !base) { set_error("%s: null argument", what); return false; }
    const void *p[] = {g->H, g->V, g->Ax, g->Ay, g->Az, g->nrm, g->Vgroup, g->cls, g->vcls,
                       g->master, g->gnext, g->colk};
    if (!check_ptrs(what, 12, p)) return false;
    if (prec != CC_F64 && prec != CC_F32_PERT) { set_error("%s: unknown precision %d", what, (int)prec); return false; }
    d = dims_of(grid);
    G = Geo{g->H, g->V, g->Ax, g->Ay, g->Az, g->nrm, g->Vgroup, g->cls, g->vcls, g->master, g->gnext, g->colk,
            g->stage_ws, g->kband, g->stage_ws ? g->nband_tiles : -1, g->side};
    double cv = phys->cp - phys->rd;
    P.rhob = base; P.rthb = base + d.nz; P.pb = base + 2 * d.nz; P.thb = base + 3 * d.nz;
    P.irthb = base + 4 * d.nz; P.rhobc = base + 5 * d.nz;
    P.g = phys->g;
    P.gam = phys->cp / cv;
    P.ux = prec == CC_F32_PERT ? phys->u0 : 0.0;
    P.vy = prec == CC_F32_PERT ? phys->v0 : 0.0;
    P.u0 = phys->u0; P.v0 = phys->v0; P.kdh = phys->kdh; P.kdv = phys->kdv;
    if (!(P.kdh >= 0.0 && P.kdv >= 0.0)) { set_error("%s: negative diffusion rate", what); return false; }
    P.zsp = phys->zsp; P.rsp = phys->rsp;
    P.ztop = d.z0 + d.nz * d.dz;
    if (phys->ztop != 0.0) {
        if (!(phys->ztop >= P.ztop * (1.0 - 1e-12)) || !std::isfinite(phys->ztop)) {
            set_error("%s: lid height %g below the grid's top %g", what, phys->ztop, P.ztop);
            return false;
        }
        P.ztop = phys->ztop;
    }
    if (!(P.rsp >= 0.0) || !std::isfinite(P.rsp) || (P.rsp != 0.0 && !std::isfinite(P.zsp))) {
        set_error("%s: invalid sponge (rate %g, bottom %g)", what, P.rsp, P.zsp);
        return false;
    }
    P.dV = d.dx * d.dy * d.dz;
    P.idV = 1.0 / P.dV;
    P.idx = 1.0 / d.dx; P.idy = 1.0 / d.dy; P.idz = 1.0 / d.dz;
    // binomial coefficients of (1+x)^gamma - 1
    P.binom[0] = P.gam;
    for (int n = 1; n < EOS_TERMS; ++n) P.binom[n] = P.binom[n - 1] * (P.gam - n) / (n + 1);
    for (int n = 0; n < EOS_TERMS; ++n) P.binomf[n] = (float)P.binom[n];
    return true;
}

inline bool state_ok(const char *what, const cc_state *q)
{
    if (!q) { set_error("%s: null state", what); return false; }
    const void *p[] = {q->rho, q->rth, q->mu, q->mv, q->mw};
    return check_ptrs(what, 5, p);
}

template <typename T>
inline SIn<T> sin_of(const cc_state *q)
{
    bool lo = sizeof(T) == 4 && q->rho_lo && q->rth_lo;
    return SIn<T>{(const T *)q->rho, (const T *)q->rth, (const T *)q->mu, (const T *)q->mv, (const T *)q->mw,
                  lo ? (const T *)q->rho_lo : nullptr, lo ? (const T *)q->rth_lo : nullptr};
}
template <typename T>
inline SOut<T> sout_of(cc_state *q)
{
    bool lo = sizeof(T) == 4 && q->rho_lo && q->rth_lo;
    return SOut<T>{(T *)q->rho, (T *)q->rth, (T *)q->mu, (T *)q->mv, (T *)q->mw,
                   lo ? (T *)q->rho_lo : nullptr, lo ? (T *)q->rth_lo : nullptr};
}

}  // namespace cc
