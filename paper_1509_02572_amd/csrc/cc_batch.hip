// Batched blocks: many grids stepped by one update and one diagnostic launch per Runge-Kutta stage
// and level, with the step sequence optionally captured into a hipGraph.
//
// Two kinds of batch share this code:
//   * ensembles: independent periodic domains, one level;
//   * refined grids (Sec. 2.2 of the paper): blocks of levels 0..L, level l with spacing and time step
//     2^-l of level 0's.  Every block is a padded box: its own cells plus ghost cells beyond each
//     side, at the block's resolution.  The box is stepped as one grid; ghost cells are integrated
//     on like the block's own cells (the paper integrates on ghost cells instead of interpolating
//     in time), so the outermost ghost layers go stale by one layer per stage while the block's
//     own cells stay exact as long as the ghost width covers the stages between refills.
//     Refills: after every stage a block's ghost cells owned by blocks of the same level are copied
//     from them; at the end of a level-l step, ghost cells of level l owned by level l+1 receive the
//     eight-point average of the fine cells, and ghost cells of level l+1 owned by level l receive
//     the coarse cell's value (Sec. 2.2).  Levels advance fine first: two steps of level l+1, then
//     one of level l.  Mass is conserved by flux matching: the fine fluxes through a coarse-fine
//     interface, accumulated over the fine final stages, replace the coarse flux of the coarse
//     final stage (the only stage that carries q^n to q^{n+1}).
#pragma clang fp contract(off)

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <vector>

#include "cc_diffuse.hpp"
#include "cc_kernels.hpp"
#include "cc_stream.hpp"

namespace cc {

// ghost-cell refill: destination block / box index, source block / box index (block numbers
// within their levels)
struct GhostEnt { int32_t dblk, didx, sblk, sidx, par = 0; };  // par: injection's fine-index parities
// an injection entry's destination index carries the parities (x, y, z in bits 0-2) of the fine
// cell's global index above bit GHOST_PAR_SHIFT (block boxes hold fewer than 2^28 slots)
constexpr int GHOST_PAR_SHIFT = 28;
constexpr int32_t GHOST_IDX_MASK = (1 << GHOST_PAR_SHIFT) - 1;
// on the device the refill lists are packed by (destination, source) block pair: chunks of at most
// 64 entries of one pair (one wavefront each, so the pair's descriptors are read once per wave), and
// the entries' destination and source box indices
struct GhostPair { int32_t didx, sidx; };
struct GhostChunk { int32_t dblk, sblk, first, count; };
constexpr int FILL_CHUNK = 64;
// fine side of one coarse-fine face: fine block, axis and the four fine sub-faces, each given as
// the box index of the cell on the +axis side of the sub-face
struct FluxSlot { int32_t fblk, axis, idx[4]; };
// coarse cell with coarse-fine faces: register slot of each face (-x,+x,-y,+y,-z,+z), -1 if none
struct CorrEnt { int32_t cblk, cidx, slot[6]; };

enum { FILL_COPY = 0, FILL_INJECT = 1, FILL_RESTRICT = 2 };

// ------------------------------------------------------------------------------------------------
// device: ghost refills
// ------------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void put_scalar(const SOut<T> &q, int64_t i, double v0, double v1)
{
    T a = (T)v0, b = (T)v1;
    q.rho[i] = a;
    q.rth[i] = b;
    if (q.rho_lo) {
        q.rho_lo[i] = (T)(v0 - (double)a);
        q.rth_lo[i] = (T)(v1 - (double)b);
    }
}

template <typename T>
__device__ __forceinline__ double get_scalar(const SOut<T> &q, int64_t i, int w)
{
    const T *hi = w ? q.rth : q.rho, *lo = w ? q.rth_lo : q.rho_lo;
    double v = (double)hi[i];
    if (lo) v += (double)lo[i];
    return v;
}

// One ghost cell and the lattice point that shares its index.  Copies within a level move the
// stored values as they are.  Between levels every value moves as a perturbation from its level's
// reference: the scalars from each level's base state, and the momentum at predicted points from the
// reference flow rhobar_c(K) U of each level's lattice level (whose base density depends on the
// spacing).  The float form stores those perturbations; FP64 stores the total momentum, so there the
// reference terms of the two lattice levels are exchanged.
template <typename T>
__global__ void __launch_bounds__(256) k_ghost_fill(const BlockDesc<T> *__restrict__ dd, int rd,
                                                    const BlockDesc<T> *__restrict__ sd, int rs,
                                                    const GhostChunk *__restrict__ ch,
                                                    const GhostPair *__restrict__ pr, int nch, int mode)
{
    const int c = blockIdx.x * (256 / FILL_CHUNK) + (int)(threadIdx.x / FILL_CHUNK);
    if (c >= nch) return;
    const int lane = threadIdx.x % FILL_CHUNK;
    // the chunk's block pair is the same on every lane of the wave
    const int dblk = __builtin_amdgcn_readfirstlane(ch[c].dblk), sblk = __builtin_amdgcn_readfirstlane(ch[c].sblk);
    const int first = __builtin_amdgcn_readfirstlane(ch[c].first), count = __builtin_amdgcn_readfirstlane(ch[c].count);
    if (lane >= count) return;
    const GhostPair g = pr[first + lane];
    const BlockDesc<T> &D = dd[dblk], &S = sd[sblk];
    const SOut<T> qd = D.q[rd], qs = S.q[rs];
    const int64_t di = g.didx & GHOST_IDX_MASK, si = g.sidx;
    const unsigned par = (unsigned)g.didx >> GHOST_PAR_SHIFT;
    if (mode == FILL_RESTRICT) {
        const int64_t sx = (int64_t)S.d.ny * S.d.nzs, sy = S.d.nzs;
        double v[2];
        for (int w = 0; w < 2; ++w) {
            double c0 = get_scalar(qs, si, w), c1 = get_scalar(qs, si + sx, w);
            double c2 = get_scalar(qs, si + sy, w), c3 = get_scalar(qs, si + sx + sy, w);
            double c4 = get_scalar(qs, si + 1, w), c5 = get_scalar(qs, si + sx + 1, w);
            double c6 = get_scalar(qs, si + sy + 1, w), c7 = get_scalar(qs, si + sx + sy + 1, w);
            v[w] = (((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7))) * 0.125;
        }
        put_scalar(qd, di, v[0], v[1]);
    } else {
        qd.rho[di] = qs.rho[si];
        qd.rth[di] = qs.rth[si];
        if (qd.rho_lo) {
            qd.rho_lo[di] = qs.rho_lo[si];
            qd.rth_lo[di] = qs.rth_lo[si];
        }
    }
    T mu = qs.mu[si], mv = qs.mv[si], mw = qs.mw[si];
    if (mode != FILL_COPY && sizeof(T) == 8 && D.G.vcls[di] == CC_PRED && S.G.vcls[si] == CC_PRED) {
        const int kd = (int)(di % D.d.nzs), ks = (int)(si % S.d.nzs);
        const double dr = D.P.rhobc[kd] - S.P.rhobc[ks];
        mu = (T)((double)mu + dr * S.P.u0);
        mv = (T)((double)mv + dr * S.P.v0);
    }
    if (mode == FILL_INJECT) {
        // the coarse field at the fine ghost's own position, where the coarse stencil allows
        const int64_t sx = (int64_t)S.d.ny * S.d.nzs, sy = S.d.nzs;
        const int ks = (int)(si % S.d.nzs);
        // scalars: a quarter cell from the parent's centre towards the child's side (weights 3/4, 1/4)
        const int64_t ox = (par & 1) ? sx : -sx, oy = (par & 2) ? sy : -sy, oz = (par & 4) ? 1 : -1;
        const bool zin = ks + oz >= 0 && ks + oz < S.d.nz;
        double a0 = 0.0, a1 = 0.0;
        bool ok = true;
        for (int c = 0; c < 8; ++c) {
            const int a = c >> 2, b = (c >> 1) & 1, e = c & 1;
            const int64_t p = si + a * ox + b * oy + (zin ? e * oz : 0);
            const double w = ((a ? 0.25 : 0.75) * (b ? 0.25 : 0.75)) * (zin ? (e ? 0.25 : 0.75) : 0.5);
            ok = ok && S.G.V[p] > 0.0;
            a0 += w * get_scalar(qs, p, 0);
            a1 += w * get_scalar(qs, p, 1);
        }
        if (ok) put_scalar(qd, di, a0, a1);
        // momentum: the mean of the coarse lattice points around the fine one (the point at the halved
        // index, and the next one along every axis where the fine index is odd), as perturbations; an
        // odd fine level over a coarse level that is not predicted (the ground) takes the level above
        const bool zup = (par & 4) && ks + 1 < S.d.nz;
        const bool predd = D.G.vcls[di] == CC_PRED;
        const bool shift = zup && S.G.vcls[si] != CC_PRED && S.G.vcls[si + 1] == CC_PRED;
        const int64_t base = si + (shift ? 1 : 0);
        const int kb = ks + (shift ? 1 : 0);
        const double rd = sizeof(T) == 8 ? D.P.rhobc[(int)(di % D.d.nzs)] : 0.0;
        if (shift && predd) {  // the fallback: the coarse point above, as a perturbation
            const double rb = sizeof(T) == 8 ? S.P.rhobc[kb] : 0.0;
            mu = (T)((double)qs.mu[base] - rb * S.P.u0 + rd * S.P.u0);
            mv = (T)((double)qs.mv[base] - rb * S.P.v0 + rd * S.P.v0);
            mw = qs.mw[base];
        }
        const bool oddx = par & 1, oddy = par & 2, oddz = zup && !shift;
        bool okm = predd;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        int n = 0;
        for (int c = 0; c < 8; ++c) {
            const int a = c >> 2, b = (c >> 1) & 1, e = c & 1;
            if ((a && !oddx) || (b && !oddy) || (e && !oddz)) continue;
            const int64_t p = base + a * sx + b * sy + e;
            okm = okm && S.G.vcls[p] == CC_PRED;
            const double ref = sizeof(T) == 8 ? S.P.rhobc[kb + e] : 0.0;  // FP64 stores the total
            s0 += (double)qs.mu[p] - ref * S.P.u0;
            s1 += (double)qs.mv[p] - ref * S.P.v0;
            s2 += (double)qs.mw[p];
            ++n;
        }
        if (okm) {
            mu = (T)(s0 / n + rd * S.P.u0);
            mv = (T)(s1 / n + rd * S.P.v0);
            mw = (T)(s2 / n);
        }
    }
    qd.mu[di] = mu;
    qd.mv[di] = mv;
    qd.mw[di] = mw;
}

// ------------------------------------------------------------------------------------------------
// device: face fluxes of open regular faces (coarse-fine interfaces lie away from the terrain)
// ------------------------------------------------------------------------------------------------
// Total fluxes of rho' and (rho theta)' (kg/s and kg K/s) through the face at the lower side of box
// cell (i,j,k) along `axis`, positive along +axis.  The perturbation part is evaluated exactly as
// the update kernel evaluates it (same operands, same order: bitwise the same value); the part
// carried by the base state and the reference flow (float form only) is added in double.
template <typename T>
__device__ void face_total_flux(const BlockDesc<T> &B, const SIn<T> &q, int axis, int i, int j, int k, double F[2],
                                bool &regular)
{
    using R = typename Compute<T>::R;
    const Dims &d = B.d;
    const Geo &G = B.G;
    const Phy &P = B.P;
    int im = i - (axis == 0), jm = j - (axis == 1), km = k - (axis == 2);
    int64_t up = cidx(d, i, j, k), lo = cidx(d, im, jm, km);
    regular = G.cls[up] == CC_OPEN && G.cls[lo] == CC_OPEN && G.gnext[up] == -1 && G.gnext[lo] == -1 &&
              G.V[up] == 1.0 && G.V[lo] == 1.0;
    R s4, AS, UAS, b0, b1;
    double S, Un;
    if (axis == 0) {
        R a[3], b[3], c[3], e[3];
        lat_vel<T>(d, G, P, q, i, j, k, a); lat_vel<T>(d, G, P, q, i, j + 1, k, b);
        lat_vel<T>(d, G, P, q, i, j, k + 1, c); lat_vel<T>(d, G, P, q, i, j + 1, k + 1, e);
        s4 = (a[0] + b[0]) + (c[0] + e[0]);
        S = d.dy * d.dz; Un = P.ux;
        AS = (R)(0.25 * 1.0 * S); UAS = (R)(P.ux * 1.0 * S);
        b0 = (R)P.rhob[k]; b1 = (R)P.rthb[k];
    } else if (axis == 1) {
        R a[3], b[3], c[3], e[3];
        lat_vel<T>(d, G, P, q, i, j, k, a); lat_vel<T>(d, G, P, q, i + 1, j, k, b);
        lat_vel<T>(d, G, P, q, i, j, k + 1, c); lat_vel<T>(d, G, P, q, i + 1, j, k + 1, e);
        s4 = (a[1] + b[1]) + (c[1] + e[1]);
        S = d.dz * d.dx; Un = P.vy;
        AS = (R)(0.25 * 1.0 * S); UAS = (R)(P.vy * 1.0 * S);
        b0 = (R)P.rhob[k]; b1 = (R)P.rthb[k];
    } else {
        R a[3], b[3], c[3], e[3];
        lat_vel<T>(d, G, P, q, i, j, k, a); lat_vel<T>(d, G, P, q, i + 1, j, k, b);
        lat_vel<T>(d, G, P, q, i, j + 1, k, c); lat_vel<T>(d, G, P, q, i + 1, j + 1, k, e);
        s4 = (a[2] + b[2]) + (c[2] + e[2]);
        S = d.dx * d.dy; Un = 0.0;
        AS = (R)(0.25 * 1.0 * S); UAS = (R)0;
        b0 = (R)P.rhobc[k]; b1 = (R)(k > 0 ? 0.5 * (P.rthb[k - 1] + P.rthb[k]) : P.rthb[0]);
    }
    R f0, f1;
    scalar_face_flux<R>(s4, AS, UAS, b0, b1, (R)q.rho[lo], (R)q.rho[up], (R)q.rth[lo], (R)q.rth[up], f0, f1);
    // base-state / reference-flow part (zero in the double form, where Un = 0)
    double h0 = axis == 2 ? 0.0 : P.rhob[k] * Un * S, h1 = axis == 2 ? 0.0 : P.rthb[k] * Un * S;
    F[0] = (double)f0 + h0;
    F[1] = (double)f1 + h1;
}

// fine side: after a fine final stage, add dt_f x (sum of the four sub-face fluxes) to each slot
template <typename T>
__global__ void k_flux_accumulate(const BlockDesc<T> *__restrict__ fd, int rs, const FluxSlot *__restrict__ sl,
                                  int n, double dtf, double *__restrict__ reg, int64_t *st)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const FluxSlot s = sl[t];
    const BlockDesc<T> &B = fd[s.fblk];
    const SIn<T> q = as_in(B.q[rs]);
    double a0 = 0.0, a1 = 0.0;
    bool ok = true;
    for (int f = 0; f < 4; ++f) {
        int i, j, k;
        unidx(B.d, s.idx[f], i, j, k);
        double F[2];
        bool reg_ok;
        face_total_flux<T>(B, q, s.axis, i, j, k, F, reg_ok);
        ok = ok && reg_ok;
        a0 += F[0];
        a1 += F[1];
    }
    reg[2 * t] += dtf * a0;
    reg[2 * t + 1] += dtf * a1;
    if (!ok) count_status(st, ST_INTERFACE);
}

// coarse side: after the coarse final stage, replace dt x (coarse face flux) by the accumulated
// fine fluxes in every coarse cell with coarse-fine faces, then clear the slots
template <typename T>
__global__ void k_flux_correct(const BlockDesc<T> *__restrict__ cd, int rs, int ro, const CorrEnt *__restrict__ ce,
                               int n, double dt, double *__restrict__ reg, int64_t *st)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const CorrEnt e = ce[t];
    const BlockDesc<T> &B = cd[e.cblk];
    const SIn<T> q = as_in(B.q[rs]);
    int i, j, k;
    unidx(B.d, e.cidx, i, j, k);
    double c0 = 0.0, c1 = 0.0;
    bool ok = true;
    for (int f = 0; f < 6; ++f) {
        int r = e.slot[f];
        if (r < 0) continue;
        int axis = f >> 1, plus = f & 1;
        double F[2];
        bool reg_ok;
        face_total_flux<T>(B, q, axis, i + (plus && axis == 0), j + (plus && axis == 1), k + (plus && axis == 2), F,
                           reg_ok);
        ok = ok && reg_ok;
        double sg = plus ? 1.0 : -1.0;
        c0 += sg * (dt * F[0] - reg[2 * r]);
        c1 += sg * (dt * F[1] - reg[2 * r + 1]);
        reg[2 * r] = 0.0;
        reg[2 * r + 1] = 0.0;
    }
    const SOut<T> &qo = B.q[ro];
    double vol = B.G.Vgroup[e.cidx] * B.P.dV;
    double v0 = get_scalar(qo, e.cidx, 0) + c0 / vol;
    double v1 = get_scalar(qo, e.cidx, 1) + c1 / vol;
    put_scalar(qo, e.cidx, v0, v1);
    if (!ok) count_status(st, ST_INTERFACE);
}

}  // namespace cc

using namespace cc;

// ------------------------------------------------------------------------------------------------
// host: batch state
// ------------------------------------------------------------------------------------------------
struct Level {
    int nblk = 0, ntiles = 0, ntilesr = 0, ncols = 0, cur = 0;  // band-point tiles, regular-point tiles, columns
    size_t desc_off = 0;
    size_t same_off = 0, inj_off = 0, res_off = 0, slot_off = 0, corr_off = 0, reg_off = 0;
    int nsame = 0, ninj = 0, nres = 0, nslot = 0, ncorr = 0;
    int nsame_near = 0;  // the first same-level entries: ghost cells within NEAR_GHOST of the update range
    // packed refill lists: chunk tables (the entries follow each table in the workspace)
    size_t same_ch = 0, inj_ch = 0, res_ch = 0;
    int csame = 0, csame_near = 0, cinj = 0, cres = 0;  // chunks
};

struct cc_batch_s {
    cc_prec prec;
    int tile = 0;
    int btile = 0;  // band-point tiles: 0 8x8x1, 1 4x4x4, 2 2x2x16
    bool diffuse = false;  // some block has a non-zero artificial-diffusion or sponge rate
    char *ws = nullptr;  // caller workspace: descriptors, refill tables, flux registers
    std::vector<Level> lev;
    hipStream_t cap = nullptr;  // private stream used only for graph capture
    // side stream of the band-point launches, forked from and joined to the stepping stream with
    // events (created with the batch, outside any capture; null: band launches stay on the stream)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    struct Graph { int nsteps; double dt; int64_t *st; std::vector<int> cur0, cur1; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

template <typename T>
const BlockDesc<T> *descs(const cc_batch_s *b, int l) { return (const BlockDesc<T> *)(b->ws + b->lev[l].desc_off); }

// the band points of a level on the side stream, `regular` (the regular-point launch) on s, then the
// join
template <typename T, typename F>
void batch_stage_split(const cc_batch_s *b, int l, int rn, int rs, int ro, double cdt, int fin, int64_t *st,
                       hipStream_t s, F regular)
{
    const Level &L = b->lev[l];
    // the points below their column's band top, on the side stream beside the regular points (the
    // two launches write disjoint points and read only inputs)
    hipStream_t sb = s;
    if (L.ntiles > 0 && b->side && hipEventRecord(b->fork, s) == hipSuccess &&
        hipStreamWaitEvent(b->side, b->fork, 0) == hipSuccess)
        sb = b->side;
    if (L.ntiles > 0) {
        if (b->btile == 0)
            hipLaunchKernelGGL((k_stage_batch<T, 8, 8, 1, 0, 1, 2>), dim3(L.ntiles), dim3(64), 0, sb, descs<T>(b, l),
                               L.nblk, L.ntiles, rn, rs, ro, cdt, fin, st);
        else if (b->btile == 1)
            hipLaunchKernelGGL((k_stage_batch<T, 4, 4, 4, 0, 1, 2>), dim3(L.ntiles), dim3(64), 0, sb, descs<T>(b, l),
                               L.nblk, L.ntiles, rn, rs, ro, cdt, fin, st);
        else
            hipLaunchKernelGGL((k_stage_batch<T, 2, 2, 16, 0, 1, 2>), dim3(L.ntiles), dim3(64), 0, sb, descs<T>(b, l),
                               L.nblk, L.ntiles, rn, rs, ro, cdt, fin, st);
    }
    if (L.ntilesr > 0) regular();  // the points at or above their column's band top
    // join: later work on s waits for the band launch (should the join fail, the host waits)
    if (sb != s && (hipEventRecord(b->join, sb) != hipSuccess || hipStreamWaitEvent(s, b->join, 0) != hipSuccess))
        (void)hipStreamSynchronize(sb);
}

template <typename T, int TX, int TY, int TZ, int MINW>
void launch_batch_stage(const cc_batch_s *b, int l, int rn, int rs, int ro, double cdt, int fin, int64_t *st,
                        hipStream_t s)
{
    const Level &L = b->lev[l];
    batch_stage_split<T>(b, l, rn, rs, ro, cdt, fin, st, s, [&] {
        hipLaunchKernelGGL((k_stage_batch<T, TX, TY, TZ, 0, MINW, 1>), dim3(L.ntilesr), dim3(TX * TY * TZ), 0, s,
                           descs<T>(b, l), L.nblk, L.ntilesr, rn, rs, ro, cdt, fin, st);
    });
}

// refill of level ld's ghost cells from level ls: nch chunks of the table at chunk offset ch, whose
// entries start at entry offset off
template <typename T>
void fill(const cc_batch_s *b, int ld, int ls, size_t ch, size_t off, int nch, int mode, hipStream_t s)
{
    if (nch <= 0) return;
    hipLaunchKernelGGL(k_ghost_fill<T>, dim3(blocks_for(nch, 256 / FILL_CHUNK)), dim3(256), 0, s, descs<T>(b, ld),
                       b->lev[ld].cur, descs<T>(b, ls), b->lev[ls].cur, (const GhostChunk *)(b->ws + ch),
                       (const GhostPair *)(b->ws + off), nch, mode);
}

// one Runge-Kutta stage of level l: update, flux matching in the final stage, diagnostics, then
// same-level ghost refill of the stage output
template <typename T>
void level_stage(cc_batch_s *b, int l, int rn, int rs, int ro, double cdt, int fin, double dt, int64_t *st,
                 hipStream_t s)
{
    const Level &L = b->lev[l];
    if (b->tile >= STREAM_ID_MIN && b->tile <= STREAM_ID_MAX) {  // streaming form (whole grids only)
        batch_stage_split<T>(b, l, rn, rs, ro, cdt, fin, st, s, [&] {
            launch_stream_batch<T>(b->tile, descs<T>(b, l), L.nblk, L.ntilesr, rn, rs, ro, cdt, fin, st, s);
        });
    } else switch (b->tile) {
    case 1: launch_batch_stage<T, 4, 4, 16, 1>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    case 6: launch_batch_stage<T, 4, 4, 32, 1>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    case 11: launch_batch_stage<T, 4, 4, 16, 8>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    case 8: launch_batch_stage<T, 2, 2, 64, 1>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    case 9: launch_batch_stage<T, 8, 8, 8, 6>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    case 7: launch_batch_stage<T, 8, 8, 16, 1>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    case 12: launch_batch_stage<T, 4, 8, 16, 6>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    default: launch_batch_stage<T, 8, 8, 8, 1>(b, l, rn, rs, ro, cdt, fin, st, s); break;
    }
    // the artificial diffusion and the sponge of the stage input, after the update as on a single
    // grid (the flux matching below covers the advective fluxes)
    if (b->diffuse) launch_diffuse_batch<T>(descs<T>(b, l), L.nblk, L.ncols, rs, ro, cdt, fin, s);
    if (fin) {
        if (l > 0 && b->lev[l - 1].nslot > 0) {  // this level is the fine side of level l-1's interfaces
            const Level &C = b->lev[l - 1];
            hipLaunchKernelGGL(k_flux_accumulate<T>, dim3(blocks_for(C.nslot, 64)), dim3(64), 0, s, descs<T>(b, l), rs,
                               (const FluxSlot *)(b->ws + C.slot_off), C.nslot, dt, (double *)(b->ws + C.reg_off), st);
        }
        if (L.ncorr > 0)
            hipLaunchKernelGGL(k_flux_correct<T>, dim3(blocks_for(L.ncorr, 64)), dim3(64), 0, s, descs<T>(b, l), rs, ro,
                               (const CorrEnt *)(b->ws + L.corr_off), L.ncorr, dt, (double *)(b->ws + L.reg_off), st);
    }
    // ghost cells of the same level were not updated: they take their owners' values before the
    // diagnostics (whose nearest-plane walk reads neighbouring columns: every listed ghost cell) and
    // again after them (the ghost cells the next stage's update reads: the near ones)
    auto refill = [&](int nch) {
        if (nch > 0)
            hipLaunchKernelGGL(k_ghost_fill<T>, dim3(blocks_for(nch, 256 / FILL_CHUNK)), dim3(256), 0, s,
                               descs<T>(b, l), ro, descs<T>(b, l), ro, (const GhostChunk *)(b->ws + L.same_ch),
                               (const GhostPair *)(b->ws + L.same_off), nch, (int)FILL_COPY);
    };
    refill(L.csame);
    hipLaunchKernelGGL(k_diagnose_batch<T>, dim3(blocks_for(L.ncols, DIAG_COLS)), dim3(DIAG_THREADS), 0, s, descs<T>(b, l), L.nblk,
                       L.ncols, ro, st);
    refill(L.csame_near);
}

// one step of level l (dt), preceded by two steps of level l+1 and followed by the exchange with it
template <typename T>
void level_step(cc_batch_s *b, int l, double dt, int64_t *st, hipStream_t s)
{
    int nl = (int)b->lev.size();
    if (l + 1 < nl) {
        level_step<T>(b, l + 1, 0.5 * dt, st, s);
        level_step<T>(b, l + 1, 0.5 * dt, st, s);
    }
    Level &L = b->lev[l];
    int a = L.cur, o = 1 - L.cur, c = 2;
    level_stage<T>(b, l, a, a, o, dt / 3.0, 0, dt, st, s);
    level_stage<T>(b, l, a, o, c, dt / 2.0, 0, dt, st, s);
    level_stage<T>(b, l, a, c, o, dt, 1, dt, st, s);
    L.cur = o;
    if (l + 1 < nl) {
        fill<T>(b, l, l + 1, L.res_ch, L.res_off, L.cres, FILL_RESTRICT, s);  // level l <- level l+1
        const Level &F = b->lev[l + 1];
        fill<T>(b, l + 1, l, F.inj_ch, F.inj_off, F.cinj, FILL_INJECT, s);    // level l+1 <- level l
    }
}

template <typename T>
void batch_enqueue(cc_batch_s *b, double dt, int nsteps, int64_t *st, hipStream_t s)
{
    for (int n = 0; n < nsteps; ++n) level_step<T>(b, 0, dt, st, s);
}

void enqueue(cc_batch_s *b, double dt, int nsteps, int64_t *st, hipStream_t s)
{
    if (b->prec == CC_F64) batch_enqueue<double>(b, dt, nsteps, st, s);
    else batch_enqueue<float>(b, dt, nsteps, st, s);
}

// all ghost cells from the current states: same level, coarse-to-fine and fine-to-coarse
template <typename T>
void sync_all(cc_batch_s *b, hipStream_t s)
{
    int nl = (int)b->lev.size();
    for (int l = 0; l < nl; ++l) {
        const Level &L = b->lev[l];
        fill<T>(b, l, l, L.same_ch, L.same_off, L.csame, FILL_COPY, s);
        if (l + 1 < nl) fill<T>(b, l, l + 1, L.res_ch, L.res_off, L.cres, FILL_RESTRICT, s);
        if (l > 0) fill<T>(b, l, l - 1, L.inj_ch, L.inj_off, L.cinj, FILL_INJECT, s);
    }
}

// ------------------------------------------------------------------------------------------------
// host: descriptors and refill / flux-matching tables
// ------------------------------------------------------------------------------------------------
struct Tables {
    std::vector<std::vector<int>> members;  // block ids per level
    std::vector<int> local;                 // block id -> number within its level
    std::vector<std::vector<GhostEnt>> same, inj, res;
    std::vector<std::vector<FluxSlot>> slots;
    std::vector<std::vector<CorrEnt>> corr;
    std::vector<std::array<int, 6>> range;  // per block: cells to update [lo, hi) (empty: the whole grid)
    std::vector<int> near;                  // per level: same-level entries within NEAR_GHOST (listed first)
};

inline int64_t pmod(int64_t a, int64_t n) { a %= n; return a < 0 ? a + n : a; }

// owner map of one level: the block number owning each unit box of the level's cells
struct OwnerMap {
    int64_t N[3] = {0, 0, 0}, u[3] = {1, 1, 1}, nu[3] = {0, 0, 0};
    std::vector<int32_t> own;
    int at(int64_t x, int64_t y, int64_t z) const  // x, y periodic; z must be in range
    {
        if (z < 0 || z >= N[2]) return -1;
        x = pmod(x, N[0]); y = pmod(y, N[1]);
        return own[((x / u[0]) * nu[1] + y / u[1]) * nu[2] + z / u[2]];
    }
};

// Same-level ghost cells a stage reads, by distance (cells, along the furthest axis) from the cells
// whose values matter (the block's own cells and its ghost cells owned by other levels): the update
// reads up to two cells beyond them, three for the members and face corners of a merged group at
// their edge (NEAR_GHOST); the nearest-plane walk of the diagnostics reads predicted velocities up to
// four lattice points sideways, with the densities of the cells around them (DIAG_GHOST), and only
// at heights near the terrain (below the block's highest diagnosed level plus DIAG_RISE).  Other
// ghost cells of the same level are never read by those cells and are not refilled (the update
// computes them with the rest of its box; their values are never used).
constexpr int NEAR_GHOST = 3, DIAG_GHOST = 5, DIAG_RISE = 8;

// cells of a box within Chebyshev distance r of a marked cell (separable: a window of 2r+1 per axis)
static std::vector<uint8_t> dilate(const std::vector<uint8_t> &m, int nx, int ny, int nz, int r)
{
    std::vector<uint8_t> a = m, b(m.size());
    const int n[3] = {nx, ny, nz};
    const int64_t st[3] = {(int64_t)ny * nz, nz, 1};
    for (int ax = 0; ax < 3; ++ax) {
        std::fill(b.begin(), b.end(), 0);
        for (int64_t c = 0; c < (int64_t)a.size(); ++c) {
            if (!a[c]) continue;
            const int pos = (int)((c / st[ax]) % n[ax]);
            const int lo = std::max(0, pos - r), hi = std::min(n[ax] - 1, pos + r);
            for (int q = lo; q <= hi; ++q) b[c + (int64_t)(q - pos) * st[ax]] = 1;
        }
        std::swap(a, b);
    }
    return a;
}

// ktop: per block, the level below which its diagnostics read (empty: every level, the upper bound
// of the table sizes)
bool build_tables(const cc_block *B, int n, const int32_t dom0[3], Tables &t, const char *what,
                  const std::vector<int> &ktop = {})
{
    int nl = 0;
    for (int m = 0; m < n; ++m) {
        if (B[m].level < 0 || B[m].level > 12) { set_error("%s: block %d has level %d", what, m, B[m].level); return false; }
        if ((int64_t)B[m].grid.nx * B[m].grid.ny * B[m].grid.nzs > GHOST_IDX_MASK) {
            set_error("%s: block %d: a box of %lld slots exceeds the 2^28 of a refill entry", what, m,
                      (long long)B[m].grid.nx * B[m].grid.ny * B[m].grid.nzs);
            return false;
        }
        nl = std::max(nl, B[m].level + 1);
    }
    t.members.assign(nl, {});
    t.local.assign(n, 0);
    for (int m = 0; m < n; ++m) {
        t.local[m] = (int)t.members[B[m].level].size();
        t.members[B[m].level].push_back(m);
    }
    for (int l = 0; l < nl; ++l)
        if (t.members[l].empty()) { set_error("%s: no block on level %d", what, l); return false; }
    const cc_block &R0 = B[t.members[0][0]];
    std::vector<OwnerMap> om(nl);
    for (int l = 0; l < nl; ++l) {
        OwnerMap &M = om[l];
        for (int a = 0; a < 3; ++a) {
            M.N[a] = (int64_t)dom0[a] << l;
            int64_t g = 0;
            for (int m : t.members[l]) {
                const cc_block &b = B[m];
                g = std::gcd(g, (int64_t)(b.org[a] + b.ilo[a]));
                g = std::gcd(g, (int64_t)(b.ihi[a] - b.ilo[a]));
            }
            g = std::gcd(g, M.N[a]);
            M.u[a] = g > 0 ? g : 1;
            M.nu[a] = M.N[a] / M.u[a];
        }
        M.own.assign((size_t)(M.nu[0] * M.nu[1] * M.nu[2]), -1);
        double f = (double)(1 << l);
        for (int m : t.members[l]) {
            const cc_block &b = B[m];
            const int box[3] = {b.grid.nx, b.grid.ny, b.grid.nz};
            const double sp[3] = {b.grid.dx, b.grid.dy, b.grid.dz}, sp0[3] = {R0.grid.dx, R0.grid.dy, R0.grid.dz};
            for (int a = 0; a < 3; ++a) {
                int64_t g0 = b.org[a] + b.ilo[a], g1 = b.org[a] + b.ihi[a];
                if (b.ilo[a] < 0 || b.ihi[a] > box[a] || b.ilo[a] >= b.ihi[a] || g0 < 0 || g1 > M.N[a]) {
                    set_error("%s: block %d: own cells [%d,%d) of a %d-cell box at origin %d leave the level-%d "
                              "domain of %lld cells", what, m, b.ilo[a], b.ihi[a], box[a], b.org[a], l, (long long)M.N[a]);
                    return false;
                }
                if (std::fabs(sp[a] * f - sp0[a]) > 1e-9 * sp0[a]) {
                    set_error("%s: block %d: spacing %g is not 2^-%d of level 0's %g", what, m, sp[a], l, sp0[a]);
                    return false;
                }
            }
            for (int64_t x = b.org[0] + b.ilo[0]; x < b.org[0] + b.ihi[0]; x += M.u[0])
                for (int64_t y = b.org[1] + b.ilo[1]; y < b.org[1] + b.ihi[1]; y += M.u[1])
                    for (int64_t z = b.org[2] + b.ilo[2]; z < b.org[2] + b.ihi[2]; z += M.u[2]) {
                        int32_t &o = M.own[((x / M.u[0]) * M.nu[1] + y / M.u[1]) * M.nu[2] + z / M.u[2]];
                        if (o >= 0) { set_error("%s: blocks %d and %d overlap on level %d", what, t.members[l][o], m, l); return false; }
                        o = t.local[m];
                    }
        }
    }
    // box index of global level-l cell g inside block m (g lies in m's own cells)
    auto box_index = [&](int m, int l, const int64_t g[3]) -> int32_t {
        const cc_block &b = B[m];
        int64_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = b.ilo[a] + pmod(g[a] - (b.org[a] + b.ilo[a]), om[l].N[a]);
        return (int32_t)((c[0] * b.grid.ny + c[1]) * b.grid.nzs + c[2]);
    };
    t.same.assign(nl, {}); t.inj.assign(nl, {}); t.res.assign(nl, {});
    t.slots.assign(nl, {}); t.corr.assign(nl, {});
    t.near.assign(nl, 0);
    // cells a block must update: its own cells and the ghost cells of other levels (integrated on
    // between refills); ghosts of the same level are refilled after every stage
    t.range.assign(n, {0, 0, 0, 0, 0, 0});
    for (int m = 0; m < n; ++m)
        t.range[m] = {B[m].ilo[0], B[m].ilo[1], B[m].ilo[2], B[m].ihi[0], B[m].ihi[1], B[m].ihi[2]};
    auto grow = [&](int m, int i, int j, int k) {
        std::array<int, 6> &r = t.range[m];
        r[0] = std::min(r[0], i); r[1] = std::min(r[1], j); r[2] = std::min(r[2], k);
        r[3] = std::max(r[3], i + 1); r[4] = std::max(r[4], j + 1); r[5] = std::max(r[5], k + 1);
    };
    for (int l = 0; l < nl; ++l) {
        std::vector<GhostEnt> far;  // same-level entries read by the diagnostics only
        for (int m : t.members[l]) {
            const cc_block &b = B[m];
            std::vector<std::array<int, 3>> at;  // box position of each same-level entry of this block
            const size_t first = t.same[l].size();
            // the cells whose values matter: own cells and ghost cells owned by another level
            const int bx = b.grid.nx, by = b.grid.ny, bz = b.grid.nz;
            std::vector<uint8_t> real((size_t)bx * by * bz, 0);
            auto mark = [&](int i, int j, int k) { real[((size_t)i * by + j) * bz + k] = 1; };
            for (int i = b.ilo[0]; i < b.ihi[0]; ++i)
                for (int j = b.ilo[1]; j < b.ihi[1]; ++j)
                    for (int k = b.ilo[2]; k < b.ihi[2]; ++k) mark(i, j, k);
            for (int i = 0; i < b.grid.nx; ++i)
                for (int j = 0; j < b.grid.ny; ++j)
                    for (int k = 0; k < b.grid.nz; ++k) {
                        if (i >= b.ilo[0] && i < b.ihi[0] && j >= b.ilo[1] && j < b.ihi[1] && k >= b.ilo[2] && k < b.ihi[2])
                            continue;
                        int64_t g[3] = {pmod(b.org[0] + i, om[l].N[0]), pmod(b.org[1] + j, om[l].N[1]), (int64_t)b.org[2] + k};
                        if (g[2] < 0 || g[2] >= om[l].N[2]) continue;
                        int32_t didx = (int32_t)(((int64_t)i * b.grid.ny + j) * b.grid.nzs + k);
                        int o = om[l].at(g[0], g[1], g[2]);
                        if (o >= 0) {
                            t.same[l].push_back({t.local[m], didx, o, box_index(t.members[l][o], l, g)});
                            at.push_back({i, j, k});
                            continue;
                        }
                        if (l > 0) {
                            int64_t gc[3] = {g[0] >> 1, g[1] >> 1, g[2] >> 1};
                            int oc = om[l - 1].at(gc[0], gc[1], gc[2]);
                            if (oc >= 0) {
                                const int32_t par = (int32_t)((g[0] & 1) | ((g[1] & 1) << 1) | ((g[2] & 1) << 2));
                                t.inj[l].push_back({t.local[m], didx, oc, box_index(t.members[l - 1][oc], l - 1, gc), par});
                                grow(m, i, j, k);
                                mark(i, j, k);
                                continue;
                            }
                        }
                        if (l + 1 < nl) {
                            int64_t gf[3] = {2 * g[0], 2 * g[1], 2 * g[2]};
                            int of = om[l + 1].at(gf[0], gf[1], gf[2]);
                            if (of >= 0) {
                                for (int c = 1; c < 8; ++c)
                                    if (om[l + 1].at(gf[0] + (c >> 2), gf[1] + ((c >> 1) & 1), gf[2] + (c & 1)) != of) {
                                        set_error("%s: the children of level-%d cell (%lld,%lld,%lld) are split between "
                                                  "blocks", what, l, (long long)g[0], (long long)g[1], (long long)g[2]);
                                        return false;
                                    }
                                t.res[l].push_back({t.local[m], didx, of, box_index(t.members[l + 1][of], l + 1, gf)});
                                grow(m, i, j, k);
                                mark(i, j, k);
                            }
                        }
                    }
            // keep the same-level entries a stage reads: the near ones in place, the diagnostic-only
            // ones aside
            const std::vector<uint8_t> near = dilate(real, bx, by, bz, NEAR_GHOST);
            const std::vector<uint8_t> diag = dilate(real, bx, by, bz, DIAG_GHOST);
            size_t w = first;
            for (size_t e = first; e < t.same[l].size(); ++e) {
                const std::array<int, 3> &p = at[e - first];
                const size_t c = ((size_t)p[0] * by + p[1]) * bz + p[2];
                if (near[c]) t.same[l][w++] = t.same[l][e];
                else if (diag[c] && (ktop.empty() || p[2] < ktop[m])) far.push_back(t.same[l][e]);
            }
            t.same[l].resize(w);
        }
        t.near[l] = (int)t.same[l].size();
        t.same[l].insert(t.same[l].end(), far.begin(), far.end());
        if (l + 1 >= nl) continue;
        // coarse-fine faces of level l's own cells
        for (int m : t.members[l]) {
            const cc_block &b = B[m];
            for (int i = b.ilo[0]; i < b.ihi[0]; ++i)
                for (int j = b.ilo[1]; j < b.ihi[1]; ++j)
                    for (int k = b.ilo[2]; k < b.ihi[2]; ++k) {
                        CorrEnt ce{t.local[m], (int32_t)(((int64_t)i * b.grid.ny + j) * b.grid.nzs + k), {-1, -1, -1, -1, -1, -1}};
                        bool any = false;
                        const int64_t g[3] = {(int64_t)b.org[0] + i, (int64_t)b.org[1] + j, (int64_t)b.org[2] + k};
                        for (int f = 0; f < 6; ++f) {
                            int a = f >> 1, sg = (f & 1) ? 1 : -1;
                            int64_t gn[3] = {g[0], g[1], g[2]};
                            gn[a] += sg;
                            if (a == 2 && (gn[2] < 0 || gn[2] >= om[l].N[2])) continue;
                            if (om[l].at(gn[0], gn[1], gn[2]) >= 0) continue;
                            int64_t gf[3] = {2 * gn[0], 2 * gn[1], 2 * gn[2]};
                            int of = om[l + 1].at(gf[0], gf[1], gf[2]);
                            if (of < 0) continue;
                            int fb = t.members[l + 1][of];
                            const cc_block &F = B[fb];
                            FluxSlot fs{of, a, {0, 0, 0, 0}};
                            int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;  // the two other axes, increasing
                            for (int s = 0; s < 4; ++s) {
                                int64_t c[3];
                                c[a] = gf[a] + (sg > 0 ? 0 : 1);  // the fine child next to the face
                                c[b1] = gf[b1] + (s & 1);
                                c[b2] = gf[b2] + (s >> 1);
                                if (om[l + 1].at(c[0], c[1], c[2]) != of) {
                                    set_error("%s: coarse-fine face of level-%d cell (%lld,%lld,%lld) has sub-faces in "
                                              "several fine blocks", what, l, (long long)g[0], (long long)g[1], (long long)g[2]);
                                    return false;
                                }
                                int32_t ci = box_index(fb, l + 1, c);
                                if (sg < 0) {  // the face is at the child's upper side: take the cell above it
                                    int64_t stride = a == 0 ? (int64_t)F.grid.ny * F.grid.nzs : (a == 1 ? F.grid.nzs : 1);
                                    ci = (int32_t)(ci + stride);
                                    int cc3[3] = {(int)(ci / ((int64_t)F.grid.ny * F.grid.nzs)), (int)((ci / F.grid.nzs) % F.grid.ny),
                                                  (int)(ci % F.grid.nzs)};
                                    const int fbox[3] = {F.grid.nx, F.grid.ny, F.grid.nz};
                                    if (cc3[a] >= fbox[a]) {
                                        set_error("%s: fine block %d has no ghost cell beyond its side", what, fb);
                                        return false;
                                    }
                                }
                                fs.idx[s] = ci;
                            }
                            ce.slot[f] = (int32_t)t.slots[l].size();
                            t.slots[l].push_back(fs);
                            any = true;
                        }
                        if (any) t.corr[l].push_back(ce);
                    }
        }
    }
    return true;
}

template <typename T>
bool build_descs(const cc_block *B, const std::vector<int> &ids, cc_prec prec, int TX, int TY, int TZ, int BX,
                 int BY, int BZ, bool own_range, const Tables &t, std::vector<char> &host, Level &L, const char *what)
{
    host.assign(sizeof(BlockDesc<T>) * ids.size(), 0);
    BlockDesc<T> *h = (BlockDesc<T> *)host.data();
    int tiles = 0, tilesr = 0, cols = 0;
    for (size_t m = 0; m < ids.size(); ++m) {
        const cc_block &b = B[ids[m]];
        Dims d; Geo G; Phy P;
        if (!make_views(what, &b.grid, &b.phys, &b.geom, b.base, prec, d, G, P)) return false;
        for (int r = 0; r < 3; ++r) {
            if (!state_ok(what, &b.q[r])) return false;
            if (sizeof(T) == 4 && (!b.q[r].rho_lo || !b.q[r].rth_lo)) {
                set_error("%s: the float form of a batch needs the low-order state arrays", what);
                return false;
            }
            h[m].q[r] = sout_of<T>(const_cast<cc_state *>(&b.q[r]));
        }
        h[m].d = d; h[m].G = G; h[m].P = P;
        const int box[3] = {d.nx, d.ny, d.nz};
        for (int a = 0; a < 3; ++a) {  // own cells and update range: from the tables for refined grids,
            h[m].ilo[a] = own_range ? b.ilo[a] : 0;             // the whole grid otherwise
            h[m].ihi[a] = own_range ? b.ihi[a] : box[a];
            h[m].rlo[a] = own_range ? t.range[ids[m]][a] : 0;
            h[m].rhi[a] = own_range ? t.range[ids[m]][3 + a] : box[a];
        }
        h[m].nbx = (h[m].rhi[0] - h[m].rlo[0] + TX - 1) / TX;
        h[m].nby = (h[m].rhi[1] - h[m].rlo[1] + TY - 1) / TY;
        h[m].nbz = (h[m].rhi[2] - h[m].rlo[2] + TZ - 1) / TZ;
        // band-point tiles: the range's levels below the highest column band top (every level when it
        // is unknown)
        const int kband = (G.kband >= 1 && G.kband <= d.nz) ? G.kband : d.nz;
        const int nlev = std::min(kband, h[m].rhi[2]) - h[m].rlo[2];
        h[m].nbxb = (h[m].rhi[0] - h[m].rlo[0] + BX - 1) / BX;
        h[m].nbyb = (h[m].rhi[1] - h[m].rlo[1] + BY - 1) / BY;
        h[m].nbzb = nlev > 0 ? (nlev + BZ - 1) / BZ : 0;
        // a whole-grid block whose stage workspace lists its band tiles in this shape takes the list
        const BandTile own = band_tile_of(d.nx, d.ny, d.nz);
        h[m].blist = !own_range && G.ws && G.nband >= 0 && own.bx == BX && own.by == BY && own.bz == BZ;
        h[m].tile0 = tiles;
        h[m].tile0r = tilesr;
        h[m].col0 = cols;
        tiles += h[m].blist ? G.nband : h[m].nbxb * h[m].nbyb * h[m].nbzb;
        tilesr += h[m].nbx * h[m].nby * h[m].nbz;
        cols += (h[m].rhi[0] - h[m].rlo[0]) * (h[m].rhi[1] - h[m].rlo[1]);
    }
    L.nblk = (int)ids.size();
    L.ntiles = tiles;
    L.ntilesr = tilesr;
    L.ncols = cols;
    return true;
}

// tile shape of a batch: the requested one if every block holds a tile in x and y; a streaming form
// (TX = its chunk of planes) for batches of whole grids when its planes fit in LDS
int batch_tile(const cc_block *B, int n, int tile, bool own_range, int prec_bytes, int &TX, int &TY, int &TZ)
{
    auto offsets_fit = [&] {
        for (int m = 0; m < n; ++m)
            if (!stream_offsets_fit(B[m].grid.nx, B[m].grid.ny, B[m].grid.nzs, prec_bytes)) return false;
        return true;
    };
    if (!own_range && stream_shape(tile, prec_bytes, TY, TZ, TX) && offsets_fit()) return tile;
    auto fits = [&](int tx, int ty) {
        for (int m = 0; m < n; ++m)
            if (B[m].grid.nx < tx || B[m].grid.ny < ty) return false;
        return true;
    };
    int id = (tile == 1 || tile == 6 || tile == 7 || tile == 8 || tile == 9 || tile == 11 || tile == 12) ? tile : 0;
    auto shape = [&](int i) {
        TX = (i == 1 || i == 6 || i == 11 || i == 12) ? 4 : (i == 8 ? 2 : 8);
        TY = (i == 1 || i == 6 || i == 11) ? 4 : (i == 8 ? 2 : 8);
        TZ = i == 6 ? 32 : ((i == 1 || i == 7 || i == 11 || i == 12) ? 16 : (i == 8 ? 64 : 8));
    };
    shape(id);
    if (!fits(TX, TY)) { id = fits(4, 4) ? 1 : 8; shape(id); }
    return id;
}

// one-wave tile shape of the band-point launch: 8x8x1 if every block holds it in x and y, else 4x4x4,
// else 2x2x16
int band_tile(const cc_block *B, int n, int &BX, int &BY, int &BZ)
{
    int id = 0;
    for (int m = 0; m < n; ++m) {
        if (B[m].grid.nx < 4 || B[m].grid.ny < 4) id = 2;
        else if ((B[m].grid.nx < 8 || B[m].grid.ny < 8) && id < 1) id = 1;
    }
    BX = id == 0 ? 8 : (id == 1 ? 4 : 2);
    BY = BX;
    BZ = id == 0 ? 1 : (id == 1 ? 4 : 16);
    return id;
}

// a refill list packed for the device: entries [0, nfirst) and [nfirst, n) are each ordered by
// (destination, source) block pair (stably, so box order is kept within a pair) and cut into chunks
// of at most FILL_CHUNK entries of one pair; the first part's chunks come first
struct Packed {
    std::vector<GhostPair> pairs;
    std::vector<GhostChunk> chunks;
    int nchunks_first = 0;
};

static Packed pack(const std::vector<GhostEnt> &v, size_t nfirst)
{
    Packed p;
    auto part = [&](size_t lo, size_t hi) {
        std::vector<GhostEnt> e(v.begin() + lo, v.begin() + hi);
        std::stable_sort(e.begin(), e.end(), [](const GhostEnt &a, const GhostEnt &b) {
            return a.dblk != b.dblk ? a.dblk < b.dblk : a.sblk < b.sblk;
        });
        for (size_t a = 0; a < e.size();) {
            size_t z = a;
            while (z < e.size() && z - a < (size_t)FILL_CHUNK && e[z].dblk == e[a].dblk && e[z].sblk == e[a].sblk) ++z;
            p.chunks.push_back({e[a].dblk, e[a].sblk, (int32_t)p.pairs.size(), (int32_t)(z - a)});
            for (size_t q = a; q < z; ++q) p.pairs.push_back({e[q].didx | (e[q].par << GHOST_PAR_SHIFT), e[q].sidx});
            a = z;
        }
    };
    part(0, nfirst);
    p.nchunks_first = (int)p.chunks.size();
    part(nfirst, v.size());
    return p;
}

// layout of the workspace and (when `b` is given) the host images to upload
struct Plan {
    size_t bytes = 0;
    std::vector<std::vector<char>> desc;
    std::vector<Packed> same, inj, res;  // per level
};

bool plan_batch(const cc_block *B, int n, cc_prec prec, int tile, bool own_range, const Tables &t, cc_batch_s *b,
                Plan &plan, const char *what)
{
    int TX, TY, TZ, BX, BY, BZ;
    int id = batch_tile(B, n, tile, own_range, prec == CC_F64 ? 8 : 4, TX, TY, TZ);
    int bid = band_tile(B, n, BX, BY, BZ);
    int nl = (int)t.members.size();
    std::vector<Level> lev(nl);
    plan.desc.assign(nl, {});
    plan.same.assign(nl, {}); plan.inj.assign(nl, {}); plan.res.assign(nl, {});
    size_t off = 0;
    for (int l = 0; l < nl; ++l) {
        bool ok = prec == CC_F64
                      ? build_descs<double>(B, t.members[l], prec, TX, TY, TZ, BX, BY, BZ, own_range, t, plan.desc[l],
                                            lev[l], what)
                      : build_descs<float>(B, t.members[l], prec, TX, TY, TZ, BX, BY, BZ, own_range, t, plan.desc[l],
                                           lev[l], what);
        if (!ok) return false;
        lev[l].desc_off = off;
        off = align256(off + plan.desc[l].size());
    }
    for (int l = 0; l < nl; ++l) {
        Level &L = lev[l];
        L.nsame = (int)t.same[l].size();
        L.nsame_near = t.near.empty() ? L.nsame : t.near[l];
        L.ninj = (int)t.inj[l].size();
        L.nres = (int)t.res[l].size();
        plan.same[l] = pack(t.same[l], (size_t)L.nsame_near);
        plan.inj[l] = pack(t.inj[l], t.inj[l].size());
        plan.res[l] = pack(t.res[l], t.res[l].size());
        auto put = [&](const Packed &p, size_t &ch, size_t &pe, int &nch) {
            nch = (int)p.chunks.size();
            ch = off; off = align256(off + sizeof(GhostChunk) * p.chunks.size());
            pe = off; off = align256(off + sizeof(GhostPair) * p.pairs.size());
        };
        put(plan.same[l], L.same_ch, L.same_off, L.csame);
        L.csame_near = plan.same[l].nchunks_first;
        put(plan.inj[l], L.inj_ch, L.inj_off, L.cinj);
        put(plan.res[l], L.res_ch, L.res_off, L.cres);
        L.nslot = (int)t.slots[l].size(); L.slot_off = off; off = align256(off + sizeof(FluxSlot) * L.nslot);
        L.ncorr = (int)t.corr[l].size(); L.corr_off = off; off = align256(off + sizeof(CorrEnt) * L.ncorr);
        L.reg_off = off; off = align256(off + sizeof(double) * 2 * L.nslot);
    }
    plan.bytes = off;
    if (b) {
        b->prec = prec;
        b->tile = id;
        b->btile = bid;
        b->lev = lev;
        b->diffuse = false;
        for (int m = 0; m < n; ++m)
            b->diffuse = b->diffuse || B[m].phys.kdh != 0.0 || B[m].phys.kdv != 0.0 || B[m].phys.rsp != 0.0;
    }
    return true;
}

// side stream and fork/join events of a batch; without them the band launches stay on the stepping
// stream
void make_side(cc_batch_s *b)
{
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess) { b->side = nullptr; return; }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(b->side);
        b->side = nullptr;
    }
}

bool upload(cc_batch_s *b, const Plan &plan, const Tables *t, hipStream_t s, const char *what)
{
    hipError_t e = hipSuccess;
    int nl = (int)b->lev.size();
    for (int l = 0; l < nl && e == hipSuccess; ++l) {
        const Level &L = b->lev[l];
        e = hipMemcpyAsync(b->ws + L.desc_off, plan.desc[l].data(), plan.desc[l].size(), hipMemcpyHostToDevice, s);
        if (!t) continue;
        auto put = [&](size_t off, const void *p, size_t nb) {
            if (e == hipSuccess && nb) e = hipMemcpyAsync(b->ws + off, p, nb, hipMemcpyHostToDevice, s);
        };
        put(L.same_ch, plan.same[l].chunks.data(), sizeof(GhostChunk) * plan.same[l].chunks.size());
        put(L.same_off, plan.same[l].pairs.data(), sizeof(GhostPair) * plan.same[l].pairs.size());
        put(L.inj_ch, plan.inj[l].chunks.data(), sizeof(GhostChunk) * plan.inj[l].chunks.size());
        put(L.inj_off, plan.inj[l].pairs.data(), sizeof(GhostPair) * plan.inj[l].pairs.size());
        put(L.res_ch, plan.res[l].chunks.data(), sizeof(GhostChunk) * plan.res[l].chunks.size());
        put(L.res_off, plan.res[l].pairs.data(), sizeof(GhostPair) * plan.res[l].pairs.size());
        put(L.slot_off, t->slots[l].data(), sizeof(FluxSlot) * L.nslot);
        put(L.corr_off, t->corr[l].data(), sizeof(CorrEnt) * L.ncorr);
        if (e == hipSuccess && L.nslot) e = hipMemsetAsync(b->ws + L.reg_off, 0, sizeof(double) * 2 * L.nslot, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host images are freed on return
    if (e != hipSuccess) { set_error("%s: %s", what, hipGetErrorString(e)); return false; }
    return true;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// entry points
// ------------------------------------------------------------------------------------------------
extern "C" size_t amr_batch_workspace_bytes(int32_t nblocks, cc_prec prec)
{
    size_t one = prec == CC_F64 ? sizeof(BlockDesc<double>) : sizeof(BlockDesc<float>);
    return align256(one * (size_t)(nblocks > 0 ? nblocks : 0));
}

extern "C" cc_status amr_batch_create(const cc_block *blocks, int32_t nblocks, cc_prec prec, int32_t tile,
                                      void *workspace, cc_batch *out, cc_stream_t stream)
{
    CC_REQUIRE(blocks && nblocks > 0 && workspace && out, "amr_batch_create: null or empty argument");
    CC_REQUIRE(prec == CC_F64 || prec == CC_F32_PERT, "amr_batch_create: unknown precision");
    for (int m = 0; m < nblocks; ++m)
        CC_REQUIRE(blocks[m].level == 0, "amr_batch_create: block %d has level %d; a batch of independent domains "
                                         "holds level-0 blocks only (refined grids: amr_hierarchy_create)", m, blocks[m].level);
    Tables t;
    t.members.assign(1, {});
    for (int m = 0; m < nblocks; ++m) t.members[0].push_back(m);
    t.same.assign(1, {}); t.inj.assign(1, {}); t.res.assign(1, {}); t.slots.assign(1, {}); t.corr.assign(1, {});
    t.near.assign(1, 0);
    cc_batch_s *b = new cc_batch_s();
    Plan plan;
    if (!plan_batch(blocks, nblocks, prec, tile, false, t, b, plan, "amr_batch_create")) { delete b; return CC_EINVAL; }
    b->ws = (char *)workspace;
    make_side(b);
    if (!upload(b, plan, nullptr, (hipStream_t)stream, "amr_batch_create")) { amr_batch_destroy(b); return CC_EDEVICE; }
    *out = b;
    return CC_OK;
}

extern "C" cc_status amr_hierarchy_workspace_bytes(const cc_block *blocks, int32_t nblocks, cc_prec prec,
                                                   const int32_t domain0[3], size_t *bytes)
{
    CC_REQUIRE(blocks && nblocks > 0 && domain0 && bytes, "amr_hierarchy_workspace_bytes: null or empty argument");
    CC_REQUIRE(prec == CC_F64 || prec == CC_F32_PERT, "amr_hierarchy_workspace_bytes: unknown precision");
    Tables t;
    if (!build_tables(blocks, nblocks, domain0, t, "amr_hierarchy_workspace_bytes")) return CC_EINVAL;
    Plan plan;
    if (!plan_batch(blocks, nblocks, prec, 0, true, t, nullptr, plan, "amr_hierarchy_workspace_bytes")) return CC_EINVAL;
    *bytes = plan.bytes;
    return CC_OK;
}

extern "C" cc_status amr_hierarchy_create(const cc_block *blocks, int32_t nblocks, cc_prec prec, int32_t tile,
                                          const int32_t domain0[3], void *workspace, size_t workspace_bytes,
                                          cc_batch *out, cc_stream_t stream)
{
    CC_REQUIRE(blocks && nblocks > 0 && domain0 && workspace && out, "amr_hierarchy_create: null or empty argument");
    CC_REQUIRE(prec == CC_F64 || prec == CC_F32_PERT, "amr_hierarchy_create: unknown precision");
    CC_REQUIRE(domain0[0] > 0 && domain0[1] > 0 && domain0[2] > 0, "amr_hierarchy_create: empty level-0 domain");
    // the level below which each block's diagnostics read: its highest diagnosed level (column
    // bands written by cutcell_merge_map) plus DIAG_RISE
    std::vector<int> ktop(nblocks, 0);
    for (int m = 0; m < nblocks; ++m) {
        const cc_grid &g = blocks[m].grid;
        CC_REQUIRE(blocks[m].geom.colk, "amr_hierarchy_create: block %d has no column bands", m);
        std::vector<int32_t> ck((size_t)g.nx * g.ny);
        hipError_t e = hipMemcpyAsync(ck.data(), blocks[m].geom.colk + 2 * (size_t)g.nx * g.ny,
                                      sizeof(int32_t) * ck.size(), hipMemcpyDeviceToHost, (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) {
            set_error("amr_hierarchy_create: %s", hipGetErrorString(e));
            return CC_EDEVICE;
        }
        int top = 0;
        for (int32_t v : ck) top = std::max(top, (int)v);
        ktop[m] = top + DIAG_RISE;
    }
    Tables t;
    if (!build_tables(blocks, nblocks, domain0, t, "amr_hierarchy_create", ktop)) return CC_EINVAL;
    cc_batch_s *b = new cc_batch_s();
    Plan plan;
    if (!plan_batch(blocks, nblocks, prec, tile, true, t, b, plan, "amr_hierarchy_create")) { delete b; return CC_EINVAL; }
    if (plan.bytes > workspace_bytes) {
        set_error("amr_hierarchy_create: workspace of %zu bytes, %zu needed", workspace_bytes, plan.bytes);
        delete b;
        return CC_EINVAL;
    }
    b->ws = (char *)workspace;
    make_side(b);
    if (!upload(b, plan, &t, (hipStream_t)stream, "amr_hierarchy_create")) { amr_batch_destroy(b); return CC_EDEVICE; }
    *out = b;
    return CC_OK;
}

extern "C" cc_status amr_hierarchy_sync(cc_batch b, cc_stream_t stream)
{
    CC_REQUIRE(b, "amr_hierarchy_sync: null batch");
    if (b->prec == CC_F64) sync_all<double>(b, (hipStream_t)stream);
    else sync_all<float>(b, (hipStream_t)stream);
    return launch_status("amr_hierarchy_sync");
}

extern "C" cc_status amr_block_step(cc_batch b, double dt, int32_t nsteps, int32_t use_graph, int64_t *st,
                                    cc_stream_t stream)
{
    CC_REQUIRE(b && nsteps >= 0, "amr_block_step: bad batch or step count");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        enqueue(b, dt, nsteps, st, s);
        return launch_status("amr_block_step");
    }
    std::vector<int> cur0;
    for (const Level &L : b->lev) cur0.push_back(L.cur);
    for (auto &g : b->graphs)
        if (g.nsteps == nsteps && g.dt == dt && g.st == st && g.cur0 == cur0) {
            hipError_t e = hipGraphLaunch(g.exec, s);
            if (e != hipSuccess) { set_error("amr_block_step: %s", hipGetErrorString(e)); return CC_EDEVICE; }
            for (size_t l = 0; l < b->lev.size(); ++l) b->lev[l].cur = g.cur1[l];
            return CC_OK;
        }
    // capture the step sequence once on a private stream, then launch it on the caller's stream
    hipError_t e = hipSuccess;
    if (!b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue(b, dt, nsteps, st, b->cap);
        e = hipStreamEndCapture(b->cap, &graph);
    }
    std::vector<int> cur1;
    for (const Level &L : b->lev) cur1.push_back(L.cur);
    for (size_t l = 0; l < b->lev.size(); ++l) b->lev[l].cur = cur0[l];
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) {
        set_error("amr_block_step (graph): %s", hipGetErrorString(e));
        return CC_EDEVICE;
    }
    b->graphs.push_back({nsteps, dt, st, cur0, cur1, exec});
    for (size_t l = 0; l < b->lev.size(); ++l) b->lev[l].cur = cur1[l];
    return CC_OK;
}

extern "C" int32_t amr_batch_current(cc_batch b, int32_t level)
{
    if (!b || level < 0 || level >= (int32_t)b->lev.size()) return -1;
    return b->lev[level].cur;
}

extern "C" int32_t amr_batch_levels(cc_batch b) { return b ? (int32_t)b->lev.size() : 0; }

extern "C" cc_status amr_batch_info(cc_batch b, int32_t level, int64_t out[8])
{
    CC_REQUIRE(b && out && level >= 0 && level < (int32_t)b->lev.size(), "amr_batch_info: bad batch or level");
    const Level &L = b->lev[level];
    const int64_t v[8] = {L.nblk, L.ntilesr, L.ntiles, L.ncols, L.nsame, L.nsame_near, L.ninj, L.nres};
    for (int a = 0; a < 8; ++a) out[a] = v[a];
    return CC_OK;
}

extern "C" cc_status amr_batch_destroy(cc_batch b)
{
    if (!b) return CC_OK;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    delete b;
    return CC_OK;
}
