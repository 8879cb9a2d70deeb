// Explicit source terms applied after the update: the fourth-order artificial diffusion of the
// prognostic fields (the D terms of every equation of Sec. 2.1; 5-point stencils per direction,
// Sec. 2.2; a second-order term where the stencil lacks fluid neighbours, with the terrain as
// boundary, Sec. 2.4) and the sponge layer below the lid (Sec. 3).
//
// Diffusion, flux form.  Through a face between two cells (or lattice points) L and U along an axis,
// the flux is the third difference of the four values straddling it,
// phi(U+1) - 3 phi(U) + 3 phi(L) - phi(L-1), or -4 (phi(U) - phi(L)) when one of the two outer values
// is missing (a solid cell, a point that is not predicted, beyond the ground or the lid), and zero
// through a closed face; a point's term is -rate x (outgoing - incoming flux).  In the interior this
// is -rate x the 5-point fourth difference.  Scalars use group values (the master's), the faces'
// apertures and the group volume, as the advective fluxes do, and so stay conserved; momentum uses
// the perturbation from the reference flow, rho u - rhobar_c (u0, v0, 0), at predicted points.
// Evaluated in double in the order the CPU reference uses: members of a group from the master along
// gnext, faces -x,+x,-y,+y,-z,+z, axes x, y, z for momentum.  Where the cells and lattice points
// within two of the centre are regular (by the column band tops) the flux form collapses to the
// 5-point fourth differences in x and y and to the plain flux form along the column (shortened at
// the ground and the lid), which a launch of its own evaluates directly in the compute precision
// (float for the float form); a second launch takes the remaining points near the terrain in the
// general flux form.
//
// Sponge: Rayleigh damping -tau(z) q of (rho theta)' at group masters (cell-centre height) and of the
// momentum perturbation at predicted points (lattice height), tau = rsp sin^2(pi/2 (z - zsp)/(ztop -
// zsp)) above zsp; rho' is not damped.
//
// Launched after the update (or tendency) kernel, which it follows on the stream:
// q_out += scale x (D(q_s) + S(q_s)).  With the diffusion off, only the levels that reach into the
// sponge are launched.
#pragma clang fp contract(off)

#include "cc_diffuse.hpp"

namespace cc {

template <typename T>
__device__ __forceinline__ double group_value(const Geo &G, const SIn<T> &q, int64_t c, int w)
{
    const int32_t m = G.master[c];
    return w == 0 ? (double)q.rho[m] : (double)q.rth[m];
}

// flux of both scalars through the face between L = (i,j,k) - e_a and U = (i,j,k), along +a
template <typename T>
__device__ void scalar_diff_flux(const Dims &d, const Geo &G, const SIn<T> &q, int a, int i, int j, int k,
                                 double F[2])
{
    F[0] = F[1] = 0.0;
    if (a == 2 && (k - 1 < 0 || k >= d.nz)) return;  // ground and lid
    const int e0 = a == 0, e1 = a == 1, e2 = a == 2;
    const int64_t U = cidx(d, i, j, k), L = cidx(d, i - e0, j - e1, k - e2);
    const double A = a == 0 ? G.Ax[U] : (a == 1 ? G.Ay[U] : G.Az[U]);
    if (A == 0.0 || G.master[L] == G.master[U]) return;  // closed or internal face
    const int k2l = k - 2 * e2, k2u = k + e2;
    bool outer = k2l >= 0 && k2u < d.nz;
    int64_t L2 = 0, U2 = 0;
    if (outer) {
        L2 = cidx(d, i - 2 * e0, j - 2 * e1, k2l);
        U2 = cidx(d, i + e0, j + e1, k2u);
        outer = G.V[L2] > 0.0 && G.V[U2] > 0.0;
    }
    for (int w = 0; w < 2; ++w) {
        const double pl = group_value(G, q, L, w), pu = group_value(G, q, U, w);
        F[w] = outer ? ((group_value(G, q, U2, w) - 3.0 * pu) + 3.0 * pl) - group_value(G, q, L2, w)
                     : -4.0 * (pu - pl);
    }
}

__device__ __forceinline__ bool predicted(const Dims &d, const Geo &G, int I, int J, int K)
{
    return K >= 0 && K < d.nz && G.vcls[cidx(d, I, J, K)] == CC_PRED;
}

// momentum perturbation component c at lattice point p of level K
template <typename T>
__device__ __forceinline__ double mom_pert(const Phy &P, const SIn<T> &q, int64_t p, int K, int c)
{
    const double m = c == 0 ? (double)q.mu[p] : (c == 1 ? (double)q.mv[p] : (double)q.mw[p]);
    if (sizeof(T) == 4 || c == 2) return m;  // the float form stores the perturbation
    const double rbc = 0.5 * (P.rhob[K - 1] + P.rhob[K]);
    return m - rbc * (c == 0 ? P.u0 : P.v0);
}

// flux of the momentum perturbation through the face between lattice points P = (I,J,K) and P + e_a
template <typename T>
__device__ void lattice_diff_flux(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &q, int a, int I,
                                  int J, int K, double F[3])
{
    const int e0 = a == 0, e1 = a == 1, e2 = a == 2;
    F[0] = F[1] = F[2] = 0.0;
    if (!predicted(d, G, I, J, K) || !predicted(d, G, I + e0, J + e1, K + e2)) return;
    const int64_t p = cidx(d, I, J, K), qq = cidx(d, I + e0, J + e1, K + e2);
    const bool outer = predicted(d, G, I - e0, J - e1, K - e2) && predicted(d, G, I + 2 * e0, J + 2 * e1, K + 2 * e2);
    const int64_t p2 = outer ? cidx(d, I - e0, J - e1, K - e2) : 0, q2 = outer ? cidx(d, I + 2 * e0, J + 2 * e1, K + 2 * e2) : 0;
    for (int c = 0; c < 3; ++c) {
        const double mp = mom_pert(P, q, p, K, c), mq = mom_pert(P, q, qq, K + e2, c);
        F[c] = outer ? ((mom_pert(P, q, q2, K + 2 * e2, c) - 3.0 * mq) + 3.0 * mp) - mom_pert(P, q, p2, K - e2, c)
                     : -4.0 * (mq - mp);
    }
}

// sponge rate at height z: 0 below the layer
__device__ __forceinline__ double sponge_tau(const Phy &P, double z)
{
    if (P.rsp == 0.0 || z <= P.zsp || P.zsp >= P.ztop) return 0.0;
    const double s = sin(0.5 * 3.14159265358979323846 * (z - P.zsp) / (P.ztop - P.zsp));
    return P.rsp * (s * s);
}

// which parts of point (i, j, k) take the direct stencil, from the column band tops (colk: first k
// of the regular cells, first K of the predicted lattice points): the cell (ic) when the cells two
// apart in x and y at its level and those of its own column within two levels are regular; the
// lattice point (ip) when it is predicted and so are the points two apart in x and y at its level
// and those of its own column within two levels that exist.  Every level at or above kall (two above
// the band height) qualifies.
__device__ __forceinline__ void direct_parts(const Dims &d, const Geo &G, int i, int j, int k, int kall, bool &ic,
                                             bool &ip)
{
    if (k >= kall) { ic = ip = true; return; }
    const int64_t nc = (int64_t)d.nx * d.ny;
    int hc = 0, hl = 0;
    const int oi[8] = {-2, -1, 1, 2, 0, 0, 0, 0}, oj[8] = {0, 0, 0, 0, -2, -1, 1, 2};
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const int64_t cc = (int64_t)wrap(i + oi[n], d.nx) * d.ny + wrap(j + oj[n], d.ny);
        hc = max(hc, G.colk[cc]);
        hl = max(hl, G.colk[nc + cc]);
    }
    const int64_t c0 = (int64_t)i * d.ny + j;
    const int kc = G.colk[c0], kl = G.colk[nc + c0];
    ic = hc <= k && kc <= max(k - 2, 0);
    ip = hl <= k && kl <= k && kl <= max(k - 2, 1);
}

// add scale x (D + S) at one cell / lattice point
template <typename T>
__device__ __forceinline__ void apply_scalars(const SOut<T> &qo, int64_t c, double scale, int final_stage,
                                              double D0, double D1)
{
    double x0 = (double)qo.rho[c], x1 = (double)qo.rth[c];
    const bool lo = final_stage && qo.rho_lo;
    if (lo) {
        x0 += (double)qo.rho_lo[c];
        x1 += (double)qo.rth_lo[c];
    }
    x0 = x0 + scale * D0;
    x1 = x1 + scale * D1;
    const T a = (T)x0, b = (T)x1;
    qo.rho[c] = a;
    qo.rth[c] = b;
    if (lo) {
        qo.rho_lo[c] = (T)(x0 - (double)a);
        qo.rth_lo[c] = (T)(x1 - (double)b);
    }
}

// INNER: the direct-stencil launch over levels [k0, k1): the parts of each point direct_parts
// selects, 5-point fourth differences in x and y and the flux form along the column in z (where the
// ground and the lid shorten it), in the compute precision.  Otherwise the flux form over levels
// [k0, k1), for the parts the direct launch left (all of them when kall < 0).
template <typename T, bool INNER>
__device__ __forceinline__ void diffuse_point(const Dims &d, const Geo &G, const Phy &P, const SIn<T> &q,
                                              const SOut<T> &qo, double scale, int final_stage, int i, int j, int k,
                                              int kall)
{
    using R = typename Compute<T>::R;
    const int64_t col = (int64_t)i * d.ny + j;
    const int64_t c = col * d.nzs + k;
    const int nz = d.nz;
    const bool diff = P.kdh != 0.0 || P.kdv != 0.0;
    bool ic = false, ip = false;
    if (diff && kall >= 0) direct_parts(d, G, i, j, k, kall, ic, ip);
    const int8_t cl = G.cls[c];
    const bool master = cl == CC_OPEN || cl == CC_ORPHAN, pred = G.vcls[c] == CC_PRED;
    const double tau_c = sponge_tau(P, d.z0 + (k + 0.5) * d.dz);
    const double tau_p = sponge_tau(P, d.z0 + k * d.dz);
    if (INNER) {
        if (!ic && !(ip && pred)) return;
        int64_t xm[2], xp[2], ym[2], yp[2];
        if (i >= 2 && i + 2 < d.nx && j >= 2 && j + 2 < d.ny) {  // no periodic wrap: plain strides
            const int64_t sx = (int64_t)d.ny * d.nzs, sy = d.nzs;
            xm[0] = c - sx; xm[1] = c - 2 * sx; xp[0] = c + sx; xp[1] = c + 2 * sx;
            ym[0] = c - sy; ym[1] = c - 2 * sy; yp[0] = c + sy; yp[1] = c + 2 * sy;
        } else {
            xm[0] = cidx(d, i - 1, j, k); xm[1] = cidx(d, i - 2, j, k);
            xp[0] = cidx(d, i + 1, j, k); xp[1] = cidx(d, i + 2, j, k);
            ym[0] = cidx(d, i, j - 1, k); ym[1] = cidx(d, i, j - 2, k);
            yp[0] = cidx(d, i, j + 1, k); yp[1] = cidx(d, i, j + 2, k);
        }
        auto d4h = [&](auto v) {
            const R v0 = v(c);
            const R dx4 = (((v(xp[1]) - (R)4 * v(xp[0])) + (R)6 * v0) - (R)4 * v(xm[0])) + v(xm[1]);
            const R dy4 = (((v(yp[1]) - (R)4 * v(yp[0])) + (R)6 * v0) - (R)4 * v(ym[0])) + v(ym[1]);
            return dx4 + dy4;
        };
        if (ic) {  // a regular cell: its own master, V = 1, open faces
            R Dv[2];
            const T *f2[2] = {q.rho, q.rth};
            for (int w = 0; w < 2; ++w) {
                const T *f = f2[w];
                auto v = [&](int64_t p) { return (R)f[p]; };
                // z flux through the face at level ff (between ff-1 and ff); none through ground and lid
                auto Fz = [&](int ff) -> R {
                    if (ff <= 0 || ff >= nz) return (R)0;
                    const int64_t u = c + (ff - k), l = u - 1;
                    if (ff - 2 >= 0 && ff + 1 < nz) return (((R)f[u + 1] - (R)3 * (R)f[u]) + (R)3 * (R)f[l]) - (R)f[l - 1];
                    return (R)-4 * ((R)f[u] - (R)f[l]);
                };
                Dv[w] = -((R)P.kdh * d4h(v) + (R)P.kdv * (Fz(k + 1) - Fz(k)));
            }
            double D1 = (double)Dv[1];
            if (tau_c != 0.0) D1 += -tau_c * (double)q.rth[c];
            apply_scalars<T>(qo, c, scale, final_stage, (double)Dv[0], D1);
        }
        if (ip && pred) {
            const int64_t c0 = (int64_t)i * d.ny + j;
            const int kl = G.colk[(int64_t)d.nx * d.ny + c0];
            auto pk = [&](int K) { return K >= kl && K <= nz - 1; };  // predicted points of the column
            T *mo[3] = {qo.mu, qo.mv, qo.mw};
            for (int cc = 0; cc < 3; ++cc) {
                auto m = [&](int64_t p, int K) { return (R)mom_pert(P, q, p, K, cc); };
                auto v = [&](int64_t p) { return m(p, k); };
                // z flux between the points at levels ff and ff+1 of the column
                auto Gz = [&](int ff) -> R {
                    if (!pk(ff) || !pk(ff + 1)) return (R)0;
                    const int64_t a = c + (ff - k);
                    if (pk(ff - 1) && pk(ff + 2))
                        return ((m(a + 2, ff + 2) - (R)3 * m(a + 1, ff + 1)) + (R)3 * m(a, ff)) - m(a - 1, ff - 1);
                    return (R)-4 * (m(a + 1, ff + 1) - m(a, ff));
                };
                double S = (double)(-((R)P.kdh * d4h(v) + (R)P.kdv * (Gz(k) - Gz(k - 1))));
                if (tau_p != 0.0) S += -tau_p * mom_pert(P, q, c, k, cc);
                mo[cc][c] = (T)((double)mo[cc][c] + scale * S);
            }
        }
        return;
    }
    // ---- flux form: scalars at a group master ----
    if (!ic && master && (diff || tau_c != 0.0)) {
        double D0 = 0.0, D1 = 0.0;
        if (diff) {
            double acc[2] = {0.0, 0.0};
            int64_t mem = c;
            for (int guard = 0; mem >= 0 && guard <= CC_MAX_GROUP; ++guard) {
                int mi, mj, mk;
                unidx(d, mem, mi, mj, mk);
                for (int f = 0; f < 6; ++f) {
                    const int a = f >> 1, plus = f & 1;
                    const int fi = mi + (a == 0 && plus), fj = mj + (a == 1 && plus), fk = mk + (a == 2 && plus);
                    if (a == 2 && (fk <= 0 || fk >= d.nz)) continue;
                    const int64_t fu = cidx(d, fi, fj, fk);
                    const double A = a == 0 ? G.Ax[fu] : (a == 1 ? G.Ay[fu] : G.Az[fu]);
                    const double kr = a == 2 ? P.kdv : P.kdh;
                    double F[2];
                    scalar_diff_flux<T>(d, G, q, a, fi, fj, fk, F);
                    for (int w = 0; w < 2; ++w) {
                        const double term = (kr * A) * F[w];
                        acc[w] = plus ? acc[w] + term : acc[w] - term;
                    }
                }
                mem = G.gnext[mem];
            }
            const double vg = G.Vgroup[c];
            D0 = -acc[0] / vg;
            D1 = -acc[1] / vg;
        }
        if (tau_c != 0.0) D1 += -tau_c * (double)q.rth[c];
        apply_scalars<T>(qo, c, scale, final_stage, D0, D1);
    }
    // ---- flux form: momentum at a predicted point ----
    if (!ip && pred && (diff || tau_p != 0.0)) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int a = 0; diff && a < 3; ++a) {
            const double kr = a == 2 ? P.kdv : P.kdh;
            double Fp[3], Fm[3];
            lattice_diff_flux<T>(d, G, P, q, a, i, j, k, Fp);
            lattice_diff_flux<T>(d, G, P, q, a, i - (a == 0), j - (a == 1), k - (a == 2), Fm);
            for (int cc = 0; cc < 3; ++cc) acc[cc] += kr * (Fp[cc] - Fm[cc]);
        }
        double S[3] = {-acc[0], -acc[1], -acc[2]};
        if (tau_p != 0.0)
            for (int cc = 0; cc < 3; ++cc) S[cc] += -tau_p * mom_pert(P, q, c, k, cc);
        qo.mu[c] = (T)((double)qo.mu[c] + scale * S[0]);
        qo.mv[c] = (T)((double)qo.mv[c] + scale * S[1]);
        qo.mw[c] = (T)((double)qo.mw[c] + scale * S[2]);
    }
}

template <typename T, bool INNER>
__global__ void __launch_bounds__(256) k_diffuse(Dims d, Geo G, Phy P, SIn<T> q, SOut<T> qo, double scale,
                                                 int final_stage, int k0, int k1, int kall)
{
    const int nk = k1 - k0;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * nk) return;
    const int k = k0 + (int)(t % nk);
    const int64_t col = t / nk;
    diffuse_point<T, INNER>(d, G, P, q, qo, scale, final_stage, (int)(col / d.ny), (int)(col % d.ny), k, kall);
}

// Blocks of a batch: the diffusion in flux form and the sponge over each block's update range [rlo, rhi), whose
// columns are numbered from the block's col0 as for the batched diagnostics; DIFF_KS threads share a
// column, each taking every DIFF_KS-th level.
constexpr int DIFF_KS = 4;

template <typename T>
__global__ void __launch_bounds__(256) k_diffuse_batch(const BlockDesc<T> *__restrict__ desc, int nblk, int ncols,
                                                       int rs, int ro, double scale, int final_stage)
{
    const int t = blockIdx.x * (256 / DIFF_KS) + (int)(threadIdx.x / DIFF_KS);
    const int ks = threadIdx.x % DIFF_KS;
    if (t >= ncols) return;
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].col0 <= t) lo = mid;
        else hi = mid - 1;
    }
    const BlockDesc<T> &D = desc[lo];
    const int wy = D.rhi[1] - D.rlo[1], r = t - D.col0;
    const int i = D.rlo[0] + r / wy, j = D.rlo[1] + r % wy;
    const SIn<T> q = as_in(D.q[rs]);
    for (int k = D.rlo[2] + ks; k < D.rhi[2]; k += DIFF_KS)
        diffuse_point<T, false>(D.d, D.G, D.P, q, D.q[ro], scale, final_stage, i, j, k, -1);
}

template <typename T>
void launch_diffuse_batch(const void *desc, int nblk, int ncols, int rs, int ro, double scale, int final_stage,
                          hipStream_t s)
{
    if (ncols <= 0) return;
    hipLaunchKernelGGL(k_diffuse_batch<T>, dim3(blocks_for(ncols, 256 / DIFF_KS)), dim3(256), 0, s,
                       (const BlockDesc<T> *)desc, nblk, ncols, rs, ro, scale, final_stage);
}

template void launch_diffuse_batch<float>(const void *, int, int, int, int, double, int, hipStream_t);
template void launch_diffuse_batch<double>(const void *, int, int, int, int, double, int, hipStream_t);

template <typename T>
void launch_diffuse(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, cc_state *qo, double scale,
                    int final_stage, hipStream_t s)
{
    const bool diff = P.kdh != 0.0 || P.kdv != 0.0;
    const bool sponge = P.rsp != 0.0 && P.zsp < P.ztop;
    if (!diff && !sponge) return;
    const int64_t nc = (int64_t)d.nx * d.ny;
    if (!diff) {  // levels below the layer feel nothing: start one level under the first one reaching in
        const double kz = std::floor((P.zsp - d.z0) / d.dz) - 1.0;
        const int kmin = kz <= 0.0 ? 0 : (kz >= d.nz ? d.nz : (int)kz);
        if (kmin >= d.nz) return;
        hipLaunchKernelGGL((k_diffuse<T, false>), dim3(blocks_for(nc * (d.nz - kmin), 256)), dim3(256), 0, s, d, G,
                           P, sin_of<T>(qs), sout_of<T>(qo), scale, final_stage, kmin, d.nz, -1);
        return;
    }
    // the direct stencils over every level (every column from two levels above the band height, below
    // it where the column band tops allow), then the flux form for what they left below that height
    const int kall = (G.kband >= 1 && G.kband <= d.nz) ? G.kband + 2 : d.nz;
    hipLaunchKernelGGL((k_diffuse<T, true>), dim3(blocks_for(nc * d.nz, 256)), dim3(256), 0, s, d, G, P,
                       sin_of<T>(qs), sout_of<T>(qo), scale, final_stage, 0, d.nz, kall);
    const int kb = kall < d.nz ? kall : d.nz;
    hipLaunchKernelGGL((k_diffuse<T, false>), dim3(blocks_for(nc * kb, 256)), dim3(256), 0, s, d, G, P,
                       sin_of<T>(qs), sout_of<T>(qo), scale, final_stage, 0, kb, kall);
}

template void launch_diffuse<float>(const Dims &, const Geo &, const Phy &, const cc_state *, cc_state *, double,
                                    int, hipStream_t);
template void launch_diffuse<double>(const Dims &, const Geo &, const Phy &, const cc_state *, cc_state *, double,
                                     int, hipStream_t);

}  // namespace cc
