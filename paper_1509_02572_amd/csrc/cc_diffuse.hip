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
// gnext, faces -x,+x,-y,+y,-z,+z, axes x, y, z for momentum.  Where every cell and lattice point
// within two of the centre is regular (from two levels above the band height to three below the lid)
// the flux form collapses to the 5-point fourth difference, which a launch of its own evaluates
// directly; the flux form covers the levels below and above.
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

// interior form of the fourth difference along the three axes: -(kdh (d4x + d4y) + kdv d4z) of the
// values v(o) at offsets o from the centre (the flux form collapses to it where every cell and point
// within two of the centre is regular)
template <typename V>
__device__ __forceinline__ double interior_d4(const Phy &P, V v, int64_t c, const int64_t xm[2], const int64_t xp[2],
                                              const int64_t ym[2], const int64_t yp[2])
{
    const double v0 = v(c, 0);
    const double dx4 = (((v(xp[1], 0) - 4.0 * v(xp[0], 0)) + 6.0 * v0) - 4.0 * v(xm[0], 0)) + v(xm[1], 0);
    const double dy4 = (((v(yp[1], 0) - 4.0 * v(yp[0], 0)) + 6.0 * v0) - 4.0 * v(ym[0], 0)) + v(ym[1], 0);
    const double dz4 = (((v(c + 2, 2) - 4.0 * v(c + 1, 1)) + 6.0 * v0) - 4.0 * v(c - 1, -1)) + v(c - 2, -2);
    return -(P.kdh * (dx4 + dy4) + P.kdv * dz4);
}

// FAST: levels [k0, k1) where every cell and lattice point within two of the centre is regular
// (k >= band height + 2, k <= nz - 3), interior stencils; otherwise the flux form over levels
// [k0, k1) and [kt, nz).
template <typename T, bool FAST>
__global__ void __launch_bounds__(256) k_diffuse(Dims d, Geo G, Phy P, SIn<T> q, SOut<T> qo, double scale,
                                                 int final_stage, int k0, int k1, int kt)
{
    const int nlo = k1 - k0, nk = nlo + (FAST ? 0 : d.nz - kt);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * nk) return;
    const int l = (int)(t % nk);
    const int k = l < nlo ? k0 + l : kt + (l - nlo);
    const int64_t col = t / nk;
    const int j = (int)(col % d.ny), i = (int)(col / d.ny);
    const int64_t c = col * d.nzs + k;
    const bool diff = P.kdh != 0.0 || P.kdv != 0.0;
    // the flux-form launch takes the interior form too where the column band tops show every cell and
    // point within two of the centre regular (most columns away from the terrain)
    bool inner = FAST;
    if (!FAST && diff && k >= 2 && k <= d.nz - 3) {
        const int64_t nc = (int64_t)d.nx * d.ny;
        auto top = [&](int ii, int jj) {
            const int64_t cc = (int64_t)wrap(ii, d.nx) * d.ny + wrap(jj, d.ny);
            return max(G.colk[cc], G.colk[nc + cc]);
        };
        inner = k - 2 >= top(i, j) && k >= top(i - 1, j) && k >= top(i - 2, j) && k >= top(i + 1, j) &&
                k >= top(i + 2, j) && k >= top(i, j - 1) && k >= top(i, j - 2) && k >= top(i, j + 1) &&
                k >= top(i, j + 2);
    }
    int64_t xm[2], xp[2], ym[2], yp[2];
    if (inner) {
        xm[0] = cidx(d, i - 1, j, k); xm[1] = cidx(d, i - 2, j, k);
        xp[0] = cidx(d, i + 1, j, k); xp[1] = cidx(d, i + 2, j, k);
        ym[0] = cidx(d, i, j - 1, k); ym[1] = cidx(d, i, j - 2, k);
        yp[0] = cidx(d, i, j + 1, k); yp[1] = cidx(d, i, j + 2, k);
    }
    // ---- scalars at a group master ----
    const int8_t cl = G.cls[c];
    const double tau_c = sponge_tau(P, d.z0 + (k + 0.5) * d.dz);
    if ((cl == CC_OPEN || cl == CC_ORPHAN) && (diff || tau_c != 0.0)) {
        double D0 = 0.0, D1 = 0.0;
        if (inner) {
            D0 = interior_d4(P, [&](int64_t p, int) { return (double)q.rho[p]; }, c, xm, xp, ym, yp);
            D1 = interior_d4(P, [&](int64_t p, int) { return (double)q.rth[p]; }, c, xm, xp, ym, yp);
        } else if (diff) {
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
    // ---- momentum at a predicted point ----
    const double tau_p = sponge_tau(P, d.z0 + k * d.dz);
    if (G.vcls[c] == CC_PRED && (diff || tau_p != 0.0)) {
        double S[3] = {0.0, 0.0, 0.0};
        if (inner) {
            for (int cc = 0; cc < 3; ++cc)
                S[cc] = interior_d4(P, [&](int64_t p, int dk) { return mom_pert(P, q, p, k + dk, cc); }, c, xm, xp,
                                    ym, yp);
        } else if (diff) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 3; ++a) {
                const double kr = a == 2 ? P.kdv : P.kdh;
                double Fp[3], Fm[3];
                lattice_diff_flux<T>(d, G, P, q, a, i, j, k, Fp);
                lattice_diff_flux<T>(d, G, P, q, a, i - (a == 0), j - (a == 1), k - (a == 2), Fm);
                for (int cc = 0; cc < 3; ++cc) acc[cc] += kr * (Fp[cc] - Fm[cc]);
            }
            for (int cc = 0; cc < 3; ++cc) S[cc] = -acc[cc];
        }
        if (tau_p != 0.0)
            for (int cc = 0; cc < 3; ++cc) S[cc] += -tau_p * mom_pert(P, q, c, k, cc);
        qo.mu[c] = (T)((double)qo.mu[c] + scale * S[0]);
        qo.mv[c] = (T)((double)qo.mv[c] + scale * S[1]);
        qo.mw[c] = (T)((double)qo.mw[c] + scale * S[2]);
    }
}

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
                           P, sin_of<T>(qs), sout_of<T>(qo), scale, final_stage, kmin, d.nz, d.nz);
        return;
    }
    // interior levels [kf, nz - 2) when the band height is known, the flux form below and above
    int kf = d.nz, ke = d.nz;
    if (G.kband >= 1 && G.kband <= d.nz && G.kband + 2 < d.nz - 2) {
        kf = G.kband + 2;
        ke = d.nz - 2;
    }
    if (kf < ke)
        hipLaunchKernelGGL((k_diffuse<T, true>), dim3(blocks_for(nc * (ke - kf), 256)), dim3(256), 0, s, d, G, P,
                           sin_of<T>(qs), sout_of<T>(qo), scale, final_stage, kf, ke, ke);
    const int nslow = kf + (d.nz - ke);
    hipLaunchKernelGGL((k_diffuse<T, false>), dim3(blocks_for(nc * nslow, 256)), dim3(256), 0, s, d, G, P,
                       sin_of<T>(qs), sout_of<T>(qo), scale, final_stage, 0, kf, ke);
}

template void launch_diffuse<float>(const Dims &, const Geo &, const Phy &, const cc_state *, cc_state *, double,
                                    int, hipStream_t);
template void launch_diffuse<double>(const Dims &, const Geo &, const Phy &, const cc_state *, cc_state *, double,
                                     int, hipStream_t);

}  // namespace cc
