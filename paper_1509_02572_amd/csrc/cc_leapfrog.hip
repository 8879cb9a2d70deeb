// The paper's own time stepping (Sec. 2.2): leap-frog with the Robert-Asselin filter, with the
// perturbation pressure p' as the prognostic thermodynamic variable (Sec. 2.1, eq. heat).
//
// A state in p' form holds p' in the slot the (rho theta)' form uses for (rho theta)'.  One step
// (driven by cutcell_lf_step) runs the Runge-Kutta update kernels once, as a stage of step 2 dt:
// q_s = q(n) with (rho theta)' from its p' (equation of state), q_n = qbar(n-1) with a zero
// thermodynamic slot, so the update leaves qbar(n-1) + 2 dt L for rho' and the momentum and 2 dt times
// the (rho theta)' tendency in the thermodynamic slot (the diffusion and sponge launch adds its part
// as after any stage).  The finishing kernel below turns the latter into p' of q(n+1): qbar(n-1)'s p'
// plus (cp/cv) p / (rho theta) times it (the chain rule of p = p0 (R rho theta / p0)^(cp/cv), equal to
// the factor (cp/cv) R (p/p0)^(R/cp) of eq. heat, with p and rho theta of q(n)), and applies the
// filter qbar(n) = q(n) + nu (qbar(n-1) - 2 q(n) + q(n+1)).  The first step is a forward step (q_n =
// q(0), dt).  Per-cell arithmetic in double; the float form carries the low-order parts of rho' and
// p' through update, finish and filter, so mass stays conserved.
#pragma clang fp contract(off)

#include "cc_leapfrog.hpp"

namespace cc {

__device__ __forceinline__ double p_from_rth(double rthp, double rthbar, double pbar, double gam)
{
    return pbar * expm1(gam * log1p(rthp / rthbar));
}

__device__ __forceinline__ double rth_from_p(double pp, double rthbar, double pbar, double gam)
{
    return rthbar * expm1(log1p(pp / pbar) / gam);
}

template <typename T>
__device__ __forceinline__ double with_lo(const T *hi, const T *lo, int64_t c)
{
    return lo ? (double)hi[c] + (double)lo[c] : (double)hi[c];
}

template <typename T>
__device__ __forceinline__ void store_split(T *hi, T *lo, int64_t c, double x)
{
    const T a = (T)x;
    hi[c] = a;
    if (lo) lo[c] = (T)(x - (double)a);
}

template <typename T>
__global__ void __launch_bounds__(256) k_pform(Dims d, Geo G, Phy P, SOut<T> q, int to_p)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    const int k = (int)(t % d.nz);
    const int64_t c = (t / d.nz) * d.nzs + k;
    if (G.cls[c] == CC_SOLID) return;
    // a merged group's value belongs to its master: members convert with the master's level (they
    // mirror the master's value, so each thread converts its own copy)
    const int km = (int)(G.master[c] % d.nzs);
    const double x = with_lo<T>(q.rth, q.rth_lo, c);
    const double y = to_p ? p_from_rth(x, P.rthb[km], P.pb[km], P.gam) : rth_from_p(x, P.rthb[km], P.pb[km], P.gam);
    store_split<T>(q.rth, q.rth_lo, c, y);
}

// (rho theta)' of the p' form state q into rthp, and zeros into z0 (and z1 when given): the
// thermodynamic slot of the q_n view of the update
template <typename T>
__global__ void __launch_bounds__(256) k_rthp(Dims d, Geo G, Phy P, SIn<T> q, T *rthp, T *z0, T *z1)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    const int k = (int)(t % d.nz);
    const int64_t c = (t / d.nz) * d.nzs + k;
    if (G.cls[c] == CC_SOLID) {
        rthp[c] = (T)0;
    } else {
        const int km = (int)(G.master[c] % d.nzs);  // members convert with their master's level
        rthp[c] = (T)rth_from_p(with_lo<T>(q.rth, q.rth_lo, c), P.rthb[km], P.pb[km], P.gam);
    }
    z0[c] = (T)0;
    if (z1) z1[c] = (T)0;
}

// qp's thermodynamic slot holds h x the (rho theta)' tendency: make it qb's p' + coef x that; then,
// unless first, filter q0 with qb and qp
template <typename T>
__global__ void __launch_bounds__(256) k_lf_finish(Dims d, Geo G, Phy P, SIn<T> qb, SOut<T> q0, SOut<T> qp,
                                                   double nu, int first, int64_t *st)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    const int k = (int)(t % d.nz);
    const int64_t c = (t / d.nz) * d.nzs + k;
    const int8_t cl = G.cls[c];
    if (cl == CC_OPEN || cl == CC_ORPHAN) {
        const double p0 = with_lo<T>(q0.rth, q0.rth_lo, c), pbb = with_lo<T>(qb.rth, qb.rth_lo, c);
        const double coef = P.gam * (P.pb[k] + p0) / (P.rthb[k] + rth_from_p(p0, P.rthb[k], P.pb[k], P.gam));
        const double pn = pbb + coef * with_lo<T>(qp.rth, qp.rth_lo, c);
        store_split<T>(qp.rth, qp.rth_lo, c, pn);
        if (!isfinite(pn)) count_status(st, ST_NONFINITE);
        if (!first) {
            const double r0 = with_lo<T>(q0.rho, q0.rho_lo, c), rb = with_lo<T>(qb.rho, qb.rho_lo, c);
            const double rn = with_lo<T>(qp.rho, qp.rho_lo, c);
            store_split<T>(q0.rho, q0.rho_lo, c, r0 + nu * ((rb - 2.0 * r0) + rn));
            store_split<T>(q0.rth, q0.rth_lo, c, p0 + nu * ((pbb - 2.0 * p0) + pn));
        }
    }
    if (!first && G.vcls[c] == CC_PRED) {
        const T *mb[3] = {qb.mu, qb.mv, qb.mw};
        T *m0[3] = {q0.mu, q0.mv, q0.mw};
        const T *mp[3] = {qp.mu, qp.mv, qp.mw};
        for (int a = 0; a < 3; ++a) {
            const double x0 = (double)m0[a][c];
            m0[a][c] = (T)(x0 + nu * (((double)mb[a][c] - 2.0 * x0) + (double)mp[a][c]));
        }
    }
}

template <typename T>
void launch_pform(const Dims &d, const Geo &G, const Phy &P, cc_state *q, int to_p, hipStream_t s)
{
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_pform<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, G, P, sout_of<T>(q), to_p);
}

template <typename T>
void launch_rthp(const Dims &d, const Geo &G, const Phy &P, const cc_state *q, T *rthp, T *z0, T *z1,
                 hipStream_t s)
{
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_rthp<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, G, P, sin_of<T>(q), rthp, z0, z1);
}

template <typename T>
void launch_lf_finish(const Dims &d, const Geo &G, const Phy &P, const cc_state *qb, cc_state *q0, cc_state *qp,
                      double nu, int first, int64_t *st, hipStream_t s)
{
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_lf_finish<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, G, P, sin_of<T>(qb),
                       sout_of<T>(q0), sout_of<T>(qp), nu, first, st);
}

template void launch_pform<float>(const Dims &, const Geo &, const Phy &, cc_state *, int, hipStream_t);
template void launch_pform<double>(const Dims &, const Geo &, const Phy &, cc_state *, int, hipStream_t);
template void launch_rthp<float>(const Dims &, const Geo &, const Phy &, const cc_state *, float *, float *, float *,
                                 hipStream_t);
template void launch_rthp<double>(const Dims &, const Geo &, const Phy &, const cc_state *, double *, double *,
                                  double *, hipStream_t);
template void launch_lf_finish<float>(const Dims &, const Geo &, const Phy &, const cc_state *, cc_state *,
                                      cc_state *, double, int, int64_t *, hipStream_t);
template void launch_lf_finish<double>(const Dims &, const Geo &, const Phy &, const cc_state *, cc_state *,
                                       cc_state *, double, int, int64_t *, hipStream_t);

}  // namespace cc
