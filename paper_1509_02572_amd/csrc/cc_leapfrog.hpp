// Leap-frog time stepping with the Robert-Asselin filter in p' form (cc_leapfrog.hip): declarations
// shared with the stage entry points.
#pragma once

#include "cc_kernels.hpp"

namespace cc {

// Convert the thermodynamic slot of q in place at every non-solid cell through the equation of
// state: to_p != 0: (rho theta)' -> p', else p' -> (rho theta)' (low-order parts carried when q has
// them).
template <typename T>
void launch_pform(const Dims &d, const Geo &G, const Phy &P, cc_state *q, int to_p, hipStream_t s);

// (rho theta)' of the p' form state q into rthp (T, cells x nzs; 0 at solid cells) and zeros into
// z0 and, when not null, z1 (the thermodynamic slot and its low-order part of the q_n view).
template <typename T>
void launch_rthp(const Dims &d, const Geo &G, const Phy &P, const cc_state *q, T *rthp, T *z0, T *z1,
                 hipStream_t s);

// After the update of a leap-frog step: qp's thermodynamic slot (h x the (rho theta)' tendency) becomes
// qb's p' + (cp/cv) p / (rho theta) x that, p and rho theta of q0, at group masters; then, unless
// first, q0 += nu (qb - 2 q0 + qp) at group masters (rho', p') and predicted points (momentum).
// Non-finite p' counts into st[2].
template <typename T>
void launch_lf_finish(const Dims &d, const Geo &G, const Phy &P, const cc_state *qb, cc_state *q0, cc_state *qp,
                      double nu, int first, int64_t *st, hipStream_t s);

}  // namespace cc
