// Fourth-order artificial diffusion (cc_diffuse.hip): declarations shared with the stage entry points.
#pragma once

#include "cc_kernels.hpp"

namespace cc {

// Add scale x (D(q_s) + S(q_s)) (diffusion and sponge) to q_out at group masters (rho', (rho theta)')
// and predicted lattice points (momentum) on stream s: scale = the stage's c dt after an update, 1
// after a tendency evaluation.
// final_stage: q_out's low-order parts (float form) are carried.  Nothing is launched when the
// diffusion rates and the sponge rate of P are all zero.
template <typename T>
void launch_diffuse(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, cc_state *qo, double scale,
                    int final_stage, hipStream_t s);

// The diffusion (flux form) and the sponge of a batch's blocks: scale x (D(q_s) + S(q_s)) added to
// q_out over every block's update range, desc being the level's BlockDesc<T> table whose col0 number
// the range's columns (ncols in all), rs / ro the state slots of q_s and q_out.
template <typename T>
void launch_diffuse_batch(const void *desc, int nblk, int ncols, int rs, int ro, double scale, int final_stage,
                          hipStream_t s);

}  // namespace cc
