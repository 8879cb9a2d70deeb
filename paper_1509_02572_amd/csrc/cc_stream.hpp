// Streaming regular-point update (cc_stream.hip): declarations shared with the stage entry points.
#pragma once

#include "cc_kernels.hpp"

namespace cc {

// tile ids of the streaming form (TY x TZ threads over a j-k cross-section, chunks of CH planes in x,
// barriers per plane): 21 8x32, 32, 2; 22 8x32, 32, 1; 23 8x16, 32, 1; 24 8x32, 64, 2; 25 8x32, 64, 1;
// 26 8x16, 32, 2
constexpr int STREAM_ID_MIN = 21, STREAM_ID_MAX = 26;

// Launch the regular points (at or above their column's band top) of the update with streaming form
// `id` on stream s.  Returns false (and launches nothing) for an id that is not a streaming form or
// whose planes do not fit in the LDS of a workgroup in this precision.
template <typename T>
bool launch_stream(int id, const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                   cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s);

}  // namespace cc
