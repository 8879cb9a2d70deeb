// Streaming regular-point update (cc_stream.hip): declarations shared with the stage entry points.
#pragma once

#include "cc_kernels.hpp"

namespace cc {

// tile ids of the streaming form (TY x TZ threads over a j-k cross-section, chunks of CH planes in x,
// barriers per plane): 21 8x32, 32, 2; 22 8x32, 32, 1; 23 8x16, 32, 1; 24 8x32, 64, 2; 25 8x32, 64, 1;
// 26 8x16, 32, 2; 27 16x16, 32, 1; 28 16x16, 32, 2; 29 16x32, 32, 2
constexpr int STREAM_ID_MIN = 21, STREAM_ID_MAX = 29;

// True when every array of an nx x ny x nzs grid at prec_bytes per value stays within 4 GiB: the
// streaming kernels address it with 32-bit byte offsets.
bool stream_offsets_fit(int nx, int ny, int nzs, int prec_bytes);

// Launch the regular points (at or above their column's band top) of the update with streaming form
// `id` on stream s.  Returns false (and launches nothing) for an id that is not a streaming form, whose
// planes do not fit in the LDS of a workgroup in this precision, or whose arrays exceed 4 GiB.
template <typename T>
bool launch_stream(int id, const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                   cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s);

// Shape of streaming form `id` (TY x TZ threads, chunks of CH planes); false when `id` is not a
// streaming form or its planes do not fit in the LDS of a workgroup at prec_bytes per value.
bool stream_shape(int id, int prec_bytes, int &TY, int &TZ, int &CH);

// The regular points of a batch of whole grids (ensemble members) with streaming form `id`: desc is
// the level's BlockDesc<T> table, whose tile0r / nby / nbz count the streaming decomposition
// (CH-plane chunks x TY x TZ); ntiles workgroups in all.  Nothing is launched for a form that
// stream_shape refuses.
template <typename T>
void launch_stream_batch(int id, const void *desc, int nblk, int ntiles, int rn, int rs, int ro, double cdt,
                         int final_stage, int64_t *st, hipStream_t s);

}  // namespace cc
