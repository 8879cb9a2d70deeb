// Internal declarations shared by the HIP translation units of libcutcell (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "cutcell.h"

namespace cc {

// Grid description passed by value to every kernel.
struct Dims {
    int nx, ny, nz, nzs;
    double dx, dy, dz;
    int nsub;
    double z0;  // height of the bottom face
};

__host__ __device__ __forceinline__ int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}
// linear index of cell / lattice point (i,j,k) with periodic i and j (k must be in range)
__host__ __device__ __forceinline__ int64_t cidx(const Dims &d, int i, int j, int k)
{
    return ((int64_t)wrap(i, d.nx) * d.ny + wrap(j, d.ny)) * d.nzs + k;
}
__host__ __device__ __forceinline__ int64_t hidx(const Dims &d, int i, int j)
{
    return (int64_t)wrap(i, d.nx) * d.ny + wrap(j, d.ny);
}
// inverse of cidx for an in-range linear index
__host__ __device__ __forceinline__ void unidx(const Dims &d, int64_t c, int &i, int &j, int &k)
{
    k = (int)(c % d.nzs);
    int64_t col = c / d.nzs;
    j = (int)(col % d.ny);
    i = (int)(col / d.ny);
}

// status counters (see cutcell.h)
enum { ST_UNMERGEABLE = 0, ST_NOPLANE = 1, ST_NONFINITE = 2, ST_TERRAIN = 3, ST_GROUPSIZE = 4, ST_INTERFACE = 5,
       ST_STALE = 6 };

// band top of a column from its cell band (one above its highest cell that is not regular) and its
// lattice band (one above its highest lattice point that is not predicted): the ground row K = 0 is
// never predicted, so a lattice band of 1 adds nothing.  Every point at or above the band top takes
// the regular update.
__host__ __device__ __forceinline__ int band_top(int kcell, int klat)
{
    const int kl = klat > 1 ? klat : 0;
    return kcell > kl ? kcell : kl;
}

// One-wave tiles of the band-point update: 8x8x1, or 4x4x4 / 2x2x16 on grids narrower than 8 / 4
// columns (the periodic index arithmetic wraps at most once)
struct BandTile { int bx, by, bz, nbx, nby, nbz; };
inline BandTile band_tile_of(int nx, int ny, int nz)
{
    BandTile t;
    if (nx >= 8 && ny >= 8) { t.bx = 8; t.by = 8; t.bz = 1; }
    else if (nx >= 4 && ny >= 4) { t.bx = 4; t.by = 4; t.bz = 4; }
    else { t.bx = 2; t.by = 2; t.bz = 16; }
    t.nbx = (nx + t.bx - 1) / t.bx;
    t.nby = (ny + t.by - 1) / t.by;
    t.nbz = (nz + t.bz - 1) / t.bz;
    return t;
}
// The stage workspace starts with the list of band tiles that hold band points (one int32 each),
// room for every tile of the grid, rounded up to 256 bytes; the two-pass arrays follow it.
inline size_t band_list_bytes(int nx, int ny, int nz)
{
    const BandTile t = band_tile_of(nx, ny, nz);
    const size_t b = sizeof(int32_t) * (size_t)t.nbx * t.nby * t.nbz;
    return (b + 255) / 256 * 256;
}

__device__ __forceinline__ void count_status(int64_t *st, int which, int64_t n = 1)
{
    if (st) atomicAdd(reinterpret_cast<unsigned long long *>(st + which), (unsigned long long)n);
}

void set_error(const char *fmt, ...);
cc_status launch_status(const char *what);
Dims dims_of(const cc_grid *g);
// host-side argument checks; on failure set the error text and return false
bool check_grid(const cc_grid *g);
bool check_ptrs(const char *what, int n, const void *const *ptrs);

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace cc

#define CC_REQUIRE(cond, ...)                  \
    do {                                       \
        if (!(cond)) {                         \
            ::cc::set_error(__VA_ARGS__);      \
            return CC_EINVAL;                  \
        }                                      \
    } while (0)
