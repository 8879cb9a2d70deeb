// Host-side plumbing of the C ABI: error text, argument checks, status mapping.
#include <cstring>
#include <string>

#include "cc_internal.hpp"

namespace cc {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

cc_status launch_status(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return CC_EDEVICE;
    }
    return CC_OK;
}

Dims dims_of(const cc_grid *g)
{
    return Dims{g->nx, g->ny, g->nz, g->nzs, g->dx, g->dy, g->dz, g->nsub, g->z0};
}

bool check_grid(const cc_grid *g)
{
    if (!g) { set_error("null grid"); return false; }
    if (g->nx < 2 || g->ny < 2 || g->nz < 3) {
        set_error("grid %dx%dx%d: need nx, ny >= 2 and nz >= 3", g->nx, g->ny, g->nz);
        return false;
    }
    if (!(g->z0 >= 0.0 && g->z0 < 1e7)) { set_error("grid bottom z0=%g out of range", g->z0); return false; }
    if (g->nzs < g->nz) { set_error("padded stride nzs=%d below nz=%d", g->nzs, g->nz); return false; }
    if (!(g->dx > 0.0 && g->dy > 0.0 && g->dz > 0.0)) { set_error("spacings must be positive"); return false; }
    if (g->nsub < 1 || g->nsub > 1024 || (g->nsub & (g->nsub - 1))) {
        set_error("nsub=%d must be a power of two in [1, 1024]", g->nsub);
        return false;
    }
    // the kernels form column and cell indices with 24-bit multiplies (__umul24): the column count
    // nx*ny and the padded stride must stay below 2^24
    if ((int64_t)g->nx * g->ny >= ((int64_t)1 << 24) || g->nzs >= (1 << 24)) {
        set_error("grid %dx%d columns (stride %d) exceeds the 2^24 column and stride limit", g->nx, g->ny, g->nzs);
        return false;
    }
    if ((int64_t)g->nx * g->ny * g->nzs >= ((int64_t)1 << 31)) {
        set_error("grid of %lld slots exceeds 32-bit cell indices", (long long)g->nx * g->ny * g->nzs);
        return false;
    }
    return true;
}

bool check_ptrs(const char *what, int n, const void *const *ptrs)
{
    for (int i = 0; i < n; ++i)
        if (!ptrs[i]) {
            set_error("%s: null array argument #%d", what, i);
            return false;
        }
    return true;
}

}  // namespace cc

extern "C" const char *cutcell_version(void) { return "libcutcell 0.1 (gfx950)"; }

extern "C" const char *cutcell_last_error(void) { return cc::g_last_error.c_str(); }

extern "C" cc_status cutcell_check_status(const int64_t *dev_status, int64_t *host, cc_stream_t stream)
{
    CC_REQUIRE(dev_status && host, "cutcell_check_status: null argument");
    hipError_t e = hipMemcpyAsync(host, dev_status, sizeof(int64_t) * CC_NSTATUS, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        cc::set_error("cutcell_check_status: %s", hipGetErrorString(e));
        return CC_EDEVICE;
    }
    if (host[cc::ST_UNMERGEABLE]) return CC_EUNMERGEABLE;
    if (host[cc::ST_NOPLANE]) return CC_ENOPLANE;
    if (host[cc::ST_NONFINITE]) return CC_ENONFINITE;
    if (host[cc::ST_TERRAIN] || host[cc::ST_GROUPSIZE] || host[cc::ST_INTERFACE]) return CC_ETERRAIN;
    return CC_OK;
}
