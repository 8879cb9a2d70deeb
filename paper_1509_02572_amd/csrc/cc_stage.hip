// Uniform-grid entry points of the cut-cell stage (Sec. 2.4 of the paper): initial state,
// diagnostics, tendency, Runge-Kutta stage and the conservation sums, for both storage precisions.
#pragma clang fp contract(off)

#include <mutex>

#include "cc_kernels.hpp"
#include "cc_stream.hpp"
#include "cc_diffuse.hpp"
#include "cc_leapfrog.hpp"

namespace cc {

// ------------------------------------------------------------------------------------------------
// Stage context: the caller's side stream for the band-point launch of an update (the two launches
// of an update write disjoint points and read only the inputs, so they may run side by side).  Fork
// and join go through events, so a capture of the caller's stream takes the side stream's work in.
// ------------------------------------------------------------------------------------------------
}  // namespace cc

struct cc_stage_ctx_s {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

namespace cc {

// ------------------------------------------------------------------------------------------------
// Initial state: theta' at constant pressure on group masters, (rho theta)' = 0, inflow (u0, v0, 0)
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_init_cells(Dims d, Geo G, Phy P, const double *noise, SOut<T> q)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int k = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int64_t c = colI * d.nzs + k;
    int8_t cl = G.cls[c];
    double r = 0.0;
    if (cl == CC_OPEN || cl == CC_ORPHAN) {
        // rho' = (rho theta)bar/(thetabar + theta') - rhobar without the cancellation
        double thp = noise ? noise[c] : 0.0;
        r = thp != 0.0 ? -(P.rhob[k] * thp) / (P.thb[k] + thp) : 0.0;
    }
    q.rho[c] = (T)r;
    q.rth[c] = (T)0;
    if (q.rho_lo) { q.rho_lo[c] = (T)(r - (double)(T)r); q.rth_lo[c] = (T)0; }
    q.mu[c] = (T)0; q.mv[c] = (T)0; q.mw[c] = (T)0;
}

// perturbation form: m' = rho_c U0 - rhobar_c U0 = rho'_c (u0, v0, 0)
__global__ void k_init_momentum_pert(Dims d, Geo G, Phy P, SOut<float> q)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int K = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int J = (int)(colI % d.ny), I = (int)(colI / d.ny);
    int64_t p = cidx(d, I, J, K);
    if (G.vcls[p] != CC_PRED) return;
    double sp = 0.0;
    for (int s = 0; s < 8; ++s)
        sp += (double)q.rho[cidx(d, I - 1 + (s & 1), J - 1 + ((s >> 1) & 1), K - 1 + (s >> 2))];
    double rpc = 0.125 * sp;
    q.mu[p] = (float)(rpc * P.ux);
    q.mv[p] = (float)(rpc * P.vy);
    q.mw[p] = 0.0f;
}

// paper variables: momentum = mean of the eight surrounding cell densities x (u0, v0, 0)
__global__ void k_init_momentum_full(Dims d, Geo G, Phy P, double u0, double v0, SOut<double> q)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.nx * d.ny * d.nz) return;
    int K = (int)(t % d.nz);
    int64_t colI = t / d.nz;
    int J = (int)(colI % d.ny), I = (int)(colI / d.ny);
    int64_t p = cidx(d, I, J, K);
    if (G.vcls[p] != CC_PRED) return;
    auto rt = [&](int a, int b, int kk) { return P.rhob[kk] + q.rho[cidx(d, I + a, J + b, kk)]; };
    double s0 = (rt(-1, -1, K - 1) + rt(0, -1, K - 1)) + (rt(-1, 0, K - 1) + rt(0, 0, K - 1));
    double s1 = (rt(-1, -1, K) + rt(0, -1, K)) + (rt(-1, 0, K) + rt(0, 0, K));
    double rc = 0.125 * (s0 + s1);
    q.mu[p] = rc * u0;
    q.mv[p] = rc * v0;
    q.mw[p] = 0.0;
}

// ------------------------------------------------------------------------------------------------
// Conservation sums: fixed grid, fixed per-thread order, fixed tree -> bitwise reproducible.  Each
// thread sums its grid-stride cells in order; a wavefront combines its 64 lanes with a butterfly of
// cross-lane shuffles; the block's waves are then added in wave order, and the final pass adds the
// block partials the same way.  No float atomics.
// ------------------------------------------------------------------------------------------------
constexpr int RED_BLOCKS = 1024, RED_THREADS = 256, RED_WAVES = RED_THREADS / 64;

// sum of v over the 64 lanes of the wavefront (every lane receives the same bits: the butterfly
// adds the same pairs in the same order on every lane)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// the four sums of a block, in wave order, into out[0..3] (thread 0 writes)
__device__ __forceinline__ void block_sum4(double acc[4], double *out)
{
    __shared__ double sh[4][RED_WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double w = wave_sum(acc[a]);
        if (lane == 0) sh[a][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < RED_WAVES; ++w) t += sh[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_reduce_partial(Dims d, Geo G, Phy P, SIn<T> q,
                                                                double *part)
{
    using R = typename Compute<T>::R;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t n = (int64_t)d.nx * d.ny * d.nz;
    for (int64_t t = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; t < n;
         t += (int64_t)RED_BLOCKS * RED_THREADS) {
        int k = (int)(t % d.nz);
        int64_t colI = t / d.nz;
        int j = (int)(colI % d.ny), i = (int)(colI / d.ny);
        int64_t c = colI * d.nzs + k;
        int8_t cl = G.cls[c];
        if (cl == CC_OPEN || cl == CC_ORPHAN) {
            double vg = G.Vgroup[c] * P.dV;
            double rp = (double)q.rho[c], tp = (double)q.rth[c];
            if (q.rho_lo) { rp += (double)q.rho_lo[c]; tp += (double)q.rth_lo[c]; }
            double rho = P.rhob[k] + rp;
            double p = P.pb[k] + P.pb[k] * expm1(P.gam * log1p(tp / P.rthb[k]));
            double z = d.z0 + ((double)k + 0.5) * d.dz;
            acc[0] += vg * rp;
            acc[1] += vg * tp;
            acc[2] += vg * rho;
            acc[3] += vg * (p / (P.gam - 1.0) + rho * P.g * z);
        }
        if (G.vcls[c] == CC_PRED) {
            R u[3];
            lat_vel<T>(d, G, P, q, i, j, k, u);
            double rpc = 0.0;
            for (int s = 0; s < 8; ++s)
                rpc += (double)q.rho[cidx(d, i - 1 + (s & 1), j - 1 + ((s >> 1) & 1), k - 1 + (s >> 2))];
            double rc = 0.5 * (P.rhob[k - 1] + P.rhob[k]) + 0.125 * rpc;
            double uu = (double)u[0] + P.ux, vv = (double)u[1] + P.vy, ww = (double)u[2];
            acc[3] += P.dV * 0.5 * rc * (uu * uu + vv * vv + ww * ww);
        }
    }
    block_sum4(acc, part + (int64_t)blockIdx.x * 4);
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_final(const double *part, double *out)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < RED_BLOCKS; b += RED_THREADS)
        for (int a = 0; a < 4; ++a) acc[a] += part[b * 4 + a];
    block_sum4(acc, out);
}

// Scratch of the allocation-free reduction: the block partials, one copy per device (file-scope
// device array; host code uses the address hipGetSymbolAddress returns for the current device,
// never the array's name).
static __device__ __align__(256) double scratch[4 * RED_BLOCKS];
constexpr size_t SCRATCH_BYTES = sizeof(double) * 4 * RED_BLOCKS;
constexpr int MAX_SCRATCH_DEVICES = 64;
static void *g_scratch[MAX_SCRATCH_DEVICES];
static std::mutex g_scratch_mu;

// device address of `scratch` on the current device, looked up once per device; null on failure
// (the error text is set)
static double *scratch_of_current_device()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_SCRATCH_DEVICES) {
        set_error("cutcell_reduce_noalloc: no usable current device (%s)", hipGetErrorString(e));
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("cutcell_reduce_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = ptr;
    }
    return (double *)g_scratch[dev];
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
template <typename T>
static void launch_diagnose(const Dims &d, const Geo &G, const Phy &P, cc_state *q, int64_t *st, hipStream_t s)
{
    int64_t nc = (int64_t)d.nx * d.ny;
    hipLaunchKernelGGL(k_diagnose<T>, dim3(blocks_for(nc, DIAG_COLS)), dim3(DIAG_THREADS), 0, s, d, G, P, sout_of<T>(q), st);
}

// tile shapes of the update kernel (id -> TX x TY x TZ, minimum waves per SIMD the register
// allocation must allow); id 0 is the default
struct TileShape { int tx, ty, tz, minw; };
constexpr TileShape TILES[] = {{8, 8, 8, 1}, {4, 4, 16, 1}, {8, 4, 16, 1}, {4, 8, 16, 1}, {8, 8, 8, 1},
                               {2, 4, 32, 1}, {4, 4, 32, 1}, {8, 8, 16, 1}, {2, 2, 64, 1},
                               {8, 8, 8, 6}, {8, 8, 8, 8}, {4, 4, 16, 8}, {4, 8, 16, 6},
                               {8, 8, 16, 4}, {8, 8, 16, 6}, {8, 8, 8, 6},  // 13-15: two points per thread in k
                               {8, 8, 8, 8}, {4, 4, 16, 8}, {8, 8, 8, 4}, {8, 8, 16, 6},  // 16-19: 2-4 points
                               {1, 1, 1, 1}};  // 20: two-pass (prepare, then one point per thread)
constexpr int NTILES = sizeof(TILES) / sizeof(TILES[0]);

template <typename T, int TX, int TY, int TZ, int MODE>
static void launch_band(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                        cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s)
{
    int nbx = (d.nx + TX - 1) / TX, nby = (d.ny + TY - 1) / TY, nbz = (G.kband + TZ - 1) / TZ;
    const int n = G.nband >= 0 ? G.nband : nbx * nby * nbz;  // the listed tiles, else all below kband
    if (n > 0)
        hipLaunchKernelGGL((k_stage_tiled<T, TX, TY, TZ, MODE, 1, 1, false, 2>), dim3(n), dim3(TX * TY * TZ), 0, s, d,
                           G, P, sin_of<T>(qs), sin_of<T>(qn), sout_of<T>(qo), cdt, final_stage, nbx, nby, nbz, 0, st);
}

// One update split by point: the band points (below their column's band top) in one-wave tiles of
// the full kernel over k < kband, then the regular points by `regular` on s.  With a stage context
// the band launch goes to its side stream, forked from s and joined back into it; otherwise it runs
// on s first.
template <typename T, int MODE, typename F>
static void launch_split(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                         cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s, F regular)
{
    cc_stage_ctx x = G.side;
    hipStream_t sb = s;
    if (x && hipEventRecord(x->fork, s) == hipSuccess && hipStreamWaitEvent(x->side, x->fork, 0) == hipSuccess)
        sb = x->side;
    if (d.nx >= 8 && d.ny >= 8)
        launch_band<T, 8, 8, 1, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, sb);
    else if (d.nx >= 4 && d.ny >= 4)
        launch_band<T, 4, 4, 4, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, sb);
    else
        launch_band<T, 2, 2, 16, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, sb);
    regular();
    // join: later work on s waits for the band launch (should the join fail, the host waits)
    if (sb != s && (hipEventRecord(x->join, sb) != hipSuccess || hipStreamWaitEvent(s, x->join, 0) != hipSuccess))
        (void)hipStreamSynchronize(sb);
}

template <typename T, int TX, int TY, int TZ, int MODE, int MINW = 1, int KP = 1>
static void launch_tiled(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                         cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s)
{
    constexpr int KT = TZ * KP;
    int nbx = (d.nx + TX - 1) / TX, nby = (d.ny + TY - 1) / TY, nbz = (d.nz + KT - 1) / KT;
    if (!(MODE == 0 && G.kband >= 1 && G.kband <= d.nz)) {  // band height unknown: the full kernel
        hipLaunchKernelGGL((k_stage_tiled<T, TX, TY, TZ, MODE, MINW, KP>), dim3(nbx * nby * nbz), dim3(TX * TY * TZ),
                           0, s, d, G, P, sin_of<T>(qs), sin_of<T>(qn), sout_of<T>(qo), cdt, final_stage, nbx, nby,
                           nbz, 0, st);
        return;
    }
    // the points at or above the band top: the kernel without the band paths over the whole grid
    launch_split<T, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, s, [&] {
        hipLaunchKernelGGL((k_stage_tiled<T, TX, TY, TZ, MODE, MINW, KP, true, 1>), dim3(nbx * nby * nbz),
                           dim3(TX * TY * TZ), 0, s, d, G, P, sin_of<T>(qs), sin_of<T>(qn), sout_of<T>(qo), cdt,
                           final_stage, nbx, nby, nbz, 0, st);
    });
}

// the tile of a grid: the requested shape if the grid holds at least one tile per direction in x
// and y (the periodic index arithmetic wraps at most once), else 4x4x16, else 2x2x64
static int pick_tile(int id, const Dims &d)
{
    if (id >= STREAM_ID_MIN && id <= STREAM_ID_MAX) return id;
    if (id <= 0 || id >= NTILES) id = 0;
    if (d.nx >= TILES[id].tx && d.ny >= TILES[id].ty) return id;
    if (d.nx >= 4 && d.ny >= 4) return 1;
    return 8;
}

// the workspace of the two-pass update fits in 32-bit indices
static bool two_pass_ok(const Dims &d)
{
    return (int64_t)d.nx * d.ny * (d.nzs + 3 * (int64_t)lattice_stride(d.nzs)) < ((int64_t)1 << 31);
}

template <typename T, int MODE>
static void launch_two_pass(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                            cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s)
{
    using R = typename Compute<T>::R;
    R *ws = (R *)((char *)G.ws + band_list_bytes(d.nx, d.ny, d.nz));
    int64_t ncol = (int64_t)d.nx * d.ny;
    hipLaunchKernelGGL(k_prepare<T>, dim3(blocks_for(ncol * lattice_stride(d.nzs), 256)), dim3(256), 0, s, d, G, P,
                       sin_of<T>(qs), ws);
    hipLaunchKernelGGL((k_stage_points<T, MODE>), dim3(blocks_for(ncol * d.nz, 256)), dim3(256), 0, s, d, G, P,
                       sin_of<T>(qs), sin_of<T>(qn), sout_of<T>(qo), (const R *)ws, cdt, final_stage, st);
}

template <typename T, int MODE>
static void launch_stage(const Dims &d, const Geo &G, const Phy &P, const cc_state *qs, const cc_state *qn,
                         cc_state *qo, double cdt, int final_stage, int64_t *st, hipStream_t s, int tile)
{
    int id = pick_tile(tile, d);
    if (id >= STREAM_ID_MIN && id <= STREAM_ID_MAX) {
        // streaming form of the regular points (needs the band height; else the default tile)
        if (MODE == 0 && G.kband >= 1 && G.kband <= d.nz) {
            bool ok = true;
            launch_split<T, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, s, [&] {
                ok = launch_stream<T>(id, d, G, P, qs, qn, qo, cdt, final_stage, st, s);
                if (!ok)  // a form whose planes do not fit in LDS in this precision: the default tile
                    hipLaunchKernelGGL((k_stage_tiled<T, 8, 8, 8, MODE, 1, 1, true, 1>),
                                       dim3(((d.nx + 7) / 8) * ((d.ny + 7) / 8) * ((d.nz + 7) / 8)), dim3(512), 0, s,
                                       d, G, P, sin_of<T>(qs), sin_of<T>(qn), sout_of<T>(qo), cdt, final_stage,
                                       (d.nx + 7) / 8, (d.ny + 7) / 8, (d.nz + 7) / 8, 0, st);
            });
            return;
        }
        id = pick_tile(0, d);
    }
    if (id == 20) {
        if (MODE == 0 && G.ws && two_pass_ok(d)) {
            launch_two_pass<T, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, s);
            return;
        }
        id = pick_tile(0, d);  // no workspace: the default tile
    }
    if (MODE == 1) id = (d.nx >= 4 && d.ny >= 4) ? 1 : 8;  // tendency evaluation: fixed shapes
    switch (id) {
#define CC_TILE_CASE(ID, X, Y, Z) \
    case ID: launch_tiled<T, X, Y, Z, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    CC_TILE_CASE(0, 8, 8, 8)
    CC_TILE_CASE(1, 4, 4, 16)
    CC_TILE_CASE(2, 8, 4, 16)
    CC_TILE_CASE(3, 4, 8, 16)
    CC_TILE_CASE(4, 8, 8, 8)
    CC_TILE_CASE(5, 2, 4, 32)
    CC_TILE_CASE(6, 4, 4, 32)
    CC_TILE_CASE(7, 8, 8, 16)
#define CC_TILE_CASE_W(ID, X, Y, Z, W) \
    case ID: launch_tiled<T, X, Y, Z, MODE, W>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    CC_TILE_CASE_W(9, 8, 8, 8, 6)
    CC_TILE_CASE_W(10, 8, 8, 8, 8)
    CC_TILE_CASE_W(11, 4, 4, 16, 8)
    CC_TILE_CASE_W(12, 4, 8, 16, 6)
#undef CC_TILE_CASE_W
    case 13: launch_tiled<T, 8, 8, 8, MODE, 4, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    case 14: launch_tiled<T, 8, 8, 8, MODE, 6, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    case 15: launch_tiled<T, 8, 8, 4, MODE, 6, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    case 16: launch_tiled<T, 8, 8, 2, MODE, 8, 4>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    case 17: launch_tiled<T, 4, 4, 8, MODE, 8, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    case 18: launch_tiled<T, 8, 8, 4, MODE, 4, 2>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    case 19: launch_tiled<T, 8, 8, 4, MODE, 6, 4>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
    default: launch_tiled<T, 2, 2, 64, MODE>(d, G, P, qs, qn, qo, cdt, final_stage, st, s); break;
#undef CC_TILE_CASE
    }
}

}  // namespace cc

using namespace cc;

extern "C" cc_status cutcell_stage_ctx_create(cc_stage_ctx *out)
{
    CC_REQUIRE(out, "cutcell_stage_ctx_create: null output");
    cc_stage_ctx x = new cc_stage_ctx_s();
    hipError_t e = hipStreamCreateWithFlags(&x->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&x->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&x->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        set_error("cutcell_stage_ctx_create: %s", hipGetErrorString(e));
        cutcell_stage_ctx_destroy(x);
        return CC_EDEVICE;
    }
    *out = x;
    return CC_OK;
}

extern "C" cc_status cutcell_stage_ctx_destroy(cc_stage_ctx x)
{
    if (!x) return CC_OK;
    if (x->join) (void)hipEventDestroy(x->join);
    if (x->fork) (void)hipEventDestroy(x->fork);
    if (x->side) (void)hipStreamDestroy(x->side);
    delete x;
    return CC_OK;
}

extern "C" cc_status cutcell_init_state(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                        const double *base, cc_prec prec, const double *noise,
                                        cc_state *q, int64_t *st, cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_init_state", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_init_state", q)) return CC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t n = (int64_t)d.nx * d.ny * d.nz;
    dim3 gb(blocks_for(n, 256)), tb(256);
    if (prec == CC_F64) {
        hipLaunchKernelGGL(k_init_cells<double>, gb, tb, 0, s, d, G, P, noise, sout_of<double>(q));
        hipLaunchKernelGGL(k_init_momentum_full, gb, tb, 0, s, d, G, P, phys->u0, phys->v0, sout_of<double>(q));
        launch_diagnose<double>(d, G, P, q, st, s);
    } else {
        hipLaunchKernelGGL(k_init_cells<float>, gb, tb, 0, s, d, G, P, noise, sout_of<float>(q));
        hipLaunchKernelGGL(k_init_momentum_pert, gb, tb, 0, s, d, G, P, sout_of<float>(q));
        launch_diagnose<float>(d, G, P, q, st, s);
    }
    return launch_status("cutcell_init_state");
}

extern "C" cc_status cutcell_diagnose(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                      const double *base, cc_prec prec, cc_state *q, int64_t *st,
                                      cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_diagnose", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_diagnose", q)) return CC_EINVAL;
    if (prec == CC_F64) launch_diagnose<double>(d, G, P, q, st, (hipStream_t)stream);
    else launch_diagnose<float>(d, G, P, q, st, (hipStream_t)stream);
    return launch_status("cutcell_diagnose");
}

extern "C" cc_status cutcell_tendency(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                      const double *base, cc_prec prec, const cc_state *q, cc_state *dq,
                                      cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_tendency", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_tendency", q) || !state_ok("cutcell_tendency", dq)) return CC_EINVAL;
    CC_REQUIRE(q->rho != dq->rho, "cutcell_tendency: output aliases input");
    hipStream_t s = (hipStream_t)stream;
    if (prec == CC_F64) {
        launch_stage<double, 1>(d, G, P, q, q, dq, 0.0, 0, nullptr, s, grid->tile);
        launch_diffuse<double>(d, G, P, q, dq, 1.0, 0, s);
    } else {
        launch_stage<float, 1>(d, G, P, q, q, dq, 0.0, 0, nullptr, s, grid->tile);
        launch_diffuse<float>(d, G, P, q, dq, 1.0, 0, s);
    }
    return launch_status("cutcell_tendency");
}

extern "C" cc_status cutcell_rk_stage(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                      const double *base, cc_prec prec, const cc_state *qn,
                                      const cc_state *qs, cc_state *qo, double cdt, int32_t final_stage,
                                      int64_t *st, cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_rk_stage", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_rk_stage", qn) || !state_ok("cutcell_rk_stage", qs) || !state_ok("cutcell_rk_stage", qo))
        return CC_EINVAL;
    CC_REQUIRE(qo->rho != qs->rho && qo->rho != qn->rho && qo->mu != qs->mu && qo->mu != qn->mu,
               "cutcell_rk_stage: q_out must not alias q_n or q_s");
    hipStream_t s = (hipStream_t)stream;
    if (prec == CC_F64) {
        launch_stage<double, 0>(d, G, P, qs, qn, qo, cdt, final_stage, st, s, grid->tile);
        launch_diffuse<double>(d, G, P, qs, qo, cdt, final_stage, s);
        launch_diagnose<double>(d, G, P, qo, st, s);
    } else {
        launch_stage<float, 0>(d, G, P, qs, qn, qo, cdt, final_stage, st, s, grid->tile);
        launch_diffuse<float>(d, G, P, qs, qo, cdt, final_stage, s);
        launch_diagnose<float>(d, G, P, qo, st, s);
    }
    return launch_status("cutcell_rk_stage");
}

extern "C" cc_status cutcell_rk_update(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                       const double *base, cc_prec prec, const cc_state *qn,
                                       const cc_state *qs, cc_state *qo, double cdt, int32_t final_stage,
                                       int64_t *st, cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_rk_update", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_rk_update", qn) || !state_ok("cutcell_rk_update", qs) || !state_ok("cutcell_rk_update", qo))
        return CC_EINVAL;
    CC_REQUIRE(qo->rho != qs->rho && qo->rho != qn->rho && qo->mu != qs->mu && qo->mu != qn->mu,
               "cutcell_rk_update: q_out must not alias q_n or q_s");
    hipStream_t s = (hipStream_t)stream;
    if (prec == CC_F64) {
        launch_stage<double, 0>(d, G, P, qs, qn, qo, cdt, final_stage, st, s, grid->tile);
        launch_diffuse<double>(d, G, P, qs, qo, cdt, final_stage, s);
    } else {
        launch_stage<float, 0>(d, G, P, qs, qn, qo, cdt, final_stage, st, s, grid->tile);
        launch_diffuse<float>(d, G, P, qs, qo, cdt, final_stage, s);
    }
    return launch_status("cutcell_rk_update");
}

// ---- leap-frog with the Robert-Asselin filter, p' form (Sec. 2.2, eq. heat) ----
static size_t lf_array_bytes(const cc_grid *grid, cc_prec prec)
{
    const size_t n = (size_t)grid->nx * grid->ny * grid->nzs;
    return (n * (prec == CC_F64 ? 8 : 4) + 255) / 256 * 256;
}

extern "C" size_t cutcell_lf_workspace_bytes(const cc_grid *grid, cc_prec prec)
{
    if (!check_grid(grid)) return 0;
    return 3 * lf_array_bytes(grid, prec);
}

extern "C" cc_status cutcell_pform(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                   const double *base, cc_prec prec, cc_state *q, int32_t to_p,
                                   cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_pform", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_pform", q)) return CC_EINVAL;
    if (prec == CC_F64) launch_pform<double>(d, G, P, q, to_p, (hipStream_t)stream);
    else launch_pform<float>(d, G, P, q, to_p, (hipStream_t)stream);
    return launch_status("cutcell_pform");
}

template <typename T>
static void lf_step(const cc_grid *grid, const Dims &d, const Geo &G, const Phy &P, const cc_state *qm,
                    cc_state *q0, cc_state *qp, char *work, size_t abytes, double dt, double nu, int first,
                    int64_t *st, hipStream_t s)
{
    T *w[3];
    for (int a = 0; a < 3; ++a) w[a] = (T *)(work + a * abytes);
    const bool lo = sizeof(T) == 4 && q0->rho_lo && q0->rth_lo && qp->rho_lo && qp->rth_lo;
    // q_s: q(n) with (rho theta)' from its p'; q_n: the base level with a zero thermodynamic slot
    launch_rthp<T>(d, G, P, q0, w[0], w[1], lo ? w[2] : nullptr, s);
    cc_state tin = *q0;
    tin.rth = w[0];
    tin.rho_lo = tin.rth_lo = nullptr;
    const cc_state *qb = first ? q0 : qm;
    cc_state base = *qb;
    base.rth = w[1];
    base.rth_lo = lo ? w[2] : nullptr;
    if (!lo) base.rho_lo = nullptr;
    cc_state out = *qp;
    if (!lo) out.rho_lo = out.rth_lo = nullptr;
    const double h = first ? dt : 2.0 * dt;
    launch_stage<T, 0>(d, G, P, &tin, &base, &out, h, lo ? 1 : 0, st, s, grid->tile);
    launch_diffuse<T>(d, G, P, &tin, &out, h, lo ? 1 : 0, s);
    launch_lf_finish<T>(d, G, P, qb, q0, &out, nu, first, st, s);
    launch_diagnose<T>(d, G, P, &out, st, s);
}

extern "C" cc_status cutcell_lf_step(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                     const double *base, cc_prec prec, const cc_state *q_m, cc_state *q_0,
                                     cc_state *q_p, void *work, double dt, double nu, int32_t first,
                                     int64_t *st, cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    const char *what = "cutcell_lf_step";
    if (!make_views(what, grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok(what, q_0) || !state_ok(what, q_p) || (!first && !state_ok(what, q_m))) return CC_EINVAL;
    CC_REQUIRE(work, "cutcell_lf_step: null workspace");
    CC_REQUIRE(q_p->rho != q_0->rho && q_p->mu != q_0->mu && (first || (q_p->rho != q_m->rho && q_p->mu != q_m->mu &&
                                                                         q_m->rho != q_0->rho)),
               "cutcell_lf_step: q_m, q_0 and q_p must be distinct states");
    CC_REQUIRE(dt > 0.0 && std::isfinite(dt), "cutcell_lf_step: dt must be positive");
    CC_REQUIRE(nu >= 0.0 && nu <= 0.5, "cutcell_lf_step: filter weight outside [0, 1/2]");
    const size_t ab = lf_array_bytes(grid, prec);
    hipStream_t s = (hipStream_t)stream;
    if (prec == CC_F64) lf_step<double>(grid, d, G, P, q_m, q_0, q_p, (char *)work, ab, dt, nu, first != 0, st, s);
    else lf_step<float>(grid, d, G, P, q_m, q_0, q_p, (char *)work, ab, dt, nu, first != 0, st, s);
    return launch_status(what);
}

extern "C" size_t cutcell_reduce_workspace(const cc_grid *)
{
    return sizeof(double) * 4 * RED_BLOCKS;
}

extern "C" cc_status cutcell_reduce(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                    const double *base, cc_prec prec, const cc_state *q, void *ws,
                                    double *out, cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_reduce", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_reduce", q)) return CC_EINVAL;
    CC_REQUIRE(ws && out, "cutcell_reduce: null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    double *part = (double *)ws;
    if (prec == CC_F64)
        hipLaunchKernelGGL(k_reduce_partial<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, d, G, P,
                           sin_of<double>(q), part);
    else
        hipLaunchKernelGGL(k_reduce_partial<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, d, G, P,
                           sin_of<float>(q), part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, part, out);
    return launch_status("cutcell_reduce");
}

extern "C" cc_status cutcell_reduce_noalloc(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                            const double *base, cc_prec prec, const cc_state *q, double *out,
                                            cc_stream_t stream)
{
    Dims d; Geo G; Phy P;
    if (!make_views("cutcell_reduce_noalloc", grid, phys, geom, base, prec, d, G, P)) return CC_EINVAL;
    if (!state_ok("cutcell_reduce_noalloc", q)) return CC_EINVAL;
    CC_REQUIRE(out, "cutcell_reduce_noalloc: null output");
    CC_REQUIRE(cutcell_reduce_workspace(grid) <= SCRATCH_BYTES,
               "cutcell_reduce_noalloc: %zu bytes of partial sums exceed the %zu-byte static scratch",
               cutcell_reduce_workspace(grid), SCRATCH_BYTES);
    double *part = scratch_of_current_device();
    if (!part) return CC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    // every partial is written before the final pass reads it: nothing to clear
    if (prec == CC_F64)
        hipLaunchKernelGGL(k_reduce_partial<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, d, G, P,
                           sin_of<double>(q), part);
    else
        hipLaunchKernelGGL(k_reduce_partial<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, d, G, P,
                           sin_of<float>(q), part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, part, out);
    return launch_status("cutcell_reduce_noalloc");
}

extern "C" size_t cutcell_stage_workspace_bytes(const cc_grid *grid, cc_prec prec)
{
    if (!grid || grid->nx <= 0 || grid->ny <= 0 || grid->nzs <= 0) return 0;
    size_t esz = prec == CC_F64 ? sizeof(double) : sizeof(float);
    size_t ncol = (size_t)grid->nx * grid->ny;
    return band_list_bytes(grid->nx, grid->ny, grid->nz) +
           esz * ncol * ((size_t)grid->nzs + 3 * (size_t)lattice_stride(grid->nzs));
}
