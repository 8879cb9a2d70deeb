// Batched blocks: many grids stepped by one update and one diagnostic launch per Runge-Kutta
// stage, with the step sequence optionally captured into a hipGraph.
#pragma clang fp contract(off)

#include <vector>

#include "cc_kernels.hpp"

using namespace cc;

// ------------------------------------------------------------------------------------------------
// batched blocks: descriptors, stepping, graph capture
// ------------------------------------------------------------------------------------------------
struct cc_batch_s {
    cc_prec prec;
    int nblk = 0, ntiles = 0, ncols = 0, tile = 0;
    void *desc = nullptr;            // device descriptors (caller workspace)
    std::vector<char> host;          // host image of the descriptors
    int cur = 0;                     // buffer index holding the current state
    hipStream_t cap = nullptr;       // private stream used only for graph capture
    struct Graph { int nsteps, cur; double dt; int64_t *st; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
};

namespace cc {

template <typename T, int TX, int TY, int TZ, int MINW>
static void launch_batch_stage(const cc_batch_s *b, int rn, int rs, int ro, double cdt, int fin, int64_t *st,
                               hipStream_t s)
{
    hipLaunchKernelGGL((k_stage_batch<T, TX, TY, TZ, 0, MINW>), dim3(b->ntiles), dim3(TX * TY * TZ), 0, s,
                       (const BlockDesc<T> *)b->desc, b->nblk, b->ntiles, rn, rs, ro, cdt, fin, st);
}

template <typename T>
static void batch_stage(const cc_batch_s *b, int rn, int rs, int ro, double cdt, int fin, int64_t *st, hipStream_t s)
{
    switch (b->tile) {
    case 1: launch_batch_stage<T, 4, 4, 16, 1>(b, rn, rs, ro, cdt, fin, st, s); break;
    case 8: launch_batch_stage<T, 2, 2, 64, 1>(b, rn, rs, ro, cdt, fin, st, s); break;
    case 9: launch_batch_stage<T, 8, 8, 8, 6>(b, rn, rs, ro, cdt, fin, st, s); break;
    default: launch_batch_stage<T, 8, 8, 8, 1>(b, rn, rs, ro, cdt, fin, st, s); break;
    }
    hipLaunchKernelGGL(k_diagnose_batch<T>, dim3(blocks_for(b->ncols, 64)), dim3(64), 0, s,
                       (const BlockDesc<T> *)b->desc, b->nblk, b->ncols, ro, st);
}

// nsteps three-stage steps of every block, rotating the three buffers (the state of step n is in
// buffer cur; the stages write the other two)
static void batch_enqueue(cc_batch_s *b, double dt, int nsteps, int64_t *st, hipStream_t s)
{
    for (int n = 0; n < nsteps; ++n) {
        int a = b->cur, o = 1 - b->cur, c = 2;
        if (b->prec == CC_F64) {
            batch_stage<double>(b, a, a, o, dt / 3.0, 0, st, s);
            batch_stage<double>(b, a, o, c, dt / 2.0, 0, st, s);
            batch_stage<double>(b, a, c, o, dt, 1, st, s);
        } else {
            batch_stage<float>(b, a, a, o, dt / 3.0, 0, st, s);
            batch_stage<float>(b, a, o, c, dt / 2.0, 0, st, s);
            batch_stage<float>(b, a, c, o, dt, 1, st, s);
        }
        b->cur = o;
    }
}

template <typename T>
static bool build_descs(const cc_block *blocks, int nblk, cc_prec prec, int TX, int TY, int TZ, cc_batch_s *b)
{
    b->host.assign(sizeof(BlockDesc<T>) * nblk, 0);
    BlockDesc<T> *h = (BlockDesc<T> *)b->host.data();
    int tiles = 0, cols = 0;
    for (int m = 0; m < nblk; ++m) {
        const cc_block &B = blocks[m];
        Dims d; Geo G; Phy P;
        if (!make_views("amr_batch_create", &B.grid, &B.phys, &B.geom, B.base, prec, d, G, P)) return false;
        for (int r = 0; r < 3; ++r) {
            if (!state_ok("amr_batch_create", &B.q[r])) return false;
            h[m].q[r] = sout_of<T>(const_cast<cc_state *>(&B.q[r]));
        }
        h[m].d = d; h[m].G = G; h[m].P = P;
        h[m].nbx = (d.nx + TX - 1) / TX; h[m].nby = (d.ny + TY - 1) / TY; h[m].nbz = (d.nz + TZ - 1) / TZ;
        h[m].tile0 = tiles;
        h[m].col0 = cols;
        tiles += h[m].nbx * h[m].nby * h[m].nbz;
        cols += d.nx * d.ny;
    }
    b->ntiles = tiles;
    b->ncols = cols;
    return true;
}

}  // namespace cc

extern "C" size_t amr_batch_workspace_bytes(int32_t nblocks, cc_prec prec)
{
    size_t one = prec == CC_F64 ? sizeof(cc::BlockDesc<double>) : sizeof(cc::BlockDesc<float>);
    return (one * (size_t)(nblocks > 0 ? nblocks : 0) + 255) / 256 * 256;
}

extern "C" cc_status amr_batch_create(const cc_block *blocks, int32_t nblocks, cc_prec prec, int32_t tile,
                                      void *workspace, cc_batch *out, cc_stream_t stream)
{
    using namespace cc;
    CC_REQUIRE(blocks && nblocks > 0 && workspace && out, "amr_batch_create: null or empty argument");
    CC_REQUIRE(prec == CC_F64 || prec == CC_F32_PERT, "amr_batch_create: unknown precision");
    for (int m = 0; m < nblocks; ++m) {
        CC_REQUIRE(blocks[m].level == 0, "amr_batch_create: block %d has level %d; a batch holds level-0 blocks only",
                  m, blocks[m].level);
    }
    // one tile shape for the whole batch; every block must hold a tile in x and y
    int id = tile;
    auto fits = [&](int tx, int ty) {
        for (int m = 0; m < nblocks; ++m)
            if (blocks[m].grid.nx < tx || blocks[m].grid.ny < ty) return false;
        return true;
    };
    if (id != 1 && id != 8 && id != 9) id = 0;
    int TX = id == 1 ? 4 : (id == 8 ? 2 : 8), TY = TX, TZ = id == 1 ? 16 : (id == 8 ? 64 : 8);
    if (!fits(TX, TY)) { id = fits(4, 4) ? 1 : 8; TX = id == 1 ? 4 : 2; TY = TX; TZ = id == 1 ? 16 : 64; }
    cc_batch_s *b = new cc_batch_s();
    b->prec = prec;
    b->nblk = nblocks;
    b->tile = id;
    b->desc = workspace;
    bool ok = prec == CC_F64 ? build_descs<double>(blocks, nblocks, prec, TX, TY, TZ, b)
                             : build_descs<float>(blocks, nblocks, prec, TX, TY, TZ, b);
    if (!ok) { delete b; return CC_EINVAL; }
    hipError_t e = hipMemcpyAsync(workspace, b->host.data(), b->host.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("amr_batch_create: %s", hipGetErrorString(e));
        delete b;
        return CC_EDEVICE;
    }
    *out = b;
    return CC_OK;
}

extern "C" cc_status amr_block_step(cc_batch b, double dt, int32_t nsteps, int32_t use_graph, int64_t *st,
                                    cc_stream_t stream)
{
    using namespace cc;
    CC_REQUIRE(b && nsteps >= 0, "amr_block_step: bad batch or step count");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        batch_enqueue(b, dt, nsteps, st, s);
        return launch_status("amr_block_step");
    }
    for (auto &g : b->graphs)
        if (g.nsteps == nsteps && g.cur == b->cur && g.dt == dt && g.st == st) {
            hipError_t e = hipGraphLaunch(g.exec, s);
            if (e != hipSuccess) { set_error("amr_block_step: %s", hipGetErrorString(e)); return CC_EDEVICE; }
            if (nsteps % 2) b->cur = 1 - b->cur;
            return CC_OK;
        }
    // capture the step sequence once on a private stream, then launch it on the caller's stream
    hipError_t e = hipSuccess;
    if (!b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    int cur0 = b->cur;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        batch_enqueue(b, dt, nsteps, st, b->cap);
        e = hipStreamEndCapture(b->cap, &graph);
    }
    b->cur = cur0;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) {
        set_error("amr_block_step (graph): %s", hipGetErrorString(e));
        return CC_EDEVICE;
    }
    b->graphs.push_back({nsteps, cur0, dt, st, exec});
    if (nsteps % 2) b->cur = 1 - b->cur;
    return CC_OK;
}

extern "C" int32_t amr_batch_current(cc_batch b) { return b ? b->cur : -1; }

extern "C" cc_status amr_batch_destroy(cc_batch b)
{
    if (!b) return CC_OK;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return CC_OK;
}
