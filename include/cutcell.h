/*
 * cutcell.h -- C ABI of libcutcell.so, the MI355X (gfx950) implementation of the explicit
 * finite-volume cut-cell stage of Yamazaki, Satomura & Nikiforakis, "3D cut-cell modelling for
 * high-resolution atmospheric simulations" (arXiv:1509.02572).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Memory.  Every array pointer is DEVICE memory allocated and owned by the caller; the library never
 * allocates or frees device memory on these paths and keeps no global state apart from a
 * thread-local last-error string (and the static scratch array of cutcell_reduce_noalloc).  Host
 * objects it creates (stage contexts, batch handles) are created and destroyed by explicit calls.
 * Calls are ordered on the caller's HIP stream (`stream`, a hipStream_t; NULL = the default stream)
 * and return as soon as their kernels are enqueued; the only calls that wait for the stream are the
 * ones documented to (cutcell_band_setup, cutcell_check_status, the batch set-up calls).
 *
 * Layout.  Cell (i,j,k), 0<=i<nx, 0<=j<ny, 0<=k<nz, spans [i dx,(i+1)dx] x [j dy,(j+1)dy] x
 * [k dz,(k+1)dz].  Every 3-D array is structure-of-arrays, k fastest, index ((i*ny + j)*nzs + k) with
 * the padded stride nzs >= nz; slots k >= nz are never read or written.  Lattice point (I,J,K) is the
 * cell corner (I dx, J dy, K dz) (velocity point of the semi-staggered arrangement, Sec. 2.3) and
 * uses the index of cell (I,J,K); the lid row K = nz is not stored.  Column and corner arrays are
 * [nx*ny], index (i*ny + j).  x and y are periodic.
 *
 * Precision.  CC_F64: every field is double and holds the paper's variables: rho', (rho theta)' at
 * cells, the momentum (rho u, rho v, rho w) at predicted lattice points and the diagnosed velocity
 * (u, v, w) at all other lattice points.  CC_F32_PERT: every state field is float and holds
 * perturbations: rho', (rho theta)', the momentum perturbation rho u - rhobar_c(K) (u0, v0, 0) at
 * predicted points (rhobar_c(K) = mean of the base density of levels K-1 and K) and the velocity
 * perturbation u - (u0, v0, 0) at diagnosed points.  Base state, geometry and reductions stay double.
 *
 * Errors.  Argument errors found on the host (null pointer, bad sizes, nsub not a power of two, nz<3)
 * return CC_EINVAL and launch nothing.  HIP launch failures return CC_EDEVICE.  Conditions found on
 * the device are counted into the caller's int64 status array `dev_status[CC_NSTATUS]` (never reset
 * by the library): [0] unmergeable cells, [1] corners without a nearest plane, [2] non-finite values,
 * [3] terrain corners outside [0, (nz-2) dz] (or above it for a raised block), [4] merged groups
 * larger than CC_MAX_GROUP, [5] coarse-fine interface faces of a refined grid that are not open
 * regular faces (the interface touches cut or merged cells), [6] non-finite values written to
 * ghost cells of refined-grid blocks (layers that go stale between refills and are overwritten;
 * informational, not an error).  The
 * caller synchronises and checks them (cutcell_check_status).  No exception crosses the ABI.
 * Calls are reentrant for distinct streams and buffers; calls sharing output buffers race.
 */
#ifndef CUTCELL_H
#define CUTCELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *cc_stream_t; /* hipStream_t */

typedef enum {
    CC_OK = 0,
    CC_EINVAL = 1,
    CC_EDEVICE = 2,
    CC_EUNMERGEABLE = 3,
    CC_ENOPLANE = 4,
    CC_ENONFINITE = 5,
    CC_ETERRAIN = 6
} cc_status;

typedef enum { CC_F64 = 0, CC_F32_PERT = 1 } cc_prec;

/* Stage context: a side stream and two events on one device, created by the caller
 * (cutcell_stage_ctx_create).  Given in cc_geom.side, the band-point launch of an update runs on the
 * side stream, forked from and joined to the caller's stream, beside the regular-point launch.  A
 * context serves one call at a time: grids stepped concurrently on different streams need one each. */
typedef struct cc_stage_ctx_s *cc_stage_ctx;

#define CC_NSTATUS 8
#define CC_MAX_GROUP 32

/* cell classes (cls), merge directions (dir) and lattice-point classes (vcls) */
enum { CC_SOLID = 0, CC_OPEN = 1, CC_ABSORBED = 2, CC_ORPHAN = 3 };
enum { CC_DIR_NONE = 0, CC_DIR_ZP = 1, CC_DIR_XM = 2, CC_DIR_XP = 3, CC_DIR_YM = 4, CC_DIR_YP = 5 };
enum { CC_GROUND = 0, CC_PRED = 1, CC_MFACE = 2 };

typedef struct {
    int32_t nx, ny, nz, nzs; /* cells; padded k stride (nzs >= nz) */
    double dx, dy, dz;       /* spacings [m] */
    int32_t nsub;            /* sub-columns per cell edge for volumes/apertures, power of two */
    int32_t tile;            /* tile shape of the update kernel (0 = default; 1..20 three-dimensional
                                tiles, 21..29 streaming forms, see the tuning table of the stage
                                kernels); results do not depend on it */
    double z0;               /* height of the grid's bottom face above the terrain datum [m]: 0 for
                                a grid standing on the ground; > 0 for a block of a refined grid
                                that starts higher (Sec. 2.2), whose H is then given relative to z0
                                and may be negative (terrain below the block) */
} cc_grid;

typedef struct {
    double g, rd, cp, p0; /* gravity, gas constant, specific heat at constant pressure, p_ref */
    double theta0, bvn;   /* sea-level potential temperature [K], Brunt-Vaisala frequency [1/s] */
    double u0, v0;        /* uniform inflow (reference velocity of the perturbation form) */
    double kdh, kdv;      /* rates [1/s] of the fourth-order artificial diffusion in x, y and in z
                             (Sec. 2.1 D terms; 0: none).  The 2-dx mode of a field decays at 16 kdh
                             per horizontal direction (16 kdv vertically); the explicit stage needs
                             dt (32 kdh + 16 kdv) below about 2.5.  In a batch or refined grid every
                             block applies it in flux form over its update range; the stencil reaches
                             two cells, so a refined level's stale ghost layers advance two per stage
                             (ghost width 12 covers two fine steps), and the coarse-fine flux
                             matching covers the advective fluxes only */
    double zsp, rsp;      /* sponge layer below the lid (Sec. 3, absorbing layer after Klemp & Lilly):
                             bottom height zsp [m, same datum as z0] and damping rate rsp [1/s] at the
                             lid (0: none).  Rayleigh damping -tau(z) (q - q_ref) with tau = rsp
                             sin^2(pi/2 (z - zsp)/(ztop - zsp)) above zsp, on (rho theta)' at group
                             masters (cell-centre height) and on rho u - rhobar_c (u0, v0, 0) at
                             predicted points (lattice height); rho' is not damped, so mass stays
                             conserved.  Needs dt rsp below about 2.5 */
    double ztop;          /* height of the domain's lid [m, same datum as z0] for the sponge: 0 for
                             the grid's own top z0 + nz dz; a block of a refined grid that ends below
                             the lid passes the domain's (not below its own top, else CC_EINVAL) */
} cc_phys;

/* Geometry and merge map (device arrays, caller-allocated). */
typedef struct {
    const double *H;          /* [nx*ny] terrain height at corner (I,J), input */
    double *V;                /* [cells] volume fraction in [0,1] */
    double *Ax, *Ay, *Az;     /* [cells] open fraction of the faces x = i dx, y = j dy, z = k dz */
    double *col;              /* [3][nx*ny] column centre height hc, gradients gx, gy */
    double *nrm;              /* [3][nx*ny] unit terrain normal at corner (I,J) */
    int8_t *cls, *dir, *vcls; /* [cells] */
    int32_t *master;          /* [cells] linear index of the group master, -1 for solid cells */
    int32_t *gnext;           /* [cells] next member of the master's group (increasing index), -1 */
    double *Vgroup;           /* [cells] group volume fraction, valid at masters */
    int32_t *colk;            /* [3][nx*ny] per column: first k of the regular cell interior; 1 + top
                                 K of a lattice point that is not predicted; 1 + top level of any
                                 diagnosed point, absorbed or solid cell */
    void *stage_ws;           /* optional workspace of cutcell_stage_workspace_bytes() bytes: holds the
                                 list of band tiles cutcell_merge_map writes (the band-point launch
                                 then covers only tiles with band points) and enables the two-pass
                                 update (cc_grid.tile = 20); NULL otherwise */
    int32_t kband;            /* host value set by cutcell_band_setup: the highest column band top.
                                 A column's band top is one above its highest point that is not
                                 regular (a cell that is cut, merged, or next to a closed face or a
                                 cell that is not open; a lattice point above the ground row that is
                                 not predicted).  The update runs the points at or above their
                                 column's band top with a kernel without the band paths and the rest
                                 with the full kernel over k < kband.  0 or out of [1, nz]: unknown
                                 (the full kernel everywhere) */
    int32_t nband_tiles;      /* host value set by cutcell_band_setup: number of band tiles in the list
                                 at the start of stage_ws; -1 without stage_ws (the band-point launch
                                 then covers every tile below kband).  The list lives in the
                                 workspace given to cutcell_band_setup: another workspace needs
                                 another call (or nband_tiles = -1); entries that are not tiles of
                                 the grid are skipped */
    cc_stage_ctx side;        /* optional stage context (NULL: the band points of an update run on the
                                 caller's stream before the regular points) */
} cc_geom;

/* Five prognostic fields; element type double (CC_F64) or float (CC_F32_PERT).
 * rho_lo, rth_lo (CC_F32_PERT only, float, nullable): low-order parts of rho' and (rho theta)'.  The
 * value of the state is rho + rho_lo; the stage that completes a time step adds q_n's low-order part
 * and stores the rounding remainder of its float result in q_out's, so the cell masses change only
 * by the FP64 rounding of the flux sums (mass and Theta' stay conserved with float storage).  With
 * null pointers the float state is rounded plainly.  Ignored by CC_F64. */
typedef struct {
    void *rho, *rth, *mu, *mv, *mw;
    void *rho_lo, *rth_lo;
} cc_state;

const char *cutcell_version(void);

/* Bytes of the optional stage workspace (cc_geom.stage_ws) of a grid: the band-tile list (one int32
 * per one-wave tile of the grid, rounded up to 256 bytes), then p' at every cell and the velocity at
 * every lattice point, in the storage precision's compute type. */
size_t cutcell_stage_workspace_bytes(const cc_grid *grid, cc_prec prec);
const char *cutcell_last_error(void);

/* Base state on cell centres z_k = z0 + (k+1/2) dz (Sec. 2.1 hydrostatic reference; constant N and
 * theta0 at z = 0, surface pressure p0, Sec. 3).  base: [6*nz] doubles = rhobar, (rho theta)bar,
 * pbar, thetabar, 1/(rho theta)bar, and at lattice level K the mean of rhobar at levels K-1 and K;
 * pbar follows from (rho theta)bar through the equation of state.  Every other call takes this
 * array as `base`. */
cc_status cutcell_base_state(const cc_grid *grid, const cc_phys *phys, double *base, cc_stream_t stream);

/* Cut-cell geometry (Sec. 2.3): bilinear terrain per column (eq. bilin) from the corner heights H,
 * cell volume fractions V and face apertures Ax/Ay/Az from nsub x nsub narrow sub-columns, column
 * gradients (eqs. xgrad, ygrad) and the unit terrain normal at every corner from centred gradients
 * of the column-centre heights (Sec. 2.4).  A face touching a cell with V = 0 is closed.  Writes
 * V, Ax, Ay, Az, col, nrm of `geom`; counts terrain outside [0,(nz-2)dz] into dev_status[3] (for a
 * raised block, grid.z0 > 0, only non-finite heights count). */
cc_status cutcell_geometry(const cc_grid *grid, cc_geom *geom, int64_t *dev_status, cc_stream_t stream);

/* Cell merging (Sec. 2.3, Figs. 5 and 6): a cell with V > 0 merges when its centre is below the
 * column's centre height or V < 1/2; direction from the column gradients (vertical if |gx|,|gy| <= 1,
 * else towards lower terrain, x preferred on ties).  Chains of targets that must merge themselves are
 * followed up to 8 hops to the master.  Also classifies lattice points (predicted when all eight
 * surrounding cells are available, Sec. 2.4) and fills gnext, Vgroup and colk.  Needs V, Az.. and
 * col from cutcell_geometry.  Unmergeable cells become their own master (CC_ORPHAN) and are counted
 * into dev_status[0].  Enqueues only; sets geom->kband = 0 and geom->nband_tiles = -1 (band height
 * unknown: updates run the full kernel everywhere until cutcell_band_setup is called). */
cc_status cutcell_merge_map(const cc_grid *grid, cc_geom *geom, int64_t *dev_status, cc_stream_t stream);

/* Band set-up (host query): synchronises `stream`, reads the column bands cutcell_merge_map wrote
 * (colk) and sets geom->kband, the highest column band top; with geom->stage_ws it also writes the
 * list of one-wave band tiles that hold band points at the start of stage_ws (copied before the call
 * returns) and sets geom->nband_tiles.  Updates then split into the regular-point launch and the
 * band-point launch.  Call after cutcell_merge_map, once per geometry. */
cc_status cutcell_band_setup(const cc_grid *grid, cc_geom *geom, cc_stream_t stream);

/* Stage context (see cc_stage_ctx): a non-blocking side stream and two events on the current device. */
cc_status cutcell_stage_ctx_create(cc_stage_ctx *out);
cc_status cutcell_stage_ctx_destroy(cc_stage_ctx ctx);

/* Initial state: theta' (nullable, cell layout, double) applied at constant pressure to group
 * masters, (rho theta)' = 0, uniform inflow (u0, v0, 0) as momentum at predicted points, then one
 * velocity-diagnostic pass.  Writes every slot k < nz of q. */
cc_status cutcell_init_state(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                             const double *base, cc_prec prec, const double *theta_noise, cc_state *q,
                             int64_t *dev_status, cc_stream_t stream);

/* Velocity diagnostics (Sec. 2.4, three-step procedure, steps 2-3): boundary velocity at every
 * corner from the nearest plane of predicted points and the free-slip projection (eq. 33),
 * merged-face points by linear interpolation towards the lowest predicted point above, points on or
 * below the terrain take the boundary velocity; absorbed cells mirror their master's scalars and
 * solid cells are zeroed.  Updates q in place. */
cc_status cutcell_diagnose(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                           const double *base, cc_prec prec, cc_state *q, int64_t *dev_status,
                           cc_stream_t stream);

/* Tendency L(q) (Sec. 2.4): scalar fluxes with apertures over the whole merged group divided by the
 * group volume (eqs. gauss_m, gauss_d, fvm_d and the merged-cell face split), momentum, pressure
 * gradient and buoyancy at predicted points (eqs. momentum_u_d, _v_d, _w_d), plus the fourth-order
 * artificial diffusion when phys->kdh or kdv is non-zero: in flux form, the flux through a face being
 * the third difference of the four values straddling it, or -4 x their first difference where an
 * outer one is missing (solid cell, point not predicted, ground, lid: the second-order term of
 * Sec. 2.4), zero through closed faces; scalars with apertures and group volumes (conservative),
 * momentum as the perturbation rho u - rhobar_c (u0, v0, 0); and the sponge's Rayleigh damping when
 * phys->rsp is non-zero (see cc_phys).  dqdt: same element type as q; scalars at group masters,
 * momentum at predicted points, zero elsewhere. */
cc_status cutcell_tendency(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                           const double *base, cc_prec prec, const cc_state *q, cc_state *dqdt,
                           cc_stream_t stream);

/* One explicit Runge-Kutta stage q_out = q_n + stage_dt * L(q_s) (three-stage scheme of Wicker &
 * Skamarock with stage_dt = dt/3, dt/2, dt; it replaces the paper's leap-frog, Sec. 2.2), followed
 * by the velocity diagnostics of q_out.  q_n may equal q_s; q_out must differ from both.  Non-finite
 * updated values are counted into dev_status[2].  final_stage != 0 marks the stage that completes a
 * time step (the only one that reads q_n's and writes q_out's low-order parts, CC_F32_PERT). */
cc_status cutcell_rk_stage(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                           const double *base, cc_prec prec, const cc_state *q_n, const cc_state *q_s,
                           cc_state *q_out, double stage_dt, int32_t final_stage, int64_t *dev_status,
                           cc_stream_t stream);

/* The update half of cutcell_rk_stage alone: q_out = q_n + stage_dt * L(q_s) at group masters
 * and predicted points, solid cells zeroed.  Absorbed cells and diagnosed lattice points of q_out
 * are left for a following cutcell_diagnose(q_out), which completes the stage (used to time the
 * fused update kernel separately). */
cc_status cutcell_rk_update(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                            const double *base, cc_prec prec, const cc_state *q_n, const cc_state *q_s,
                            cc_state *q_out, double stage_dt, int32_t final_stage, int64_t *dev_status,
                            cc_stream_t stream);

/* The paper's own time stepping (Sec. 2.2): leap-frog with the Robert-Asselin filter, with the
 * perturbation pressure p' as the prognostic thermodynamic variable (Sec. 2.1, eq. heat).  A state
 * in "p' form" holds p' [Pa] in its rth slot (and rth_lo for CC_F32_PERT); every other field is as in
 * the (rho theta)' form.
 *
 * cutcell_pform converts q in place at every non-solid cell through the equation of state
 * p = p0 (R rho theta / p0)^(cp/cv): to_p != 0: (rho theta)' -> p', else p' -> (rho theta)'.
 *
 * cutcell_lf_step advances one step.  first != 0: a forward step q_p = q_0 + dt L(q_0) (q_m is not
 * read and may be NULL; q_0 is left as it is).  Else q_p = q_m + 2 dt L(q_0), with q_m the filtered
 * state of the previous time level, and then q_0 is filtered in place: q_0 += nu (q_m - 2 q_0 + q_p)
 * (Robert-Asselin, weight nu in [0, 1/2]).  L is the merged-cell tendency of cutcell_tendency
 * (diffusion and sponge included) at (rho theta)' from p' of q_0, except that p' takes the (rho
 * theta)' tendency times (cp/cv) p / (rho theta) = (cp/cv) R (p/p0)^(R/cp) (the chain rule of the
 * equation of state; eq. heat).  Updates and the filter act at group masters (rho', p') and
 * predicted points (momentum); solid cells of q_p are zeroed and q_p takes the velocity-diagnostic
 * pass (absorbed cells mirror the master's p').  The filtered q_0 keeps its diagnosed points and
 * absorbed cells as they were (the scheme never reads them).  With the low-order arrays
 * (CC_F32_PERT) rho' and p' are carried with them through update and filter, so mass stays
 * conserved.  The update runs the kernels of cutcell_rk_update (grid.tile applies) as one stage of
 * step 2 dt.  work: caller-allocated device memory of cutcell_lf_workspace_bytes(grid, prec) bytes
 * ((rho theta)' of q_0 and zeroed scratch), not read across calls.  q_m, q_0, q_p distinct.
 * Non-finite results are counted into dev_status[2].  The caller rotates (q_m, q_0, q_p) <-
 * (q_0, q_p, q_m) between steps. */
size_t cutcell_lf_workspace_bytes(const cc_grid *grid, cc_prec prec);
cc_status cutcell_pform(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom, const double *base,
                        cc_prec prec, cc_state *q, int32_t to_p, cc_stream_t stream);
cc_status cutcell_lf_step(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom, const double *base,
                          cc_prec prec, const cc_state *q_m, cc_state *q_0, cc_state *q_p, void *work,
                          double dt, double nu, int32_t first, int64_t *dev_status, cc_stream_t stream);

/* Conservation sums (FP64, deterministic order): out[4] = { M' = sum Vgroup dV rho',
 * Theta' = sum Vgroup dV (rho theta)', M_total (with the base density at each master's level),
 * E = internal + potential energy of the groups + kinetic energy at predicted points }.  Mass is
 * conserved (Sec. 2.4); E is reported only.  workspace: cutcell_reduce_workspace() bytes. */
size_t cutcell_reduce_workspace(const cc_grid *grid);
cc_status cutcell_reduce(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                         const double *base, cc_prec prec, const cc_state *q, void *workspace,
                         double *out, cc_stream_t stream);

/* cutcell_reduce without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The block
 * partial sums live in a static device array of the library (4 x 1024 doubles = 32 KiB, one copy
 * per device, held until the process ends; its address is looked up once per device on the first
 * call with that device current).  The call itself allocates and frees nothing.  Every call on a
 * device shares that device's array: calls that overlap on one device (on different streams, or
 * from different threads) race and must be ordered by the caller.  Same arguments, results and
 * errors as cutcell_reduce; CC_EDEVICE when the array's address cannot be obtained. */
cc_status cutcell_reduce_noalloc(const cc_grid *grid, const cc_phys *phys, const cc_geom *geom,
                                 const double *base, cc_prec prec, const cc_state *q, double *out,
                                 cc_stream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Batched blocks.  A block is a uniform grid with its own geometry, base state and three state
 * buffers.  A batch steps all its blocks with one update launch and one diagnostic launch per
 * Runge-Kutta stage (per level); the launch enumerates the tiles of all blocks, so blocks of uneven
 * size balance by tile count (the paper gives every thread equal cubes instead, Sec. 2.2, 2.5).
 *
 *  - Ensembles (amr_batch_create): independent periodic domains, all of level 0.
 *  - Refined grids (amr_hierarchy_create, Sec. 2.2): blocks of levels 0..L over one laterally
 *    periodic domain of domain0[3] level-0 cells; level l has spacing and time step 2^-l of level
 *    0's.  Each block's grid is a padded box: the block's own cells [ilo, ihi) and ghost cells
 *    beyond them at the block's resolution (the same terrain, heights relative to the box bottom
 *    grid.z0).  Own cells of one level do not overlap; own cells of all levels tile the domain
 *    except buried regions; a coarse cell's eight children lie in one fine block.  Ghost cells are
 *    integrated on like own cells and refilled: after every stage from same-level blocks (copy);
 *    after every level-l step, level-l ghosts owned by level l+1 get the eight-point average (momentum:
 *    the coincident fine lattice point) and level-(l+1) ghosts owned by level l get the coarse field
 *    interpolated linearly to their own centre and lattice point (the parent's values where the
 *    coarse stencil meets terrain, the ground or the lid; an odd fine lattice level over a coarse
 *    level that is not predicted takes the coarse level above).  Values cross levels as
 *    perturbations from each level's reference: the scalars from its base state, the momentum at
 *    predicted points from its reference flow rhobar_c(K) (u0, v0, 0).  A level-l step follows two
 *    level-(l+1) steps (fine first).  Flux matching: the fine advective fluxes through a coarse-fine
 *    face, summed over the two fine final stages (x dt_fine), replace dt x the coarse flux in the
 *    coarse final stage, which conserves mass exactly (the diffusive fluxes are not matched).  The
 *    ghost width must cover the stages between refills and the diagnostic reach (6 cells: 2 fine
 *    steps x 3 stages; 12 with the artificial diffusion, whose stencil reaches two cells); a block
 *    box holds fewer than 2^28 slots; coarse-fine interfaces must stay clear of cut and merged cells
 *    (counted into dev_status[5] otherwise).  Diffusion and sponge act on every block (the sponge
 *    from the domain's lid height, cc_phys.ztop).
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    cc_grid grid;
    cc_phys phys;
    cc_geom geom;         /* geometry and merge map of the block (cutcell_geometry/_merge_map) */
    const double *base;   /* base state of the block (cutcell_base_state) */
    cc_state q[3];        /* three state buffers; the current state starts in q[0] (the float form
                             needs rho_lo and rth_lo in all three) */
    int32_t level;        /* refinement level (0 for ensemble members) */
    int32_t org[3];       /* level-l global index of grid cell (0,0,0) (may be negative; x and y
                             wrap periodically); ignored by amr_batch_create */
    int32_t ilo[3];       /* the block's own cells are grid cells [ilo, ihi) in each direction; */
    int32_t ihi[3];       /* the others are ghost cells; ignored by amr_batch_create */
} cc_block;

typedef struct cc_batch_s *cc_batch;

/* Device workspace (bytes) that holds the descriptors of nblocks independent blocks. */
size_t amr_batch_workspace_bytes(int32_t nblocks, cc_prec prec);

/* Describe nblocks level-0 blocks (independent periodic domains) to the device: copies the
 * descriptors into `workspace`, which must stay allocated until amr_batch_destroy, and synchronises
 * `stream`.  `tile` selects the update kernel's tile shape as cc_grid.tile does (ids 0, 1, 6, 7, 8, 9, 11, 12; one
 * shape for the batch; smaller shapes are taken when a block cannot hold it).  The handle is host
 * state owned by the caller.  Blocks with level != 0 return CC_EINVAL. */
cc_status amr_batch_create(const cc_block *blocks, int32_t nblocks, cc_prec prec, int32_t tile,
                           void *workspace, cc_batch *out, cc_stream_t stream);

/* Workspace (bytes) of a refined grid: descriptors, ghost-refill tables and flux registers.
 * Validates the layout (CC_EINVAL with the reason in cutcell_last_error). */
cc_status amr_hierarchy_workspace_bytes(const cc_block *blocks, int32_t nblocks, cc_prec prec,
                                        const int32_t domain0[3], size_t *bytes);

/* Describe a refined grid (see above) to the device: builds the refill and flux-matching tables on
 * the host, uploads them with the descriptors into `workspace` (>= the size above; kept until
 * amr_batch_destroy), clears the flux registers and synchronises `stream`. */
cc_status amr_hierarchy_create(const cc_block *blocks, int32_t nblocks, cc_prec prec, int32_t tile,
                               const int32_t domain0[3], void *workspace, size_t workspace_bytes,
                               cc_batch *out, cc_stream_t stream);

/* Refill every ghost cell of a refined grid from the current states (same level, coarse to fine,
 * fine to coarse).  Call once after the initial states are set. */
cc_status amr_hierarchy_sync(cc_batch batch, cc_stream_t stream);

/* nsteps level-0 steps of dt (Sec. 2.2: level l takes 2^l steps of dt 2^-l, finest first), in place
 * in the blocks' buffers; each step of a level is a three-stage Runge-Kutta step with one update and
 * one diagnostic launch per stage over the level's blocks, plus refills and flux matching.  Ensembles
 * have one level.  use_graph != 0: the sequence is captured once into a hipGraph (cached per nsteps,
 * dt, starting buffers and status pointer) and replayed as a single graph launch on `stream`.  Device
 * conditions are counted into dev_status as for the single-grid calls. */
cc_status amr_block_step(cc_batch batch, double dt, int32_t nsteps, int32_t use_graph, int64_t *dev_status,
                         cc_stream_t stream);

/* Index (0..2) of the buffer holding level `level`'s current state (-1 for a bad level). */
int32_t amr_batch_current(cc_batch batch, int32_t level);

/* Number of levels of the batch (1 for ensembles). */
int32_t amr_batch_levels(cc_batch batch);

/* Launch sizes of one level: out[8] = {blocks, regular-point tiles, band-point tiles, diagnostic
 * columns, same-level refill entries refilled before the diagnostics, those refilled after them (the
 * ghost cells within reach of the next stage's update), coarse-to-fine entries, fine-to-coarse
 * entries}. */
cc_status amr_batch_info(cc_batch batch, int32_t level, int64_t out[8]);

/* Release the handle (graph executables, capture stream). */
cc_status amr_batch_destroy(cc_batch batch);

/* Host helper: copies dev_status to the host (synchronising `stream`) and maps the first non-zero
 * counter to its status code. */
cc_status cutcell_check_status(const int64_t *dev_status, int64_t *host_copy, cc_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CUTCELL_H */
