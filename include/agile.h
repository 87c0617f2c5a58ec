/*
 * agile.h -- C-ABI of the MI355X block-AMR finite-volume library.
 *
 * The library advances conservation laws dU/dt + div F(U) = 0 (AGILE 1.0,
 * Sec. 2.3) on a static block-structured AMR mesh of 16^3-cell blocks with
 * two ghost layers (Sec. 3.1) on one AMD Instinct MI355X (gfx950).  One
 * update step is: ghost fill across blocks (same-level copy, restriction and
 * minmod-limited prolongation at 2:1 level jumps; Sec. 2.1.2-2.1.3), then per
 * SSP Runge-Kutta stage: conservative-to-primitive conversion, PLM
 * reconstruction (minmod or van Leer), HLL/HLLC/LF Riemann flux (Table 1),
 * flux divergence with coarse-fine flux correction, stage combination;
 * finally the CFL signal-speed reduction that sets the next dt (the "Set dt"
 * node, Sec. 2.1.2).
 *
 * Conventions for every entry point:
 *   - Return value: AGILE_OK (0) or a negative AGILE_E* code.  No exception
 *     or abort crosses the ABI (a failed host allocation inside a call is
 *     reported as AGILE_ENOMEM).  The first error on a mesh is sticky: later
 *     calls on that mesh return AGILE_ESTATE until agile_mesh_destroy.
 *     agile_last_error() gives a message for the sticky error.
 *   - Streams: all device work of a mesh is enqueued on cfg.stream (a
 *     hipStream_t, NULL = the default stream).  Calls that return host data
 *     (agile_dt, agile_readback / agile_read_ghosts into host memory)
 *     synchronise that stream; every other call is asynchronous.
 *   - Threads: one mesh must not be used from two threads at once; different
 *     meshes may be used from different threads and streams.
 *   - Ownership: the caller owns the config, block descriptors and input /
 *     output arrays; the library copies what it needs during the call and
 *     never frees caller memory.  Device memory of a mesh is allocated by the
 *     library (hipMalloc) in agile_set_blocks and freed in agile_mesh_destroy,
 *     or, with cfg.dev_pool set, carved from the caller's memory.
 *   - Layouts: a state array is float64 [nblocks][nvar][B][B][B] (x
 *     fastest, B = cfg.block_n), blocks in the caller's agile_block_desc
 *     order.  Conserved
 *     variables: Euler rho, m_x, m_y, m_z, e (Sec. 2.3.1); MHD-GLM adds
 *     B_x, B_y, B_z, psi (Sec. 2.3.3).
 */
#ifndef AGILE_H
#define AGILE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct agile_mesh agile_mesh; /* opaque, owned by the library */

enum {
    AGILE_OK = 0,
    AGILE_EINVAL = -1,        /* bad argument, config or mesh (overlap, gap, 2:1 violation) */
    AGILE_ENOMEM = -2,        /* device or host allocation failed */
    AGILE_EDEVICE = -3,       /* a HIP runtime call failed */
    AGILE_ESTATE = -4,        /* call out of order, or a sticky error is set */
    AGILE_ENONPHYSICAL = -5   /* rho <= 0, p <= 0 or NaN met by a kernel (no floors) */
};

enum { AGILE_EULER = 0, AGILE_MHD_GLM = 1, AGILE_SRHD = 2 };   /* physics (Sec. 2.3.1, 2.3.3,
                                                                  2.3.4) */
enum { AGILE_HLL = 0, AGILE_HLLC = 1, AGILE_LF = 2 }; /* Riemann solver (Table 1); LF: local
                                                      Lax-Friedrichs, the flux of Sec. 3.1 */
enum { AGILE_MINMOD = 0, AGILE_VANLEER = 1 };       /* reconstruction slope limiter */
enum { AGILE_FP64 = 0, AGILE_FP32_FLUX = 1 };       /* reconstruction + flux precision */

typedef struct {
    int physics;          /* AGILE_EULER (rho, m, e), AGILE_MHD_GLM (rho, m, e,
                             B, psi) or AGILE_SRHD (D, m, tau with c = 1;
                             riemann must be AGILE_LF) */
    int riemann;          /* AGILE_HLL, AGILE_HLLC or AGILE_LF (HLLC, LF: Euler
                             only; MHD-GLM offers HLL, Table 1) */
    int precision;        /* AGILE_FP64, or AGILE_FP32_FLUX: reconstruction and
                             Riemann flux in float, state / divergence / flux
                             correction / dt in double */
    double gamma;         /* ratio of specific heats (Sec. 2.3.1 closure; the
                             ideal-gas index of Sec. 2.3.4 for SRHD) */
    double cfl;           /* dt = cfl / max_cells sum_d (|v_d| + c_d) / dx
                             (SRHD: the largest |characteristic speed| along d) */
    double glm_alpha;     /* GLM decay parameter alpha (Sec. 2.3.3), MHD only */
    int block_n;          /* cells per block edge B: 16, 32 or 64 (the block
                             sizes of Sec. 3.1, Table 4).  A block is the unit
                             of refinement, 2:1 balance, the caller's layout
                             and the regrid estimate; the device stores and
                             updates it as (B/16)^3 tiles of 16^3 cells, whose
                             face ghosts within a block are read in place like
                             those of same-level neighbours, so every B gives
                             the same cell values.  Batch requests: 16. */
    int nghost;           /* ghost layers: must be 2 */
    int base_blocks[3];   /* blocks per axis on level 1 */
    double lo[3], hi[3];  /* periodic domain; cells must be cubic */
    int max_level;        /* finest level allowed, 1..12 */
    void *stream;         /* hipStream_t (NULL = default stream) */
    int limiter;          /* AGILE_MINMOD (0) or AGILE_VANLEER (the limiter of the
                             benchmark of Sec. 3.1); MHD: minmod */
    int rk_stages;        /* SSP Runge-Kutta stages: 2 (also 0) or 3 (the paper's
                             three-step scheme, Sec. 3.1); MHD: 2 */
    void *dev_pool;       /* optional caller-owned device memory (e.g. a torch
                             tensor's storage), 256-byte aligned, NULL = the
                             library allocates.  When set, every device array
                             of the mesh is carved from it: agile_set_blocks
                             returns AGILE_ENOMEM if dev_pool_bytes is below
                             agile_plan_stats.device_bytes, and a larger pool
                             leaves room for regrids to grow the mesh.  The
                             caller keeps it valid until agile_mesh_destroy and
                             must not touch it meanwhile; the library never
                             frees it.  Must be NULL in a batch request. */
    size_t dev_pool_bytes;/* size of dev_pool in bytes */
} agile_config;

typedef struct {
    int level;            /* 1 = base level */
    int idx[3];           /* block coordinates on that level, 0 <= idx[d] < base_blocks[d] << (level-1) */
} agile_block_desc;

/* Create an empty mesh: the host side of "Init level one" in the
 * initialisation flow chart (Sec. 2.1.2, Fig. 1), before any block exists.
 * Validates the config (block_n 16, 32 or 64, nghost == 2, cubic cells, supported
 * physics / solver / precision).  No device memory is allocated here.  *out
 * is set only on success.  Errors: AGILE_EINVAL, AGILE_ENOMEM. */
int agile_mesh_create(const agile_config *cfg, agile_mesh **out);

/* Set the leaf blocks and their interior state.  The blocks must tile the
 * periodic domain without overlap and satisfy 2:1 balance across faces.
 * Builds the neighbour, ghost-fill and flux-correction tables on the host
 * (mesh bookkeeping stays on the host, Sec. 2.1.2), allocates device memory
 * and uploads the state.  u: [nblocks][nvar][B][B][B] float64, in host
 * memory (u_on_device = 0, copied synchronously) or device memory
 * (u_on_device = 1, read on cfg.stream).  May be called again to replace the
 * mesh.  Errors: AGILE_EINVAL, AGILE_ENOMEM, AGILE_EDEVICE. */
int agile_set_blocks(agile_mesh *m, int64_t nblocks, const agile_block_desc *blocks,
                     const double *u, int u_on_device);

/* Fill the ghost data of every block from the current state: restriction
 * into coarse ghosts next to finer blocks, then prolongation into fine ghosts
 * next to coarser blocks, level by level (same-level ghosts are read in place
 * from the neighbours and need no fill).  SRHD prolongs the primitives
 * (rho, Gamma v, p) and converts the children back, which keeps them physical
 * next to strong relativistic shocks.  agile_step does this itself; this
 * call exists for inspection.  Errors: AGILE_ESTATE. */
int agile_fill_ghosts(agile_mesh *m);

/* dt = cfl / max over all leaf cells of sum_d (|v_d| + c_d)/dx_l, for the
 * current state (exact maximum, independent of reduction order); c_d is the
 * sound speed (Euler) or the fast magnetosonic speed along d (MHD).  SRHD
 * (Sec. 2.3.4): the sum of the largest |characteristic speed| along each
 * axis, from the primitives of the con2prim root in xi = Gamma^2 rho h,
 * formed with reciprocal arithmetic (a few ulp from an IEEE evaluation; the
 * same bits as the dt that agile_step_cfl takes from the last stage).
 * Blocking.  Errors: AGILE_ESTATE, AGILE_ENONPHYSICAL, AGILE_EDEVICE. */
int agile_dt(agile_mesh *m, double *dt_out);

/* One SSP Runge-Kutta step with the given dt > 0: the "Advance Solution"
 * node of the time-evolution flow chart (Sec. 2.1.2, Fig. 2) -- ghost fills
 * and, per stage, the stage update and the coarse-fine flux correction; two
 * stages (SSP-RK2, cfg.rk_stages = 0 or 2) or three (SSP-RK3,
 * cfg.rk_stages = 3, the three-step scheme of Sec. 3.1).  MHD-GLM (Sec. 2.3.3): the cleaning speed
 * is c_h = max over leaf cells of max_d (|v_d| + c_f,d) of the state at the
 * start of the step; the Dedner interface step sets (B_n, psi) at each face;
 * psi decays by the exact factor exp(-(dt/2) c_h alpha / dx_l) before and
 * after the two stages (Strang splitting of the damping term).
 * Asynchronous.  Errors: AGILE_EINVAL, AGILE_ESTATE, AGILE_EDEVICE. */
int agile_step(agile_mesh *m, double dt);

/* nsteps turns of the time-evolution loop of Fig. 2 (Sec. 2.1.2) without IO
 * or regrid: "Set dt" on the device from the CFL signal maximum of the
 * current state (the agile_dt formula; no host round trip), then one SSP
 * Runge-Kutta step as agile_step.  Asynchronous.  The dt of the last step
 * taken is returned by agile_last_dt.  Errors: AGILE_EINVAL (nsteps < 0),
 * AGILE_ESTATE, AGILE_EDEVICE. */
int agile_step_cfl(agile_mesh *m, int nsteps);

/* dt used by the most recent step (blocking). */
int agile_last_dt(agile_mesh *m, double *dt_out);

/* Copy the interior state to u_out ([nblocks][nvar][B][B][B] float64, in
 * the caller's block order): the "update host(w)" transfer before IO in the
 * time-evolution flow chart (Sec. 2.1.2, Fig. 2), or a device-to-device
 * copy.  capacity_doubles must be at least nblocks*nvar*B^3.  Host destination (out_on_device = 0): blocking; device
 * destination: asynchronous on cfg.stream.  Checks the non-physical flag.
 * Errors: AGILE_EINVAL, AGILE_ESTATE, AGILE_ENONPHYSICAL, AGILE_EDEVICE. */
int agile_readback(agile_mesh *m, double *u_out, int64_t capacity_doubles, int out_on_device);

/* Copy the face ghosts of every block as the update reads them (block_n 16
 * only; AGILE_EINVAL otherwise):
 * [nblocks][6 faces -x,+x,-y,+y,-z,+z][nvar][512], each face slab 2 cells
 * deep in (k, j, i) order with the ghost layer index increasing with the
 * coordinate.  Calls agile_fill_ghosts first.  capacity_doubles >=
 * nblocks*6*nvar*512.  Same destination rules as agile_readback. */
int agile_read_ghosts(agile_mesh *m, double *g_out, int64_t capacity_doubles, int out_on_device);

/* Host-only planning (no device work, usable without a GPU): validates a
 * block list exactly as agile_set_blocks does and reports the sizes of the
 * tables it would build and the device bytes the mesh would occupy (used by
 * admission control of the batched serving loop).  msg (may be NULL)
 * receives the validation message.  Errors: AGILE_EINVAL. */
typedef struct {
    int64_t nblocks;
    int64_t same_level_faces;   /* block faces with a same-level neighbour */
    int64_t restrict_tasks;     /* coarse block faces next to 4 finer blocks */
    int64_t prolong_tasks;      /* fine block faces next to a coarser block */
    int64_t reflux_blocks;      /* coarse blocks with coarse-fine faces */
    int64_t flux_registers;     /* stored face-flux slabs (coarse + fine sides) */
    int levels;                 /* finest level present */
    int nvar;
    int64_t device_bytes;       /* device memory of the mesh alone: what
                                   agile_set_blocks allocates, and the least
                                   dev_pool_bytes it accepts */
    int prolong_launches;       /* prolongation launches per ghost fill: levels
                                   share one unless a level reads ghosts
                                   prolonged on the level below */
    int fused_correction;       /* 1: the flux correction after a stage and the
                                   restriction of the ghost fill that follows
                                   share one launch (no coarse block with a
                                   coarse-fine face also borders a coarser
                                   block) */
} agile_plan_stats;

int agile_plan(const agile_config *cfg, int64_t nblocks, const agile_block_desc *blocks, agile_plan_stats *out,
               char *msg, int msg_len);

/* Kernel timing with HIP events recorded on the mesh's stream around every
 * launch of the selected kernel classes: AGILE_K_STAGE (the fused stage
 * update), AGILE_K_FILL (restriction + prolongation), AGILE_K_REFLUX (flux
 * correction), AGILE_K_DT (signal-speed reduction).  agile_profile(m, kinds)
 * times the classes whose bit (1 << AGILE_K_*) is set in kinds
 * (AGILE_PROFILE_ALL: every class, 0: none) and clears the totals; timed
 * steps launch eagerly (no graph replay).  With AGILE_PROFILE_KEEP or-ed
 * into kinds it only switches the timed classes, without waiting and
 * without clearing, so that a loop can time some of its steps and sum them.
 * agile_profile_read synchronises the stream and returns the summed kernel
 * time (ms) and the number of launches of one class since the last clear.
 * Errors: AGILE_EINVAL, AGILE_EDEVICE. */
enum { AGILE_K_STAGE = 0, AGILE_K_FILL = 1, AGILE_K_REFLUX = 2, AGILE_K_DT = 3 };
enum { AGILE_PROFILE_ALL = 15, AGILE_PROFILE_KEEP = 16 };
int agile_profile(agile_mesh *m, int kinds);
int agile_profile_read(agile_mesh *m, int kind, double *ms_total, int64_t *launches);

/* Stage-kernel shape and step options of a mesh.  None of them changes the
 * arithmetic of any cell, so results are bitwise identical for every value.
 *   AGILE_OPT_GRAPH: 1 = agile_step_cfl replays one captured hipGraph per
 *                    step (needs a non-NULL cfg.stream; ignored otherwise and
 *                    while kernel timing is on);
 *   AGILE_OPT_KSLAB: z-planes per workgroup of the stage kernel, 16, 8 or 4
 *                    (smaller slabs give more workgroups for small meshes),
 *                    or 0 (the default): 16 from 512 active blocks on, 8 from
 *                    256, else 4; setting it sets AGILE_OPT_KSLAB_LAST too;
 *   AGILE_OPT_XCD:   1 = each of the 8 XCDs gets one contiguous range of
 *                    blocks (neighbours share that XCD's L2), 0 = the plain
 *                    workgroup order (the default); setting it sets
 *                    AGILE_OPT_XCD_LAST too;
 *   AGILE_OPT_KSLAB_LAST, AGILE_OPT_XCD_LAST: the same for the last stage of
 *                    a step only (the one that also reduces the signal rate);
 *                    the two others then apply to the first and middle stages.
 * May be set before or after agile_set_blocks.  Errors: AGILE_EINVAL. */
enum { AGILE_OPT_GRAPH = 0, AGILE_OPT_KSLAB = 1, AGILE_OPT_XCD = 2, AGILE_OPT_KSLAB_LAST = 3, AGILE_OPT_XCD_LAST = 4 };
int agile_mesh_set_option(agile_mesh *m, int option, int value);
int agile_mesh_get_option(const agile_mesh *m, int option, int *value);

/* Autotuner: chooses the (KSLAB, XCD) shape of the first stage and that of
 * the last stage of a step (the middle SSP-RK3 stage takes the first stage's).
 * With library-allocated memory it times whole steps on a temporary device
 * copy of the state, restoring the state after each trial; with a caller-owned
 * pool (or when that copy cannot be allocated) it times single launches of
 * each stage kind reading the current state and writing only the stage
 * buffer.  The mesh state, simulated time and dt are unchanged.  Blocking.
 * Errors: AGILE_ESTATE, AGILE_EDEVICE. */
int agile_mesh_tune(agile_mesh *m);

/* Simulated time reached: the sum of the dt of all steps taken (blocking). */
int agile_mesh_time(agile_mesh *m, double *t_out);

/* ---- batched serving --------------------------------------------------------
 * A batch serves independent simulation requests (meshes) on one GPU: each
 * request is queued with its own mesh, initial state and step count; requests
 * are admitted first come, first served whenever their device footprint fits
 * in the batch's block pool (a request that arrives while others run joins at
 * the next tick); every tick advances all running requests by one SSP-RK2
 * step, each with its own CFL dt, through one batched launch sequence (ghost
 * fills, stage updates and flux corrections of all meshes and levels at
 * once), optionally replayed from a captured hipGraph; a request that reached
 * its step count stops and keeps its state until collected.  Every mesh gives
 * bitwise the same result alone (agile_mesh) and in any mix.  All meshes of a
 * batch share physics, Riemann solver and precision; gamma, CFL, domain and
 * mesh are per request.  One batch must not be used from two threads. */
typedef struct agile_batch agile_batch;

typedef struct {
    int physics, riemann, precision;  /* shared by every request: AGILE_EULER with
                                         HLL, HLLC or LF, or AGILE_SRHD with LF */
    int64_t budget_bytes;             /* device memory of the block pool (<= 0: 16 GiB) */
    int max_meshes;                   /* resident requests at most */
    int use_graph;                    /* 1: replay each tick's step from a captured hipGraph
                                         (needs a non-NULL stream) */
    int autotune;                     /* 1: tune the stage shape once per size class
                                         (power of two of running blocks) */
    void *stream;                     /* hipStream_t of all device work (NULL = default) */
    void *dev_pool;                   /* optional caller-owned device memory, 256-byte
                                         aligned: the block pool is carved from it and
                                         budget_bytes is ignored; kept valid by the
                                         caller until agile_batch_destroy */
    size_t dev_pool_bytes;
    int64_t max_active_blocks;        /* step-latency budget: a queued request is
                                         admitted only while the running requests'
                                         blocks plus its own stay within this bound
                                         (a request is always admitted into an idle
                                         batch); a tick then advances at most about
                                         this many blocks.  0: memory is the only
                                         bound */
} agile_batch_config;

typedef struct {
    int64_t queued;          /* requests waiting for admission after the tick */
    int64_t resident;        /* requests holding device memory (running or finished) */
    int64_t active;          /* requests advanced by the tick */
    int64_t admitted;        /* requests admitted during the tick */
    int64_t finished;        /* requests that reached their step count in the tick */
    int64_t active_blocks;   /* blocks updated by the tick */
    int64_t free_blocks;     /* free pool blocks after the tick */
    double admit_ms;         /* host time spent admitting requests (uploads included) */
    double build_ms;         /* host time spent rebuilding the batched tables and
                                capturing / instantiating the step graph */
    int64_t graph_builds;    /* step graphs built during the tick (0 or 1) */
} agile_tick_info;

enum { AGILE_REQ_UNKNOWN = 0, AGILE_REQ_QUEUED = 1, AGILE_REQ_RUNNING = 2, AGILE_REQ_FINISHED = 3 };

/* Create a batch; allocates the whole block pool (or carves it from
 * cfg.dev_pool).  Errors: AGILE_EINVAL, AGILE_ENOMEM. */
int agile_batch_create(const agile_batch_config *cfg, agile_batch **out);

/* Pool size and free blocks (in 16^3 blocks). */
int agile_batch_capacity(const agile_batch *b, int64_t *cap_blocks, int64_t *free_blocks);

/* Queue a request for nsteps CFL steps.  u is its initial state
 * ([nblocks][5][16][16][16] float64, caller's block order).  mesh_cfg and
 * blocks are copied.  Host u (u_on_device = 0) is copied as well.  Device u
 * (u_on_device = 1) is not: it is read on the batch's stream by the tick that
 * admits the request, so the caller keeps it valid and unchanged until the
 * request has left the queue (status no longer AGILE_REQ_QUEUED, or
 * cancelled).  tag identifies the request (unique among queued and resident
 * requests).  A request runs the batch's physics, solver and precision with
 * minmod and SSP-RK2; a config asking for anything else is rejected.
 * Errors: AGILE_EINVAL (bad mesh, config or duplicate tag), AGILE_ENOMEM
 * (larger than the whole pool), AGILE_ESTATE. */
int agile_batch_submit(agile_batch *b, const agile_config *mesh_cfg, int64_t nblocks, const agile_block_desc *blocks,
                       const double *u, int u_on_device, int64_t nsteps, uint64_t tag);

/* One tick: admit queued requests in arrival order while the head fits (in
 * memory, and within max_active_blocks), then advance every running request
 * by one step.  Returns after the step has
 * completed on the device.  Errors: AGILE_ESTATE, AGILE_EDEVICE (sticky). */
int agile_batch_tick(agile_batch *b, agile_tick_info *info);

/* Where a request is: AGILE_REQ_* and steps taken. */
int agile_batch_status(agile_batch *b, uint64_t tag, int *state, int64_t *steps_done);

/* Collect a finished request: copies its state (caller's block order) to
 * u_out (host, or device when out_on_device = 1), returns its step count and
 * simulated time, and frees its device memory.  Returns AGILE_ENONPHYSICAL
 * (after copying) if a kernel met a non-physical state in that request.
 * Errors: AGILE_EINVAL (unknown tag, small buffer), AGILE_ESTATE (still
 * running). */
int agile_batch_result(agile_batch *b, uint64_t tag, double *u_out, int64_t capacity_doubles, int out_on_device,
                       int64_t *steps_done, double *t_reached);

/* Drop a queued or resident request. */
int agile_batch_cancel(agile_batch *b, uint64_t tag);

void agile_batch_destroy(agile_batch *b);
const char *agile_batch_last_error(const agile_batch *b);

/* ------------------------------------------------------------------------
 * Regrid: device error estimate, host refine / coarsen decision, device data
 * transfer (the "AMR error estimator" and "AMR Coarsen Refine" nodes of the
 * flow charts, Fig. 1 and Fig. 2; the estimator follows Loehner's scheme,
 * named in Sec. 4.3).
 *
 * Estimator of a cell: Loehner's normalised second difference of one
 * conserved variable, summed over the three axes (face neighbours only,
 * face ghosts at block sides):
 *   E = sqrt(sum_d a_d^2 / sum_d b_d^2),  a_d = (u+ - u) - (u - u-),
 *   b_d = (|u+ - u| + |u - u-|) + eps((|u+| + 2|u|) + |u-|),
 * evaluated with IEEE arithmetic in that order (0 <= E <= 1; E = 0 where the
 * variable is zero on the whole stencil, so both sums vanish); the block
 * value is the maximum over its cells. */
typedef struct {
    int variable;       /* conserved variable index (0 = density) */
    int max_level;      /* finest level a refinement may create, 1 .. cfg.max_level */
    double refine;      /* refine a leaf whose estimate exceeds this */
    double coarsen;     /* coarsen a complete octet whose 8 estimates are all below this */
    double eps;         /* noise filter of the estimator, > 0 (0.01 is usual) */
} agile_regrid_params;

typedef struct {
    int64_t old_blocks, new_blocks;
    int64_t refined;    /* leaves replaced by their 8 children */
    int64_t coarsened;  /* octets replaced by their parent */
} agile_regrid_stats;

/* Per-block estimate of the current state into out_host[nblocks] (caller's
 * block order).  Fills the ghosts first; blocking.  Errors: AGILE_EINVAL,
 * AGILE_ESTATE, AGILE_EDEVICE. */
int agile_mesh_error(agile_mesh *m, int variable, double eps, double *out_host);

/* Host-only decision (no GPU): from a block list and its per-block estimate,
 * the new leaves sorted by (level, x, y, z): leaves above p->refine below
 * p->max_level are refined; complete octets (level >= 2) all below
 * p->coarsen and none refined are coarsened; refinement spreads to coarser
 * face neighbours and coarsening is withdrawn until 2:1 balance holds across
 * faces (one level of change per leaf).  out receives at most capacity
 * blocks; *n_out the number of new leaves (also when it exceeds capacity,
 * then AGILE_EINVAL).  stats may be NULL. */
int agile_regrid_decide(const agile_config *cfg, int64_t nblocks, const agile_block_desc *blocks,
                        const double *err, const agile_regrid_params *p, int64_t capacity, agile_block_desc *out,
                        int64_t *n_out, agile_regrid_stats *stats);

/* Regrid the mesh in place: estimate (agile_mesh_error), decide
 * (agile_regrid_decide), then fill the new leaves on the device -- a copy
 * where a leaf stays, limited linear prolongation from the parent where it
 * was refined (the ghost prolongation formula, on primitives for SRHD,
 * which is then not exactly conservative), the mean of the 8 children
 * where an octet was coarsened -- and rebuild the tables.  Afterwards the
 * mesh's blocks are the new sorted list (agile_mesh_blocks); the simulated
 * time, the last dt and the non-physical flag carry over.  The new state is
 * staged in the mesh's stage buffer when the new mesh fits in its device
 * memory; otherwise (the mesh grew) a new device pool with room for growth is
 * allocated -- or, with cfg.dev_pool, AGILE_ENOMEM is returned and the mesh
 * is left as it was (this error is not sticky).  A small task table is
 * allocated and freed inside.  stats may
 * be NULL.  Errors: AGILE_EINVAL, AGILE_ESTATE, AGILE_ENOMEM, AGILE_EDEVICE. */
int agile_mesh_regrid(agile_mesh *m, const agile_regrid_params *p, agile_regrid_stats *stats);

/* Regrid without any device allocation, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).  Does
 * what agile_mesh_regrid does, with two limits: the new mesh must fit in the
 * mesh's existing device memory (a mesh set with headroom -- a caller pool
 * larger than agile_plan_stats.device_bytes, or one grown by an earlier
 * agile_mesh_regrid -- or a regrid that does not grow it), else AGILE_ENOMEM;
 * and it may have at most AGILE_NOALLOC_MAX_BLOCKS blocks, else AGILE_EINVAL.
 * Both refusals leave the mesh as it was and are not sticky (the reason is
 * given by agile_last_error).  The remap task table lives in one static
 * device array per GPU (AGILE_NOALLOC_MAX_BLOCKS records of 40 bytes, held
 * until the process ends) that all calls on that GPU share: two calls that
 * overlap on one GPU race.  The new state is staged in the mesh's own stage
 * buffer.  The device that was current at agile_set_blocks must be current.
 * Host bookkeeping (the decision and the tables) still uses the C++ heap.
 * Blocking.  Errors: AGILE_EINVAL, AGILE_ENOMEM, AGILE_ESTATE, AGILE_EDEVICE. */
enum { AGILE_NOALLOC_MAX_BLOCKS = 65536 };
int agile_mesh_regrid_noalloc(agile_mesh *m, const agile_regrid_params *p, agile_regrid_stats *stats);

/* Regrid a running request between ticks (the regrid of the time-evolution
 * loop, Sec. 2.1.2, Fig. 2, for one request of the batch): the estimate,
 * decision and transfer of agile_mesh_regrid on that request's mesh, its
 * simulated time, dt, flags and steps taken carried over.  When the new mesh
 * fits in the pool beside the other residents it stays resident (its
 * blocks may move in the pool); otherwise its state goes to host memory and
 * the request rejoins the queue at its head, to be admitted again by its new
 * footprint as memory frees up (before any request that arrived later).  Its
 * state and the block order of agile_batch_result are then those of the new
 * sorted leaf list (agile_batch_blocks).  Blocking.  Errors: AGILE_EINVAL
 * (unknown, queued or finished request, bad parameters), AGILE_ENOMEM (the
 * new mesh is larger than the whole pool; the request is unchanged),
 * AGILE_ESTATE, AGILE_EDEVICE (sticky). */
int agile_batch_regrid(agile_batch *b, uint64_t tag, const agile_regrid_params *p, agile_regrid_stats *stats);

/* The current leaf blocks of a queued or resident request, in the order of
 * its state; *n gets the count, AGILE_EINVAL when capacity is smaller. */
int agile_batch_blocks(agile_batch *b, uint64_t tag, int64_t capacity, agile_block_desc *out, int64_t *n);

/* The mesh's current leaf blocks in its block order (the order of
 * agile_set_blocks, or the sorted order after a regrid).  *n gets the count;
 * AGILE_EINVAL when capacity is smaller. */
int agile_mesh_blocks(const agile_mesh *m, int64_t capacity, agile_block_desc *out, int64_t *n);

/* Measurement support (the bandwidth the roofline is compared with, not a
 * step of the method): copy `bytes` (a multiple of 16; both pointers device
 * memory, 16-byte aligned, not overlapping) from src to dst with a plain
 * streaming kernel, each word read and written once, enqueued on `stream`
 * (a hipStream_t, NULL = default).  Asynchronous.  Errors: AGILE_EINVAL,
 * AGILE_EDEVICE. */
int agile_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* Number of leaf blocks and conserved variables of the mesh. */
int agile_mesh_info(const agile_mesh *m, int64_t *nblocks, int *nvar);

/* Release all device and host memory of the mesh (NULL is ignored).  Waits
 * for the mesh's outstanding work. */
void agile_mesh_destroy(agile_mesh *m);

/* Static message for an error code. */
const char *agile_strerror(int code);

/* Message for the mesh's sticky error, or for the last non-sticky refusal
 * ("" if none); valid until the next call on the mesh. */
const char *agile_last_error(const agile_mesh *m);

#ifdef __cplusplus
}
#endif

#endif /* AGILE_H */
