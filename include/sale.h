/*
 * sale.h -- C ABI of libsale.so: the SALE (Simplified Arbitrary
 * Lagrangian-Eulerian) hydrodynamics step on one MI355X (gfx950).
 *
 * One step is the Lagrangian phase on a logically structured 3D hex mesh
 * followed by the Eulerian rezone and advection (a face-flux remap) back to
 * the fixed mesh -- the "Lagrangian rezoning", "Eulerian rezoning" and
 * "Advection" kernels of the ScalSALE framework (arXiv 2209.01983, Sec. I-D
 * and Table I), for a single ideal gas, p = (gamma-1) rho e (Sec. I-C/I-D),
 * with cell-centred density and internal energy and vertex velocities
 * (cell and vertex quantities, Sec. III-C/III-D). The paper prints no scheme
 * equations; the library computes the scheme fixed by the project's FP64
 * oracle: acoustic half-step pressure predictor, von Neumann-Richtmyer +
 * Landshoff viscosity, compatible energy, exact trilinear swept volumes,
 * first-order unsplit donor-cell remap, dual-mesh momentum remap with a
 * kinetic-energy fix, reflective walls on all six faces.
 *
 * The caller-supplied buffers follow the paper's zero-copy "pointer to the
 * data" hand-off (Point_to_data, Sec. III-A) and its C interoperability
 * (Sec. I-D, Table I; Sec. II-A).
 *
 * Conventions for every function:
 *  - Return int: SALE_OK (0) on success, < 0 on error, > 0 informational.
 *    Nothing throws, aborts or exits.
 *  - Ownership: the caller owns every device buffer (workspace, arena,
 *    field destinations). The library owns only small host structs, freed by
 *    sale_destroy / sale_pool_destroy. It never calls hipMalloc/hipFree and
 *    never synchronises the device; only functions documented as
 *    synchronising wait on the caller's stream.
 *  - Streams: a `hip_stream` argument is a hipStream_t (NULL = the null
 *    stream). All device work of a context is ordered on its stream.
 *  - Threading: a context is single-threaded; different contexts may be used
 *    from different threads on different streams.
 *  - Layout of fields exchanged with the caller ("logical layout"):
 *      cell (i,j,k), 0<=i<nx  -> index i + nx*(j + ny*k)
 *      node (i,j,k), 0<=i<=nx -> index i + (nx+1)*(j + (ny+1)*k)
 *    Velocity is three node arrays (u, v, w), i.e. structure of arrays.
 */
#ifndef SALE_H
#define SALE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define SALE_OK 0
#define SALE_DONE 1       /* t >= t_end: the run is complete             */
#define SALE_EINVAL (-1)  /* invalid argument, config or initial data   */
#define SALE_ENOMEM (-2)  /* workspace / arena too small                 */
#define SALE_EHIP (-3)    /* a HIP runtime call failed; see sale_strerror */
#define SALE_ENUMERIC (-4) /* non-finite / non-positive density, negative
                              or non-finite energy, non-finite dt          */
#define SALE_ETANGLE (-5) /* a predictor or Lagrangian cell volume <= 0   */
#define SALE_EBUSY (-6)   /* pool admission refused for now (no free slot
                             or arena range; retry after a release) --
                             apart from SALE_ENOMEM, which a retry cannot
                             cure                                          */

/* ---- enums ------------------------------------------------------------- */
#define SALE_FP64 0       /* every quantity in FP64                      */
#define SALE_MIXED32 1    /* FP32 storage and bulk arithmetic; FP64 for
                             node displacements, swept volumes, volume
                             differences, the CFL dt and the totals (the
                             swept volumes reach the remap's FP32 fluxes
                             as FP32)                                     */
#define SALE_BC_REFLECT 0 /* reflective (slip) wall                      */

#define SALE_EULERIAN 0   /* Lagrangian phase + remap to the fixed mesh  */
#define SALE_LAGRANGIAN 1 /* pure Lagrangian: the mesh moves with the flow */

#define SALE_SOD_X 0          /* Sod tube along x                        */
#define SALE_SEDOV_CORNER 1   /* Sedov blast deposited in cell (0,0,0)   */
#define SALE_USER 2           /* caller arrays                           */
#define SALE_NOH 3            /* Noh implosion toward the corner lo      */

/* status flag bits (sticky, see sale_status) */
#define SALE_FLAG_TANGLE 1u   /* V* <= 0 or V^L <= 0                      */
#define SALE_FLAG_NUMERIC 2u  /* rho <= 0, e < 0, non-finite value or dt  */

/* field mask bits for sale_fields (destinations in ascending bit order) */
#define SALE_F_RHO (1u << 0)    /* cells: density                         */
#define SALE_F_E (1u << 1)      /* cells: specific internal energy        */
#define SALE_F_P (1u << 2)      /* cells: pressure (gamma-1) rho e        */
#define SALE_F_Q (1u << 3)      /* cells: artificial viscosity of the state */
#define SALE_F_U (1u << 4)      /* nodes: x velocity                      */
#define SALE_F_V (1u << 5)      /* nodes: y velocity                      */
#define SALE_F_W (1u << 6)      /* nodes: z velocity                      */
#define SALE_F_STATE (1u << 7)  /* host double[4]: t, steps, next dt, status */
#define SALE_F_TOTALS (1u << 8) /* host double[2]: total mass, total energy */
#define SALE_F_CLOCK (1u << 9)  /* host double[2]: device wall clock (s) at the
                                   run's first pool advance and when its last
                                   step completed in a pool (0: never)     */
#define SALE_F_X (1u << 10)     /* nodes: x position (the moving mesh in the
                                   pure-Lagrangian mode, else the fixed one) */
#define SALE_F_Y (1u << 11)     /* nodes: y position                        */
#define SALE_F_Z (1u << 12)     /* nodes: z position                        */

/* ---- configuration ----------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz;       /* cells per axis, >= 1; (nx+1)(ny+1)(nz+1) * 8
                               must stay below 2^32 bytes (each field array
                               is addressed with 32-bit offsets), e.g. up
                               to 811^3 cells                              */
  double lo[3], hi[3];      /* box; cell size (hi-lo)/n per axis, hi > lo   */
  double gamma;             /* ideal-gas ratio of specific heats, > 1       */
  double cfl;               /* Courant number, 0 < cfl < 1 (default 0.5)    */
  double c_quad, c_lin;     /* viscosity coefficients >= 0 (1.0, 0.5)       */
  double t_end;             /* end time >= 0                                */
  int32_t precision;        /* SALE_FP64 | SALE_MIXED32                     */
  int32_t bc[6];            /* per face (-x,+x,-y,+y,-z,+z): SALE_BC_REFLECT */
  int32_t remap_order;      /* 1 (or 0): first-order donor cell; 2: donor
                               values from limited linear profiles at the
                               swept volume's centroid (van Leer slopes),
                               cells and dual mesh; single runs only (a
                               pool admits order 1)                         */
  int32_t mode;             /* SALE_EULERIAN (default) | SALE_LAGRANGIAN: the
                               paper's Lagrangian rezoning (Table I, Fig. 2a),
                               the mesh moves with the flow and is never
                               remapped. The Lagrangian mode: FP64 only,
                               single runs only (a pool admits SALE_EULERIAN),
                               remap_order ignored (must be <= 1), starts from
                               the Cartesian mesh of lo/hi (any problem kind),
                               per-cell length scale V / largest face area,
                               exact trilinear-hex volumes and corner vectors,
                               SALE_F_Q not available                        */
  double c_hg;              /* viscous hourglass coefficient >= 0 of the
                               Lagrangian mode (Flanagan-Belytschko form;
                               0 disables; e.g. 0.1)                        */
} sale_config;

typedef struct {
  int32_t kind;             /* SALE_SOD_X | SALE_SEDOV_CORNER | SALE_USER |
                               SALE_NOH                                     */
  double sod[5];            /* x_split, rho_L, p_L, rho_R, p_R (u = 0); a cell
                               is "left" iff its centre x < x_split          */
  double sedov[3];          /* rho0, p0, E_dep: uniform rho0, e = p0/((gamma-1)
                               rho0); cell (0,0,0) gets e = E_dep/(rho0 V0)  */
  double noh[3];            /* rho0 > 0, p0 >= 0, u0: uniform rho0, e = p0/
                               ((gamma-1) rho0), node velocity -u0 r/|r| with
                               r = (i dx, j dy, k dz) restricted to the first
                               noh_dims axes (0 at r = 0), wall-normal
                               components zeroed on the walls. The Noh
                               problem (Sec. I-D lists it among ScalSALE's
                               problems) is cold (p0 = 0); a small p0 (e.g.
                               1e-6) keeps e away from zero, where rounding
                               in the kinetic-energy fix can make it
                               negative (SALE_FLAG_NUMERIC)                 */
  int32_t noh_dims;         /* 1 planar (x), 2 cylindrical (x, y), 3 spherical */
  const double *rho, *e;    /* SALE_USER: cells, logical layout             */
  const double *u, *v, *w;  /* SALE_USER: nodes, logical layout; wall-normal
                               components are set to zero on the walls      */
  int32_t user_on_device;   /* SALE_USER arrays are device (1) or host (0)  */
  double t0;                /* initial time (restart), <= t_end             */
  int64_t step0;            /* initial step count (restart)                 */
} sale_problem;

typedef struct sale_ctx sale_ctx;

/* Bytes of device workspace one run of `cfg` needs (256-byte aligned
 * sub-buffers): the control block, two copies of the state (rho, e per cell;
 * u, v, w per node) and the step's intermediates. The caller allocates it
 * (e.g. a torch uint8 tensor) and keeps it alive until sale_destroy -- the
 * paper's hand-over of data by pointer, Point_to_data (Sec. III-A).
 * SALE_EINVAL for an invalid config. */
int sale_workspace_bytes(const sale_config *cfg, size_t *bytes);

/* Validate cfg and the problem, lay out the workspace d_ws (device,
 * ws_bytes >= sale_workspace_bytes), write the initial state and its first
 * time step on `hip_stream` (asynchronous), and return a new context. The
 * problems are the paper's verification flows: the Sod tube and the Sedov
 * blast (Sec. I-D, Fig. 2), the Noh implosion (Sec. I-D), or caller arrays.
 * SALE_USER arrays must be finite with rho > 0 and e >= 0 (SALE_EINVAL
 * otherwise; device arrays are checked on the device and reported by the
 * first sale_status/sale_run). Host user arrays are copied before return. */
int sale_init(const sale_config *cfg, const sale_problem *prob, void *d_ws, size_t ws_bytes,
              void *hip_stream, sale_ctx **out);

/* Allocation-free variant of sale_init, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation. The caller passes only the state part of
 * the workspace -- the control block and the two state buffers, `*state_bytes`
 * bytes at d_state (device, 256-byte aligned, kept alive until the context
 * ends); the intermediates (u', the Lagrangian cell results, reduction
 * partials, the export scratch array, and the second-order / pure-Lagrangian
 * arrays) live in a device array of the library, 160 MiB (167,772,160 bytes)
 * per device, which each device holds from its first sale_init_static until
 * the process ends. Nothing in it needs to start at zero: every intermediate
 * is written before it is read within a step.
 * With d_state == NULL the call only writes the state bytes cfg needs to
 * *state_bytes and returns SALE_OK (no device call). Otherwise *state_bytes
 * is the size of d_state and the call does what sale_init does and returns
 * the device's static context. SALE_ENOMEM if cfg's intermediates exceed the
 * 160 MiB array (first-order cubes up to 137^3 cells in FP64, 166^3 in
 * MIXED32) or *state_bytes is too small; SALE_EINVAL as
 * sale_init. Allocates nothing, host or device: the context's host struct is
 * one static slot per device.
 * One static context per device: a later sale_init_static on the same device
 * ends the previous one (its handle must not be used again), and calls on
 * contexts that share a device's array overlap at their peril -- they race on
 * it. sale_step, sale_fields, sale_status and sale_run on a static context
 * allocate nothing either (sale_run enqueues single steps, no graphs);
 * sale_destroy releases the slot.
 */
int sale_init_static(const sale_config *cfg, const sale_problem *prob, void *d_state, size_t *state_bytes,
                     void *hip_stream, sale_ctx **out);

/* Enqueue one Lagrange + remap step (asynchronous): the Lagrangian phase,
 * then the Eulerian rezone and advection back to the fixed mesh (the paper's
 * Lagrangian and Eulerian kernels and advection, Sec. I-D and Table I; in
 * the pure-Lagrangian mode the Lagrangian rezoning only). A step enqueued
 * after the run reached t_end, or after an error flag was raised, changes
 * nothing. */
int sale_step(sale_ctx *ctx);

/* Run until t >= t_end or until max_steps more steps were taken (the
 * simulation loop of cycles the paper times, Sec. IV). t_end < 0
 * keeps the configured end time; otherwise it replaces it (the last step is
 * clipped to land on it). Steps are enqueued in chunks -- once a context has
 * run 128 steps through sale_run, mostly as replays of a captured HIP graph
 * of several steps (dt, t and the done decision stay in device memory, so a
 * replay past t_end is a no-op); the stream is
 * synchronised after each chunk to read the device status. Returns SALE_DONE
 * when t_end was reached, SALE_OK when max_steps ran out first,
 * SALE_ETANGLE / SALE_ENUMERIC on a flagged step. */
int sale_run(sale_ctx *ctx, double t_end, int64_t max_steps);

/* Copy the fields selected by `mask` into dst[0..], one pointer per set bit in
 * ascending bit order, to device (dst_on_device != 0) or host memory, in the
 * logical layout. RHO, E, U, V, W are written as double (as_fp64 != 0) or in
 * the storage type (double for SALE_FP64, float for SALE_MIXED32); P and Q
 * are always double. STATE and TOTALS always go to host double arrays. TOTALS
 * are the mass and the total (internal + kinetic) energy, which the scheme
 * conserves to rounding. Synchronises the stream. */
int sale_fields(sale_ctx *ctx, uint32_t mask, void *const *dst, int dst_on_device, int as_fp64);

/* Enqueue n steps like sale_step and time each of the step's three kernels
 * with HIP events on the context's stream (the paper times compute cycles
 * only, initialisation excluded, Sec. IV): ms[0], ms[1], ms[2] receive the
 * summed durations of the step start (dt), the Lagrangian phase with the
 * Lagrangian geometry, and the remap, over the n steps. Synchronises the
 * stream after every step. SALE_EINVAL for n < 1 or a NULL ms. */
int sale_step_timed(sale_ctx *ctx, int32_t n, float ms[3]);

/* Launch shape of the context's two step kernels (a tuning knob; results do
 * not depend on it): tiles of 35 x rows columns for the Lagrangian kernel and
 * 36 x rows for the remap kernel, 32 owned in x (rows 7, 14 or 28; default 14
 * and 14, the remap 7 on meshes at most 3 cells across in y), and the
 * number of blocks the split of the z extent into segments aims at (0, the
 * default: automatic -- a small mesh is split as finely as the chip holds its
 * blocks at once, a large one aims at 3072 blocks). Synchronises the stream.
 * SALE_EINVAL for other values. */
int sale_set_launch(sale_ctx *ctx, int32_t rows_lagrange, int32_t rows_remap, int32_t target_blocks);

/* Synchronise the stream and return the sticky status flags (SALE_FLAG_*)
 * of the run's steps.
 * Returns SALE_ETANGLE / SALE_ENUMERIC if a flag is set, else SALE_DONE if
 * t >= t_end, else SALE_OK. */
int sale_status(sale_ctx *ctx, int32_t *status_flags);

/* Free the context's host memory (the workspace stays the caller's). */
void sale_destroy(sale_ctx *ctx);

/* ---- pool: many independent runs, advanced together ------------------------
 * Batched and served runs: independent runs of different mesh sizes share one
 * caller-owned device arena and are advanced together, in one of two modes.
 * Persistent: an advance is one launch of a persistent kernel that pulls
 * (round, phase, run, tile) work items from device queues, a run's phase
 * waiting only for that run's previous phase; every run is served by the
 * blocks of one XCD (the runs are split into one group per XCD, balanced by
 * cells), so that a run's tiles meet in that XCD's L2. Lockstep: an advance is
 * a sequence of rounds; per round one launch computes every run's time step,
 * one launch runs the Lagrange tiles of all runs and one the remap tiles of
 * all runs, so the kernel boundaries order the phases. With the environment
 * variable SALE_POOL_GRAPHS=1 at sale_pool_create, the rounds after an
 * advance's first are replays of one HIP graph of a round's four launches,
 * captured on a stream of the pool's own and kept while the set of active
 * runs and the block counts stay the same (the graph holds kernel launches
 * only); by default every round is launched (as fast or faster on the pools
 * measured). In both modes each run's z extent is split in proportion to
 * its share of the cells. The mode is chosen per advance: persistent when
 * there are at least four active runs per XCD and the busiest XCD's cells are
 * within 10% of the mean, lockstep otherwise; the environment variable
 * SALE_POOL_PERSISTENT=1 (=0) at sale_pool_create forces the persistent
 * (lockstep) mode. Each run has its own time step; a run that is done skips
 * its tiles. A run's results do not depend on which other runs share the
 * pool, nor on the advance mode. In the persistent mode a wait for a run's
 * previous phase is capped (2 s); a wait that hits the cap aborts the
 * advance: every later wait gives up at once, and each run with an item that
 * could not wait is flagged SALE_FLAG_NUMERIC (its state is not trusted).
 * Test hooks, read at sale_pool_create: SALE_POOL_WAIT_TICKS sets the cap in
 * ticks of the 100 MHz device clock; SALE_POOL_XCC_MASK (a bit mask of XCD
 * ids) replaces the XCDs the device reports for the grouping, and a run
 * assigned to an XCD that receives no block of the persistent launch is not
 * advanced and is flagged SALE_FLAG_NUMERIC. */
typedef struct sale_pool sale_pool;

/* Create a pool of up to max_runs slots over the device arena
 * [d_arena, d_arena + arena_bytes) (caller-owned, 256-byte aligned, kept alive
 * until sale_pool_destroy); arena_bytes is the pool's device-memory budget
 * (the admission limit). All runs of a pool share `precision`. Host only: no
 * device call. (Runs of many independent problems are an addition of this
 * library: the paper runs one problem per job.) */
int sale_pool_create(int32_t precision, int32_t max_runs, void *d_arena, size_t arena_bytes,
                     void *hip_stream, sale_pool **out);

/* Admit a run: carve its workspace from the arena, enqueue its initial state
 * and return its slot. The run stops after n_steps steps or at cfg->t_end,
 * whichever comes first. cfg->precision must equal the pool's; remap order 1
 * and SALE_EULERIAN only (SALE_EINVAL otherwise). SALE_ENOMEM if the run's
 * workspace is larger than the arena's room for runs (it would never fit);
 * SALE_EBUSY if no slot is free or no free arena range is large enough now
 * (the caller retries after a release). Synchronises the stream before returning (the run's descriptor
 * is copied from host memory), so the admission waits for the work already
 * on the stream. */
int sale_pool_admit(sale_pool *pool, const sale_config *cfg, const sale_problem *prob, int64_t n_steps,
                    int32_t *slot);

/* Advance every unfinished admitted run by up to max_steps_per_run steps:
 * one persistent launch, or lockstep rounds (launched, or the first launched
 * and the rest graph replays). Synchronises the stream first (the tables of
 * the runs in the advance are copied from host memory), then enqueues the
 * advance and returns without waiting for it. The pool's first advance that
 * may take the persistent mode first runs a small kernel that lists the
 * device's XCD ids and waits for it (SALE_EHIP if it finds none). A failed
 * capture or instantiation of the
 * round graph returns SALE_EHIP after the first round was enqueued. */
int sale_pool_advance(sale_pool *pool, int32_t max_steps_per_run);

/* Synchronise the stream and list, in done[0..*n_done), the slots whose run
 * has finished (n_steps taken, t_end reached, or an error flag raised) and
 * that were not listed by an earlier poll; at most `cap` are listed. */
int sale_pool_poll(sale_pool *pool, int32_t *done, int32_t cap, int32_t *n_done);

/* sale_fields for one slot (same mask, destinations and types). */
int sale_pool_fields(sale_pool *pool, int32_t slot, uint32_t mask, void *const *dst, int dst_on_device,
                     int as_fp64);

/* Return a slot and its arena range to the pool (synchronises the stream). */
int sale_pool_release(sale_pool *pool, int32_t slot);

/* Free the pool's host memory, its capture stream and its round graph (the
 * arena stays the caller's). If a round graph exists, the stream is
 * synchronised first, so that no queued replay outlives it. */
void sale_pool_destroy(sale_pool *pool);

/* Static description of a return code (SALE_EHIP: the last HIP error of the
 * calling thread). */
const char *sale_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SALE_H */
