/*
 * sphbuf.h -- C ABI of the MI355X (gfx950) buffer-update library for the
 * arbitrary-positioned SPH in-/outlet buffer of Zhang, Fan, Ren, Qian & Hu,
 * "Generalized and high-efficiency arbitrary-positioned buffer for smoothed
 * particle hydrodynamics" (arXiv 2406.16786).
 *
 * One update runs five steps on the GPU:
 *   1. a cell-linked list over all particles (counting sort: cell_start, cell_idx),
 *   2. per in-/outlet, candidates gathered only from the cells that overlap its
 *      check region (Section 3.1: the cell-linked lists local to each buffer),
 *   3. each candidate rotated into the buffer's local frame (Eq. 2D_transformation,
 *      Eq. 3D_transformation) so that crossing is a one-coordinate comparison,
 *   4. inlet generation: the crossing buffer particle is duplicated and recycled
 *      one buffer length back (Algorithm 1, Algorithm 3),
 *   5. outlet deletion by stream compaction (Algorithm 2, Algorithm 3), with
 *      relabelling of outlet / bidirectional buffer particles.
 *
 * Conventions
 *   - Every particle array is a caller-owned DEVICE array (structure of arrays),
 *     at least `capacity` elements long.  Positions and carried fields are FP32,
 *     labels int32 (0 = ordinary fluid, k = 1..15 = buffer k), ids int64.
 *   - The live particle count is a device-resident int64 (`n_dev`) that the
 *     library reads at the start of each call and rewrites after an update.
 *   - Rotation matrices are row-major 3x3, global -> local: r' = Q (r - O').  Row 0
 *     is the in-/outflow direction X'.  In 2-D only the upper-left 2x2 block is
 *     used and it must be a proper rotation.
 *   - All calls return sph_status; nothing throws across the ABI.  On any error
 *     an update leaves every particle array and the library's own counters as
 *     they were (checks run on the GPU before the first write).
 *   - A context is bound to one HIP stream and is not thread-safe.  All device
 *     work of a context is ordered on that stream.  Calls marked "sync" wait for
 *     the stream; the others only enqueue.  sph_config.update_path picks how the
 *     update finds its candidates (see sph_update_path); results are identical.
 *   - The library allocates its device scratch in sph_create and
 *     sph_buffer_define; build and update calls allocate nothing.
 *
 * The calls of the method, by what they do:
 *   cell-linked list ............ sph_celllist_build (view: sph_celllist_view)
 *   buffer definition ........... sph_buffer_define (frames: sph_rotation_*)
 *   one-time identification ..... sph_buffer_identify
 *   update, counts returned ..... sph_buffer_update (enqueue only:
 *                                 sph_buffer_update_async + sph_last_result)
 *   full-scan baseline .......... sph_buffer_update_fullscan[_async]
 *   event index sets ............ sph_last_events
 *   state export / import ....... sph_state_export, sph_state_import (the same
 *                                 fields as sph_state_get / sph_state_set)
 *   many domains ................ sph_batch_create, sph_batch_step (counts of
 *                                 every domain: sph_batch_results), graph
 *                                 capture and replay: sph_batch_graph_capture,
 *                                 sph_batch_graph_launch
 */
#ifndef SPHBUF_H
#define SPHBUF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_ERR_ARG = 1,              /* bad pointer, size, dimension or kind                  */
    SPH_ERR_ROTATION = 2,         /* matrix not orthonormal with det +1 (tol 1e-9)          */
    SPH_ERR_OVERLAP = 3,          /* check region intersects an existing buffer's           */
    SPH_ERR_CAPACITY = 4,         /* N - |deleted| + |generated| would exceed capacity      */
    SPH_ERR_CFL = 5,              /* a buffer particle left its buffer's check region       */
    SPH_ERR_NONFINITE = 6,        /* NaN / Inf position among the live particles            */
    SPH_ERR_TOO_MANY_BUFFERS = 7, /* more than SPH_MAX_BUFFERS buffers in one context       */
    SPH_ERR_EVENTS = 8,           /* more events in one update than max_events              */
    SPH_ERR_HIP = 9,              /* a HIP runtime call failed                              */
    SPH_ERR_STATE = 10            /* call out of order (e.g. update before any cell list)   */
} sph_status;

typedef enum { SPH_INLET = 1, SPH_OUTLET = 2, SPH_BIDIR = 3 } sph_kind;

#define SPH_MAX_BUFFERS 15
#define SPH_MAX_CARRIED 16
/* Largest max_events of a context: per update at most this many generated
 * particles and this many deleted particles (and four times as many relabelled
 * ones).  The finalize sorts and applies the events of one update on chip, so
 * the bound is fixed; an update with more events returns SPH_ERR_EVENTS and
 * changes nothing (a caller with more inflow per step splits it into smaller
 * steps).  Algorithms 1-3 themselves put no bound on the events of a step. */
#define SPH_MAX_EVENTS_LIMIT 4096

/* How an update finds its candidates.  Both give the same events and arrays.
 *   SPH_UPDATE_MERGED (default): the count pass of sph_celllist_build lists the
 *     particles of every buffer's cover cells that lie near its check region (an
 *     FP32 test widened by the guard band) as it bins them; the update runs their
 *     exact tests beside the build's scatter, then the finalize.
 *   SPH_UPDATE_CELLS: the build builds the whole cell list; the update walks the
 *     cover cells of the finished list (one wave per run of cells). */
typedef enum { SPH_UPDATE_MERGED = 0, SPH_UPDATE_CELLS = 1 } sph_update_path;

/* How sph_celllist_build sorts the particles into cells (section 2.3's cell
 * list).  Every method gives each cell the same set of particles; the order
 * inside a cell is unspecified.
 *   SPH_BUILD_AUTO (default): times both methods on the context's stream (HIP
 *     events, read once complete: the host never waits) and runs the faster, with
 *     a re-check every 64 builds; grids of more than 2^24 cells use counting.
 *   SPH_BUILD_COUNTING: count per cell (atomics), look-back scan, scatter.
 *   SPH_BUILD_BUCKETED: count per bucket of consecutive cells, bucket scatter, a
 *     counting sort of each bucket in LDS; grids of at most 2^24 cells (counting
 *     beyond). */
typedef enum { SPH_BUILD_AUTO = 0, SPH_BUILD_COUNTING = 1, SPH_BUILD_BUCKETED = 2 } sph_build_method;

typedef struct sph_ctx sph_ctx;

/* Caller-owned device arrays of one domain. */
typedef struct {
    float *pos[3];                      /* x, y, z; pos[2] ignored (may be NULL) in 2-D        */
    float *carried[SPH_MAX_CARRIED];    /* fields copied on duplication (velocity, mass, ...)  */
    int32_t n_carried;                  /* 0..SPH_MAX_CARRIED                                  */
    int32_t pad_;
    int32_t *label;                     /* 0 = fluid, k = buffer k; written by the library     */
    int64_t *id;                        /* duplicates get next_id, next_id + 1, ...            */
    int64_t *n_dev;                     /* device int64: live count, updated in place          */
    int64_t capacity;                   /* length of every array above (< 2^31)                */
} sph_particles;

typedef struct {
    int32_t dim;            /* 2 or 3                                                         */
    int32_t pad_;
    double lo[3], hi[3];    /* cell-grid bounds; particles outside are binned into edge cells */
    double cell_size;       /* cell edge (2h = 2.6 dp in the paper's setting)                 */
    double dp;              /* particle spacing: the FP32 guard band is max(1e-4 dp, bound)   */
    int64_t capacity;       /* largest particle capacity that will be passed                  */
    int64_t max_events;     /* per update, for generated and for deleted; <= 4096             */
    int64_t next_id;        /* id of the first duplicate                                      */
    void *stream;           /* hipStream_t (NULL = the null stream)                           */
    int32_t brick_log2;     /* 0: dense grid; 1..5: brick-sparse grid of 2^b cells per axis   */
    int32_t brick_margin;   /* sparse grid: active bricks = occupied ones dilated by this     */
    int32_t update_path;    /* sph_update_path (0 = SPH_UPDATE_MERGED)                         */
    int32_t build_method;   /* sph_build_method (0 = SPH_BUILD_AUTO)                           */
} sph_config;

/* Result of the last update (see sph_last_result). */
typedef struct {
    int32_t status;                      /* sph_status of the update                          */
    int32_t n_buffers;
    int64_t n_generated;                 /* |G|                                               */
    int64_t n_deleted;                   /* |D|                                               */
    int64_t n_before;                    /* N on entry                                        */
    int64_t n_after;                     /* N - |D| + |G| (== n_before on error)              */
    int64_t next_id;
    int64_t n_labelled[SPH_MAX_BUFFERS]; /* particles carrying each buffer's label afterwards  */
} sph_result;

/* ------------------------------------------------------------------ lifetime -- */

/* Create a context: validates cfg, allocates the cell grid and all scratch on the
 * current HIP device.  SPH_ERR_ARG for a bad config (dim, cell_size <= 0, empty or
 * non-finite bounds, more than 2^31 cells, capacity <= 0 or >= 2^31, max_events
 * outside 1..4096, an unknown update_path or build_method, or a grid on which FP32 binning can
 * misplace a particle by a quarter cell or more: the cell coordinate
 * fl32(fl32(x - fl32(lo)) * fl32(1/cell_size)) is off by at most
 * |lo - fl32(lo)|/cell_size + 3.0001 2^-24 (cells per axis + 1 + that offset)
 * cells, and buffer covers are widened by 1.5 times this bound, at least 1e-2
 * cell); SPH_ERR_HIP if allocation fails.  *out is NULL on error. */
sph_status sph_create(const sph_config *cfg, sph_ctx **out);
sph_status sph_destroy(sph_ctx *ctx);

/* Define one in-/outlet buffer (Section 3.1: translation O' and rotation of the
 * local frame, box of half-extents a/2, b/2, c/2 centred at O').  margin > 0 is
 * the check-region margin delta (<= 0 selects cell_size): the check region is the
 * box dilated by delta on every side and stands for the local cell-linked lists
 * that extend slightly past the buffer.  Host FP64 work (frame validation, cell
 * cover of the check region, guard band), then the buffer's range of the run
 * lists is allocated, sized for its cover in any orientation (a turn recomputes
 * the cover in place), and filled (setup: waits for the stream).
 * Errors: SPH_ERR_ARG (kind, non-positive or non-finite extents, a check region
 * wider than 2^20 cells), SPH_ERR_ROTATION, SPH_ERR_OVERLAP (check regions of two
 * buffers intersect), SPH_ERR_TOO_MANY_BUFFERS.  *buffer_id receives 1..15.
 * The next update needs a cell list built after this call. */
sph_status sph_buffer_define(sph_ctx *ctx, sph_kind kind, const double origin[3], const double rot[9],
                             const double half[3], double margin, int32_t *buffer_id);

/* ------------------------------------------------------------------ hot path -- */

/* Brick-sparse grid only (a no-op for a dense grid): activate the bricks that hold
 * live particles now, dilated by brick_margin bricks; every other brick maps to
 * one overflow cell, which joins each buffer's candidate cells when its check
 * region reaches an inactive brick.  Cell keys: slot * 2^(dim b) + local cell.
 * Re-derives the candidate cells of the defined buffers.  Setup call (sync,
 * allocates); call it again if the particles drift far from the active bricks
 * (results stay exact, only the overflow cell gets crowded). */
sph_status sph_grid_fit(sph_ctx *ctx, const sph_particles *p);

/* Step 1: counting-sort cell list of the live particles on the context stream
 * (async).  Flags non-finite positions for the next update.
 * On the merged path (the default) the count pass also classifies the particles
 * of every buffer's cover cells and emits their events (steps 2-5 decided here,
 * on these positions and carried fields; the caller must not change the arrays
 * before the update), and the scan and scatter are left for the update, which
 * runs the finalize beside the scan in one launch and then the scatter; a call
 * that reads the cell list first enqueues them itself.  Library calls that
 * change the state the events were decided on (apply_bc, rotate, identify,
 * set_fields, set_bc, buffer_define, grid_fit, state_set) drop them, and the
 * update then walks the cover cells; results are the same either way.
 * Capacities above 2^25 particles and domains without buffers take the plain
 * build. */
sph_status sph_celllist_build(sph_ctx *ctx, const sph_particles *p);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the cell-list build of
 * sph_celllist_build on a dense grid, without a context.  Every scratch array of
 * the build (cell counts, packed cell keys and ranks, scan tile states, control
 * words) lives in one library-owned device array of fixed size, one copy per GPU,
 * held until the process ends; nothing is allocated or freed, no allocating
 * library routine is called.  Calls on one GPU share that array: calls that
 * overlap on one GPU (different streams, threads) race, so order them.
 *   dim, lo, cell_size, dims: the grid (cells per axis; particles outside it are
 *     binned into the edge cells; FP32 binning as sph_create requires);
 *   x, y, z: device FP32 positions (z ignored in 2-D), at least capacity long;
 *   n_dev: device int64, the live count (clamped to [0, capacity]);
 *   cell_start: device int32 [cells + 1], cell_idx: device int32 [capacity]
 *     (caller-owned outputs, as sph_celllist_view describes them);
 *   stream: hipStream_t (NULL = the null stream).  Async.
 * SPH_ERR_ARG for a NULL pointer, a bad grid, more than SPH_NOALLOC_MAX_CELLS
 * cells or a capacity above SPH_NOALLOC_MAX_PARTICLES (nothing is launched).  The
 * first call on a GPU also clears its copy of the array (a small kernel). */
#define SPH_NOALLOC_MAX_PARTICLES (1 << 20)
#define SPH_NOALLOC_MAX_CELLS (1 << 20)
sph_status sph_celllist_build_noalloc(int32_t dim, const double lo[3], double cell_size, const int32_t dims[3],
                                      const float *x, const float *y, const float *z, const int64_t *n_dev,
                                      int64_t capacity, int32_t *cell_start, int32_t *cell_idx, void *stream);

/* Algorithm 1, identification (run once, before the first update): label k for every live
 * particle inside buffer k's box; buffer_id = -1 for all buffers.  Full pass over
 * the particles (sync).  SPH_ERR_NONFINITE leaves labels untouched. */
sph_status sph_buffer_identify(sph_ctx *ctx, sph_particles *p, int32_t buffer_id);

/* Steps 2-5 with local-cell candidates (needs sph_celllist_build on the same
 * positions first).  Sync: waits for the stream and returns |G| and |D|.
 * Errors SPH_ERR_CFL / CAPACITY / NONFINITE / EVENTS leave everything unchanged. */
sph_status sph_buffer_update(sph_ctx *ctx, sph_particles *p, int64_t *n_generated, int64_t *n_deleted);

/* Same as sph_buffer_update but only enqueues; read the outcome with
 * sph_last_result (which syncs). */
sph_status sph_buffer_update_async(sph_ctx *ctx, sph_particles *p);

/* Baseline: the same update with every live particle as a candidate of every
 * buffer (no cell list; the all-particle scan the paper replaces). Sync. */
sph_status sph_buffer_update_fullscan(sph_ctx *ctx, sph_particles *p, int64_t *n_generated,
                                      int64_t *n_deleted);
sph_status sph_buffer_update_fullscan_async(sph_ctx *ctx, sph_particles *p);

/* Sync: outcome of the last update enqueued on this context. */
sph_status sph_last_result(sph_ctx *ctx, sph_result *out);

/* Sync: sorted index sets of the last successful update (pre-update indices).
 * gen_src: sources of the duplicates; del_idx: deleted particles.  Copies at most
 * cap entries of each. */
sph_status sph_last_events(sph_ctx *ctx, int64_t *gen_src, int64_t *del_idx, int64_t cap, int64_t *n_gen,
                           int64_t *n_del);

/* Device pointers to the library-owned cell list of the last build: cell_start
 * has n_cells + 1 entries, cell_idx has N entries (pre-update indices). */
sph_status sph_celllist_view(sph_ctx *ctx, const int32_t **cell_start, const int32_t **cell_idx,
                             int64_t *n_cells, int32_t dims[3]);

/* The build method of the last build (SPH_BUILD_COUNTING or SPH_BUILD_BUCKETED;
 * SPH_BUILD_AUTO before the first) and, for SPH_BUILD_AUTO, each method's smoothed
 * build time in microseconds (count pass plus cells pass, from HIP events; index
 * 0 counting, 1 bucketed; 0 while unmeasured) and the number of timed builds it
 * rests on.  Any output may be NULL.  Host-only: reads what the context has
 * harvested, never waits. */
sph_status sph_build_stats(sph_ctx *ctx, int32_t *method, double us[2], int64_t samples[2]);

/* SPH_BUILD_AUTO: forget both methods' build times and time them again over the
 * next builds (for a flow that has changed its character, e.g. after a restart
 * from a checkpoint).  Host-only; SPH_OK also for a fixed method (no effect). */
sph_status sph_build_retune(sph_ctx *ctx);

/* Async: neighbour search on the cell list of the last build, the use a solver
 * makes of the same list (the kernel support 2h of Section 3, h = 1.3 dp, is the
 * cell size).  For every live particle i (i < N):
 *   counts[i] = #{ j != i live : |r_i - r_j| < radius },
 * the distance decided as in FP64 by ((dx*dx + dy*dy) + dz*dz) < radius*radius with
 * dx = (double)x_i - (double)x_j (dz = 0 in 2-D), every operation rounded to
 * nearest.  counts: caller-owned device int32 array of at least N entries; entries
 * past N are left alone; valid once the context's stream has reached this call.
 * The particle arrays must be those of the last sph_celllist_build, unchanged.
 * Allocates nothing: the positions are copied into cell order in the build's own
 * key scratch (the cell list itself stays as it is).
 * Errors: SPH_ERR_ARG (NULL, radius not in (0, cell size], or a grid too large for
 * FP32 cell coordinates), SPH_ERR_STATE (no current cell list).  Nothing is
 * written on error. */
sph_status sph_neighbor_count(sph_ctx *ctx, const sph_particles *p, double radius, int32_t *counts);

/* ---------------------------------- boundary conditions and moving buffers -- */

/* Roles of the caller's carried arrays: indices into sph_particles.carried of the
 * velocity components and of the density, -1 where absent.  Checked against
 * n_carried at every call that uses them (SPH_ERR_ARG). */
typedef struct {
    int32_t vel[3];
    int32_t rho;
} sph_fields;
sph_status sph_set_fields(sph_ctx *ctx, const sph_fields *fields);

typedef enum { SPH_BC_NONE = 0, SPH_BC_VELOCITY = 1, SPH_BC_PRESSURE = 2 } sph_bc_kind;
typedef enum {
    SPH_PROFILE_PLUG = 0,        /* f = 1                                            */
    SPH_PROFILE_PARABOLIC_Y = 1, /* f = 1 - (Y'/R)^2 (Eqs. 2D/3D_velocity_profile)   */
    SPH_PROFILE_PARABOLIC_R = 2  /* f = 1 - (Y'^2 + Z'^2)/(R R): a pipe's profile    */
} sph_profile;

/* In-/outlet boundary condition of one buffer (Section 4).
 * Velocity BC (Section 4.2): the buffer's particles move with the prescribed
 * local-frame velocity v' = (u f(Y', Z'), 0, 0), i.e. v = Q^T v'
 * (Eqs. 2D/3D_velocity_transformation).  Pressure BC (Section 4.1): their
 * velocity is projected on the boundary normal u_hat = Q^T e_x
 * (Eq. velocity_correction), and a particle the update recycles at this buffer
 * takes the density rho0 + p_b / c0^2 (Eq. postulate-density; EoS
 * p = c0^2 (rho - rho0)).  The momentum-equation part of the pressure BC belongs
 * to the solver.  u and p_b may change between steps (call again). */
typedef struct {
    int32_t kind;      /* sph_bc_kind                                      */
    int32_t profile;   /* sph_profile (velocity BC)                        */
    double u;          /* velocity BC: speed scale along X'                 */
    double radius;     /* velocity BC: R of the parabolic profiles (> 0)    */
    double p_b;        /* pressure BC: boundary pressure                    */
    double rho0;       /* pressure BC: reference density                    */
    double c0;         /* pressure BC: artificial sound speed (> 0)         */
} sph_bc;
/* Host validation plus one small upload on the context stream.  SPH_ERR_ARG for
 * an unknown buffer, kind or profile, a non-finite value, radius <= 0 (parabolic)
 * or c0 <= 0 (pressure). */
sph_status sph_buffer_set_bc(sph_ctx *ctx, int32_t buffer_id, const sph_bc *bc);

/* Apply every buffer's boundary condition to its particles (label k inside the
 * check region), exactly as defined in FP64 and rounded to FP32 once.  Needs a
 * cell list of the current positions (sph_celllist_build; it stays valid, the
 * positions do not change) and velocity fields.  Sync.  SPH_ERR_CFL if some
 * buffer particle lies outside its check region: those are left alone, the
 * others are set (the call is not transactional).  SPH_ERR_STATE without a
 * current cell list. */
sph_status sph_buffer_apply_bc(sph_ctx *ctx, sph_particles *p);

/* Turn buffer buffer_id rigidly about center by the orthonormal matrix m
 * (row-major, global coordinates; det +1), as the rotating sprinkler of
 * Section 5.3 turns its buffer every step: each of its particles inside the
 * check region moves to C + m (r - C), its velocity (if velocity fields are set)
 * to m v, both in FP64 rounded to FP32 once; then the frame follows,
 * O' <- C + m (O' - C), Q <- Q m^T, and the cell cover of the check region is
 * recomputed on the device (into the buffer's own range of the run lists, sized
 * at definition for any orientation; no allocation, no host work on the cells).
 * Needs a cell list of the current positions; invalidates it (rebuild before the
 * next update).  Sync: returns the outcome of the turn.  Errors: SPH_ERR_ROTATION
 * (m not orthonormal), SPH_ERR_OVERLAP (the turned check region would meet
 * another buffer's: nothing changes), SPH_ERR_CFL as for sph_buffer_apply_bc. */
sph_status sph_buffer_rotate(sph_ctx *ctx, sph_particles *p, int32_t buffer_id, const double center[3],
                             const double m[9]);
/* The same, enqueue only (argument, rotation and overlap errors are still
 * returned at once); the CFL outcome is read later with sph_last_bc_status. */
sph_status sph_buffer_rotate_async(sph_ctx *ctx, sph_particles *p, int32_t buffer_id, const double center[3],
                                   const double m[9]);
/* sph_buffer_apply_bc, enqueue only; outcome with sph_last_bc_status. */
sph_status sph_buffer_apply_bc_async(sph_ctx *ctx, sph_particles *p);
/* Sync: outcome of the last boundary-condition pass or turn enqueued (SPH_OK or
 * SPH_ERR_CFL). */
sph_status sph_last_bc_status(sph_ctx *ctx);
/* Sync: the cover of a buffer as the library holds it now (after definition,
 * grid fit or turns): runs of consecutive cell keys (first key, length), at most
 * cap of them; *n_runs receives the count (SPH_ERR_ARG if it exceeds cap). */
sph_status sph_buffer_cover(sph_ctx *ctx, int32_t buffer_id, int32_t *first, int32_t *len, int64_t cap,
                            int64_t *n_runs);

/* Library state that is not in the particle arrays: next_id and each buffer's
 * labelled count (sync).  Lets a caller checkpoint and restore a run. */
sph_status sph_state_get(sph_ctx *ctx, int64_t *next_id, int64_t n_labelled[SPH_MAX_BUFFERS]);
sph_status sph_state_set(sph_ctx *ctx, int64_t next_id, const int64_t n_labelled[SPH_MAX_BUFFERS]);
/* The same state as an opaque blob (sync): export writes SPH_STATE_BLOB_BYTES
 * bytes to blob when *len is at least that, and always sets *len to that size
 * (blob may be NULL to ask for it: SPH_ERR_ARG, *len set).  import reads a blob
 * written by export (SPH_ERR_ARG for a wrong length or tag). */
#define SPH_STATE_BLOB_BYTES 136
sph_status sph_state_export(sph_ctx *ctx, void *blob, size_t *len);
sph_status sph_state_import(sph_ctx *ctx, const void *blob, size_t len);

/* ---------------------------------------------------------------- profiling -- */

/* Kernel phases timed by the optional per-launch HIP events. */
typedef enum {
    SPH_PHASE_COUNT = 0,      /* cell keys; bucket ranks (or per-cell ranks)      */
    SPH_PHASE_SCAN = 1,       /* exclusive scan of the cell counts (batch, large grids) */
    SPH_PHASE_SCATTER = 2,    /* into bucket order (or cell order); merged step:
                                 with the candidates' exact tests beside it      */
    SPH_PHASE_CLASSIFY = 3,   /* local-cell candidates, frame, crossing tests     */
    SPH_PHASE_FULLSCAN = 4,   /* full scan: every particle, FP32 filter (baseline)*/
    SPH_PHASE_FINALIZE = 5,   /* status, sort, duplicate/recycle/relabel/compact  */
    SPH_PHASE_BC = 6,         /* boundary conditions on buffer particles          */
    SPH_PHASE_ROTATE = 7,     /* rigid turn of a buffer's particles               */
    SPH_PHASE_CANDIDATES = 8, /* full scan: the filter's candidates, exact tests  */
    SPH_PHASE_NEIGHBOR = 9,   /* neighbour counts over the cell list              */
    SPH_PHASE_COVER = 10,     /* cover cells of a turned buffer (two launches)    */
    SPH_PHASE_SORT = 11,      /* per-bucket counting sort: cell starts, cell_idx  */
    SPH_NPHASE = 12
} sph_phase;

/* When on, every kernel launch of the context is bracketed by two HIP events on
 * the context stream (events are created here, up to 8192 launches are kept).
 * Off by default; turning it on or off drops the recorded launches. */
sph_status sph_profile_enable(sph_ctx *ctx, int32_t on);
/* Sync: total milliseconds and launch counts per phase since the last reset
 * (arrays of SPH_NPHASE); reset != 0 clears them afterwards. */
sph_status sph_profile_read(sph_ctx *ctx, double ms[SPH_NPHASE], int64_t launches[SPH_NPHASE], int32_t reset);

/* ------------------------------------------------------------------ batches -- */

/* Many independent domains stepped together.  One step runs the cell-list build
 * and the local-cell update of every domain with five launches in total (count,
 * scan, scatter, classify, finalize over all domains: a static table maps each
 * block to a domain), either enqueued directly or replayed from a HIP graph
 * captured at the first step.  Member contexts keep their own results
 * (sph_last_result, sph_last_events) and must be fully set up first: a later
 * sph_buffer_define, sph_grid_fit or a change of the density field in
 * sph_set_fields on a member invalidates the batch (its launch tables hold the
 * member's grid arrays, run-list arrays and field roles): sph_batch_step then
 * returns SPH_ERR_STATE and launches nothing.  Turning a member's buffer
 * (sph_buffer_rotate) keeps the batch valid: the turned cover is recomputed on
 * the device into the same arrays. */
typedef struct sph_batch sph_batch;
typedef enum { SPH_BATCH_KERNELS = 0, SPH_BATCH_GRAPH = 1 } sph_batch_mode;

/* domains[d] is stepped with particles[d] (pointers are baked into the batch).
 * stream: hipStream_t for all batch work; NULL makes a private non-blocking
 * stream (graphs cannot be captured on the null stream).  The caller orders
 * the batch stream after any work of the members' own streams.  Allocates. */
sph_status sph_batch_create(sph_ctx *const *domains, const sph_particles *particles, int32_t n_domains,
                            void *stream, sph_batch **out);
sph_status sph_batch_destroy(sph_batch *b);
/* SPH_BATCH_KERNELS or SPH_BATCH_GRAPH (default). */
sph_status sph_batch_set_mode(sph_batch *b, int32_t mode);
/* Particles per block of the count and scatter launches (256 .. 2^20; default
 * 2048).  Sync; drops a captured graph. */
sph_status sph_batch_set_count_block(sph_batch *b, int32_t particles_per_block);
/* Cover runs (row runs of cover cells) that one classify workgroup gathers
 * (1 .. 8; default 3): fewer give more workgroups, more give each workgroup a
 * longer candidate list.  Sync; drops a captured graph. */
sph_status sph_batch_set_gather(sph_batch *b, int32_t runs_per_block);
/* The batch's launch mode, particles per count block and runs per classify
 * workgroup (outputs may be NULL). */
sph_status sph_batch_get_config(sph_batch *b, int32_t *mode, int32_t *particles_per_block,
                                int32_t *runs_per_block);
/* Async: one step (build + local-cell update) of every domain.  SPH_ERR_STATE if
 * a member was redefined since sph_batch_create (nothing is enqueued). */
sph_status sph_batch_step(sph_batch *b);
/* The step as a HIP graph: capture sets SPH_BATCH_GRAPH and records the step's
 * five launches into a graph (sync; replaces an earlier graph); launch replays it
 * on the batch stream (async; captures first if there is no graph). */
sph_status sph_batch_graph_capture(sph_batch *b);
sph_status sph_batch_graph_launch(sph_batch *b);
/* Sync: out[d] = result of domain d's last update. */
sph_status sph_batch_results(sph_batch *b, sph_result *out);
/* Per-launch timing of the five launches of a step in SPH_BATCH_KERNELS mode
 * (two HIP events on the batch stream around each; up to 8192 launches are
 * kept).  enable: sync, drops what was recorded.  read: sync; ms and launches
 * have 5 entries (count, scan, scatter, classify, finalize); reset != 0 clears. */
sph_status sph_batch_profile_enable(sph_batch *b, int32_t on);
sph_status sph_batch_profile_read(sph_batch *b, double ms[5], int64_t launches[5], int32_t reset);
/* Autotuner: times `trials` steps of each launch mode x particles-per-block
 * candidate, then of each runs-per-classify-workgroup choice at the best of
 * those, and keeps the fastest (steps are real updates of the current states;
 * sph_batch_get_config reports the choice).  cache_path (optional) holds earlier
 * choices keyed by device, domain count and total capacity; a hit skips the
 * sweep.  Outputs may be NULL. */
sph_status sph_batch_tune(sph_batch *b, int32_t trials, const char *cache_path, int32_t *mode,
                          int32_t *particles_per_block, double *ms_per_step);

/* ------------------------------------------------------------ host helpers -- */
/* Pure host FP64; usable without a GPU. */

/* Eq. (2D_transformation) embedded in 3x3: [[cos, sin, 0], [-sin, cos, 0], [0, 0, 1]]. */
sph_status sph_rotation_2d(double theta, double rot[9]);
/* Eq. (rotation_matrix) exactly as printed (active rotation by theta about unit n). */
sph_status sph_rotation_axis_angle(const double n[3], double theta, double rot[9]);
/* Global->local frame with X' along dir (Eqs. rotation_axis to 3D_transformation,
 * read with Q = R^T so that Q dir = |dir| e_x).  dir parallel to -e_x gives a half
 * turn about e_z.  SPH_ERR_ARG for a zero or non-finite dir. */
sph_status sph_rotation_from_direction(const double dir[3], double rot[9]);
/* SPH_OK if rot (2x2 block in 2-D) is orthonormal with det +1 within 1e-9. */
sph_status sph_check_rotation(int32_t dim, const double rot[9]);

/* Cells of a dense grid (lo, cell_size, dims) whose boxes, dilated by
 * max(1e-2, 1.5 E) of a cell (E: the FP32 binning bound given at sph_create) and
 * with edge cells extended to infinity, intersect the check region of a buffer
 * (separating-axis test).  Written as runs along x: first cell (linear index
 * ix + dims[0] * (iy + dims[1] * iz)) and run length, at most cap runs.
 * SPH_ERR_ARG if more than cap runs are needed (*n_runs then holds the need) or
 * if E reaches a quarter cell. */
sph_status sph_grid_cover(int32_t dim, const double lo[3], double cell_size, const int32_t dims[3],
                          const double origin[3], const double rot[9], const double half[3], double margin,
                          int32_t *run_first, int32_t *run_len, int64_t cap, int64_t *n_runs);

/* FP32 guard band of a buffer: max(1e-4 dp, 2 E) with E a bound on the FP32
 * error of a local coordinate of any candidate (hi/lo split origin). */
double sph_guard_band(int32_t dim, const double origin[3], const double half[3], double margin,
                      double cell_size, double dp);

const char *sph_status_str(sph_status s);

#ifdef __cplusplus
}
#endif
#endif
