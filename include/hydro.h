/*
 * hydro.h -- C ABI of the MI355X (gfx950) hydro library.
 *
 * The library advances the evolved fields of octree leaf subgrids by the
 * finite-volume hydro step of Octo-Tiger's new hydro module (arXiv 2107.10987,
 * section IV-B): PPM reconstruction at the 26 face, edge and corner points of
 * every cell along the 13 lines through its centre, central-upwind
 * (Kurganov-Tadmor) point fluxes with the maximum signal speed, Newton-Cotes
 * face quadrature, flux divergence with rotating-frame sources, and a
 * two-stage SSP Runge-Kutta update with dual-energy (entropy tracer) pressure.
 *
 * Leaves hold E^3 cells, E = 8 (default) or 16 (hydro_params.leaf_edge).  The
 * kernels work on 8^3 tiles with three ghost layers (a 14^3 block in LDS); a
 * 16^3 leaf is eight tiles, tile t at cell offset 8 (t & 1, (t >> 1) & 1, t >> 2).
 *
 * Data layout (device memory owned by the caller unless noted):
 *   U         double [n][7][E][E][E]  fields rho, sx, sy, sz, E, tau, X per leaf;
 *                                      cells [k][j][i], i fastest (structure of arrays)
 *   dx        double [n]               cell size of each leaf
 *   origin    double [n][3]            centre of cell (0,0,0) of each leaf; the frame
 *                                      rotates about the z axis through x = y = 0
 *   ghost_map int32  [n][T][2232]      T = (E/8)^3 tiles per leaf: source of every
 *                                      ghost cell of every tile's 14^3 block, in raster
 *                                      order (k, j, i in -3..10 relative to the tile,
 *                                      i fastest, its 8^3 cells skipped).  Entry s >= 0:
 *                                      copy cell s%E^3 of leaf s/E^3; s < 0: mean of the
 *                                      2x2x2 cells of leaf b/E^3 whose lowest cell is
 *                                      b%E^3, b = -s-1.  hydro_ghost_map builds it.
 * Every call is asynchronous on the caller's stream except where noted.
 * Return codes: 0 on success or a negative HYDRO_E* code; nothing aborts and no
 * C++ exception crosses this boundary.  A handle is not thread-safe; use one
 * handle per stream.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_OK 0
#define HYDRO_EINVAL (-1)   /* bad argument; text in hydro_last_error          */
#define HYDRO_ENOMEM (-2)   /* workspace too small or allocation failed         */
#define HYDRO_EHIP (-3)     /* HIP runtime error; its text in hydro_last_error  */
#define HYDRO_ENONPHYS (-4) /* rho <= 0 or a non-finite value was produced      */

#define HYDRO_NX 8          /* cells per leaf edge */
#define HYDRO_GHOST 3       /* ghost layers: the five-point PPM stencil       */
#define HYDRO_NF 7          /* evolved fields                                 */
#define HYDRO_NGHOST 2232   /* ghost cells per leaf: 14^3 - 8^3               */

typedef struct hydro_t hydro_t;

/* Stage-kernel schedules (hydro_params.schedule). */
#define HYDRO_SCHED_AUTO 0        /* per launch size: the autotuned table, else a built-in rule  */
#define HYDRO_SCHED_FACE 1        /* a workgroup per leaf, one face of each axis per thread       */
#define HYDRO_SCHED_COLUMN 2      /* a workgroup per leaf, lanes walk cell columns (1.71x PPM)    */
#define HYDRO_SCHED_PERSISTENT 3  /* one workgroup per compute unit pulling leaves from a queue  */
#define HYDRO_SCHED_TILED 4       /* persistent, queue of (leaf, axis) items: 3x the parallelism */
#define HYDRO_NBUCKET 16          /* autotune buckets: launch size in [2^b, 2^(b+1))             */

/* Library-wide settings fixed at creation. */
typedef struct hydro_params {
    int32_t max_leaves; /* capacity of every workspace, in leaves (> 0)             */
    int32_t device;     /* HIP device ordinal                                        */
    int32_t recon;      /* 0: plain PPM; 1: learned reconstruction with FP64 check and
                           plain-PPM fallback per cell (hydro_mlp_load first)       */
    int32_t schedule;   /* HYDRO_SCHED_*                                             */
    double eta1;        /* dual energy: e < eta1*E at a point -> e = tau^gamma (1e-3) */
    double eta2;        /* dual energy: e > eta2*E after a step -> tau = e^(1/gamma)  */
    const char *tune_cache; /* NULL, or a JSON table written by hydro_autotune: loaded
                               at creation and used by HYDRO_SCHED_AUTO            */
    int32_t mlp_batch;  /* rows of the network's training workspace (0: 4096)     */
    int32_t rk_order;   /* SSP Runge-Kutta stages per step: 2 (default, 0 = 2) or 3 */
    int32_t scheme;     /* 0: fluxes at the 9 points of every face (new scheme);
                           1: at face centres only, weight 1 (the paper's old scheme,
                           section IV-B); same reconstruction                      */
    int32_t reflux;     /* 1: flux correction at coarse/fine faces (every grid then
                           carries face_flags and the reflux list from
                           hydro_reflux_map); 0: none.                            */
    int32_t leaf_edge;  /* cells per leaf edge: 8 (0 = 8) or 16                     */
} hydro_params;

/* One set of leaves that exchange ghosts: the whole mesh of a step.  All work
 * is ordered on `stream`: the launches of one stage may run concurrently on
 * side streams of the handle, forked from `stream` and joined back to it before
 * anything that follows. */
typedef struct hydro_grid {
    int32_t n;                 /* leaves, 0 < n <= max_leaves                        */
    int32_t n_launch;          /* 0: one launch per stage; else launches over the   */
    const int32_t *launch_off; /*   host leaf ranges [launch_off[b], launch_off[b+1]) */
    double *U;                 /* device [n][7][512], conserved state                */
    const double *dx;          /* device [n]                                         */
    const double *origin;      /* device [n][3]                                      */
    const int32_t *ghost_map;  /* device [n][2232]                                   */
    double omega;              /* frame rotation rate about z                        */
    double gamma;              /* ratio of specific heats, > 1                       */
    void *stream;              /* hipStream_t; NULL = the null stream                */
    const int32_t *face_flags; /* device [n T] from hydro_reflux_map, or NULL without */
    const int32_t *reflux;     /*   reflux; device [n_reflux][26] correction list    */
    int32_t n_reflux;          /*   entries in the list (may be 0)                   */
    const int32_t *prolong;    /* device [n_prolong][8] from hydro_ghost_map_linear  */
    int32_t n_prolong;         /*   (NULL, 0 with a plain ghost map)                 */
    const int32_t *mlp_alias;  /* device [n T][384] from hydro_mlp_alias_map, or NULL */
} hydro_grid;

/* Octree description used to build the ghost map (host memory). */
typedef struct hydro_tree {
    int32_t n;              /* leaves                                                */
    int32_t nb[3];          /* level-0 leaves per axis                               */
    int32_t bc[3];          /* per axis: 0 periodic, 1 zero-gradient outflow         */
    const int32_t *level;   /* [n] refinement level of each leaf                     */
    const int32_t *coord;   /* [n][3] leaf coordinates at its level                  */
    int32_t leaf_edge;      /* cells per leaf edge: 8 (0 = 8) or 16                  */
} hydro_tree;

/* Allocate every workspace the step needs (state copy for the first stage,
 * per-tile flux differences of the column-walk schedule (86,016 B per 8^3
 * tile), per-tile signal speeds, error flags) for up to p->max_leaves leaves on
 * p->device.  No later call allocates device memory.  *out is NULL on error.
 * Source: section IV-C1 (device buffers and streams are created up front and
 * reused, because allocation synchronises the whole GPU). */
int hydro_create(const hydro_params *p, hydro_t **out);

/* Free the workspace; idempotent on NULL.  Source: section IV-C1 (the
 * handle owns every buffer it pre-allocated). */
int hydro_destroy(hydro_t *h);

/* Build the ghost map of a tree on the host into map[t->n][T][2232] (caller-owned
 * host memory; T = 1 for 8^3 leaves, 8 for 16^3 leaves).  Ghost cells take: periodic wrap or zero-gradient outflow at
 * the leaf's level; a same-level cell; the covering cell of a coarser leaf
 * (injection); or the mean of the 2x2x2 cells of a leaf one level finer.
 * Returns HYDRO_EINVAL if the tree is not 2:1 balanced or a leaf is outside
 * the box.  Synchronous; needs no handle and no GPU.  Source: section IV-B
 * (leaf sub-grids of an AMR octree) and section IV-C1 (each kernel reads
 * its sub-grid's cells and the cells of its ghost layer); the fill rules
 * themselves are not given in the paper. */
int hydro_ghost_map(const hydro_tree *t, int32_t *map);

/* hydro_ghost_map with linear-limited prolongation: a ghost cell inside a
 * coarser leaf's cell C gets, instead of C's value, U_C plus for each axis
 * (+-1/4) minmod(U_{C+e} - U_C, U_C - U_{C-e}) (the sign by the half of C the
 * ghost cell lies in; the neighbours at C's level by the same rules as ghost
 * cells; the terms added in x, y, z order).  The paper's AMR (section IV-B)
 * leaves coarse-to-fine ghost values unspecified; this is the conservative,
 * monotonicity-preserving linear choice.  Such ghost cells get map entries
 * s < -2^30 naming row -s-2^30-1 of table[capacity][8]: {C, C-x, C+x, C-y,
 * C+y, C-z, C+z (each a copy or mean entry as in the ghost map), side bits
 * (bit a: upper half along axis a)}.  *n_table receives the rows needed;
 * HYDRO_ENOMEM if that exceeds capacity.  Needs n * E^3 < 2^30.  Synchronous;
 * needs no handle and no GPU.  Pass the table as hydro_grid.prolong. */
int hydro_ghost_map_linear(const hydro_tree *t, int32_t *map, int32_t *table, int32_t capacity,
                           int32_t *n_table);

/* Coarse/fine face lists of a tree for the flux correction (host memory,
 * caller-owned).  The paper runs the scheme on an AMR octree (section IV-B)
 * and does not say how fluxes are matched where a leaf meets finer ones; the
 * library uses the conservative correction: each stage, the flux through a
 * coarse face shared with four finer cells is replaced by the mean of those
 * cells' own Simpson face fluxes.
 * The lists are per 8^3 block: a leaf itself for 8^3 leaves; for 16^3 leaves
 * block b = 8 leaf + t is the leaf's octant at cell offset
 * 8 (t & 1, (t >> 1) & 1, t >> 2), and the lists are those of the mesh of
 * octants (the same cells and levels), T = 8 blocks per leaf (T = 1 for 8^3).
 *   face_flags[t->n * T]: bit f (f = 2 axis + side, side 1 = the +axis face)
 *     set when face f of the block borders blocks one level finer (the block
 *     is corrected), bit 8+f when it borders a coarser one (the block's flux
 *     through face f is kept for its coarse neighbour).
 *   entries[t->n * T][26] (capacity): one entry per corrected block,
 *     *n_entries of them: {block, mask of bits 0-5, child[6][4]};
 *     child[f][o1 + 2 o2] is the finer block across face f whose offsets along
 *     the two other axes (in increasing axis order) are o1, o2; -1 for faces
 *     without finer blocks.
 * Returns HYDRO_EINVAL if the tree is not 2:1 balanced across a face or a
 * leaf is outside the box.  Synchronous; needs no handle and no GPU.
 * Source: section IV-B (AMR octree); the matching itself is not in the
 * paper. */
int hydro_reflux_map(const hydro_tree *t, int32_t *face_flags, int32_t *entries, int32_t *n_entries);

/* One full SSP Runge-Kutta step of all leaves, in place on g->U (Shu-Osher
 * form, ghosts refreshed from the stage input before each stage, tracer
 * resync after the last stage; section IV-B, three stages in section V-A2):
 *   order 2: U1 = U + dt L(U);  U <- U/2 + (U1 + dt L(U1))/2
 *   order 3: U1 = U + dt L(U);  U2 = 3U/4 + (U1 + dt L(U1))/4;
 *            U <- U/3 + 2(U2 + dt L(U2))/3.
 * If amax_out (host, [g->n]) is non-NULL the call synchronises the stream,
 * writes each leaf's maximum signal speed over both stages and reports
 * HYDRO_ENONPHYS if a stage produced rho <= 0 or a non-finite value.  Otherwise
 * it returns without waiting and the speeds stay in the handle
 * (hydro_amax_device).  Source: section IV-B (reconstruction at the 26
 * points, central-upwind fluxes, Newtonian face quadrature, rotating frame,
 * entropy tracer); section V-A2 (three Runge-Kutta stages per step); every
 * leaf of the call in one launch per stage is the aggregation of section
 * IV-C3. */
int hydro_step(hydro_t *h, const hydro_grid *g, double dt, double *amax_out);

/* One stage with explicit buffers (device, [n][7][512] each; Uin provides the
 * ghosts of every leaf).  stage 1: Uout = Uin + dt L(Uin); stage s > 1 of the
 * handle's order: Uout = a Un + b (Uin + dt L(Uin)) with the coefficients
 * above, and the tracer resync after the last stage.  Uout may alias Un, not
 * Uin.  amax (device [n], may be NULL) receives each leaf's maximum signal
 * speed.  g->U is not used.  Source: section IV-B (one evaluation of the
 * scheme), section V-A2 (a Runge-Kutta stage). */
int hydro_stage(hydro_t *h, const hydro_grid *g, int stage, double dt, const double *Uin,
                const double *Un, double *Uout, double *amax);

/* Maximum signal speed of each leaf for the state g->U: amax (device [n]).
 * Source: section IV-B (the central-upwind scheme's local speeds at the
 * quadrature points). */
int hydro_signal_speed(hydro_t *h, const hydro_grid *g, double *amax);

/* Reconstructed values of every interior cell at its 26 points:
 * out (device [n][7][512][26]); point d = (dx,dy,dz) is numbered
 * 9(dz+1) + 3(dy+1) + (dx+1), minus one past the centre.  8^3 leaves only.
 * Source: section IV-B (PPM along the 13 lines through the cell centre,
 * left and right values at the 26 quadrature points). */
int hydro_reconstruct(hydro_t *h, const hydro_grid *g, double *out);

/* One SSP-RK2 step driven on the device: both stages read dt from dt_dev
 * (device, one double); afterwards dt_dev holds the next step,
 * cfl * min over leaves of dx / a_max over both stages.  Never synchronises
 * and never allocates, so it can be captured into a HIP graph.  Source:
 * section IV-B (the scheme), section V-A2 (Runge-Kutta stages); the time
 * step from the signal speeds is not given in the paper (CFL 0.4 here);
 * running without host round trips answers the launch overheads of
 * section IV-C3. */
int hydro_step_dev(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev);

/* dt_dev = cfl * min over leaves of dx / a_max(g->U): the first step of a run
 * (signal-speed pre-pass; asynchronous).  Source: section IV-B (local
 * speeds of the central-upwind scheme). */
int hydro_dt(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev);

/* Capture nsteps hydro_step_dev calls on g->stream (must not be NULL) into
 * a HIP graph held by the handle, replacing any earlier one; the grid's
 * buffers and launch partition are baked in.  hydro_graph_launch replays it
 * on `stream`.  Source: section IV-C3 (many small kernels starve the GPU;
 * aggregating them is proposed there and in section VII-A as future work);
 * graphs are this library's answer, not the paper's. */
int hydro_graph_capture(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev, int nsteps);
int hydro_graph_launch(hydro_t *h, void *stream);

/* Time every schedule on stage-1 launches of 1, 2, 4, ... leaves (up to
 * g->n, each bucket from the first leaves of g) and keep the fastest per
 * size bucket for HYDRO_SCHED_AUTO; table (host [HYDRO_NBUCKET], may be
 * NULL) receives it, and cache_path (may be NULL) a JSON copy.  When g has
 * several launches per stage (which run concurrently), whole stages of that
 * partition are also timed with the table and with each schedule for every
 * launch, and as one launch over all of g's leaves with the table's
 * schedule (two interleaved rounds, each candidate's faster one counting),
 * and the fastest of these is used for stages of several launches (kept in
 * the JSON copy as "concurrent": -1 for the table, 2-4 a schedule, 5 the one
 * launch).  Uses only the
 * handle's workspace; g->U is read, not written.  Synchronous.  Source:
 * section IV-C3 (the launch configuration and sub-grids per kernel decide
 * GPU utilisation) and section VII-A (tuning the kernels is future work). */
int hydro_autotune(hydro_t *h, const hydro_grid *g, const char *cache_path, int32_t *table);

/* ---- allocation-free step ------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one SSP-RK2
 * step of hydro_step (plain PPM, the column-walk kernel, one launch per
 * stage), without a handle.  Its workspace -- the stage-1 state, the column
 * walk's flux differences, per-leaf signal speeds when amax is NULL and the
 * status word, 7.3 MB for HYDRO_NOALLOC_MAX_LEAVES leaves -- is one fixed
 * device array of the library that every GPU it runs on holds until the
 * process ends; the call allocates nothing.  It runs on the calling thread's
 * current device, in place on g->U (8^3 leaves; g->n <= HYDRO_NOALLOC_MAX_LEAVES,
 * else HYDRO_EINVAL; launch partitions are ignored; no flux correction;
 * linear-prolongation tables are used).  amax (device [g->n], may be NULL)
 * receives each leaf's maximum signal speed over both stages.  The first call
 * on a device looks up the array and uploads the ghost tables, and must not
 * be captured (HYDRO_EINVAL if it is).  sync = 0: asynchronous on g->stream,
 * graph-capturable; sync = 1: waits for the stream and reports HYDRO_ENONPHYS
 * if a stage produced rho <= 0 or a non-finite value.  Errors set
 * hydro_last_error(NULL).  Every call on a device shares that device's array:
 * calls that overlap on one device (other streams, other threads) race. */
#define HYDRO_NOALLOC_MAX_LEAVES 64
int hydro_step_noalloc(const hydro_grid *g, double dt, double eta1, double eta2, double *amax, int sync);

/* ---- learned reconstruction ----------------------------------------------
 * A 34-64-64-26 network (tanh-GELU) maps the normalised 3x3x3 neighbourhood of
 * a cell, x_k = (q_nb - q_c)/sigma with sigma = max |q_nb - q_c|, plus a
 * one-hot field id, to the 26 point values q_c + sigma*y_d.  It runs on
 * bfloat16 MFMA with FP32 accumulation; the plain limiter then acts on the
 * predicted values (clamp between the cell and its neighbour in that
 * direction, PPM monotonicity constraint on each line's pair), every value is
 * checked in FP64 (bounds, monotonicity, rho, E, tau > 0 and X >= 0) and a
 * cell any of whose fields fails takes plain PPM.  Fluxes, update and
 * conservation stay FP64.
 * Parameters: float32 vector of 8090 values, W1[64][34], b1[64], W2[64][64],
 * b2[64], W3[26][64], b3[26].  Not a method of the paper: an extension; the
 * calls below cite no section. */

/* Set the network's parameters (host [8090]); resets the Adam state.
 * Non-finite parameters are accepted: every row they touch fails the check
 * and falls back to plain PPM.  Synchronous. */
int hydro_mlp_load(hydro_t *h, const float *params);
/* Copy the current float32 parameters to host params[8090]. Synchronous. */
int hydro_mlp_save(hydro_t *h, float *params);
/* Network outputs Y (device [B][26]) for inputs X (device [B][34]),
 * B <= mlp_batch.  Asynchronous on stream. */
int hydro_mlp_forward(hydro_t *h, const float *X, int B, float *Y, void *stream);
/* Gradient of the mean-square loss over B rows and 26 outputs against
 * targets T (device [B][26]) into grad (device [8090]); loss (device, one
 * float, may be NULL).  Deterministic.  Asynchronous on stream. */
int hydro_mlp_grad(hydro_t *h, const float *X, const float *T, int B, float *grad, float *loss,
                   void *stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) at learning rate lr on a batch;
 * loss as in hydro_mlp_grad.  Asynchronous on stream. */
int hydro_mlp_train_step(hydro_t *h, const float *X, const float *T, int B, double lr, float *loss,
                         void *stream);
/* Training pairs from the plain reconstruction of g->U: rows
 * [leaf][cell][field] of the interior cells, X (device [n*3584][34]), the
 * plain PPM point values in the same normalisation T (device [n*3584][26]),
 * valid (device [n*3584], 0 where the neighbourhood is flat).  8^3 leaves only. */
int hydro_mlp_pairs(hydro_t *h, const hydro_grid *g, float *X, float *T, uint8_t *valid);
/* Rows of the learned reconstruction that two blocks share, for the learned
 * stages of a grid (host memory, built from the tree and its host ghost map,
 * plain or linear).  A face-adjacent ghost cell of block b that copies cell X
 * of block b2 (same level, or the periodic image) gets, when the 3x3x3
 * neighbourhoods of the two cells are filled from the same sources in every
 * cell, the entry b2 * 896 + slot of X (its network inputs, outputs and
 * verdict are then those of X, bit for bit); else -1.  alias[n T][384] in
 * slot order 512..895 of hydro_mlp_values.  Pass it (on the device) as
 * hydro_grid.mlp_alias: a learned stage's pre-pass then skips every ghost slab
 * all of whose cells alias blocks of the same launch, and the stage reads
 * those cells' values from the aliased rows.  HYDRO_EINVAL for a bad tree.
 * Synchronous; needs no handle and no GPU.  Not in the paper: the learned
 * reconstruction is an extension. */
int hydro_mlp_alias_map(const hydro_tree *t, const int32_t *map, int32_t *alias);

/* The learned reconstruction's pre-pass of a stage alone, for the state g->U
 * (test and inspection support).  For every 8^3 block b (T per leaf) and every
 * cell slot s its fluxes need -- the 512 interior cells by index, then the 64
 * cells of each face-adjacent ghost slab x-, x+, y-, y+, z-, z+ by their two
 * in-block coordinates in axis order (slot 512 + 64 slab + u + 8 v) --
 * val (device [n T][7][26][896], [block][field][point][slot]; points numbered
 * as in hydro_reconstruct) receives the limited FP64 point values, each the
 * cell value plus a binary32 offset rounded toward zero (the stage itself
 * keeps only the offsets: half the bytes), and ok
 * (device uint8 [n T][896]) 1 where the cell passes the FP64 check in all
 * seven fields, 0 where the stage takes plain PPM for it.  y (device float
 * [n T][7][896][26], may be NULL) receives the network's outputs of every row
 * whose neighbourhood is not flat (other rows may be left untouched).
 * With val and ok NULL the pre-pass writes the handle's own workspace exactly
 * as in a stage (skipping the ghost slabs g->mlp_alias shares); with val
 * every slot is computed.  Counts toward hydro_mlp_stats.  Asynchronous on
 * g->stream. */
int hydro_mlp_values(hydro_t *h, const hydro_grid *g, double *val, uint8_t *ok, float *y);
/* Cells reconstructed by the learned path and cells that fell back to plain
 * PPM since the previous call (synchronises): each block's interior cells,
 * 512 per block and pre-pass (a face-adjacent ghost cell is counted in the
 * block it belongs to). */
int hydro_mlp_stats(hydro_t *h, int64_t *cells, int64_t *fallback);

/* Device pointer to the maximum signal speeds of the last step, one per 8^3
 * tile ([n] for 8^3 leaves, [n][8] for 16^3 leaves).  Source: section IV-B
 * (local speeds). */
const double *hydro_amax_device(const hydro_t *h);

/* Synchronise the handle's last stream and report HYDRO_ENONPHYS if any
 * stage since the previous check produced rho <= 0 or a non-finite value;
 * clears the flag.  The paper names no floors; a non-physical state is an
 * error here. */
int hydro_check(hydro_t *h, void *stream);

/* Stage-kernel timing.  enable = 1 starts recording a HIP event pair around
 * every stage launch of a step on its stream (up to 4096 launches, then
 * recording stops; the signal-speed pre-pass of hydro_signal_speed and
 * hydro_dt is not recorded); enable = 0 stops.  If total_ms / launches are non-NULL the call
 * first waits for the recorded events and reports the summed kernel time (ms)
 * and the number of launches timed since the previous report, then clears
 * them.  Event objects are created on the first enable.  Measurement
 * support (section V-A1 reports per-kernel times); not part of the method. */
int hydro_timing(hydro_t *h, int enable, double *total_ms, int64_t *launches);

/* The attainable FP64 vector rate of the current device, for the rooflines:
 * blocks workgroups of 256 threads, each thread eight independent chains of
 * iters fused multiply-adds a = a m + c (16 iters flops per thread), chain k
 * of thread t starting at t + k; out (device double [blocks * 256]) receives
 * each thread's sum of its chains (with m = c = 1: 8 t + 28 + 8 iters).
 * Asynchronous on stream; time it with events.  Errors set
 * hydro_last_error(NULL).  Measurement support; not part of the method. */
int hydro_fp64_probe(double *out, int32_t blocks, int32_t iters, double m, double c, void *stream);

/* Text of a return code, and of the last error of a handle (NULL: of the
 * last hydro_create).  Library support; not part of the method. */
const char *hydro_strerror(int code);
const char *hydro_last_error(const hydro_t *h);

#ifdef __cplusplus
}
#endif
#endif
