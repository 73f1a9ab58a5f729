/*
 * lbm.h -- C ABI of the MI355X (gfx950) two-component pseudopotential
 * lattice Boltzmann hot path.
 *
 * Method: Chen, Wang, Tao, Yang, Chen, "Improvement of Solid-Fluid
 * Interaction Scheme in Lattice Boltzmann Immiscible Pseudopotential Models"
 * (arXiv 2505.22256):
 *   - two D2Q9 population sets, BGK collision with Guo forcing (Sec. 2.1-2.2,
 *     Eq. 1-7), one relaxation time for both components;
 *   - fluid-fluid cohesion with psi = rho on the eighth-order-isotropic (E8)
 *     24-position stencil (Eq. 8, Sec. 2.4);
 *   - second-layer stencil data at walls copied from the first layer
 *     (Sec. 2.4, Table 1);
 *   - Martys-Chen adhesion (Eq. 9) with the local, effective-density
 *     dependent parameter of component 1 (Eq. 10-12);
 *   - halfway bounce-back at solid nodes and at non-periodic domain edges
 *     (Sec. 3.1, 3.2, 3.5).
 *
 * Conventions shared by every entry point
 *   - Lattice nx x ny, node id = y*nx + x (x fastest).  Host arrays of one
 *     value per node are [ny][nx]; population arrays are [2][9][ny][nx]
 *     (component, D2Q9 direction, node) with the directions
 *     e_0 = (0,0), e_1..e_8 = (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *   - All host pointers are owned by the caller; the library copies in or
 *     out and keeps no host pointer after the call returns.  The library owns
 *     all device memory of a context.
 *   - Every int-returning call returns LBM_OK (0) or a negative LBM_E* code
 *     and never aborts; lbm_last_error() gives a message.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Work is enqueued on the context's HIP stream (lbm_set_stream); calls
 *     that return host data synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* bad argument or parameter                      */
    LBM_ESTATE = -2,    /* call out of order (e.g. step before init)       */
    LBM_ENOMEM = -3,    /* host or device allocation failed                */
    LBM_EDEVICE = -4,   /* HIP runtime error, or no usable gfx950 device   */
    LBM_EUNSTABLE = -5, /* non-finite state, or the contact angle failed   */
    LBM_EIO = -6        /* checkpoint file error                           */
};

/* Population storage.  F64 stores f and computes in FP64.  F32, F16 and
 * BF16 store the deviation g_i = f_i - w_i rho0_k (rho0_k = mean initial
 * density of component k over fluid nodes) and compute in FP32.  F32
 * rounds to nearest even; F16 and BF16 round stochastically unless
 * LBM_ROUND_NEAREST is given (see the flags below). */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_BF16 = 3 };

/* Context flags.  PERIODIC_* wrap an axis; along a non-periodic axis the
 * outside counts as solid.  The others select alternative readings of
 * points the paper leaves open:
 *   SCHEME_ORIGINAL  constant G_w1 for component 1 (Eq. 9, Sec. 2.3.1);
 *   E8_COPY_OFF      unavailable second-layer positions read 0 (no Table 1 copy);
 *   WALLPSI_SELF     unavailable first-layer positions read psi(x) instead of 0;
 *   VEL_LITERAL      u^eq = sum_k j_k / sum_k rho_k (Eq. 4-5 without the
 *                    half-force shift of Guo's scheme);
 *   FORCE_DENSITY    body force g_k per unit volume instead of rho_k g_k.
 * INLET and OUTFLOW open the x edges (x must not be periodic; EINVAL
 * otherwise), as in the confined-droplet set-up of Sec. 3.3:
 *   INLET    Zou-He velocity inlet at x = 0: the populations entering from
 *            x = -1 are rebuilt so that each component has the row's
 *            velocity (lbm_set_inlet_velocity);
 *   OUTFLOW  zero-gradient outflow at x = nx - 1: the populations entering
 *            from x = nx are those the upstream neighbour receives, i.e.
 *            pulled from (nx - 1, y - e_iy); bounce-back if that is solid.
 *   On the E8 stencil (Sec. 2.4) a first-layer position beyond an open
 *   edge reads its ghost, the node of the same row clamped into the domain
 *   (zero when that is solid), and a second-layer one takes the Table 1
 *   copy; the solid switch s of Eq. 9 there is the ghost's.
 * Rounding of F16 and BF16 stores (ignored for F64 and F32):
 *   ROUND_STOCHASTIC (the default for F16 and BF16; giving it is allowed)
 *            rounds the stored deviation up or down with probability
 *            proportional to the distance, from a counter-based hash of
 *            (node, component, direction, step): unbiased, reproducible
 *            and independent of the tiling.
 *   ROUND_NEAREST  round-to-nearest-even instead.  Its error repeats every
 *            step in a steady state and accumulates (mass drift): on the
 *            flat-wall droplet the contact angle is off by about 5 degrees
 *            (F16) and 11 degrees (BF16) after 5000 steps.
 *   Both together are EINVAL.  lbm_get_flags returns the flags in effect. */
enum {
    LBM_PERIODIC_X = 1,
    LBM_PERIODIC_Y = 2,
    LBM_SCHEME_ORIGINAL = 4,
    LBM_E8_COPY_OFF = 8,
    LBM_WALLPSI_SELF = 16,
    LBM_VEL_LITERAL = 32,
    LBM_FORCE_DENSITY = 64,
    LBM_ROUND_STOCHASTIC = 128,
    LBM_INLET = 256,
    LBM_OUTFLOW = 512,
    LBM_ROUND_NEAREST = 1024
};

/* Tile schedule bits for lbm_set_tile. */
enum { LBM_SCHED_ALIGN = 1, LBM_SCHED_BANDS = 2, LBM_SCHED_XCD_SLABS = 4, LBM_SCHED_TWO_STEP = 8, LBM_SCHED_REPULL = 16 };

/* Contact-angle wall kinds for lbm_contact_angle. */
enum { LBM_WALL_FLAT = 0, LBM_WALL_CYLINDER = 1 };

/* Create a context on the current HIP device.  nx, ny >= 5; storage one of
 * LBM_F64..LBM_BF16; flags a combination of LBM_PERIODIC_X..LBM_ROUND_NEAREST.
 * Allocates two population buffers of 18*nx*ny elements (ping-pong).  One
 * component's 9 direction arrays are addressed through one 32-bit buffer
 * range, so 9*nx*ny elements must span less than 4 GiB (at most about 60 M
 * nodes in FP64, 119 M in FP32, 238 M in FP16 or BF16); nx*ny <= 2^30.
 * Errors: EINVAL (sizes, storage, flags), ENOMEM, EDEVICE (no gfx950 GPU). */
int lbm_create(lbm_ctx **out, int nx, int ny, int storage, unsigned flags);

/* As lbm_create, but the two population buffers are the caller's device
 * memory (for instance two torch tensors' data_ptr on the current device),
 * so that a caller can read or write the state in place.  Each must hold
 * lbm_population_bytes(nx, ny, storage) bytes, be 256-byte aligned, lie on
 * the current device and not overlap the other.  The library never frees
 * them; they must stay valid until lbm_destroy.  Layout of each: the
 * storage type's elements as [component 2][direction 9][y][x], directions
 * e_0 = (0,0), e_1..e_4 = (1,0), (0,1), (-1,0), (0,-1), e_5..e_8 = (1,1),
 * (-1,1), (-1,-1), (1,-1); solid nodes hold all-ones bit patterns.
 * The buffer lbm_current_buffer names holds the post-collision populations
 * of the last step, f*(x, t-1); the next step pulls f_i(x, t) =
 * f*_i(x - e_i, t-1), or the bounce-back f*_opp(i)(x, t-1) at a wall link,
 * from it.  After lbm_init_fields or lbm_set_populations it holds the state
 * set, streamed backwards (f*_j(z) = f_j(z + e_j), or f_opp(j)(z) where
 * z + e_j is solid) so that this pull returns it.  The other buffer is
 * the next step's output: the step overwrites every fluid-node slot of it,
 * so a caller may use those in between, but it writes no solid-node slot
 * (they keep the all-ones pattern that marks solid nodes to the step after
 * it); a caller must leave those slots, in either buffer, unchanged.
 * For F32, F16 and BF16 storage the values are the deviations of the
 * storage-type comment above.  Errors: as lbm_create, and EINVAL for a null,
 * misaligned, too small, overlapping or non-device buffer. */
int lbm_create_ex(lbm_ctx **out, int nx, int ny, int storage, unsigned flags, void *buf_a, void *buf_b,
                  size_t bytes_each);
/* Bytes of one population buffer: 18*nx*ny elements of the storage type
 * (0 for sizes or a storage lbm_create refuses). */
size_t lbm_population_bytes(int nx, int ny, int storage);
/* 0 for buf_a, 1 for buf_b: the buffer that holds the current state. */
int lbm_current_buffer(const lbm_ctx *c);
/* Flags in effect: those given at creation with the storage's rounding
 * resolved (LBM_ROUND_STOCHASTIC set for F16 and BF16 unless
 * LBM_ROUND_NEAREST was given; neither bit for F64 and F32).  0 for a null
 * context. */
unsigned lbm_get_flags(const lbm_ctx *c);

/* Solid mask, ny*nx bytes, 0 = fluid, non-zero = solid (the switch s(x) of
 * Eq. 9).  Copied.  Invalidates the populations (init again). */
int lbm_set_geometry(lbm_ctx *c, const uint8_t *solid);

/* Physical parameters: cohesion G_c (Eq. 8), adhesion G_ads and relaxation
 * time tau (Eq. 2).  Adhesion mapping: G_w2 = G_c, G_w1 = G_c + 2 G_ads,
 * delta = 0.8 (Sec. 2.3.2: G_w2 = G12, lambda = G_w1/G_w2 = 1 + 2 G_ads/G_c).
 * EINVAL if tau <= 0.5, if a value is non-finite, or, for the improved
 * scheme, if lambda <= 0 or G_w1 + G_w2 == 0. */
int lbm_set_params(lbm_ctx *c, double G_c, double G_ads, double tau);

/* Paper-native adhesion parameters of Eq. 9-12 (after lbm_set_params).
 * EINVAL if delta <= 0 or, for the improved scheme, G_w1 + G_w2 == 0. */
int lbm_set_adhesion(lbm_ctx *c, double G_w1, double G_w2, double delta);

/* Body acceleration g_k of each component (force rho_k g_k, Sec. 3.1). */
int lbm_set_body_accel(lbm_ctx *c, double g1x, double g1y, double g2x, double g2y);

/* Sliding walls (the Couette set-up of Sec. 3.1): solid nodes, and
 * positions outside a non-periodic y edge, in rows y < ny/2 move with
 * (ubx, uby), the others with (utx, uty).  A bounce-back link from a moving
 * wall gains 6 w_i rho*_k (e_i . u_w) (Ladd's momentum term), rho*_k being
 * the node's own post-collision density.  All zero (the default): resting
 * walls.  EINVAL on a non-finite value. */
int lbm_set_wall_velocity(lbm_ctx *c, double ubx, double uby, double utx, double uty);

/* Inlet velocity of each row (ux, uy: ny FP64 each, copied), used with
 * LBM_INLET, e.g. the Poiseuille profile u_x = 4 U_m eta (1 - eta) of
 * Sec. 3.3.  Default zero.  EINVAL if a value is non-finite or ux >= 1. */
int lbm_set_inlet_velocity(lbm_ctx *c, const double *ux, const double *uy);

/* Initial densities (ny*nx each, FP64): f_i = w_i rho_k, u = 0, t = 0,
 * i.e. the equilibrium of Eq. 6 at rest (the paper starts from the two
 * phases' densities without stating the populations).  Solid entries are
 * ignored.  EINVAL on a non-finite fluid density, ESTATE before
 * lbm_set_geometry. */
int lbm_init_fields(lbm_ctx *c, const double *rho1, const double *rho2);

/* Pre-collision populations f(x, t) as [2][9][ny][nx] FP64; solid entries
 * ignored on input, returned as 0.  set_populations resets t to 0.  The
 * state set by init_fields or set_populations is taken as given: the open
 * and moving boundary conditions act from the first step's streaming on. */
int lbm_set_populations(lbm_ctx *c, const double *f);
int lbm_get_populations(lbm_ctx *c, double *f);

/* Pre-collision populations f(x, t) of the w x h window whose lower-left
 * node is (x0, y0), as [2][9][h][w] FP64 (solid -> 0).  The window wraps
 * along periodic axes; EINVAL if it leaves a non-periodic domain or
 * w, h < 1.  Synchronous. */
int lbm_get_populations_window(lbm_ctx *c, int x0, int y0, int w, int h, double *f);

/* Advance n >= 0 time steps of Eq. 1: densities and momenta (Eq. 3-4),
 * cohesion on the E8 stencil with the Table 1 second-layer copy (Eq. 8,
 * Sec. 2.4), adhesion with the local G of component 1 (Eq. 9-12), body
 * force, the Guo-shifted velocity (Eq. 5), BGK collision with the Guo
 * forcing term (Eq. 2, 6, 7), then pull streaming with halfway bounce-back
 * (Sec. 3.1-3.2).  Asynchronous: the kernels are enqueued on the context
 * stream.  ESTATE before geometry, parameters and initial fields; EINVAL
 * for n < 0; EDEVICE when a launch fails. */
int lbm_step(lbm_ctx *c, int n);

/* Fused diagnostics: with every > 0, every step whose start time t is a
 * multiple of `every` also accumulates the lbm_reduce() quantities of time
 * t inside the step kernel (no extra pass over the populations); the
 * latest record stays on the device until lbm_get_diag copies it (with its
 * time in *t_diag).  every = 0 turns this off.  ESTATE if no record exists. */
int lbm_set_diag_interval(lbm_ctx *c, int every);
int lbm_get_diag(lbm_ctx *c, double out[8], long *t_diag);

/* Wait for all work of the context; EDEVICE if a kernel failed. */
int lbm_synchronize(lbm_ctx *c);

/* Number of steps taken since the last initialisation. */
long lbm_time(const lbm_ctx *c);

/* Densities rho_k and the common velocity u^eq (Eq. 3-5 with the Guo
 * half-force shift) at the current time, ny*nx FP64 each; NULL skips an
 * output; solid nodes give 0.  Synchronous. */
int lbm_get_fields(lbm_ctx *c, double *rho1, double *rho2, double *ux, double *uy);

/* Whole-lattice diagnostics at the current time, FP64 with a deterministic
 * compensated two-pass sum: out = {M1, M2, Px, Py, max|u|, min rho1,
 * max rho1, number of fluid nodes with a non-finite rho or u}, where
 * M_k = sum rho_k (Eq. 3; conserved by Eq. 1-2) and P = sum (rho_1 +
 * rho_2) u^eq with u^eq of Eq. 5 (the spurious-current measure of Sec. 3.2
 * is max|u|).  Fluid nodes only; a node with a non-finite value is counted
 * in out[7] and left out of the rest.  With no fluid node, min and max
 * rho1 are 0.  Synchronous; ESTATE before initialisation. */
int lbm_reduce(lbm_ctx *c, double out[8]);

/* lbm_reduce for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * eight diagnostics, written to d_out, the caller's device memory (8
 * doubles, 8-byte aligned), enqueued on the context's stream and not
 * synchronised (read d_out after lbm_synchronize or a stream wait).  No
 * device or host allocation and no copy: the workgroup partials go to a
 * 1 MiB device array that the library holds on each GPU it runs on until
 * the process ends, so at most 16384 workgroup records: EINVAL for a
 * lattice that needs more (the pass runs 252-column strips in segments of
 * the tile's seg_rows rows, 64 when that is 0: ceil(nx / 252) times
 * ceil(ny / seg_rows), rounded up to a multiple of 8, must not exceed
 * 16384).  Every call on one GPU uses the same
 * array: calls that overlap in time on one GPU (other streams, other
 * contexts, other threads) race and must be serialised by the caller; the
 * array needs no clearing (every record is written before it is read).
 * ESTATE before initialisation; EINVAL for a null or misaligned d_out. */
int lbm_reduce_noalloc(lbm_ctx *c, double *d_out);

/* Static contact angle (degrees, measured through component 1).  Interface
 * points where rho^e = (rho1 - rho2)/(rho1 + rho2) (Eq. 10) changes sign
 * along x- and y-links between fluid nodes, by linear interpolation; points
 * closer than 3 lattice units to the wall are dropped; algebraic circle fit
 * refined by Gauss-Newton, in FP64 on the device.
 *   wall_kind LBM_WALL_FLAT:     wall[0] = wall line y_w (drop above it);
 *   wall_kind LBM_WALL_CYLINDER: wall[0..1] = centre, wall[2] = surface radius.
 * EUNSTABLE if fewer than 3 points remain or the fit fails. */
int lbm_contact_angle(lbm_ctx *c, int wall_kind, const double wall[3], double *theta_deg);

/* Tables the step kernel derives from the geometry (Sec. 2.3-2.4: the
 * bounce-back links of halfway bounce-back, and the E8 stencil positions
 * after the Table 1 second-layer rule), for checking:
 *   link[ny*nx]: bit i-1 set when the pull source x - e_i of fluid node x is
 *     unavailable (bounce-back); 0 on solid nodes;
 *   nw_list[n_nw]: fluid nodes with an unavailable E8 stencil position,
 *     ascending;
 *   nw_src[24*n_nw]: per listed node and stencil position n = 1..24, the node
 *     whose psi is used after the wall rules, or -1 for zero.  Stencil order:
 *     1-8 the D2Q9 links e_1..e_8, 9-16 twice e_1..e_8, then (2,1) (-1,2)
 *     (-2,-1) (1,-2) (1,2) (-2,1) (-1,-2) (2,-1).
 * Pass nw_list = NULL to query n_nw only.  Synchronous. */
int lbm_get_tables(lbm_ctx *c, uint8_t *link, int32_t *nw_list, int32_t *nw_src, int *n_nw);

/* Use an existing HIP stream (hipStream_t, e.g. a torch stream handle);
 * NULL selects the library's own stream. */
int lbm_set_stream(lbm_ctx *c, void *hip_stream);

/* Tile shape of the step kernel: block in {64, 128, 256} threads (strip
 * width block - 4 columns) and rows per workgroup segment.  seg_rows = 0
 * is persistent scheduling: one work unit per resident workgroup, each
 * taking an equal share of the strip rows.  Default after lbm_create:
 * FP32 block 128 (64 with LBM_INLET or LBM_OUTFLOW), seg_rows 24,
 * LBM_SCHED_TWO_STEP | LBM_SCHED_BANDS; FP16 and BF16 block 64,
 * seg_rows 32, LBM_SCHED_TWO_STEP | LBM_SCHED_BANDS, except that with
 * LBM_INLET or LBM_OUTFLOW BF16, and FP16 with stochastic rounding (its
 * default), take block 128, seg_rows 16, LBM_SCHED_BANDS; FP64 block 64,
 * seg_rows 48, LBM_SCHED_TWO_STEP | LBM_SCHED_BANDS.  Results do not
 * depend on the tile shape (bitwise).  sched bits: LBM_SCHED_ALIGN makes
 * strips a multiple of 128 bytes wide from x = 0, so that stores never
 * cover part of a cache line shared with another workgroup;
 * LBM_SCHED_BANDS (fixed segments only) runs units across the strips
 * first, so concurrent workgroups cover whole rows; LBM_SCHED_XCD_SLABS
 * gives each of the 8 XCDs one contiguous slab of rows, one workgroup per
 * strip marching down it (seg_rows is ignored).  LBM_SCHED_TWO_STEP (FP32,
 * FP16, BF16: any block; FP64: block 64 or 128, EINVAL otherwise)
 * fuses two time steps per launch: the first step's
 * post-collision rows stay in LDS and the second step pulls them from
 * there, so HBM is read and written once per two steps (strips lose 5
 * columns of halo on each side instead of 2); the diagnostics of either
 * step are recorded in the same launch; an odd last step (and every step
 * when diagnostics are due every step) runs alone.  Populations are
 * bitwise those of single steps; diagnostics agree to rounding (the sums
 * run in another order).  lbm_autotune times the
 * current tile and then every candidate for `steps` steps each on the
 * current state (restoring state and time afterwards); a candidate replaces
 * the best so far only when it is at least 2 % faster, so timing noise does
 * not move the choice between near-equal tiles.  LBM_SCHED_REPULL (with
 * LBM_SCHED_TWO_STEP, 64- or 128-thread strips, closed lattices without
 * sliding walls) makes the first of the two fused steps pull each row
 * again when it finishes it instead of holding the pulled rows in
 * registers: fewer registers per thread, one more read of each row
 * through the caches; results are unchanged (bitwise). */
int lbm_set_tile(lbm_ctx *c, int block, int seg_rows, unsigned sched);
int lbm_get_tile(const lbm_ctx *c, int *block, int *seg_rows, unsigned *sched);
int lbm_autotune(lbm_ctx *c, int steps);

/* Checkpoint: populations, time, parameters, wall and inlet velocities.
 * EIO on file errors; load requires a context of the same size, storage
 * and flags. */
int lbm_save(lbm_ctx *c, const char *path);
int lbm_load(lbm_ctx *c, const char *path);

/* Number of fluid nodes (after set_geometry), and the algorithmic bytes per
 * fluid-node update of the step for this storage: 2 components x 9
 * populations x (read + write) + 1 byte of geometry. */
long lbm_fluid_nodes(const lbm_ctx *c);
int lbm_bytes_per_update(const lbm_ctx *c);

const char *lbm_last_error(const lbm_ctx *c);
void lbm_destroy(lbm_ctx *c);

/* ------------------------------------------------------------------ */
/* Batching: many independent runs in one launch per time step          */
/* ------------------------------------------------------------------ */

/* One run of a batch.  Arrays are ny*nx and copied at creation.  accel may
 * be NULL (no body force). */
typedef struct {
    int nx, ny;
    unsigned flags;
    double G_c, G_ads, tau;
    int wall_kind;
    double wall[3];
    const uint8_t *solid;
    const double *rho1, *rho2;
    const double *accel; /* g1x, g1y, g2x, g2y or NULL */
} lbm_run_desc;

/* Create a batch of nruns runs with one storage type.  Every run is advanced
 * by one kernel launch per time step over a (run, strip, segment) work list;
 * with `use_graph` non-zero, lbm_batch_step replays a captured HIP graph.
 * Each run's result is bitwise that of a single context with the same
 * inputs and tile shape. */
int lbm_batch_create(lbm_batch **out, int nruns, const lbm_run_desc *runs, int storage);
/* (The rounding of F16 and BF16 stores is a property of the launch: every
 * run of a batch must resolve to the same mode, i.e. LBM_ROUND_NEAREST on
 * all runs or on none; LBM_EINVAL otherwise.) */
int lbm_batch_set_tile(lbm_batch *b, int block, int seg_rows);
/* Tile of the batched kernel by measurement: times the current tile and
 * then block in {64, 128, 256} x seg_rows in {8, 16, 24, 32, 48, 64, 128,
 * 256}, with one step
 * per launch and (except FP64) two fused steps, for `steps` steps each (no
 * graph), keeps the fastest (a candidate needs a 2 % margin over the best
 * so far) and restores every run's state and the step counter.
 * Synchronous. */
int lbm_batch_autotune(lbm_batch *b, int steps);
int lbm_batch_get_tile(const lbm_batch *b, int *block, int *seg_rows);
/* LBM_SCHED_TWO_STEP (FP32 / FP16 / BF16, any block) fuses two time
 * steps per launch as for a single lattice; 0 runs one step per launch.
 * Other bits are LBM_EINVAL.  The autotuner also tries both. */
int lbm_batch_set_sched(lbm_batch *b, unsigned sched);
unsigned lbm_batch_get_sched(const lbm_batch *b);
int lbm_batch_step(lbm_batch *b, int n);
int lbm_batch_use_graph(lbm_batch *b, int use_graph, int steps_per_graph);
int lbm_batch_get_fields(lbm_batch *b, int run, double *rho1, double *rho2, double *ux, double *uy);
int lbm_batch_contact_angles(lbm_batch *b, double *theta_deg);
int lbm_batch_set_stream(lbm_batch *b, void *hip_stream);
long lbm_batch_fluid_nodes(const lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);
void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
