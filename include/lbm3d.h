/*
 * lbm3d.h -- C ABI of the three-dimensional form of the two-component
 * pseudopotential lattice Boltzmann hot path on MI355X (gfx950).
 *
 * Method: arXiv 2505.22256 (Chen, Wang, Tao, Yang, Chen), Sec. 3.5: the
 * improved solid-fluid interaction checked on static contact angles of a
 * droplet on a sphere.  The paper states the set-up but not the 3-D lattice;
 * this library implements:
 *   - two D3Q19 population sets, BGK collision with Guo forcing (Eq. 1-7 in
 *     three dimensions), c_s^2 = 1/3, one relaxation time;
 *   - cohesion with psi = rho (Eq. 8) and adhesion (Eq. 9) on the
 *     eighth-order isotropic stencil of the 5x5x5 neighbourhood: the 92
 *     positions with |e|^2 in {1,2,3,4,5,6,8}, weights 4/45, 1/21, 2/105,
 *     5/504, 1/315, 1/630, 1/5040 (sum W e_x^2 = 1; summed over e_z they
 *     are the 2-D E8 weights);
 *   - the second-layer rule of Sec. 2.4 / Table 1 in 3-D: an unavailable
 *     position with a coordinate of magnitude 2 takes what its first-layer
 *     partner (sgn e_x, sgn e_y, sgn e_z) resolves to;
 *   - the local adhesion parameter of component 1 (Eq. 10-12);
 *   - halfway bounce-back at solid nodes and non-periodic faces.
 *
 * Conventions
 *   - Lattice nx x ny x nz (each >= 5), node id = (z*ny + y)*nx + x.  Host
 *     arrays of one value per node are [nz][ny][nx]; population arrays are
 *     [2][19][nz][ny][nx] with the D3Q19 directions
 *       e_0 = 0; e_1..e_6 = (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1);
 *       e_7..e_18 = (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *                   (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *     (each odd direction followed by its opposite), weights 1/3, 1/18,
 *     1/36.
 *   - Host pointers are the caller's; the library copies in or out and
 *     keeps none.  It owns all device memory of a context.
 *   - Every int-returning call returns LBM_OK (0) or a negative LBM_E*
 *     code (the values of lbm.h) and never aborts; lbm3d_last_error gives a
 *     message.  A context is not thread-safe; separate contexts are
 *     independent.  Work is enqueued on the context's HIP stream; calls
 *     that return host data synchronise it.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx lbm3d_ctx;

/* Flags: LBM_PERIODIC_X, LBM_PERIODIC_Y, LBM3D_PERIODIC_Z wrap an axis
 * (outside a non-periodic face counts as solid); LBM_SCHEME_ORIGINAL,
 * LBM_E8_COPY_OFF, LBM_WALLPSI_SELF, LBM_VEL_LITERAL, LBM_FORCE_DENSITY,
 * LBM_ROUND_STOCHASTIC and LBM_ROUND_NEAREST mean what they mean in lbm.h
 * (F16 and BF16 round stochastically unless LBM_ROUND_NEAREST is given).
 * LBM_INLET and LBM_OUTFLOW are not available in 3-D (EINVAL). */
enum { LBM3D_PERIODIC_Z = 2048 };

/* Contact-angle wall kinds for lbm3d_contact_angle. */
enum { LBM3D_WALL_FLAT = 0, LBM3D_WALL_SPHERE = 1 };

/* Create a context on the current HIP device; storage LBM_F64..LBM_BF16.
 * Allocates two population buffers of 38 nx ny nz elements (ping-pong).
 * EINVAL for sizes below 5, more than 2^31 nodes, a buffer range of 4 GiB
 * or more per component, a bad storage or flag; ENOMEM; EDEVICE (no
 * gfx950 device). */
int lbm3d_create(lbm3d_ctx **out, int nx, int ny, int nz, int storage, unsigned flags);
/* Flags in effect (rounding resolved as in lbm_get_flags); 0 for NULL. */
unsigned lbm3d_get_flags(const lbm3d_ctx *c);

/* Solid mask nz*ny*nx bytes (0 fluid, non-zero solid: the switch s of
 * Eq. 9); copied.  Invalidates the populations. */
int lbm3d_set_geometry(lbm3d_ctx *c, const uint8_t *solid);

/* G_c (Eq. 8), G_ads and tau (Eq. 2) with G_w2 = G_c, G_w1 = G_c + 2 G_ads,
 * delta = 0.8 (lambda = G_w1 / G_w2, Sec. 2.3.2).  EINVAL as lbm_set_params. */
int lbm3d_set_params(lbm3d_ctx *c, double G_c, double G_ads, double tau);
/* Paper-native adhesion parameters of Eq. 9-12 (after lbm3d_set_params). */
int lbm3d_set_adhesion(lbm3d_ctx *c, double G_w1, double G_w2, double delta);
/* Body acceleration g_k of each component: g[0..2] component 1, g[3..5]
 * component 2 (force rho_k g_k, or g_k with LBM_FORCE_DENSITY). */
int lbm3d_set_body_accel(lbm3d_ctx *c, const double g[6]);

/* Initial densities (nz*ny*nx each): f_i = w_i rho_k (Eq. 6 at rest), t = 0.
 * Solid entries ignored; EINVAL on a non-finite fluid density; ESTATE
 * before lbm3d_set_geometry. */
int lbm3d_init_fields(lbm3d_ctx *c, const double *rho1, const double *rho2);
/* Pre-collision populations f(x, t), [2][19][nz][ny][nx] FP64 (solid: ignored
 * on input, 0 on output).  set resets t to 0. */
int lbm3d_set_populations(lbm3d_ctx *c, const double *f);
int lbm3d_get_populations(lbm3d_ctx *c, double *f);

/* Advance n >= 0 time steps of Eq. 1 in 3-D: densities and momenta
 * (Eq. 3-4), cohesion on the 92-position stencil with the second-layer
 * copy (Eq. 8, Sec. 2.4), adhesion with the local G (Eq. 9-12), body force,
 * u^eq (Eq. 5), BGK + Guo collision (Eq. 2, 6, 7), pull streaming with
 * halfway bounce-back (Sec. 3.5).  Asynchronous.  ESTATE before geometry,
 * parameters and fields; EINVAL for n < 0; EDEVICE when a launch fails. */
int lbm3d_step(lbm3d_ctx *c, int n);
int lbm3d_synchronize(lbm3d_ctx *c);
long lbm3d_time(const lbm3d_ctx *c);

/* rho_k and u^eq (Eq. 3-5) at the current time, nz*ny*nx FP64 each; NULL
 * skips; solid nodes give 0.  Synchronous. */
int lbm3d_get_fields(lbm3d_ctx *c, double *rho1, double *rho2, double *ux, double *uy, double *uz);

/* out = {M1, M2, Px, Py, Pz, max|u|, min rho1, max rho1, non-finite count}
 * over fluid nodes (as lbm_reduce), FP64, deterministic compensated sums.
 * Synchronous. */
int lbm3d_reduce(lbm3d_ctx *c, double out[9]);

/* Static contact angle in degrees, through component 1: interface points
 * where rho^e (Eq. 10) changes sign along x, y and z links between fluid
 * nodes of the largest region of each phase (6-connected, not across
 * periodic seams), at least 3 lattice units from the wall; algebraic sphere
 * fit refined by Gauss-Newton, FP64 on the device.
 *   LBM3D_WALL_FLAT:   wall[0] = wall plane z_w (droplet above);
 *   LBM3D_WALL_SPHERE: wall[0..2] centre, wall[3] surface radius;
 *   cos theta = -(z_c - z_w)/r, or (R^2 + r^2 - d^2) / (2 R r).
 * EUNSTABLE with fewer than 4 points or a failed fit.  Synchronous. */
int lbm3d_contact_angle(lbm3d_ctx *c, int wall_kind, const double wall[4], double *theta_deg);

/* Brick of the collide pass: bx x by x bz nodes per workgroup of
 * bx * by * tz threads (tz threads per column, each finishing every tz-th
 * plane of it), one of 32 x 8 x 4 with tz 1, 2 or 4, 32 x 8 x 8 with tz 1
 * or 2, and 64 x 4 x 4 with tz 2; EINVAL otherwise.  The default is
 * 32 x 8 x 4 with tz 2 for FP32 and with tz 1 for the other storages.  Each
 * step runs a density pass (psi = rho of every node from the pulled
 * populations, 2 values per node) and then the collide pass, which stages
 * psi of its brick and a 2-node halo in LDS and pulls the populations of
 * its own nodes.  Results do not depend on the brick (bitwise). */
int lbm3d_set_tile(lbm3d_ctx *c, int bx, int by, int bz, int tz);
int lbm3d_get_tile(const lbm3d_ctx *c, int *bx, int *by, int *bz, int *tz);

int lbm3d_set_stream(lbm3d_ctx *c, void *hip_stream);
/* Fluid nodes, and the algorithmic bytes per fluid-node update: 2
 * components x 19 populations x (read + write) x element + 1 byte. */
long lbm3d_fluid_nodes(const lbm3d_ctx *c);
int lbm3d_bytes_per_update(const lbm3d_ctx *c);
const char *lbm3d_last_error(const lbm3d_ctx *c);
void lbm3d_destroy(lbm3d_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* LBM3D_H */
