/*
 * FP64 CPU oracle of the three-dimensional form of the two-component
 * pseudopotential lattice Boltzmann method with the improved solid-fluid
 * adhesion (arXiv 2505.22256, Sec. 3.5: static contact angles on a sphere).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, serial-order FP64 code used to
 * check the GPU library.  It shares no code, header, table or constant with
 * the GPU path (nor with the 2-D oracle, apart from living in the same
 * shared object).  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.
 *
 * The paper gives the 3-D set-up but not the 3-D lattice; the readings
 * implemented here:
 *   - D3Q19 velocity set, c_s^2 = 1/3, weights 1/3, 1/18 (6 axis links),
 *     1/36 (12 face diagonals); directions 1-6 = +-x, +-y, +-z, then the
 *     diagonals, each odd direction followed by its opposite;
 *   - cohesion (Eq. 8) and adhesion (Eq. 9) on the eighth-order isotropic
 *     3-D stencil of the 5x5x5 neighbourhood: the 92 positions with
 *     |e|^2 in {1, 2, 3, 4, 5, 6, 8}, weights fixed by sum W e_x^2 = 1 and
 *     isotropy of the 4th, 6th and 8th moment tensors;
 *   - the second-layer rule of Sec. 2.4 / Table 1 in 3-D: an unavailable
 *     position with a coordinate of magnitude 2 takes the value its
 *     first-layer partner (sgn e_x, sgn e_y, sgn e_z) resolves to, which is
 *     what Table 1 does in 2-D;
 *   - everything else (Eq. 10-12, Guo forcing, BGK, halfway bounce-back,
 *     the readings of the 2-D oracle) unchanged.
 *
 * Conventions
 *   lattice nx x ny x nz, node id = (z*ny + y)*nx + x (x fastest);
 *   populations f[k][i][node], k = 0,1, i = 0..18;
 *   the state is the pre-collision population set at time t;
 *   solid nodes carry no populations (entries ignored / zero).
 */
#ifndef LBM_ORACLE3D_H
#define LBM_ORACLE3D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OR3_OK = 0,
    OR3_EINVAL = -1,
    OR3_ESTATE = -2,
    OR3_ENOMEM = -3,
    OR3_EUNSTABLE = -5
};

/* Flags: the 2-D oracle's bit values where they mean the same. */
enum {
    OR3_PERIODIC_X = 1,
    OR3_PERIODIC_Y = 2,
    OR3_SCHEME_ORIGINAL = 4,
    OR3_E8_COPY_OFF = 8,
    OR3_WALLPSI_SELF = 16,
    OR3_VEL_LITERAL = 32,
    OR3_FORCE_DENSITY = 64,
    OR3_PERIODIC_Z = 2048
};

typedef struct oracle3d_ctx oracle3d_ctx;

int  oracle3d_create(oracle3d_ctx **out, int nx, int ny, int nz, unsigned flags);
void oracle3d_destroy(oracle3d_ctx *c);
const char *oracle3d_last_error(const oracle3d_ctx *c);

int oracle3d_set_geometry(oracle3d_ctx *c, const uint8_t *solid);
int oracle3d_set_params(oracle3d_ctx *c, double G_c, double G_ads, double tau);
int oracle3d_set_adhesion(oracle3d_ctx *c, double G_w1, double G_w2, double delta);
int oracle3d_set_body_accel(oracle3d_ctx *c, const double g[6]); /* g1 (x,y,z), g2 (x,y,z) */
int oracle3d_init_fields(oracle3d_ctx *c, const double *rho1, const double *rho2);
int oracle3d_set_populations(oracle3d_ctx *c, const double *f);
int oracle3d_get_populations(const oracle3d_ctx *c, double *f);
int oracle3d_step(oracle3d_ctx *c, int nsteps);
long oracle3d_time(const oracle3d_ctx *c);

/* rho_k and u^eq at time t; NULL skips; solid nodes give 0. */
int oracle3d_get_fields(oracle3d_ctx *c, double *rho1, double *rho2, double *ux, double *uy, double *uz);
/* out = {M1, M2, Px, Py, Pz, max|u|, min rho1, max rho1, non-finite count}. */
int oracle3d_reduce(oracle3d_ctx *c, double out[9]);

/* Per-node pieces (x, y, z of a fluid node, densities of time t):
 * parts[18] = [coh1 coh2 ads1 ads2 body1 body2] x (x, y, z); S[3]. */
int oracle3d_node_forces(oracle3d_ctx *c, int x, int y, int z, double parts[18]);
int oracle3d_adhesion_vector(const oracle3d_ctx *c, int x, int y, int z, double S[3]);

/* Constants: D3Q19 (19 entries each) and the 3-D stencil (92 entries;
 * copy_from = 0-based first-layer partner, or -1). */
void oracle3d_d3q19(int ex[19], int ey[19], int ez[19], double w[19], int opp[19]);
int  oracle3d_stencil(int ex[92], int ey[92], int ez[92], double W[92], int copy_from[92]);
void oracle3d_equilibrium(double rho, const double u[3], double feq[19]);
void oracle3d_forcing(const double F[3], const double u[3], double Fi[19]);

/* Contact angle.  kind 0: flat wall z = wall[0] (droplet above);
 * kind 1: sphere of centre wall[0..2] and surface radius wall[3].
 * Interface points where rho^e changes sign along x, y and z links between
 * fluid nodes of the largest region of each phase (6-connected, not across
 * periodic seams), at least 3 lattice units from the wall; sphere fit
 * (algebraic, then Gauss-Newton). */
int oracle3d_interface_points(oracle3d_ctx *c, int kind, const double wall[4], double *px, double *py,
                              double *pz, int cap, int *n_out);
int oracle3d_sphere_fit(const double *px, const double *py, const double *pz, int n, double out[4]);
int oracle3d_contact_angle(oracle3d_ctx *c, int kind, const double wall[4], double *theta_deg);

#ifdef __cplusplus
}
#endif
#endif /* LBM_ORACLE3D_H */
