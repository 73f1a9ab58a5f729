/*
 * FP64 CPU oracle for the two-component immiscible pseudopotential (Shan-Chen,
 * psi = rho) lattice Boltzmann method with the improved, effective-density
 * dependent solid-fluid adhesion and the eighth-order-isotropic (E8) stencil
 * with second-layer copying at walls.
 *
 * Paper: Chen, Wang, Tao, Yang, Chen, "Improvement of Solid-Fluid Interaction
 * Scheme in Lattice Boltzmann Immiscible Pseudopotential Models"
 * (arXiv 2505.22256), Sec. 2.1-2.4, Eq. 1-12, Table 1.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial-order FP64
 * implementation used to check the GPU library.  It shares no code, header,
 * table or constant with the GPU path.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.
 *
 * Conventions
 *   lattice nx x ny, node id = y*nx + x (x fastest);
 *   populations f[k][i][node], k = 0,1 (components 1,2), i = 0..8;
 *   the state is the pre-collision population set at time t;
 *   solid nodes carry no populations (their entries are ignored / zero).
 *
 * Every entry point returns ORC_OK (0) or a negative error code; the last
 * error message is kept in the context.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ESTATE = -2,
    ORC_ENOMEM = -3,
    ORC_EUNSTABLE = -5
};

/* Context flags.  Bits 0-1 select periodic axes; the rest select the
 * alternative readings of passages the paper leaves open. */
enum {
    ORC_PERIODIC_X = 1,
    ORC_PERIODIC_Y = 2,
    ORC_SCHEME_ORIGINAL = 4,   /* constant G_w1 (Eq. 9) instead of Eq. 11   */
    ORC_E8_COPY_OFF = 8,       /* unavailable second layer -> 0, no copy    */
    ORC_WALLPSI_SELF = 16,     /* unavailable first layer -> psi(x), not 0  */
    ORC_VEL_LITERAL = 32,      /* u^eq = sum j / sum rho (Eq. 4-5 literal)  */
    ORC_FORCE_DENSITY = 64,    /* body force = g_k, not rho_k g_k           */
    ORC_INLET = 256,           /* Zou-He velocity inlet at x = 0 (Sec. 3.3) */
    ORC_OUTFLOW = 512,         /* zero-gradient outflow at x = nx - 1       */
    /* Reading exploration (CPU only, no device counterpart): S(x) of Eq. 9
     * with the D2Q9 weights w_i over the eight links, the literal "w_i" of
     * the printed equation, instead of the E8 stencil. */
    ORC_ADH_D2Q9 = 4096
};

typedef struct oracle_ctx oracle_ctx;

int  oracle_create(oracle_ctx **out, int nx, int ny, unsigned flags);
void oracle_destroy(oracle_ctx *c);
const char *oracle_last_error(const oracle_ctx *c);

int oracle_set_geometry(oracle_ctx *c, const uint8_t *solid);
/* G_w2 = G_c, G_w1 = G_c + 2 G_ads, delta = 0.8 */
int oracle_set_params(oracle_ctx *c, double G_c, double G_ads, double tau);
/* paper-native adhesion parameters of Eq. 9-12 */
int oracle_set_adhesion(oracle_ctx *c, double G_w1, double G_w2, double delta);
int oracle_set_body_accel(oracle_ctx *c, double g1x, double g1y, double g2x, double g2y);
/* Open and moving boundaries (Sec. 3.1 sliding walls, Sec. 3.3 inlet and
 * outflow).  Solid nodes (and positions outside a non-periodic y edge) in
 * rows y < ny/2 move with (ubx, uby), the others with (utx, uty); a
 * bounce-back link from a moving wall gains 6 w_i rho*_k (e_i . u_w)
 * (Ladd), rho*_k being the node's own post-collision density.  The inlet
 * velocity of row y is (ux[y], uy[y]) (arrays of ny, copied). */
int oracle_set_wall_velocity(oracle_ctx *c, double ubx, double uby, double utx, double uty);
int oracle_set_inlet_velocity(oracle_ctx *c, const double *ux, const double *uy);
/* f_i = w_i rho_k (u = 0) on fluid nodes */
int oracle_init_fields(oracle_ctx *c, const double *rho1, const double *rho2);
int oracle_set_populations(oracle_ctx *c, const double *f);
int oracle_get_populations(const oracle_ctx *c, double *f);
int oracle_step(oracle_ctx *c, int n);
long oracle_time(const oracle_ctx *c);
/* rho_k and u^eq at the current time; solid nodes -> 0; NULL skips */
int oracle_get_fields(oracle_ctx *c, double *rho1, double *rho2, double *ux, double *uy);
/* M1, M2, Px, Py, max|u|, min rho1, max rho1, count of non-finite nodes */
int oracle_reduce(oracle_ctx *c, double out[8]);
/* Contact angle (the paper gives no measuring method): points where
 * rho^e = (rho1 - rho2)/(rho1 + rho2) changes sign along an x or y link of
 * two fluid nodes, placed by linear interpolation, kept when the link joins
 * the largest rho^e > 0 region to the largest rho^e <= 0 region (4-connected,
 * not across periodic seams) and the point lies at least 3 lattice units
 * from the wall; circle fit; angle measured through component 1.
 * wall_kind 0: flat wall below the drop, wall[0] = wall line y_w.
 * wall_kind 1: cylinder, wall[0..1] = centre, wall[2] = surface radius. */
int oracle_contact_angle(oracle_ctx *c, int wall_kind, const double wall[3], double *theta_deg);
int oracle_interface_points(oracle_ctx *c, int wall_kind, const double wall[3],
                            double *px, double *py, int cap, int *n);
/* link[N]: bit i-1 set when the pull source x - e_i is unavailable (fluid
 * nodes only, 0 on solid).  nw_list: fluid nodes with an unavailable E8
 * position, ascending.  nw_src[24 per entry]: node whose psi feeds stencil
 * position n after the unavailable-position rules, or -1 for "zero". */
int oracle_get_tables(const oracle_ctx *c, uint8_t *link, int32_t *nw_list,
                      int32_t *nw_src, int *n_nw);

/* OpenMP threads the row loops use (1 without OpenMP). */
int oracle_threads(void);
int oracle_set_threads(int n);

/* ---- pieces exposed for unit pins ---- */
void oracle_d2q9(int ex[9], int ey[9], double w[9], int opp[9]);
void oracle_e8(int ex[24], int ey[24], double W[24], int copy_from[24]);
double oracle_local_G(double rho_e, double G_w1, double G_w2, double delta);
void oracle_equilibrium(double rho, const double u[2], double feq[9]);
void oracle_forcing(const double F[2], const double u[2], double Fi[9]);
/* out: Fcoh1(x,y) Fcoh2(x,y) Fads1 Fads2 Fbody1 Fbody2 (12 doubles) */
int oracle_node_forces(oracle_ctx *c, int x, int y, double out[12]);
int oracle_adhesion_vector(const oracle_ctx *c, int x, int y, double S[2]);
int oracle_circle_fit(const double *px, const double *py, int n, double abr[3]);

#ifdef __cplusplus
}
#endif
#endif
