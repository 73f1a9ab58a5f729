/*
 * FP64 CPU oracle -- see lbm_oracle.h for scope and conventions.
 *
 * TEST INFRASTRUCTURE ONLY: plain, serial-order FP64 code written from the
 * paper (arXiv 2505.22256).  No blocking, fusion or reordering beyond what
 * the equations state.  OpenMP splits node loops by rows only; no reduction
 * happens inside a parallel region, so results do not depend on the thread
 * count.
 *
 * One time step (Sec. 2.1-2.4):
 *   1. rho_k = sum_i f_i^k, j_k = sum_i f_i^k e_i             (Eq. 3-4)
 *   2. psi_k = rho_k (Sec. 2.2, text after Eq. 8)
 *   3. cohesion on the E8 stencil with second-layer copying     (Eq. 8, Sec. 2.4, Table 1)
 *   4. adhesion with the local parameter G(x)                   (Eq. 9-11)
 *   5. body force, u^eq (Guo half-force shift)                  (Eq. 5, Sec. 3.1)
 *   6. equilibrium, forcing term, BGK collision                 (Eq. 1, 2, 6, 7)
 *   7. streaming with halfway bounce-back at unavailable links  (Eq. 1 LHS, Sec. 3.2, 3.5),
 *      optionally from moving walls (Sec. 3.1), with a Zou-He velocity
 *      inlet and a zero-gradient outflow (Sec. 3.3)
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Lattice constants                                                   */
/* ------------------------------------------------------------------ */

/* D2Q9 velocity set: rest, four axis links, four diagonals (Sec. 2.1). */
static const int QX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int QY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double QW[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int QOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0; /* lattice sound speed squared */

/* E8 stencil (Sec. 2.4, Fig. 2a): 24 positions in two layers.
 * 1-8 are the D2Q9 links, 9-16 are the D2Q9 links doubled, 17-24 are the
 * knight moves.  Positions n and n+2 (within each group of four) are
 * opposite, so the stencil can be summed over 12 opposite pairs. */
static const int SX[24] = {1, 0, -1, 0,  1, -1, -1, 1,
                           2, 0, -2, 0,  2, -2, -2, 2,
                           2, -1, -2, 1, 1, -2, -1, 2};
static const int SY[24] = {0, 1, 0, -1,  1, 1, -1, -1,
                           0, 2, 0, -2,  2, 2, -2, -2,
                           1, 2, -1, -2, 2, 1, -2, -1};

/* Eighth-order isotropic weights as a function of |e|^2
 * (normalised so that sum W e_x^2 = 1). */
static double e8_weight(int e2)
{
    switch (e2) {
    case 1: return 4.0 / 21.0;
    case 2: return 4.0 / 45.0;
    case 4: return 1.0 / 60.0;
    case 5: return 2.0 / 315.0;
    case 8: return 1.0 / 5040.0;
    default: return 0.0;
    }
}

/* Table 1: second-layer position n (1-based) takes the first-layer position
 * n-8 (n = 9..16), n-12 (n = 17..20) or n-16 (n = 21..24).  Returns the
 * 0-based source, or -1 for first-layer positions. */
static int table1_source(int n0)
{
    int n = n0 + 1;
    if (n <= 8) return -1;
    if (n <= 16) return n - 8 - 1;
    if (n <= 20) return n - 12 - 1;
    return n - 16 - 1;
}

/* ------------------------------------------------------------------ */
/* Context                                                             */
/* ------------------------------------------------------------------ */

struct oracle_ctx {
    int nx, ny, n;
    unsigned flags;
    uint8_t *solid;
    double *f;     /* [2][9][n] pre-collision populations at time t */
    double *fpost; /* [2][9][n] post-collision populations           */
    double *rho;   /* [2][n] */
    double Gc, Gw1, Gw2, delta, tau;
    double acc[2][2];
    double uw[2][2];  /* wall velocity: [0] rows y < ny/2, [1] the others */
    int moving;       /* any wall velocity nonzero */
    double *inlet;    /* [2][ny] inlet velocity per row */
    int have_geom, have_params, have_fields;
    long t;
    char err[256];
};

static int fail(oracle_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

#define F_AT(c, k, i, node) ((c)->f[((size_t)(k) * 9 + (i)) * (size_t)(c)->n + (size_t)(node)])
#define FP_AT(c, k, i, node) ((c)->fpost[((size_t)(k) * 9 + (i)) * (size_t)(c)->n + (size_t)(node)])
#define RHO_AT(c, k, node) ((c)->rho[(size_t)(k) * (size_t)(c)->n + (size_t)(node)])

/* Node id of lattice position (x, y) after periodic wrapping, or -1 when the
 * position lies outside the domain along a non-periodic axis. */
static int node_at(const oracle_ctx *c, int x, int y)
{
    if (x < 0 || x >= c->nx) {
        if (!(c->flags & ORC_PERIODIC_X)) return -1;
        x %= c->nx;
        if (x < 0) x += c->nx;
    }
    if (y < 0 || y >= c->ny) {
        if (!(c->flags & ORC_PERIODIC_Y)) return -1;
        y %= c->ny;
        if (y < 0) y += c->ny;
    }
    return y * c->nx + x;
}

/* A position is available when it is inside the domain and fluid. */
static int available(const oracle_ctx *c, int x, int y)
{
    int id = node_at(c, x, y);
    return id >= 0 && !c->solid[id];
}

/* A position beyond an open x edge (the inlet left of x = 0, the outflow
 * right of x = nx - 1): its ghost is the node of the same row clamped into
 * the domain.  Returns the ghost's node id, -1 when the ghost is solid or
 * outside, or -2 when the position does not lie beyond an open edge. */
static int open_ghost(const oracle_ctx *c, int x, int y)
{
    int cx;
    if (x < 0 && (c->flags & ORC_INLET)) cx = 0;
    else if (x >= c->nx && (c->flags & ORC_OUTFLOW)) cx = c->nx - 1;
    else return -2;
    return available(c, cx, y) ? node_at(c, cx, y) : -1;
}

/* s(P) of Eq. 9: 1 on a solid position or one outside a closed edge; a
 * position beyond an open edge takes its ghost's value. */
static double solid_switch(const oracle_ctx *c, int x, int y)
{
    if (available(c, x, y)) return 0.0;
    int g = open_ghost(c, x, y);
    if (g == -2) return 1.0;
    return g >= 0 ? 0.0 : 1.0;
}

int oracle_create(oracle_ctx **out, int nx, int ny, unsigned flags)
{
    if (!out) return ORC_EINVAL;
    *out = NULL;
    if (nx < 5 || ny < 5) return ORC_EINVAL;
    if (flags & ~(127u | ORC_INLET | ORC_OUTFLOW | ORC_ADH_D2Q9)) return ORC_EINVAL;
    if ((flags & (ORC_INLET | ORC_OUTFLOW)) && (flags & ORC_PERIODIC_X)) return ORC_EINVAL;
    oracle_ctx *c = (oracle_ctx *)calloc(1, sizeof *c);
    if (!c) return ORC_ENOMEM;
    c->nx = nx;
    c->ny = ny;
    c->n = nx * ny;
    c->flags = flags;
    c->solid = (uint8_t *)calloc((size_t)c->n, 1);
    c->f = (double *)calloc((size_t)c->n * 18, sizeof(double));
    c->fpost = (double *)calloc((size_t)c->n * 18, sizeof(double));
    c->rho = (double *)calloc((size_t)c->n * 2, sizeof(double));
    c->inlet = (double *)calloc((size_t)ny * 2, sizeof(double));
    if (!c->solid || !c->f || !c->fpost || !c->rho || !c->inlet) {
        oracle_destroy(c);
        return ORC_ENOMEM;
    }
    c->delta = 0.8;
    *out = c;
    return ORC_OK;
}

void oracle_destroy(oracle_ctx *c)
{
    if (!c) return;
    free(c->solid);
    free(c->f);
    free(c->fpost);
    free(c->rho);
    free(c->inlet);
    free(c);
}

const char *oracle_last_error(const oracle_ctx *c) { return c ? c->err : "null context"; }

int oracle_set_geometry(oracle_ctx *c, const uint8_t *solid)
{
    if (!c || !solid) return ORC_EINVAL;
    for (int i = 0; i < c->n; ++i) c->solid[i] = solid[i] ? 1 : 0;
    c->have_geom = 1;
    c->have_fields = 0;
    return ORC_OK;
}

static int check_adhesion(oracle_ctx *c, double Gw1, double Gw2, double delta)
{
    if (!(delta > 0.0)) return fail(c, ORC_EINVAL, "delta must be > 0");
    if (!(c->flags & ORC_SCHEME_ORIGINAL) && Gw1 + Gw2 == 0.0)
        return fail(c, ORC_EINVAL, "improved scheme needs G_w1 + G_w2 != 0");
    if (!isfinite(Gw1) || !isfinite(Gw2)) return fail(c, ORC_EINVAL, "non-finite adhesion");
    return ORC_OK;
}

int oracle_set_params(oracle_ctx *c, double G_c, double G_ads, double tau)
{
    if (!c) return ORC_EINVAL;
    if (!(tau > 0.5) || !isfinite(tau)) return fail(c, ORC_EINVAL, "tau must be > 0.5");
    if (!isfinite(G_c) || !isfinite(G_ads)) return fail(c, ORC_EINVAL, "non-finite parameter");
    double Gw2 = G_c, Gw1 = G_c + 2.0 * G_ads;
    if (!(c->flags & ORC_SCHEME_ORIGINAL)) {
        /* lambda = G_w1 / G_w2 must stay positive */
        if (!(Gw2 != 0.0 && Gw1 / Gw2 > 0.0))
            return fail(c, ORC_EINVAL, "lambda = 1 + 2 G_ads / G_c must be > 0");
    }
    int rc = check_adhesion(c, Gw1, Gw2, 0.8);
    if (rc) return rc;
    c->Gc = G_c;
    c->Gw1 = Gw1;
    c->Gw2 = Gw2;
    c->delta = 0.8;
    c->tau = tau;
    c->have_params = 1;
    return ORC_OK;
}

int oracle_set_adhesion(oracle_ctx *c, double G_w1, double G_w2, double delta)
{
    if (!c) return ORC_EINVAL;
    if (!c->have_params) return fail(c, ORC_ESTATE, "set_params first");
    int rc = check_adhesion(c, G_w1, G_w2, delta);
    if (rc) return rc;
    c->Gw1 = G_w1;
    c->Gw2 = G_w2;
    c->delta = delta;
    return ORC_OK;
}

int oracle_set_body_accel(oracle_ctx *c, double g1x, double g1y, double g2x, double g2y)
{
    if (!c) return ORC_EINVAL;
    c->acc[0][0] = g1x;
    c->acc[0][1] = g1y;
    c->acc[1][0] = g2x;
    c->acc[1][1] = g2y;
    return ORC_OK;
}

int oracle_set_wall_velocity(oracle_ctx *c, double ubx, double uby, double utx, double uty)
{
    if (!c) return ORC_EINVAL;
    if (!isfinite(ubx) || !isfinite(uby) || !isfinite(utx) || !isfinite(uty))
        return fail(c, ORC_EINVAL, "non-finite wall velocity");
    c->uw[0][0] = ubx;
    c->uw[0][1] = uby;
    c->uw[1][0] = utx;
    c->uw[1][1] = uty;
    c->moving = ubx != 0.0 || uby != 0.0 || utx != 0.0 || uty != 0.0;
    return ORC_OK;
}

int oracle_set_inlet_velocity(oracle_ctx *c, const double *ux, const double *uy)
{
    if (!c || !ux || !uy) return ORC_EINVAL;
    for (int y = 0; y < c->ny; ++y) {
        if (!isfinite(ux[y]) || !isfinite(uy[y]) || !(ux[y] < 1.0))
            return fail(c, ORC_EINVAL, "inlet velocity must be finite with u_x < 1");
        c->inlet[y] = ux[y];
        c->inlet[c->ny + y] = uy[y];
    }
    return ORC_OK;
}

int oracle_init_fields(oracle_ctx *c, const double *rho1, const double *rho2)
{
    if (!c || !rho1 || !rho2) return ORC_EINVAL;
    if (!c->have_geom) return fail(c, ORC_ESTATE, "set_geometry first");
    for (int id = 0; id < c->n; ++id) {
        double r[2] = {rho1[id], rho2[id]};
        for (int k = 0; k < 2; ++k) {
            if (!c->solid[id] && !isfinite(r[k])) return fail(c, ORC_EINVAL, "non-finite density");
            for (int i = 0; i < 9; ++i) F_AT(c, k, i, id) = c->solid[id] ? 0.0 : QW[i] * r[k];
        }
    }
    c->have_fields = 1;
    c->t = 0;
    return ORC_OK;
}

int oracle_set_populations(oracle_ctx *c, const double *f)
{
    if (!c || !f) return ORC_EINVAL;
    if (!c->have_geom) return fail(c, ORC_ESTATE, "set_geometry first");
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i)
            for (int id = 0; id < c->n; ++id) {
                double v = f[((size_t)k * 9 + i) * (size_t)c->n + id];
                if (!c->solid[id] && !isfinite(v)) return fail(c, ORC_EINVAL, "non-finite population");
                F_AT(c, k, i, id) = c->solid[id] ? 0.0 : v;
            }
    c->have_fields = 1;
    c->t = 0;
    return ORC_OK;
}

int oracle_get_populations(const oracle_ctx *c, double *f)
{
    if (!c || !f) return ORC_EINVAL;
    memcpy(f, c->f, (size_t)c->n * 18 * sizeof(double));
    return ORC_OK;
}

long oracle_time(const oracle_ctx *c) { return c ? c->t : -1; }

/* ------------------------------------------------------------------ */
/* Pieces of the method                                                */
/* ------------------------------------------------------------------ */

/* Eq. 6: second-order equilibrium with the common velocity u^eq. */
void oracle_equilibrium(double rho, const double u[2], double feq[9])
{
    double uu = u[0] * u[0] + u[1] * u[1];
    for (int i = 0; i < 9; ++i) {
        double eu = QX[i] * u[0] + QY[i] * u[1];
        feq[i] = QW[i] * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Eq. 7: Guo forcing term, with the tensor contraction written out:
 * F_i = w_i [ e_i.F / cs^2 + (u F + F u) : (e_i e_i - cs^2 I) / (2 cs^4) ]. */
void oracle_forcing(const double F[2], const double u[2], double Fi[9])
{
    double A[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) A[a][b] = u[a] * F[b] + F[a] * u[b];
    for (int i = 0; i < 9; ++i) {
        double e[2] = {(double)QX[i], (double)QY[i]};
        double eF = e[0] * F[0] + e[1] * F[1];
        double contr = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double Bab = e[a] * e[b] - (a == b ? CS2 : 0.0);
                contr += A[a][b] * Bab;
            }
        Fi[i] = QW[i] * (eF / CS2 + contr / (2.0 * CS2 * CS2));
    }
}

/* Eq. 11: local adhesion parameter of component 1 as a function of the
 * effective density (Eq. 10).  Coefficients as printed below Eq. 11. */
double oracle_local_G(double rho_e, double Gw1, double Gw2, double delta)
{
    double s1 = 2.0 * Gw1 * Gw2 / (Gw1 + Gw2);
    double t1 = s1;
    double s2 = 2.0 * (Gw1 - s1) / delta;
    double s3 = -s2 / (2.0 * delta);
    double t2 = 2.0 * (t1 - Gw2) / delta;
    double t3 = t2 / (2.0 * delta);
    if (rho_e > delta) return Gw1;
    if (rho_e > 0.0) return s1 + s2 * rho_e + s3 * rho_e * rho_e;
    if (rho_e > -delta) return t1 + t2 * rho_e + t3 * rho_e * rho_e;
    return Gw2;
}

void oracle_d2q9(int ex[9], int ey[9], double w[9], int opp[9])
{
    for (int i = 0; i < 9; ++i) {
        ex[i] = QX[i];
        ey[i] = QY[i];
        w[i] = QW[i];
        opp[i] = QOPP[i];
    }
}

void oracle_e8(int ex[24], int ey[24], double W[24], int copy_from[24])
{
    for (int n = 0; n < 24; ++n) {
        ex[n] = SX[n];
        ey[n] = SY[n];
        W[n] = e8_weight(SX[n] * SX[n] + SY[n] * SY[n]);
        copy_from[n] = table1_source(n);
    }
}

/* Stencil position n as seen from node (x, y): the node id that feeds it
 * after the unavailable-position rules, or -1 for the value zero.
 *   first layer : available ? neighbour : beyond an open edge with a fluid
 *                 ghost ? ghost : (WALLPSI_SELF ? self : zero)
 *   second layer: available ? neighbour : (COPY_OFF ? zero : value of m(n))
 * (Sec. 2.4 and Table 1 for the copy, which the paper applies at velocity
 * boundaries as at walls; Eq. 8-9 for what a wall contributes.) */
static void resolve_sources(const oracle_ctx *c, int x, int y, int src[24])
{
    int self = y * c->nx + x;
    for (int n = 0; n < 24; ++n) {
        int px = x + SX[n], py = y + SY[n];
        if (available(c, px, py)) {
            src[n] = node_at(c, px, py);
            continue;
        }
        int m = table1_source(n);
        if (m < 0) {
            int g = open_ghost(c, px, py);
            if (g >= 0) src[n] = g;
            else src[n] = (c->flags & ORC_WALLPSI_SELF) ? self : -1;
        } else {
            src[n] = (c->flags & ORC_E8_COPY_OFF) ? -1 : src[m];
        }
    }
}

/* S(x) = sum_n W_n s(x + e_n) e_n with s = 1 on unavailable positions
 * (Eq. 9, summed over the E8 stencil, by opposite pairs). */
static void adhesion_vector(const oracle_ctx *c, int x, int y, double S[2])
{
    S[0] = 0.0;
    S[1] = 0.0;
    if (c->flags & ORC_ADH_D2Q9) {
        /* the alternative reading: D2Q9 weights over the eight links */
        for (int i = 1; i < 9; ++i) {
            double s = solid_switch(c, x + QX[i], y + QY[i]);
            S[0] += QW[i] * s * QX[i];
            S[1] += QW[i] * s * QY[i];
        }
        return;
    }
    for (int g = 0; g < 6; ++g)
        for (int h = 0; h < 2; ++h) {
            int n = 4 * g + h, o = n + 2; /* o is the position opposite n */
            double sn = solid_switch(c, x + SX[n], y + SY[n]);
            double so = solid_switch(c, x + SX[o], y + SY[o]);
            double W = e8_weight(SX[n] * SX[n] + SY[n] * SY[n]);
            S[0] += W * SX[n] * (sn - so);
            S[1] += W * SY[n] * (sn - so);
        }
}

int oracle_adhesion_vector(const oracle_ctx *c, int x, int y, double S[2])
{
    if (!c || x < 0 || y < 0 || x >= c->nx || y >= c->ny) return ORC_EINVAL;
    adhesion_vector(c, x, y, S);
    return ORC_OK;
}

static void compute_density(oracle_ctx *c)
{
    int n = c->n;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            int id = y * c->nx + x;
            for (int k = 0; k < 2; ++k) {
                double r = 0.0;
                if (!c->solid[id])
                    for (int i = 0; i < 9; ++i) r += F_AT(c, k, i, id);
                RHO_AT(c, k, id) = r;
            }
        }
    (void)n;
}

/* Forces on both components at fluid node (x, y) from the densities in
 * c->rho (psi = rho).  parts: [coh1 coh2 ads1 ads2 body1 body2] x (x, y). */
static void node_forces(const oracle_ctx *c, int x, int y, double parts[6][2])
{
    int id = y * c->nx + x;
    double rho[2] = {RHO_AT(c, 0, id), RHO_AT(c, 1, id)};

    /* Psi_n^k for the 24 stencil positions */
    int src[24];
    resolve_sources(c, x, y, src);
    double Psi[2][24];
    for (int k = 0; k < 2; ++k)
        for (int n = 0; n < 24; ++n) Psi[k][n] = src[n] < 0 ? 0.0 : RHO_AT(c, k, src[n]);

    /* Eq. 8: F_k = -G_c psi_k(x) sum_n W_n Psi_n^{other} e_n, summed by
     * opposite pairs (n, n+2) in each group of four positions. */
    for (int k = 0; k < 2; ++k) {
        int other = 1 - k;
        double sx = 0.0, sy = 0.0;
        for (int g = 0; g < 6; ++g)
            for (int h = 0; h < 2; ++h) {
                int n = 4 * g + h, o = n + 2;
                double W = e8_weight(SX[n] * SX[n] + SY[n] * SY[n]);
                double d = Psi[other][n] - Psi[other][o];
                sx += W * SX[n] * d;
                sy += W * SY[n] * d;
            }
        parts[k][0] = -c->Gc * rho[k] * sx;
        parts[k][1] = -c->Gc * rho[k] * sy;
    }

    /* Eq. 9-11: adhesion with G_w1 replaced by the local G(x) of Eq. 11 for
     * component 1; component 2 keeps the constant G_w2. */
    double S[2];
    adhesion_vector(c, x, y, S);
    double G1 = c->Gw1;
    if (!(c->flags & ORC_SCHEME_ORIGINAL)) {
        double rho_e = (rho[0] - rho[1]) / (rho[0] + rho[1]); /* Eq. 10 */
        G1 = oracle_local_G(rho_e, c->Gw1, c->Gw2, c->delta);
    }
    double G[2] = {G1, c->Gw2};
    for (int k = 0; k < 2; ++k) {
        parts[2 + k][0] = -G[k] * rho[k] * S[0];
        parts[2 + k][1] = -G[k] * rho[k] * S[1];
    }

    /* body force: acceleration g_k (or a constant force density) */
    for (int k = 0; k < 2; ++k) {
        double scale = (c->flags & ORC_FORCE_DENSITY) ? 1.0 : rho[k];
        parts[4 + k][0] = scale * c->acc[k][0];
        parts[4 + k][1] = scale * c->acc[k][1];
    }
}

/* Moments, total forces and u^eq at fluid node id (Eq. 3-5). */
static void node_macro(const oracle_ctx *c, int x, int y, double rho[2], double j[2][2],
                       double F[2][2], double u[2])
{
    int id = y * c->nx + x;
    for (int k = 0; k < 2; ++k) {
        rho[k] = RHO_AT(c, k, id);
        j[k][0] = 0.0;
        j[k][1] = 0.0;
        for (int i = 0; i < 9; ++i) {
            j[k][0] += F_AT(c, k, i, id) * QX[i];
            j[k][1] += F_AT(c, k, i, id) * QY[i];
        }
    }
    double parts[6][2];
    node_forces(c, x, y, parts);
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 2; ++a) F[k][a] = parts[k][a] + parts[2 + k][a] + parts[4 + k][a];
    /* Eq. 5; with Guo forcing the force enters the velocity with weight 1/2 */
    double half = (c->flags & ORC_VEL_LITERAL) ? 0.0 : 0.5;
    for (int a = 0; a < 2; ++a)
        u[a] = ((j[0][a] + half * F[0][a]) + (j[1][a] + half * F[1][a])) / (rho[0] + rho[1]);
}

int oracle_node_forces(oracle_ctx *c, int x, int y, double out[12])
{
    if (!c || x < 0 || y < 0 || x >= c->nx || y >= c->ny) return ORC_EINVAL;
    if (!c->have_fields || !c->have_params) return fail(c, ORC_ESTATE, "fields/params missing");
    compute_density(c);
    double parts[6][2];
    node_forces(c, x, y, parts);
    for (int p = 0; p < 6; ++p) {
        out[2 * p] = parts[p][0];
        out[2 * p + 1] = parts[p][1];
    }
    return ORC_OK;
}

static int ready(oracle_ctx *c)
{
    if (!c) return ORC_EINVAL;
    if (!c->have_geom) return fail(c, ORC_ESTATE, "set_geometry first");
    if (!c->have_params) return fail(c, ORC_ESTATE, "set_params first");
    if (!c->have_fields) return fail(c, ORC_ESTATE, "init_fields first");
    return ORC_OK;
}

/* Streaming into fluid node (x, y), component k.  The source is x - e_i,
 * except right of the outflow, where it is (x, y - e_iy): the node whose
 * population the upstream neighbour at x - 1 receives (zero normal
 * gradient).  Then
 *   f_i(x, t+1) = f*_i(source, t) when the source is available;
 *   a source left of the inlet: Zou-He unknown (below);
 *   otherwise halfway bounce-back f*_opp(i)(x, t), plus 6 w_i rho*_k
 *     (e_i . u_w) when the wall at the source moves (Ladd), rho*_k being
 *     the node's own post-collision density sum_j f*_j(x, t).
 * Zou-He at the inlet (west edge, velocity (U, V) of the row): with the
 * known populations, rho = [f0 + f2 + f4 + 2 (f3 + f6 + f7)] / (1 - U),
 * f1 = f3 + 2/3 rho U, f5 = f7 - (f2 - f4)/2 + rho U/6 + rho V/2,
 * f8 = f6 + (f2 - f4)/2 + rho U/6 - rho V/2. */
static void stream_node(oracle_ctx *c, int k, int x, int y)
{
    int id = y * c->nx + x;
    double f[9];
    int unknown = 0;
    double rpost = 0.0;
    if (c->moving)
        for (int j = 0; j < 9; ++j) rpost += FP_AT(c, k, j, id);
    for (int i = 0; i < 9; ++i) {
        int sx = x - QX[i], sy = y - QY[i];
        if (sx >= c->nx && (c->flags & ORC_OUTFLOW)) sx = x;
        if (available(c, sx, sy)) {
            f[i] = FP_AT(c, k, i, node_at(c, sx, sy));
        } else if (sx < 0 && (c->flags & ORC_INLET)) {
            f[i] = 0.0;
            unknown = 1;
        } else {
            f[i] = FP_AT(c, k, QOPP[i], id);
            if (c->moving) {
                const double *u = c->uw[sy < c->ny / 2 ? 0 : 1];
                f[i] += 6.0 * QW[i] * rpost * (QX[i] * u[0] + QY[i] * u[1]);
            }
        }
    }
    if (unknown) {
        double U = c->inlet[y], V = c->inlet[c->ny + y];
        double rho = (((f[0] + f[2]) + f[4]) + 2.0 * ((f[3] + f[6]) + f[7])) / (1.0 - U);
        f[1] = f[3] + (2.0 / 3.0) * rho * U;
        f[5] = ((f[7] - 0.5 * (f[2] - f[4])) + (1.0 / 6.0) * rho * U) + 0.5 * rho * V;
        f[8] = ((f[6] + 0.5 * (f[2] - f[4])) + (1.0 / 6.0) * rho * U) - 0.5 * rho * V;
    }
    for (int i = 0; i < 9; ++i) F_AT(c, k, i, id) = f[i];
}

int oracle_step(oracle_ctx *c, int nsteps)
{
    int rc = ready(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(c, ORC_EINVAL, "negative step count");
    for (int s = 0; s < nsteps; ++s) {
        compute_density(c);
        /* collision (Eq. 1-2, 6-7) */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                int id = y * c->nx + x;
                if (c->solid[id]) continue;
                double rho[2], j[2][2], F[2][2], u[2];
                node_macro(c, x, y, rho, j, F, u);
                for (int k = 0; k < 2; ++k) {
                    double feq[9], Fi[9];
                    oracle_equilibrium(rho[k], u, feq);
                    oracle_forcing(F[k], u, Fi);
                    for (int i = 0; i < 9; ++i) {
                        double fi = F_AT(c, k, i, id);
                        FP_AT(c, k, i, id) =
                            fi + (feq[i] - fi) / c->tau + (1.0 - 1.0 / (2.0 * c->tau)) * Fi[i];
                    }
                }
            }
        /* streaming */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                int id = y * c->nx + x;
                if (c->solid[id]) continue;
                for (int k = 0; k < 2; ++k) stream_node(c, k, x, y);
            }
        c->t += 1;
    }
    return ORC_OK;
}

int oracle_get_fields(oracle_ctx *c, double *rho1, double *rho2, double *ux, double *uy)
{
    int rc = ready(c);
    if (rc) return rc;
    compute_density(c);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            int id = y * c->nx + x;
            double rho[2] = {0.0, 0.0}, j[2][2], F[2][2], u[2] = {0.0, 0.0};
            if (!c->solid[id]) node_macro(c, x, y, rho, j, F, u);
            if (rho1) rho1[id] = rho[0];
            if (rho2) rho2[id] = rho[1];
            if (ux) ux[id] = u[0];
            if (uy) uy[id] = u[1];
        }
    return ORC_OK;
}

int oracle_reduce(oracle_ctx *c, double out[8])
{
    int rc = ready(c);
    if (rc) return rc;
    size_t n = (size_t)c->n;
    double *r1 = (double *)malloc(n * sizeof(double)), *r2 = (double *)malloc(n * sizeof(double));
    double *ux = (double *)malloc(n * sizeof(double)), *uy = (double *)malloc(n * sizeof(double));
    if (!r1 || !r2 || !ux || !uy) {
        free(r1); free(r2); free(ux); free(uy);
        return fail(c, ORC_ENOMEM, "out of memory");
    }
    oracle_get_fields(c, r1, r2, ux, uy);
    double M1 = 0, M2 = 0, Px = 0, Py = 0, umax = 0, rmin = INFINITY, rmax = -INFINITY, bad = 0;
    for (size_t id = 0; id < n; ++id) {
        if (c->solid[id]) continue;
        if (!isfinite(r1[id]) || !isfinite(r2[id]) || !isfinite(ux[id]) || !isfinite(uy[id])) {
            bad += 1.0;
            continue;
        }
        double rt = r1[id] + r2[id];
        M1 += r1[id];
        M2 += r2[id];
        Px += rt * ux[id];
        Py += rt * uy[id];
        double um = sqrt(ux[id] * ux[id] + uy[id] * uy[id]);
        if (um > umax) umax = um;
        if (r1[id] < rmin) rmin = r1[id];
        if (r1[id] > rmax) rmax = r1[id];
    }
    out[0] = M1; out[1] = M2; out[2] = Px; out[3] = Py;
    out[4] = umax; out[5] = rmin; out[6] = rmax; out[7] = bad;
    free(r1); free(r2); free(ux); free(uy);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Tables                                                              */
/* ------------------------------------------------------------------ */

int oracle_get_tables(const oracle_ctx *c, uint8_t *link, int32_t *nw_list, int32_t *nw_src,
                      int *n_nw)
{
    if (!c || !c->have_geom) return ORC_ESTATE;
    int count = 0;
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            int id = y * c->nx + x;
            if (link) {
                uint8_t b = 0;
                if (!c->solid[id])
                    for (int i = 1; i < 9; ++i)
                        if (!available(c, x - QX[i], y - QY[i])) b |= (uint8_t)(1u << (i - 1));
                link[id] = b;
            }
            if (c->solid[id]) continue;
            int near = 0;
            for (int n = 0; n < 24; ++n)
                if (!available(c, x + SX[n], y + SY[n])) near = 1;
            if (!near) continue;
            if (nw_list) {
                int src[24];
                resolve_sources(c, x, y, src);
                nw_list[count] = id;
                if (nw_src)
                    for (int n = 0; n < 24; ++n) nw_src[(size_t)count * 24 + n] = src[n];
            }
            ++count;
        }
    if (n_nw) *n_nw = count;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Contact angle: sign changes of rho^e along links, circle fit         */
/* ------------------------------------------------------------------ */

/* Solve the 3x3 system A x = b by Gaussian elimination with partial pivoting. */
static int solve3(double A[3][3], double b[3], double xout[3])
{
    double M[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) M[r][q] = A[r][q];
        M[r][3] = b[r];
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int q = 0; q < 4; ++q) {
                double tmp = M[col][q];
                M[col][q] = M[piv][q];
                M[piv][q] = tmp;
            }
        for (int r = col + 1; r < 3; ++r) {
            double fct = M[r][col] / M[col][col];
            for (int q = col; q < 4; ++q) M[r][q] -= fct * M[col][q];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = M[r][3];
        for (int q = r + 1; q < 3; ++q) s -= M[r][q] * xout[q];
        xout[r] = s / M[r][r];
    }
    return 0;
}

/* Algebraic (Kasa) circle fit on mean-centred points, refined by
 * Gauss-Newton on the geometric distances.  abr = centre x, centre y, radius. */
int oracle_circle_fit(const double *px, const double *py, int n, double abr[3])
{
    if (!px || !py || n < 3) return ORC_EINVAL;
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < n; ++i) {
        mx += px[i];
        my += py[i];
    }
    mx /= n;
    my /= n;
    double A[3][3] = {{0}}, b[3] = {0};
    for (int i = 0; i < n; ++i) {
        double u = px[i] - mx, v = py[i] - my, z = u * u + v * v;
        double row[3] = {u, v, 1.0};
        for (int r = 0; r < 3; ++r) {
            for (int q = 0; q < 3; ++q) A[r][q] += row[r] * row[q];
            b[r] -= row[r] * z;
        }
    }
    double DEF[3];
    if (solve3(A, b, DEF)) return ORC_EINVAL;
    double a = mx - DEF[0] / 2.0, bb = my - DEF[1] / 2.0;
    double r2 = DEF[0] * DEF[0] / 4.0 + DEF[1] * DEF[1] / 4.0 - DEF[2];
    if (!(r2 > 0.0)) return ORC_EINVAL;
    double r = sqrt(r2);
    for (int it = 0; it < 100; ++it) {
        double JJ[3][3] = {{0}}, Jr[3] = {0};
        for (int i = 0; i < n; ++i) {
            double dx = px[i] - a, dy = py[i] - bb;
            double d = sqrt(dx * dx + dy * dy);
            if (d == 0.0) continue;
            double J[3] = {-dx / d, -dy / d, -1.0};
            double res = d - r;
            for (int p = 0; p < 3; ++p) {
                for (int q = 0; q < 3; ++q) JJ[p][q] += J[p] * J[q];
                Jr[p] -= J[p] * res;
            }
        }
        double dlt[3];
        if (solve3(JJ, Jr, dlt)) break;
        a += dlt[0];
        bb += dlt[1];
        r += dlt[2];
        double step = fabs(dlt[0]) + fabs(dlt[1]) + fabs(dlt[2]);
        if (step <= 1e-13 * (1.0 + fabs(r))) break;
    }
    abr[0] = a;
    abr[1] = bb;
    abr[2] = r;
    return ORC_OK;
}

static double wall_distance(int kind, const double wall[3], double x, double y)
{
    if (kind == 0) return y - wall[0];
    double dx = x - wall[0], dy = y - wall[1];
    return sqrt(dx * dx + dy * dy) - wall[2];
}

/* Label the 4-connected regions (links along x and y, not across the
 * periodic seams, the same links the interface points are taken on) of
 * fluid nodes with rho^e > 0 and of fluid nodes with rho^e <= 0, by a
 * breadth-first flood fill in scan order.  best[1] / best[0] receive the
 * label of the largest region of each phase (ties: the region met first in
 * scan order, i.e. the one holding the smallest node index), -1 if none.
 * Only the interface between these two regions, the droplet and the fluid
 * around it, enters the fit: pockets trapped inside the droplet and
 * satellite droplets are left out. */
static int largest_regions(const oracle_ctx *c, const double *re, int *lab, int best[2])
{
    size_t n = (size_t)c->n;
    int *queue = (int *)malloc(n * sizeof(int));
    if (!queue) return -1;
    for (size_t id = 0; id < n; ++id) lab[id] = -1;
    int nlab = 0, best_size[2] = {0, 0};
    best[0] = best[1] = -1;
    for (int seed = 0; seed < c->n; ++seed) {
        if (c->solid[seed] || lab[seed] >= 0) continue;
        const int phase = re[seed] > 0.0;
        int head = 0, tail = 0;
        queue[tail++] = seed;
        lab[seed] = nlab;
        while (head < tail) {
            const int a = queue[head++];
            const int x = a % c->nx, y = a / c->nx;
            const int nb[4][2] = {{x + 1, y}, {x - 1, y}, {x, y + 1}, {x, y - 1}};
            for (int k = 0; k < 4; ++k) {
                const int xx = nb[k][0], yy = nb[k][1];
                if (xx < 0 || yy < 0 || xx >= c->nx || yy >= c->ny) continue;
                const int b = yy * c->nx + xx;
                if (c->solid[b] || lab[b] >= 0 || (re[b] > 0.0) != phase) continue;
                lab[b] = nlab;
                queue[tail++] = b;
            }
        }
        if (tail > best_size[phase]) {
            best_size[phase] = tail;
            best[phase] = nlab;
        }
        ++nlab;
    }
    free(queue);
    return 0;
}

int oracle_interface_points(oracle_ctx *c, int kind, const double wall[3], double *px, double *py,
                            int cap, int *n_out)
{
    int rc = ready(c);
    if (rc) return rc;
    if ((kind != 0 && kind != 1) || !wall) return fail(c, ORC_EINVAL, "bad wall description");
    size_t n = (size_t)c->n;
    double *r1 = (double *)malloc(n * sizeof(double)), *r2 = (double *)malloc(n * sizeof(double));
    double *re = (double *)malloc(n * sizeof(double));
    int *lab = (int *)malloc(n * sizeof(int));
    int best[2];
    if (!r1 || !r2 || !re || !lab) {
        free(r1); free(r2); free(re); free(lab);
        return fail(c, ORC_ENOMEM, "out of memory");
    }
    oracle_get_fields(c, r1, r2, NULL, NULL);
    for (size_t id = 0; id < n; ++id) re[id] = c->solid[id] ? 0.0 : (r1[id] - r2[id]) / (r1[id] + r2[id]);
    if (largest_regions(c, re, lab, best)) {
        free(r1); free(r2); free(re); free(lab);
        return fail(c, ORC_ENOMEM, "out of memory");
    }
    int count = 0;
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            int a = y * c->nx + x;
            if (c->solid[a]) continue;
            for (int dir = 0; dir < 2; ++dir) {
                int x2 = x + (dir == 0), y2 = y + (dir == 1);
                if (x2 >= c->nx || y2 >= c->ny) continue;
                int bnode = y2 * c->nx + x2;
                if (c->solid[bnode]) continue;
                if ((re[a] > 0.0) == (re[bnode] > 0.0)) continue;
                if (lab[a] != best[re[a] > 0.0] || lab[bnode] != best[re[bnode] > 0.0]) continue;
                double tpar = re[a] / (re[a] - re[bnode]);
                double qx = x + tpar * (x2 - x), qy = y + tpar * (y2 - y);
                if (wall_distance(kind, wall, qx, qy) < 3.0) continue;
                if (count < cap && px && py) {
                    px[count] = qx;
                    py[count] = qy;
                }
                ++count;
            }
        }
    free(r1); free(r2); free(re); free(lab);
    if (n_out) *n_out = count;
    return ORC_OK;
}

int oracle_contact_angle(oracle_ctx *c, int kind, const double wall[3], double *theta_deg)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!theta_deg) return fail(c, ORC_EINVAL, "null output");
    int npts = 0;
    rc = oracle_interface_points(c, kind, wall, NULL, NULL, 0, &npts);
    if (rc) return rc;
    if (npts < 3) return fail(c, ORC_EUNSTABLE, "fewer than 3 interface points");
    double *px = (double *)malloc((size_t)npts * sizeof(double));
    double *py = (double *)malloc((size_t)npts * sizeof(double));
    if (!px || !py) {
        free(px); free(py);
        return fail(c, ORC_ENOMEM, "out of memory");
    }
    oracle_interface_points(c, kind, wall, px, py, npts, &npts);
    double abr[3];
    rc = oracle_circle_fit(px, py, npts, abr);
    free(px);
    free(py);
    if (rc) return fail(c, ORC_EUNSTABLE, "circle fit failed");
    double cth;
    if (kind == 0) {
        cth = -(abr[1] - wall[0]) / abr[2];
    } else {
        double dx = abr[0] - wall[0], dy = abr[1] - wall[1];
        double d2 = dx * dx + dy * dy, Rs = wall[2], r = abr[2];
        cth = (Rs * Rs + r * r - d2) / (2.0 * Rs * r);
    }
    if (cth > 1.0) cth = 1.0;
    if (cth < -1.0) cth = -1.0;
    *theta_deg = acos(cth) * 180.0 / M_PI;
    return ORC_OK;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the row loops from now on (n >= 1); results do not depend
 * on it.  Returns the previous count. */
int oracle_set_threads(int n)
{
    int prev = oracle_threads();
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return prev;
}
