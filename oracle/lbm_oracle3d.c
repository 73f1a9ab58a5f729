/*
 * FP64 CPU oracle, three dimensions -- see lbm_oracle3d.h for the readings.
 *
 * TEST INFRASTRUCTURE ONLY: plain, serial-order FP64 code written from the
 * paper (arXiv 2505.22256).  OpenMP splits node loops by planes only; no sum
 * crosses a thread, so results do not depend on the thread count.
 *
 * One time step, as in two dimensions (Sec. 2.1-2.4):
 *   1. rho_k = sum_i f_i^k, j_k = sum_i f_i^k e_i            (Eq. 3-4)
 *   2. psi_k = rho_k
 *   3. cohesion on the 3-D stencil with the second-layer copy (Eq. 8, Sec. 2.4)
 *   4. adhesion with the local parameter G(x)                  (Eq. 9-11)
 *   5. body force, u^eq with Guo's half-force shift            (Eq. 5)
 *   6. equilibrium, forcing term, BGK collision                (Eq. 1, 2, 6, 7)
 *   7. streaming with halfway bounce-back at unavailable links (Sec. 3.5)
 */
#include "lbm_oracle3d.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define NS 92

/* D3Q19: rest, six axis links, twelve face diagonals; each odd direction
 * is followed by its opposite. */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double CS2 = 1.0 / 3.0;

static double d3q19_weight(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int d3q19_opp(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }

/* Eighth-order isotropic 3-D weights by |e|^2 (sum W e_x^2 = 1). */
static double e8_weight3(int e2)
{
    switch (e2) {
    case 1: return 4.0 / 45.0;
    case 2: return 1.0 / 21.0;
    case 3: return 2.0 / 105.0;
    case 4: return 5.0 / 504.0;
    case 5: return 1.0 / 315.0;
    case 6: return 1.0 / 630.0;
    case 8: return 1.0 / 5040.0;
    default: return 0.0;
    }
}

/* The stencil, built once: positions of the 5x5x5 neighbourhood with a
 * nonzero weight, ordered so that position 2m+1 is the opposite of 2m
 * (the first of each pair is the lexicographically positive one). */
static int SXs[NS], SYs[NS], SZs[NS], COPYs[NS];
static int stencil_ready = 0;

static int sgn(int v) { return (v > 0) - (v < 0); }

static void build_stencil(void)
{
    if (stencil_ready) return;
    int n = 0;
    for (int z = -2; z <= 2; ++z)
        for (int y = -2; y <= 2; ++y)
            for (int x = -2; x <= 2; ++x) {
                int e2 = x * x + y * y + z * z;
                if (e8_weight3(e2) == 0.0) continue;
                /* lexicographically positive: first nonzero of (z, y, x) > 0 */
                int lead = z != 0 ? z : (y != 0 ? y : x);
                if (lead < 0) continue;
                SXs[n] = x; SYs[n] = y; SZs[n] = z;
                SXs[n + 1] = -x; SYs[n + 1] = -y; SZs[n + 1] = -z;
                n += 2;
            }
    /* second layer -> index of the first-layer partner (sgn of each axis) */
    for (int a = 0; a < NS; ++a) {
        COPYs[a] = -1;
        if (abs(SXs[a]) < 2 && abs(SYs[a]) < 2 && abs(SZs[a]) < 2) continue;
        int px = sgn(SXs[a]), py = sgn(SYs[a]), pz = sgn(SZs[a]);
        for (int b = 0; b < NS; ++b)
            if (SXs[b] == px && SYs[b] == py && SZs[b] == pz) COPYs[a] = b;
    }
    stencil_ready = 1;
}

static double stencil_weight(int a) { return e8_weight3(SXs[a] * SXs[a] + SYs[a] * SYs[a] + SZs[a] * SZs[a]); }

struct oracle3d_ctx {
    int nx, ny, nz;
    long n;
    unsigned flags;
    uint8_t *solid;
    double *f, *fpost, *rho;
    double Gc, Gw1, Gw2, delta, tau;
    double acc[2][3];
    int have_geom, have_params, have_fields;
    long t;
    char err[256];
};

static int fail(oracle3d_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

#define F3(c, k, i, id) ((c)->f[((size_t)(k) * Q + (i)) * (size_t)(c)->n + (size_t)(id)])
#define FP3(c, k, i, id) ((c)->fpost[((size_t)(k) * Q + (i)) * (size_t)(c)->n + (size_t)(id)])
#define R3(c, k, id) ((c)->rho[(size_t)(k) * (size_t)(c)->n + (size_t)(id)])

/* Node id after periodic wrapping, or -1 outside a non-periodic axis. */
static long node3(const oracle3d_ctx *c, int x, int y, int z)
{
    if (x < 0 || x >= c->nx) {
        if (!(c->flags & OR3_PERIODIC_X)) return -1;
        x %= c->nx;
        if (x < 0) x += c->nx;
    }
    if (y < 0 || y >= c->ny) {
        if (!(c->flags & OR3_PERIODIC_Y)) return -1;
        y %= c->ny;
        if (y < 0) y += c->ny;
    }
    if (z < 0 || z >= c->nz) {
        if (!(c->flags & OR3_PERIODIC_Z)) return -1;
        z %= c->nz;
        if (z < 0) z += c->nz;
    }
    return ((long)z * c->ny + y) * c->nx + x;
}

static int avail3(const oracle3d_ctx *c, int x, int y, int z)
{
    long id = node3(c, x, y, z);
    return id >= 0 && !c->solid[id];
}

int oracle3d_create(oracle3d_ctx **out, int nx, int ny, int nz, unsigned flags)
{
    if (!out) return OR3_EINVAL;
    *out = NULL;
    if (nx < 5 || ny < 5 || nz < 5) return OR3_EINVAL;
    if (flags & ~(127u | OR3_PERIODIC_Z)) return OR3_EINVAL;
    build_stencil();
    oracle3d_ctx *c = (oracle3d_ctx *)calloc(1, sizeof *c);
    if (!c) return OR3_ENOMEM;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->n = (long)nx * ny * nz;
    c->flags = flags;
    c->solid = (uint8_t *)calloc((size_t)c->n, 1);
    c->f = (double *)calloc((size_t)c->n * 2 * Q, sizeof(double));
    c->fpost = (double *)calloc((size_t)c->n * 2 * Q, sizeof(double));
    c->rho = (double *)calloc((size_t)c->n * 2, sizeof(double));
    if (!c->solid || !c->f || !c->fpost || !c->rho) {
        oracle3d_destroy(c);
        return OR3_ENOMEM;
    }
    c->delta = 0.8;
    *out = c;
    return OR3_OK;
}

void oracle3d_destroy(oracle3d_ctx *c)
{
    if (!c) return;
    free(c->solid);
    free(c->f);
    free(c->fpost);
    free(c->rho);
    free(c);
}

const char *oracle3d_last_error(const oracle3d_ctx *c) { return c ? c->err : "null context"; }

int oracle3d_set_geometry(oracle3d_ctx *c, const uint8_t *solid)
{
    if (!c || !solid) return OR3_EINVAL;
    for (long i = 0; i < c->n; ++i) c->solid[i] = solid[i] ? 1 : 0;
    c->have_geom = 1;
    c->have_fields = 0;
    return OR3_OK;
}

static int check_adh(oracle3d_ctx *c, double Gw1, double Gw2, double delta)
{
    if (!(delta > 0.0)) return fail(c, OR3_EINVAL, "delta must be > 0");
    if (!isfinite(Gw1) || !isfinite(Gw2)) return fail(c, OR3_EINVAL, "non-finite adhesion");
    if (!(c->flags & OR3_SCHEME_ORIGINAL) && Gw1 + Gw2 == 0.0)
        return fail(c, OR3_EINVAL, "improved scheme needs G_w1 + G_w2 != 0");
    return OR3_OK;
}

int oracle3d_set_params(oracle3d_ctx *c, double G_c, double G_ads, double tau)
{
    if (!c) return OR3_EINVAL;
    if (!(tau > 0.5) || !isfinite(tau)) return fail(c, OR3_EINVAL, "tau must be > 0.5");
    if (!isfinite(G_c) || !isfinite(G_ads)) return fail(c, OR3_EINVAL, "non-finite parameter");
    double Gw2 = G_c, Gw1 = G_c + 2.0 * G_ads; /* lambda = G_w1 / G_w2 */
    if (!(c->flags & OR3_SCHEME_ORIGINAL) && !(Gw2 != 0.0 && Gw1 / Gw2 > 0.0))
        return fail(c, OR3_EINVAL, "lambda = 1 + 2 G_ads / G_c must be > 0");
    int rc = check_adh(c, Gw1, Gw2, 0.8);
    if (rc) return rc;
    c->Gc = G_c;
    c->Gw1 = Gw1;
    c->Gw2 = Gw2;
    c->delta = 0.8;
    c->tau = tau;
    c->have_params = 1;
    return OR3_OK;
}

int oracle3d_set_adhesion(oracle3d_ctx *c, double G_w1, double G_w2, double delta)
{
    if (!c) return OR3_EINVAL;
    if (!c->have_params) return fail(c, OR3_ESTATE, "set_params first");
    int rc = check_adh(c, G_w1, G_w2, delta);
    if (rc) return rc;
    c->Gw1 = G_w1;
    c->Gw2 = G_w2;
    c->delta = delta;
    return OR3_OK;
}

int oracle3d_set_body_accel(oracle3d_ctx *c, const double g[6])
{
    if (!c || !g) return OR3_EINVAL;
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 3; ++a) c->acc[k][a] = g[3 * k + a];
    return OR3_OK;
}

int oracle3d_init_fields(oracle3d_ctx *c, const double *rho1, const double *rho2)
{
    if (!c || !rho1 || !rho2) return OR3_EINVAL;
    if (!c->have_geom) return fail(c, OR3_ESTATE, "set_geometry first");
    for (long id = 0; id < c->n; ++id) {
        double r[2] = {rho1[id], rho2[id]};
        for (int k = 0; k < 2; ++k) {
            if (!c->solid[id] && !isfinite(r[k])) return fail(c, OR3_EINVAL, "non-finite density");
            for (int i = 0; i < Q; ++i) F3(c, k, i, id) = c->solid[id] ? 0.0 : d3q19_weight(i) * r[k];
        }
    }
    c->have_fields = 1;
    c->t = 0;
    return OR3_OK;
}

int oracle3d_set_populations(oracle3d_ctx *c, const double *f)
{
    if (!c || !f) return OR3_EINVAL;
    if (!c->have_geom) return fail(c, OR3_ESTATE, "set_geometry first");
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < Q; ++i)
            for (long id = 0; id < c->n; ++id) {
                double v = f[((size_t)k * Q + i) * (size_t)c->n + id];
                if (!c->solid[id] && !isfinite(v)) return fail(c, OR3_EINVAL, "non-finite population");
                F3(c, k, i, id) = c->solid[id] ? 0.0 : v;
            }
    c->have_fields = 1;
    c->t = 0;
    return OR3_OK;
}

int oracle3d_get_populations(const oracle3d_ctx *c, double *f)
{
    if (!c || !f) return OR3_EINVAL;
    memcpy(f, c->f, (size_t)c->n * 2 * Q * sizeof(double));
    return OR3_OK;
}

long oracle3d_time(const oracle3d_ctx *c) { return c ? c->t : -1; }

/* ------------------------------------------------------------------ */
/* Pieces of the method                                                */
/* ------------------------------------------------------------------ */

void oracle3d_d3q19(int ex[19], int ey[19], int ez[19], double w[19], int opp[19])
{
    for (int i = 0; i < Q; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        ez[i] = EZ[i];
        w[i] = d3q19_weight(i);
        opp[i] = d3q19_opp(i);
    }
}

int oracle3d_stencil(int ex[92], int ey[92], int ez[92], double W[92], int copy_from[92])
{
    build_stencil();
    for (int a = 0; a < NS; ++a) {
        ex[a] = SXs[a];
        ey[a] = SYs[a];
        ez[a] = SZs[a];
        W[a] = stencil_weight(a);
        copy_from[a] = COPYs[a];
    }
    return NS;
}

/* Eq. 6 with u^eq (three dimensions). */
void oracle3d_equilibrium(double rho, const double u[3], double feq[19])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        feq[i] = d3q19_weight(i) * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Eq. 7: F_i = w_i [ e_i.F / cs^2 + (u F + F u) : (e_i e_i - cs^2 I) / (2 cs^4) ]. */
void oracle3d_forcing(const double F[3], const double u[3], double Fi[19])
{
    double A[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = u[a] * F[b] + F[a] * u[b];
    for (int i = 0; i < Q; ++i) {
        double e[3] = {(double)EX[i], (double)EY[i], (double)EZ[i]};
        double eF = e[0] * F[0] + e[1] * F[1] + e[2] * F[2];
        double contr = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) contr += A[a][b] * (e[a] * e[b] - (a == b ? CS2 : 0.0));
        Fi[i] = d3q19_weight(i) * (eF / CS2 + contr / (2.0 * CS2 * CS2));
    }
}

/* Eq. 11 (same as in two dimensions). */
static double local_G3(double re, double Gw1, double Gw2, double delta)
{
    double s1 = 2.0 * Gw1 * Gw2 / (Gw1 + Gw2), t1 = s1;
    double s2 = 2.0 * (Gw1 - s1) / delta, s3 = -s2 / (2.0 * delta);
    double t2 = 2.0 * (t1 - Gw2) / delta, t3 = t2 / (2.0 * delta);
    if (re > delta) return Gw1;
    if (re > 0.0) return s1 + s2 * re + s3 * re * re;
    if (re > -delta) return t1 + t2 * re + t3 * re * re;
    return Gw2;
}

/* Stencil position a seen from (x, y, z): the node id that feeds it after
 * the unavailable-position rules, or -1 for zero (Sec. 2.4):
 *   first layer : available ? neighbour : (WALLPSI_SELF ? self : zero)
 *   second layer: available ? neighbour : (COPY_OFF ? zero : what the
 *                 first-layer partner resolved to). */
static void resolve3(const oracle3d_ctx *c, int x, int y, int z, long src[NS])
{
    long self = node3(c, x, y, z);
    /* first layer first, so that second-layer positions can copy */
    for (int pass = 0; pass < 2; ++pass)
        for (int a = 0; a < NS; ++a) {
            int second = COPYs[a] >= 0;
            if (second != pass) continue;
            int px = x + SXs[a], py = y + SYs[a], pz = z + SZs[a];
            if (avail3(c, px, py, pz)) {
                src[a] = node3(c, px, py, pz);
            } else if (!second) {
                src[a] = (c->flags & OR3_WALLPSI_SELF) ? self : -1;
            } else {
                src[a] = (c->flags & OR3_E8_COPY_OFF) ? -1 : src[COPYs[a]];
            }
        }
}

/* S(x) = sum_n W_n s(x + e_n) e_n, s = 1 on unavailable positions (Eq. 9),
 * by opposite pairs. */
static void adhesion3(const oracle3d_ctx *c, int x, int y, int z, double S[3])
{
    S[0] = S[1] = S[2] = 0.0;
    for (int a = 0; a < NS; a += 2) {
        double sa = avail3(c, x + SXs[a], y + SYs[a], z + SZs[a]) ? 0.0 : 1.0;
        double sb = avail3(c, x + SXs[a + 1], y + SYs[a + 1], z + SZs[a + 1]) ? 0.0 : 1.0;
        double W = stencil_weight(a);
        S[0] += W * SXs[a] * (sa - sb);
        S[1] += W * SYs[a] * (sa - sb);
        S[2] += W * SZs[a] * (sa - sb);
    }
}

int oracle3d_adhesion_vector(const oracle3d_ctx *c, int x, int y, int z, double S[3])
{
    if (!c || x < 0 || y < 0 || z < 0 || x >= c->nx || y >= c->ny || z >= c->nz) return OR3_EINVAL;
    adhesion3(c, x, y, z, S);
    return OR3_OK;
}

static void density3(oracle3d_ctx *c)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (long id = (long)z * c->nx * c->ny; id < (long)(z + 1) * c->nx * c->ny; ++id)
            for (int k = 0; k < 2; ++k) {
                double r = 0.0;
                if (!c->solid[id])
                    for (int i = 0; i < Q; ++i) r += F3(c, k, i, id);
                R3(c, k, id) = r;
            }
}

/* Forces at fluid node (x, y, z) from the densities in c->rho:
 * parts [coh1 coh2 ads1 ads2 body1 body2] x (x, y, z). */
static void forces3(const oracle3d_ctx *c, int x, int y, int z, double parts[6][3])
{
    long id = node3(c, x, y, z);
    double rho[2] = {R3(c, 0, id), R3(c, 1, id)};
    long src[NS];
    resolve3(c, x, y, z, src);
    /* Eq. 8: F_k = -G_c psi_k(x) sum_n W_n Psi_n^{other} e_n */
    for (int k = 0; k < 2; ++k) {
        int o = 1 - k;
        double s[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < NS; a += 2) {
            double pa = src[a] < 0 ? 0.0 : R3(c, o, src[a]);
            double pb = src[a + 1] < 0 ? 0.0 : R3(c, o, src[a + 1]);
            double W = stencil_weight(a);
            s[0] += W * SXs[a] * (pa - pb);
            s[1] += W * SYs[a] * (pa - pb);
            s[2] += W * SZs[a] * (pa - pb);
        }
        for (int d = 0; d < 3; ++d) parts[k][d] = -c->Gc * rho[k] * s[d];
    }
    /* Eq. 9-11 */
    double S[3];
    adhesion3(c, x, y, z, S);
    double G1 = c->Gw1;
    if (!(c->flags & OR3_SCHEME_ORIGINAL)) G1 = local_G3((rho[0] - rho[1]) / (rho[0] + rho[1]), c->Gw1, c->Gw2, c->delta);
    double G[2] = {G1, c->Gw2};
    for (int k = 0; k < 2; ++k)
        for (int d = 0; d < 3; ++d) parts[2 + k][d] = -G[k] * rho[k] * S[d];
    for (int k = 0; k < 2; ++k) {
        double scale = (c->flags & OR3_FORCE_DENSITY) ? 1.0 : rho[k];
        for (int d = 0; d < 3; ++d) parts[4 + k][d] = scale * c->acc[k][d];
    }
}

static void macro3(const oracle3d_ctx *c, int x, int y, int z, double rho[2], double F[2][3], double u[3])
{
    long id = node3(c, x, y, z);
    double j[2][3];
    for (int k = 0; k < 2; ++k) {
        rho[k] = R3(c, k, id);
        j[k][0] = j[k][1] = j[k][2] = 0.0;
        for (int i = 0; i < Q; ++i) {
            double fi = F3(c, k, i, id);
            j[k][0] += fi * EX[i];
            j[k][1] += fi * EY[i];
            j[k][2] += fi * EZ[i];
        }
    }
    double parts[6][3];
    forces3(c, x, y, z, parts);
    for (int k = 0; k < 2; ++k)
        for (int d = 0; d < 3; ++d) F[k][d] = parts[k][d] + parts[2 + k][d] + parts[4 + k][d];
    double half = (c->flags & OR3_VEL_LITERAL) ? 0.0 : 0.5;
    for (int d = 0; d < 3; ++d) u[d] = ((j[0][d] + half * F[0][d]) + (j[1][d] + half * F[1][d])) / (rho[0] + rho[1]);
}

int oracle3d_node_forces(oracle3d_ctx *c, int x, int y, int z, double out[18])
{
    if (!c || x < 0 || y < 0 || z < 0 || x >= c->nx || y >= c->ny || z >= c->nz) return OR3_EINVAL;
    if (!c->have_fields || !c->have_params) return fail(c, OR3_ESTATE, "fields/params missing");
    density3(c);
    double parts[6][3];
    forces3(c, x, y, z, parts);
    for (int p = 0; p < 6; ++p)
        for (int d = 0; d < 3; ++d) out[3 * p + d] = parts[p][d];
    return OR3_OK;
}

static int ready3(oracle3d_ctx *c)
{
    if (!c) return OR3_EINVAL;
    if (!c->have_geom) return fail(c, OR3_ESTATE, "set_geometry first");
    if (!c->have_params) return fail(c, OR3_ESTATE, "set_params first");
    if (!c->have_fields) return fail(c, OR3_ESTATE, "init_fields first");
    return OR3_OK;
}

int oracle3d_step(oracle3d_ctx *c, int nsteps)
{
    int rc = ready3(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(c, OR3_EINVAL, "negative step count");
    for (int s = 0; s < nsteps; ++s) {
        density3(c);
        /* collision (Eq. 1-2, 6-7) */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    long id = node3(c, x, y, z);
                    if (c->solid[id]) continue;
                    double rho[2], F[2][3], u[3];
                    macro3(c, x, y, z, rho, F, u);
                    for (int k = 0; k < 2; ++k) {
                        double feq[Q], Fi[Q];
                        oracle3d_equilibrium(rho[k], u, feq);
                        oracle3d_forcing(F[k], u, Fi);
                        for (int i = 0; i < Q; ++i) {
                            double fi = F3(c, k, i, id);
                            FP3(c, k, i, id) = fi + (feq[i] - fi) / c->tau + (1.0 - 1.0 / (2.0 * c->tau)) * Fi[i];
                        }
                    }
                }
        /* streaming, halfway bounce-back where the source is unavailable */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    long id = node3(c, x, y, z);
                    if (c->solid[id]) continue;
                    for (int k = 0; k < 2; ++k)
                        for (int i = 0; i < Q; ++i) {
                            int sx = x - EX[i], sy = y - EY[i], sz = z - EZ[i];
                            F3(c, k, i, id) = avail3(c, sx, sy, sz) ? FP3(c, k, i, node3(c, sx, sy, sz))
                                                                    : FP3(c, k, d3q19_opp(i), id);
                        }
                }
        c->t += 1;
    }
    return OR3_OK;
}

int oracle3d_get_fields(oracle3d_ctx *c, double *rho1, double *rho2, double *ux, double *uy, double *uz)
{
    int rc = ready3(c);
    if (rc) return rc;
    density3(c);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long id = node3(c, x, y, z);
                double rho[2] = {0.0, 0.0}, F[2][3], u[3] = {0.0, 0.0, 0.0};
                if (!c->solid[id]) macro3(c, x, y, z, rho, F, u);
                if (rho1) rho1[id] = rho[0];
                if (rho2) rho2[id] = rho[1];
                if (ux) ux[id] = u[0];
                if (uy) uy[id] = u[1];
                if (uz) uz[id] = u[2];
            }
    return OR3_OK;
}

int oracle3d_reduce(oracle3d_ctx *c, double out[9])
{
    int rc = ready3(c);
    if (rc) return rc;
    size_t n = (size_t)c->n;
    double *r1 = (double *)malloc(n * sizeof(double)), *r2 = (double *)malloc(n * sizeof(double));
    double *u[3];
    for (int d = 0; d < 3; ++d) u[d] = (double *)malloc(n * sizeof(double));
    if (!r1 || !r2 || !u[0] || !u[1] || !u[2]) {
        free(r1); free(r2); free(u[0]); free(u[1]); free(u[2]);
        return fail(c, OR3_ENOMEM, "out of memory");
    }
    oracle3d_get_fields(c, r1, r2, u[0], u[1], u[2]);
    double M1 = 0, M2 = 0, P[3] = {0, 0, 0}, umax = 0, rmin = INFINITY, rmax = -INFINITY, bad = 0;
    for (size_t id = 0; id < n; ++id) {
        if (c->solid[id]) continue;
        if (!isfinite(r1[id]) || !isfinite(r2[id]) || !isfinite(u[0][id]) || !isfinite(u[1][id]) ||
            !isfinite(u[2][id])) {
            bad += 1.0;
            continue;
        }
        double rt = r1[id] + r2[id];
        M1 += r1[id];
        M2 += r2[id];
        for (int d = 0; d < 3; ++d) P[d] += rt * u[d][id];
        double um = sqrt(u[0][id] * u[0][id] + u[1][id] * u[1][id] + u[2][id] * u[2][id]);
        if (um > umax) umax = um;
        if (r1[id] < rmin) rmin = r1[id];
        if (r1[id] > rmax) rmax = r1[id];
    }
    out[0] = M1; out[1] = M2; out[2] = P[0]; out[3] = P[1]; out[4] = P[2];
    out[5] = umax; out[6] = rmin; out[7] = rmax; out[8] = bad;
    free(r1); free(r2); free(u[0]); free(u[1]); free(u[2]);
    return OR3_OK;
}

/* ------------------------------------------------------------------ */
/* Contact angle: interface points, sphere fit                          */
/* ------------------------------------------------------------------ */

/* Gaussian elimination with partial pivoting, n <= 4. */
static int solve_n(int n, double A[4][4], double b[4], double x[4])
{
    double M[4][5];
    for (int r = 0; r < n; ++r) {
        for (int q = 0; q < n; ++q) M[r][q] = A[r][q];
        M[r][n] = b[r];
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int q = 0; q <= n; ++q) {
                double t = M[col][q];
                M[col][q] = M[piv][q];
                M[piv][q] = t;
            }
        for (int r = col + 1; r < n; ++r) {
            double fct = M[r][col] / M[col][col];
            for (int q = col; q <= n; ++q) M[r][q] -= fct * M[col][q];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = M[r][n];
        for (int q = r + 1; q < n; ++q) s -= M[r][q] * x[q];
        x[r] = s / M[r][r];
    }
    return 0;
}

/* Algebraic sphere fit x^2 + y^2 + z^2 + D x + E y + F z + G = 0 on
 * mean-centred points, then Gauss-Newton on the geometric distances.
 * out = centre (x, y, z), radius. */
int oracle3d_sphere_fit(const double *px, const double *py, const double *pz, int n, double out[4])
{
    if (!px || !py || !pz || n < 4) return OR3_EINVAL;
    double m[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        m[0] += px[i];
        m[1] += py[i];
        m[2] += pz[i];
    }
    for (int d = 0; d < 3; ++d) m[d] /= n;
    double A[4][4] = {{0}}, b[4] = {0};
    for (int i = 0; i < n; ++i) {
        double p[3] = {px[i] - m[0], py[i] - m[1], pz[i] - m[2]};
        double row[4] = {p[0], p[1], p[2], 1.0};
        double w = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        for (int r = 0; r < 4; ++r) {
            for (int q = 0; q < 4; ++q) A[r][q] += row[r] * row[q];
            b[r] -= row[r] * w;
        }
    }
    double D[4];
    if (solve_n(4, A, b, D)) return OR3_EINVAL;
    double cx = m[0] - D[0] / 2.0, cy = m[1] - D[1] / 2.0, cz = m[2] - D[2] / 2.0;
    double r2 = (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) / 4.0 - D[3];
    if (!(r2 > 0.0)) return OR3_EINVAL;
    double r = sqrt(r2);
    for (int it = 0; it < 100; ++it) {
        double JJ[4][4] = {{0}}, Jr[4] = {0};
        for (int i = 0; i < n; ++i) {
            double dx = px[i] - cx, dy = py[i] - cy, dz = pz[i] - cz;
            double dd = sqrt(dx * dx + dy * dy + dz * dz);
            if (dd == 0.0) continue;
            double J[4] = {-dx / dd, -dy / dd, -dz / dd, -1.0};
            double res = dd - r;
            for (int p = 0; p < 4; ++p) {
                for (int q = 0; q < 4; ++q) JJ[p][q] += J[p] * J[q];
                Jr[p] -= J[p] * res;
            }
        }
        double dl[4];
        if (solve_n(4, JJ, Jr, dl)) break;
        cx += dl[0];
        cy += dl[1];
        cz += dl[2];
        r += dl[3];
        double step = fabs(dl[0]) + fabs(dl[1]) + fabs(dl[2]) + fabs(dl[3]);
        if (step <= 1e-13 * (1.0 + fabs(r))) break;
    }
    out[0] = cx;
    out[1] = cy;
    out[2] = cz;
    out[3] = r;
    return OR3_OK;
}

static double wall_dist3(int kind, const double w[4], double x, double y, double z)
{
    if (kind == 0) return z - w[0];
    double dx = x - w[0], dy = y - w[1], dz = z - w[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - w[3];
}

/* Largest 6-connected region of each phase (rho^e > 0, rho^e <= 0) among
 * fluid nodes, links not across periodic seams; breadth-first in scan
 * order, ties to the region met first. */
static int regions3(const oracle3d_ctx *c, const double *re, long *lab, long best[2])
{
    long n = c->n;
    long *queue = (long *)malloc((size_t)n * sizeof(long));
    if (!queue) return -1;
    for (long i = 0; i < n; ++i) lab[i] = -1;
    long nlab = 0, bsize[2] = {0, 0};
    best[0] = best[1] = -1;
    for (long seed = 0; seed < n; ++seed) {
        if (c->solid[seed] || lab[seed] >= 0) continue;
        int ph = re[seed] > 0.0;
        long head = 0, tail = 0;
        queue[tail++] = seed;
        lab[seed] = nlab;
        while (head < tail) {
            long a = queue[head++];
            int x = (int)(a % c->nx), y = (int)((a / c->nx) % c->ny), z = (int)(a / ((long)c->nx * c->ny));
            int nb[6][3] = {{x + 1, y, z}, {x - 1, y, z}, {x, y + 1, z}, {x, y - 1, z}, {x, y, z + 1}, {x, y, z - 1}};
            for (int k = 0; k < 6; ++k) {
                int xx = nb[k][0], yy = nb[k][1], zz = nb[k][2];
                if (xx < 0 || yy < 0 || zz < 0 || xx >= c->nx || yy >= c->ny || zz >= c->nz) continue;
                long b = ((long)zz * c->ny + yy) * c->nx + xx;
                if (c->solid[b] || lab[b] >= 0 || (re[b] > 0.0) != ph) continue;
                lab[b] = nlab;
                queue[tail++] = b;
            }
        }
        if (tail > bsize[ph]) {
            bsize[ph] = tail;
            best[ph] = nlab;
        }
        ++nlab;
    }
    free(queue);
    return 0;
}

int oracle3d_interface_points(oracle3d_ctx *c, int kind, const double wall[4], double *px, double *py,
                              double *pz, int cap, int *n_out)
{
    int rc = ready3(c);
    if (rc) return rc;
    if ((kind != 0 && kind != 1) || !wall) return fail(c, OR3_EINVAL, "bad wall description");
    size_t n = (size_t)c->n;
    double *r1 = (double *)malloc(n * sizeof(double)), *r2 = (double *)malloc(n * sizeof(double));
    double *re = (double *)malloc(n * sizeof(double));
    long *lab = (long *)malloc(n * sizeof(long));
    long best[2];
    if (!r1 || !r2 || !re || !lab) {
        free(r1); free(r2); free(re); free(lab);
        return fail(c, OR3_ENOMEM, "out of memory");
    }
    oracle3d_get_fields(c, r1, r2, NULL, NULL, NULL);
    for (size_t id = 0; id < n; ++id) re[id] = c->solid[id] ? 0.0 : (r1[id] - r2[id]) / (r1[id] + r2[id]);
    if (regions3(c, re, lab, best)) {
        free(r1); free(r2); free(re); free(lab);
        return fail(c, OR3_ENOMEM, "out of memory");
    }
    int count = 0;
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long a = ((long)z * c->ny + y) * c->nx + x;
                if (c->solid[a]) continue;
                for (int dir = 0; dir < 3; ++dir) {
                    int x2 = x + (dir == 0), y2 = y + (dir == 1), z2 = z + (dir == 2);
                    if (x2 >= c->nx || y2 >= c->ny || z2 >= c->nz) continue;
                    long b = ((long)z2 * c->ny + y2) * c->nx + x2;
                    if (c->solid[b]) continue;
                    if ((re[a] > 0.0) == (re[b] > 0.0)) continue;
                    if (lab[a] != best[re[a] > 0.0] || lab[b] != best[re[b] > 0.0]) continue;
                    double tp = re[a] / (re[a] - re[b]);
                    double qx = x + tp * (x2 - x), qy = y + tp * (y2 - y), qz = z + tp * (z2 - z);
                    if (wall_dist3(kind, wall, qx, qy, qz) < 3.0) continue;
                    if (count < cap && px && py && pz) {
                        px[count] = qx;
                        py[count] = qy;
                        pz[count] = qz;
                    }
                    ++count;
                }
            }
    free(r1); free(r2); free(re); free(lab);
    if (n_out) *n_out = count;
    return OR3_OK;
}

int oracle3d_contact_angle(oracle3d_ctx *c, int kind, const double wall[4], double *theta_deg)
{
    int rc = ready3(c);
    if (rc) return rc;
    if (!theta_deg) return fail(c, OR3_EINVAL, "null output");
    int np = 0;
    rc = oracle3d_interface_points(c, kind, wall, NULL, NULL, NULL, 0, &np);
    if (rc) return rc;
    if (np < 4) return fail(c, OR3_EUNSTABLE, "fewer than 4 interface points");
    double *px = (double *)malloc((size_t)np * sizeof(double));
    double *py = (double *)malloc((size_t)np * sizeof(double));
    double *pz = (double *)malloc((size_t)np * sizeof(double));
    if (!px || !py || !pz) {
        free(px); free(py); free(pz);
        return fail(c, OR3_ENOMEM, "out of memory");
    }
    oracle3d_interface_points(c, kind, wall, px, py, pz, np, &np);
    double s[4];
    rc = oracle3d_sphere_fit(px, py, pz, np, s);
    free(px); free(py); free(pz);
    if (rc) return fail(c, OR3_EUNSTABLE, "sphere fit failed");
    double cth;
    if (kind == 0) {
        cth = -(s[2] - wall[0]) / s[3];
    } else {
        double dx = s[0] - wall[0], dy = s[1] - wall[1], dz = s[2] - wall[2];
        double d2 = dx * dx + dy * dy + dz * dz, Rs = wall[3], r = s[3];
        cth = (Rs * Rs + r * r - d2) / (2.0 * Rs * r);
    }
    if (cth > 1.0) cth = 1.0;
    if (cth < -1.0) cth = -1.0;
    *theta_deg = acos(cth) * 180.0 / M_PI;
    return OR3_OK;
}
