// Host side of the 3-D C ABI declared in include/lbm3d.h: contexts,
// parameter mapping, launches, diagnostics and the contact angle.
#include "lbm3d.h"
#include "lbm3d_contact.hpp"
#include "lbm3d_launch.hpp"
#include "lbm_params.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace lbm3;
using namespace lbm3_host;

struct lbm3d_ctx {
    int nx = 0, ny = 0, nz = 0, storage = 0;
    unsigned flags = 0;
    long long N = 0;
    int device = 0;
    hipStream_t stream = nullptr, own_stream = nullptr;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t *d_solid = nullptr;
    double *d_tmp = nullptr;  // staging: fields (5N doubles) or populations (38N)
    size_t tmp_bytes = 0;
    double *d_partials = nullptr;
    size_t partials_cap = 0;
    double *d_out = nullptr;  // 9 diagnostics + 7 contact-angle results
    int *d_cc = nullptr;      // phase-region labels (2N + 2 ints)
    std::vector<uint8_t> solid;
    long long n_fluid = 0;
    double Gc = 0, Gw1 = 0, Gw2 = 0, delta = 0.8, tau = 1.0;
    double acc[2][3] = {{0, 0, 0}, {0, 0, 0}};
    double rho0[2] = {0, 0};
    bool have_geom = false, have_params = false, have_fields = false;
    long t = 0;
    int bx = 32, by = 8, bz = 4, tz = 1;  // collide-pass brick and threads in z
    void *d_psi = nullptr;        // density-pass output: psi of both components per node
    std::string err;
};

namespace {

int fail(lbm3d_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char b[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(b, sizeof b, fmt, ap);
        va_end(ap);
        c->err = b;
    }
    return code;
}

#define HIPCHK3(c, call)                                                                                   \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) return fail((c), LBM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t esize(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32 ? 4 : 2; }

int ensure_tmp(lbm3d_ctx *c, size_t bytes)
{
    if (c->tmp_bytes >= bytes) return LBM_OK;
    if (c->d_tmp) (void)hipFree(c->d_tmp);
    c->d_tmp = nullptr;
    c->tmp_bytes = 0;
    if (hipMalloc(&c->d_tmp, bytes) != hipSuccess) return fail(c, LBM_ENOMEM, "device allocation of %zu bytes failed", bytes);
    c->tmp_bytes = bytes;
    return LBM_OK;
}

int ensure_partials(lbm3d_ctx *c, size_t n)
{
    if (c->partials_cap >= n) return LBM_OK;
    if (c->d_partials) (void)hipFree(c->d_partials);
    c->d_partials = nullptr;
    c->partials_cap = 0;
    if (hipMalloc(&c->d_partials, n * 9 * sizeof(double)) != hipSuccess) return fail(c, LBM_ENOMEM, "partials allocation failed");
    c->partials_cap = n;
    return LBM_OK;
}

template <class C>
KParams3<C> make_params3(const lbm3d_ctx *c, const void *A, void *B, int bx, int by, int bz)
{
    KParams3<C> p;
    std::memset(&p, 0, sizeof p);
    p.A = A;
    p.B = B;
    p.nx = c->nx;
    p.ny = c->ny;
    p.nz = c->nz;
    p.flags = c->flags;
    p.bricks_x = (c->nx + bx - 1) / bx;
    p.bricks_y = (c->ny + by - 1) / by;
    p.bricks_z = (c->nz + bz - 1) / bz;
    p.n_units = p.bricks_x * p.bricks_y * p.bricks_z;
    p.psi = (PsiPair<C> *)c->d_psi;
    p.tick = (unsigned)c->t;
    p.N = c->N;
    const double tau = c->tau;
    p.omega = (C)(1.0 / tau);
    p.omw = (C)(1.0 - 1.0 / tau);
    p.cf3 = (C)(3.0 * (1.0 - 1.0 / (2.0 * tau)));
    p.cf9 = (C)(9.0 * (1.0 - 1.0 / (2.0 * tau)));
    p.half = (c->flags & LBM_VEL_LITERAL) ? (C)0 : (C)0.5;
    p.negGc = (C)(-c->Gc);
    p.Gw1 = (C)c->Gw1;
    p.Gw2 = (C)c->Gw2;
    p.delta = (C)c->delta;
    if (!(c->flags & LBM_SCHEME_ORIGINAL)) {
        // Eq. 11 coefficients (s1 = t1 = harmonic mean of G_w1 and G_w2)
        const double s1 = 2.0 * c->Gw1 * c->Gw2 / (c->Gw1 + c->Gw2);
        const double s2 = 2.0 * (c->Gw1 - s1) / c->delta;
        const double t2 = 2.0 * (s1 - c->Gw2) / c->delta;
        p.s1 = (C)s1;
        p.s2 = (C)s2;
        p.s3 = (C)(-s2 / (2.0 * c->delta));
        p.t2 = (C)t2;
        p.t3 = (C)(t2 / (2.0 * c->delta));
    }
    const bool dev = c->storage != LBM_F64;
    for (int k = 0; k < 2; ++k) {
        for (int d = 0; d < 3; ++d) p.g[k][d] = (C)c->acc[k][d];
        p.rho0[k] = dev ? (C)c->rho0[k] : (C)0;
        p.omega_rho0[k] = dev ? (C)(c->rho0[k] / tau) : (C)0;
    }
    return p;
}

template <int S>
int run_pass3_t(lbm3d_ctx *c, Pass3 pass, double *fields, int *nparts)
{
    using C = typename lbm::Traits<S>::C;
    const bool fp = pass == P3_FIELDS_REDUCE;
    KParams3<C> p = make_params3<C>(c, c->buf[c->cur], c->buf[c->cur ^ 1], fp ? 32 : c->bx, fp ? 8 : c->by,
                                    fp ? 4 : c->bz);
    const int grid = ((p.n_units + 7) / 8) * 8;
    if (nparts) *nparts = grid;
    if (pass != P3_STEP) {
        int rc = ensure_partials(c, (size_t)grid);
        if (rc) return rc;
        p.partials = c->d_partials;
    }
    if (fields) {
        p.out_rho1 = fields;
        p.out_rho2 = fields + c->N;
        p.out_ux = fields + 2 * c->N;
        p.out_uy = fields + 3 * c->N;
        p.out_uz = fields + 4 * c->N;
    }
    const bool sr = (S == lbm::ST_F16 || S == lbm::ST_BF16) && (c->flags & LBM_ROUND_STOCHASTIC);
    const hipError_t e = launch3<S>(p, pass, c->bx, c->by, c->bz, c->tz, sr, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return LBM_OK;
}

int run_pass3(lbm3d_ctx *c, Pass3 pass, double *fields, int *nparts)
{
    switch (c->storage) {
    case LBM_F64: return run_pass3_t<lbm::ST_F64>(c, pass, fields, nparts);
    case LBM_F32: return run_pass3_t<lbm::ST_F32>(c, pass, fields, nparts);
    case LBM_F16: return run_pass3_t<lbm::ST_F16>(c, pass, fields, nparts);
    default: return run_pass3_t<lbm::ST_BF16>(c, pass, fields, nparts);
    }
}

template <int S>
int inverse3_t(lbm3d_ctx *c, const double *fsrc, const double *rho)
{
    using C = typename lbm::Traits<S>::C;
    KParams3<C> p = make_params3<C>(c, nullptr, c->buf[c->cur], 32, 8, 4);
    const long long blocks = (c->N + 255) / 256;
    hipLaunchKernelGGL((k_inverse3<S>), dim3((unsigned)blocks), dim3(256), 0, c->stream, p, c->d_solid, fsrc, rho);
    HIPCHK3(c, hipGetLastError());
    return LBM_OK;
}

int inverse3(lbm3d_ctx *c, const double *fsrc, const double *rho)
{
    switch (c->storage) {
    case LBM_F64: return inverse3_t<lbm::ST_F64>(c, fsrc, rho);
    case LBM_F32: return inverse3_t<lbm::ST_F32>(c, fsrc, rho);
    case LBM_F16: return inverse3_t<lbm::ST_F16>(c, fsrc, rho);
    default: return inverse3_t<lbm::ST_BF16>(c, fsrc, rho);
    }
}

template <int S>
int pull_all_t(lbm3d_ctx *c, double *out)
{
    using C = typename lbm::Traits<S>::C;
    KParams3<C> p = make_params3<C>(c, c->buf[c->cur], nullptr, 32, 8, 4);
    const long long blocks = (c->N + 255) / 256;
    hipLaunchKernelGGL((k_pull3_all<S>), dim3((unsigned)blocks), dim3(256), 0, c->stream, p, out);
    HIPCHK3(c, hipGetLastError());
    return LBM_OK;
}

int pull_all(lbm3d_ctx *c, double *out)
{
    switch (c->storage) {
    case LBM_F64: return pull_all_t<lbm::ST_F64>(c, out);
    case LBM_F32: return pull_all_t<lbm::ST_F32>(c, out);
    case LBM_F16: return pull_all_t<lbm::ST_F16>(c, out);
    default: return pull_all_t<lbm::ST_BF16>(c, out);
    }
}

int ready3(lbm3d_ctx *c)
{
    if (!c) return LBM_EINVAL;
    if (!c->have_geom) return fail(c, LBM_ESTATE, "set_geometry first");
    if (!c->have_params) return fail(c, LBM_ESTATE, "set_params first");
    if (!c->have_fields) return fail(c, LBM_ESTATE, "init_fields or set_populations first");
    return LBM_OK;
}

int check_adh3(lbm3d_ctx *c, double Gw1, double Gw2, double delta)
{
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(c, LBM_EINVAL, "delta must be > 0");
    if (!std::isfinite(Gw1) || !std::isfinite(Gw2)) return fail(c, LBM_EINVAL, "non-finite adhesion parameter");
    if (!(c->flags & LBM_SCHEME_ORIGINAL) && Gw1 + Gw2 == 0.0)
        return fail(c, LBM_EINVAL, "improved scheme needs G_w1 + G_w2 != 0");
    return LBM_OK;
}

// Fields + diagnostics pass into d_tmp (5N doubles) and d_out[0..8].
int fields_reduce3(lbm3d_ctx *c)
{
    int rc = ensure_tmp(c, (size_t)c->N * 5 * sizeof(double));
    if (rc) return rc;
    int nparts = 0;
    rc = run_pass3(c, P3_FIELDS_REDUCE, c->d_tmp, &nparts);
    if (rc) return rc;
    hipLaunchKernelGGL(k_reduce3_final, dim3(1), dim3(256), 0, c->stream, c->d_partials, nparts, c->d_out);
    HIPCHK3(c, hipGetLastError());
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm3d_create(lbm3d_ctx **out, int nx, int ny, int nz, int storage, unsigned flags)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (nx < 5 || ny < 5 || nz < 5) return LBM_EINVAL;
    const long long N = (long long)nx * ny * nz;
    if (N > (1LL << 31) - 1) return LBM_EINVAL;
    if (storage < LBM_F64 || storage > LBM_BF16) return LBM_EINVAL;
    const unsigned allowed = LBM_PERIODIC_X | LBM_PERIODIC_Y | LBM3D_PERIODIC_Z | LBM_SCHEME_ORIGINAL |
                             LBM_E8_COPY_OFF | LBM_WALLPSI_SELF | LBM_VEL_LITERAL | LBM_FORCE_DENSITY |
                             LBM_ROUND_STOCHASTIC | LBM_ROUND_NEAREST;
    if (flags & ~allowed) return LBM_EINVAL;
    if ((flags & LBM_ROUND_STOCHASTIC) && (flags & LBM_ROUND_NEAREST)) return LBM_EINVAL;
    // one component's 19 direction arrays are addressed through a 32-bit range
    if (N * 19 * (long long)esize(storage) >= (1LL << 32)) return LBM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LBM_EDEVICE;
    lbm3d_ctx *c = new (std::nothrow) lbm3d_ctx();
    if (!c) return LBM_ENOMEM;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->N = N;
    c->storage = storage;
    c->flags = lbm_host::resolve_rounding(flags, storage);
    // FP32: two threads per column, whose 512-thread workgroups fit two to
    // a CU at the four waves per SIMD its collide kernel is built for
    if (storage == LBM_F32) c->tz = 2;
    hipDeviceProp_t prop;
    if (hipGetDevice(&c->device) != hipSuccess || hipGetDeviceProperties(&prop, c->device) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete c;
        return LBM_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return LBM_EDEVICE;
    }
    c->stream = c->own_stream;
    const size_t bytes = (size_t)N * 38 * esize(storage);
    const size_t psi_bytes = (size_t)N * 2 * (storage == LBM_F64 ? sizeof(double) : sizeof(float));
    const bool ok = hipMalloc(&c->buf[0], bytes) == hipSuccess && hipMalloc(&c->buf[1], bytes) == hipSuccess &&
                    hipMalloc(&c->d_psi, psi_bytes) == hipSuccess && hipMalloc(&c->d_solid, (size_t)N) == hipSuccess &&
                    hipMalloc(&c->d_out, 32 * sizeof(double)) == hipSuccess;
    if (!ok) {
        lbm3d_destroy(c);
        return LBM_ENOMEM;
    }
    c->solid.assign((size_t)N, 0);
    *out = c;
    return LBM_OK;
}

unsigned lbm3d_get_flags(const lbm3d_ctx *c) { return c ? c->flags : 0u; }

void lbm3d_destroy(lbm3d_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *p : {c->buf[0], c->buf[1], c->d_psi, (void *)c->d_solid, (void *)c->d_tmp, (void *)c->d_partials,
                    (void *)c->d_out, (void *)c->d_cc})
        if (p) (void)hipFree(p);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

const char *lbm3d_last_error(const lbm3d_ctx *c) { return c ? c->err.c_str() : "null context"; }

int lbm3d_set_stream(lbm3d_ctx *c, void *hip_stream)
{
    if (!c) return LBM_EINVAL;
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    c->stream = hip_stream ? (hipStream_t)hip_stream : c->own_stream;
    return LBM_OK;
}

int lbm3d_set_geometry(lbm3d_ctx *c, const uint8_t *solid)
{
    if (!c || !solid) return LBM_EINVAL;
    long long nf = 0;
    for (long long i = 0; i < c->N; ++i) {
        c->solid[(size_t)i] = solid[i] ? 1 : 0;
        nf += solid[i] ? 0 : 1;
    }
    HIPCHK3(c, hipMemcpyAsync(c->d_solid, c->solid.data(), (size_t)c->N, hipMemcpyHostToDevice, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    c->n_fluid = nf;
    c->have_geom = true;
    c->have_fields = false;
    return LBM_OK;
}

int lbm3d_set_params(lbm3d_ctx *c, double G_c, double G_ads, double tau)
{
    if (!c) return LBM_EINVAL;
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(c, LBM_EINVAL, "tau must be > 0.5");
    if (!std::isfinite(G_c) || !std::isfinite(G_ads)) return fail(c, LBM_EINVAL, "non-finite parameter");
    const double Gw2 = G_c, Gw1 = G_c + 2.0 * G_ads;
    if (!(c->flags & LBM_SCHEME_ORIGINAL) && !(Gw2 != 0.0 && Gw1 / Gw2 > 0.0))
        return fail(c, LBM_EINVAL, "lambda = 1 + 2 G_ads / G_c must be > 0");
    int rc = check_adh3(c, Gw1, Gw2, 0.8);
    if (rc) return rc;
    c->Gc = G_c;
    c->Gw1 = Gw1;
    c->Gw2 = Gw2;
    c->delta = 0.8;
    c->tau = tau;
    c->have_params = true;
    return LBM_OK;
}

int lbm3d_set_adhesion(lbm3d_ctx *c, double G_w1, double G_w2, double delta)
{
    if (!c) return LBM_EINVAL;
    if (!c->have_params) return fail(c, LBM_ESTATE, "set_params first");
    int rc = check_adh3(c, G_w1, G_w2, delta);
    if (rc) return rc;
    c->Gw1 = G_w1;
    c->Gw2 = G_w2;
    c->delta = delta;
    return LBM_OK;
}

int lbm3d_set_body_accel(lbm3d_ctx *c, const double g[6])
{
    if (!c || !g) return LBM_EINVAL;
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(g[q])) return fail(c, LBM_EINVAL, "non-finite acceleration");
    for (int k = 0; k < 2; ++k)
        for (int d = 0; d < 3; ++d) c->acc[k][d] = g[3 * k + d];
    return LBM_OK;
}

int lbm3d_init_fields(lbm3d_ctx *c, const double *rho1, const double *rho2)
{
    if (!c || !rho1 || !rho2) return LBM_EINVAL;
    if (!c->have_geom) return fail(c, LBM_ESTATE, "set_geometry first");
    double s[2] = {0, 0};
    for (long long i = 0; i < c->N; ++i) {
        if (c->solid[(size_t)i]) continue;
        if (!std::isfinite(rho1[i]) || !std::isfinite(rho2[i])) return fail(c, LBM_EINVAL, "non-finite density");
        s[0] += rho1[i];
        s[1] += rho2[i];
    }
    c->rho0[0] = c->n_fluid ? s[0] / (double)c->n_fluid : 0.0;
    c->rho0[1] = c->n_fluid ? s[1] / (double)c->n_fluid : 0.0;
    int rc = ensure_tmp(c, (size_t)c->N * 2 * sizeof(double));
    if (rc) return rc;
    HIPCHK3(c, hipMemcpyAsync(c->d_tmp, rho1, (size_t)c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK3(c, hipMemcpyAsync(c->d_tmp + c->N, rho2, (size_t)c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const size_t bytes = (size_t)c->N * 38 * esize(c->storage);
    HIPCHK3(c, hipMemsetAsync(c->buf[0], 0xff, bytes, c->stream));
    HIPCHK3(c, hipMemsetAsync(c->buf[1], 0xff, bytes, c->stream));
    c->cur = 0;
    rc = inverse3(c, nullptr, c->d_tmp);
    if (rc) return rc;
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    c->have_fields = true;
    c->t = 0;
    return LBM_OK;
}

int lbm3d_set_populations(lbm3d_ctx *c, const double *f)
{
    if (!c || !f) return LBM_EINVAL;
    if (!c->have_geom) return fail(c, LBM_ESTATE, "set_geometry first");
    double s[2] = {0, 0};
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 19; ++i)
            for (long long z = 0; z < c->N; ++z) {
                if (c->solid[(size_t)z]) continue;
                const double v = f[(size_t)(k * 19 + i) * c->N + z];
                if (!std::isfinite(v)) return fail(c, LBM_EINVAL, "non-finite population");
                s[k] += v;
            }
    c->rho0[0] = c->n_fluid ? s[0] / (double)c->n_fluid : 0.0;
    c->rho0[1] = c->n_fluid ? s[1] / (double)c->n_fluid : 0.0;
    int rc = ensure_tmp(c, (size_t)c->N * 38 * sizeof(double));
    if (rc) return rc;
    HIPCHK3(c, hipMemcpyAsync(c->d_tmp, f, (size_t)c->N * 38 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const size_t bytes = (size_t)c->N * 38 * esize(c->storage);
    HIPCHK3(c, hipMemsetAsync(c->buf[0], 0xff, bytes, c->stream));
    HIPCHK3(c, hipMemsetAsync(c->buf[1], 0xff, bytes, c->stream));
    c->cur = 0;
    rc = inverse3(c, c->d_tmp, nullptr);
    if (rc) return rc;
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    c->have_fields = true;
    c->t = 0;
    return LBM_OK;
}

int lbm3d_get_populations(lbm3d_ctx *c, double *f)
{
    int rc = ready3(c);
    if (rc) return rc;
    if (!f) return fail(c, LBM_EINVAL, "null output");
    rc = ensure_tmp(c, (size_t)c->N * 38 * sizeof(double));
    if (rc) return rc;
    rc = pull_all(c, c->d_tmp);
    if (rc) return rc;
    HIPCHK3(c, hipMemcpyAsync(f, c->d_tmp, (size_t)c->N * 38 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm3d_step(lbm3d_ctx *c, int n)
{
    int rc = ready3(c);
    if (rc) return rc;
    if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
    for (int s = 0; s < n; ++s) {
        rc = run_pass3(c, P3_STEP, nullptr, nullptr);
        if (rc) return rc;
        c->cur ^= 1;
        c->t += 1;
    }
    return LBM_OK;
}

int lbm3d_synchronize(lbm3d_ctx *c)
{
    if (!c) return LBM_EINVAL;
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

long lbm3d_time(const lbm3d_ctx *c) { return c ? c->t : -1; }

int lbm3d_get_fields(lbm3d_ctx *c, double *rho1, double *rho2, double *ux, double *uy, double *uz)
{
    int rc = ready3(c);
    if (rc) return rc;
    rc = fields_reduce3(c);
    if (rc) return rc;
    double *outs[5] = {rho1, rho2, ux, uy, uz};
    for (int q = 0; q < 5; ++q)
        if (outs[q])
            HIPCHK3(c, hipMemcpyAsync(outs[q], c->d_tmp + (size_t)q * c->N, (size_t)c->N * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm3d_reduce(lbm3d_ctx *c, double out[9])
{
    int rc = ready3(c);
    if (rc) return rc;
    if (!out) return fail(c, LBM_EINVAL, "null output");
    rc = fields_reduce3(c);
    if (rc) return rc;
    HIPCHK3(c, hipMemcpyAsync(out, c->d_out, 9 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    if (c->n_fluid == 0) {
        out[6] = 0.0;
        out[7] = 0.0;
    }
    return LBM_OK;
}

int lbm3d_contact_angle(lbm3d_ctx *c, int wall_kind, const double wall[4], double *theta_deg)
{
    int rc = ready3(c);
    if (rc) return rc;
    if (!wall || !theta_deg || (wall_kind != LBM3D_WALL_FLAT && wall_kind != LBM3D_WALL_SPHERE))
        return fail(c, LBM_EINVAL, "bad wall description");
    rc = fields_reduce3(c);
    if (rc) return rc;
    if (!c->d_cc && hipMalloc(&c->d_cc, ((size_t)c->N * 2 + 2) * sizeof(int)) != hipSuccess) {
        c->d_cc = nullptr;
        return fail(c, LBM_ENOMEM, "label allocation failed");
    }
    int *par = c->d_cc, *cnt = c->d_cc + c->N, *best = c->d_cc + 2 * c->N;
    const double *r1 = c->d_tmp, *r2 = c->d_tmp + c->N;
    long long bx = (c->N + 255) / 256;
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(k_cc3_init, dim3((unsigned)bx), dim3(256), 0, c->stream, c->N, c->d_solid, par, cnt);
    hipLaunchKernelGGL(k_cc3_hook, dim3((unsigned)bx), dim3(256), 0, c->stream, c->nx, c->ny, c->nz, r1, r2, c->d_solid,
                       par);
    hipLaunchKernelGGL(k_cc3_count, dim3((unsigned)bx), dim3(256), 0, c->stream, c->N, c->d_solid, par, cnt);
    hipLaunchKernelGGL(k_cc3_pick, dim3(1), dim3(256), 0, c->stream, c->N, r1, r2, c->d_solid, (const int *)par,
                       (const int *)cnt, best);
    Wall3 wd;
    wd.kind = wall_kind;
    for (int q = 0; q < 4; ++q) wd.w[q] = wall[q];
    hipLaunchKernelGGL(k_contact3, dim3(1), dim3(256), 0, c->stream, c->nx, c->ny, c->nz, r1, r2, c->d_solid,
                       (const int *)par, (const int *)best, wd, c->d_out + 16);
    HIPCHK3(c, hipGetLastError());
    double res[7];
    HIPCHK3(c, hipMemcpyAsync(res, c->d_out + 16, 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    if (res[6] != 0.0)
        return fail(c, LBM_EUNSTABLE, res[6] == 1.0 ? "fewer than 4 interface points" : "sphere fit failed");
    *theta_deg = res[0];
    return LBM_OK;
}

int lbm3d_set_tile(lbm3d_ctx *c, int bx, int by, int bz, int tz)
{
    if (!c) return LBM_EINVAL;
    const bool ok = (bx == 32 && by == 8 && bz == 4 && (tz == 1 || tz == 2 || tz == 4)) ||
                    (bx == 32 && by == 8 && bz == 8 && (tz == 1 || tz == 2)) || (bx == 64 && by == 4 && bz == 4 && tz == 2);
    if (!ok) return fail(c, LBM_EINVAL, "brick %d x %d x %d with %d threads in z not available", bx, by, bz, tz);
    c->bx = bx;
    c->by = by;
    c->bz = bz;
    c->tz = tz;
    return LBM_OK;
}

int lbm3d_get_tile(const lbm3d_ctx *c, int *bx, int *by, int *bz, int *tz)
{
    if (!c) return LBM_EINVAL;
    if (bx) *bx = c->bx;
    if (by) *by = c->by;
    if (bz) *bz = c->bz;
    if (tz) *tz = c->tz;
    return LBM_OK;
}

long lbm3d_fluid_nodes(const lbm3d_ctx *c) { return c ? (long)c->n_fluid : -1; }

int lbm3d_bytes_per_update(const lbm3d_ctx *c) { return c ? (int)(38 * 2 * esize(c->storage) + 1) : -1; }

}  // extern "C"
