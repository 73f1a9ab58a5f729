// Three-dimensional step kernel of the two-component pseudopotential LBM
// for gfx950 (arXiv 2505.22256, Sec. 3.5: contact angles on a sphere; the
// method of Sec. 2.1-2.4 on a 3-D lattice).
//
// Lattice: D3Q19 (directions 1-6 = +-x, +-y, +-z, then the twelve face
// diagonals, each odd direction followed by its opposite).  Cohesion
// (Eq. 8) and adhesion (Eq. 9) use the eighth-order isotropic stencil of
// the 5x5x5 neighbourhood (92 positions, |e|^2 in {1,2,3,4,5,6,8}); an
// unavailable position with a coordinate of magnitude 2 takes what its
// first-layer partner (sgn e_x, sgn e_y, sgn e_z) resolves to, which is
// the rule of Table 1 carried to 3-D.
//
// Data layout in HBM: SoA [component][direction 19][node], node =
// (z * ny + y) * nx + x, deviations g = f - w_i rho0 for F32/F16/BF16,
// all-ones sentinels in every slot of a solid node (as in 2-D).
//
// Two passes per step.  The density pass pulls every node's populations
// (Eq. 1 streaming with halfway bounce-back) and writes psi = rho of both
// components (8 B per node in FP32).  The collide pass gives each
// workgroup a brick of nodes: it stages psi of the brick and a 2-node halo
// in LDS, pulls the populations of its own nodes only (the halo costs 8 B
// of psi, not 38 populations), and computes the stencil sums from LDS,
// the forces, the collision and the store.  Against a fused pass whose
// halo nodes pull all their populations to get their density, this reads
// the populations twice per step but never for halo nodes.
#pragma once

#include "lbm_device.hpp"

namespace lbm3 {

using lbm::Axis;
using lbm::make_axis;
using lbm::make_axis_near;
using lbm::PsiPair;
using lbm::Traits;
using lbm::lds_sent;
using lbm::lds_sentinel;

enum : unsigned { F3_PERIODIC_X = 1u, F3_PERIODIC_Y = 2u, F3_ORIGINAL = 4u, F3_COPY_OFF = 8u,
                  F3_WALLPSI_SELF = 16u, F3_VEL_LITERAL = 32u, F3_FORCE_DENSITY = 64u,
                  F3_ROUND_STOCHASTIC = 128u, F3_ROUND_NEAREST = 1024u, F3_PERIODIC_Z = 2048u };

enum : int { K3_STORE = 1, K3_REDUCE = 2, K3_FIELDS = 4, K3_SR = 16 };

// ---------------------------------------------------------------------------
// D3Q19
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int dx3(int i)
{
    return i == 1 || i == 7 || i == 9 || i == 11 || i == 13 ? 1 : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14 ? -1 : 0);
}
__host__ __device__ constexpr int dy3(int i)
{
    return i == 3 || i == 7 || i == 10 || i == 15 || i == 17 ? 1 : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18 ? -1 : 0);
}
__host__ __device__ constexpr int dz3(int i)
{
    return i == 5 || i == 11 || i == 14 || i == 15 || i == 18 ? 1 : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17 ? -1 : 0);
}
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// ---------------------------------------------------------------------------
// The 92-position stencil, grouped by shell, each position followed by its
// opposite; weights normalised to sum W e_x^2 = 1.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr double e8w3(int e2)
{
    return e2 == 1 ? 4.0 / 45.0 : e2 == 2 ? 1.0 / 21.0 : e2 == 3 ? 2.0 / 105.0 : e2 == 4 ? 5.0 / 504.0
         : e2 == 5 ? 1.0 / 315.0 : e2 == 6 ? 1.0 / 630.0 : e2 == 8 ? 1.0 / 5040.0 : 0.0;
}

constexpr int NS3 = 92;

struct Stencil3 {
    signed char x[NS3], y[NS3], z[NS3];
    signed char partner[NS3];  // first-layer partner of a second-layer position, else -1
};

constexpr Stencil3 make_stencil3()
{
    Stencil3 s{};
    const int shells[7] = {1, 2, 3, 4, 5, 6, 8};
    int n = 0;
    for (int k = 0; k < 7; ++k)
        for (int a = -2; a <= 2; ++a)
            for (int b = -2; b <= 2; ++b)
                for (int c = -2; c <= 2; ++c) {
                    if (a * a + b * b + c * c != shells[k]) continue;
                    // keep the half whose first nonzero coordinate (x, then y, then z) is positive
                    const int lead = a != 0 ? a : (b != 0 ? b : c);
                    if (lead < 0) continue;
                    s.x[n] = (signed char)a;
                    s.y[n] = (signed char)b;
                    s.z[n] = (signed char)c;
                    s.x[n + 1] = (signed char)-a;
                    s.y[n + 1] = (signed char)-b;
                    s.z[n + 1] = (signed char)-c;
                    n += 2;
                }
    for (int m = 0; m < NS3; ++m) {
        s.partner[m] = -1;
        const bool second = s.x[m] * s.x[m] == 4 || s.y[m] * s.y[m] == 4 || s.z[m] * s.z[m] == 4;
        if (!second) continue;
        const int px = (s.x[m] > 0) - (s.x[m] < 0), py = (s.y[m] > 0) - (s.y[m] < 0), pz = (s.z[m] > 0) - (s.z[m] < 0);
        for (int q = 0; q < NS3; ++q)
            if (s.x[q] == px && s.y[q] == py && s.z[q] == pz) s.partner[m] = (signed char)q;
    }
    return s;
}

static constexpr Stencil3 kS3 = make_stencil3();

__host__ __device__ constexpr int s3x(int n) { return kS3.x[n]; }
__host__ __device__ constexpr int s3y(int n) { return kS3.y[n]; }
__host__ __device__ constexpr int s3z(int n) { return kS3.z[n]; }
__host__ __device__ constexpr int s3p(int n) { return kS3.partner[n]; }
__host__ __device__ constexpr double s3w(int n) { return e8w3(s3x(n) * s3x(n) + s3y(n) * s3y(n) + s3z(n) * s3z(n)); }

// ---------------------------------------------------------------------------
// Parameters of a 3-D run (kernel argument)
// ---------------------------------------------------------------------------
template <class C> struct KParams3 {
    const void *A;  // post-collision set at t-1 (read)
    void *B;        // post-collision set at t   (written)
    int nx, ny, nz;
    unsigned flags;
    int bricks_x, bricks_y, bricks_z, n_units;
    PsiPair<C> *psi;  // psi = rho of both components per node (density pass output)
    unsigned tick;
    long long N;
    C omega, half, negGc, Gw1, Gw2, s1, s2, s3, t2, t3, delta;
    C omw, cf3, cf9;
    C omega_rho0[2];
    C g[2][3];
    C rho0[2];
    double *out_rho1, *out_rho2, *out_ux, *out_uy, *out_uz;
    double *partials;
};

template <int S> struct PopMem3 {
    __amdgpu_buffer_rsrc_t r[2];
    uint32_t dstride;
};

template <int S>
__device__ __forceinline__ PopMem3<S> make_mem3(const void *base, long long N)
{
    using R = typename Traits<S>::raw_t;
    PopMem3<S> m;
    const uint32_t ds = (uint32_t)(N * (long long)sizeof(R));
    for (int k = 0; k < 2; ++k)
        m.r[k] = __builtin_amdgcn_make_buffer_rsrc((char *)base + (long long)k * 19 * N * (long long)sizeof(R),
                                                   (short)0, (int)(19u * ds), lbm::BUF_RSRC_WORD3);
    m.dstride = ds;
    return m;
}

template <int S>
__device__ __forceinline__ typename Traits<S>::raw_t load3(const PopMem3<S> &m, int k, int i, uint32_t voff)
{
    using R = typename Traits<S>::raw_t;
    const int soff = (int)((uint32_t)i * m.dstride);
    if constexpr (sizeof(R) == 8) {
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(m.r[k], voff, soff, 0));
    } else if constexpr (sizeof(R) == 4) {
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(m.r[k], voff, soff, 0));
    } else {
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b16(m.r[k], voff, soff, 0));
    }
}

template <int S>
__device__ __forceinline__ void store3(const PopMem3<S> &m, int k, int i, uint32_t voff, typename Traits<S>::raw_t v)
{
    using R = typename Traits<S>::raw_t;
    const int soff = (int)((uint32_t)i * m.dstride);
    if constexpr (sizeof(R) == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v),
                                              m.r[k], voff, soff, 0);
    } else if constexpr (sizeof(R) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), m.r[k], voff, soff, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), m.r[k], voff, soff, 0);
    }
}

template <int S> struct Raw3 {
    typename Traits<S>::raw_t v[2][19];
};

// Source x - e_i of direction i for a node with axes (ax, ay, az), and
// whether it lies inside the domain.
__device__ __forceinline__ uint32_t src_node3(int i, const Axis &ax, const Axis &ay, const Axis &az, int nx, int ny,
                                              bool &ok)
{
    const int ex = dx3(i), ey = dy3(i), ez = dz3(i);
    const int col = ex == 1 ? ax.m : (ex == -1 ? ax.p : ax.c);
    const int row = ey == 1 ? ay.m : (ey == -1 ? ay.p : ay.c);
    const int pl = ez == 1 ? az.m : (ez == -1 ? az.p : az.c);
    ok = (ex == 1 ? ax.okm : (ex == -1 ? ax.okp : true)) && (ey == 1 ? ay.okm : (ey == -1 ? ay.okp : true)) &&
         (ez == 1 ? az.okm : (ez == -1 ? az.okp : true));
    return ((uint32_t)pl * (uint32_t)ny + (uint32_t)row) * (uint32_t)nx + (uint32_t)col;
}

// Issue the loads of f*_i(x - e_i, t-1) of one node (pull streaming,
// Eq. 1); sources outside the domain and invalid nodes get an out-of-range
// offset (the load returns 0 without traffic).
template <int S>
__device__ __forceinline__ void issue3(const PopMem3<S> &m, int nx, int ny, const Axis &ax, const Axis &ay,
                                       const Axis &az, bool valid, Raw3<S> &q)
{
    using R = typename Traits<S>::raw_t;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        bool ok;
        const uint32_t src = src_node3(i, ax, ay, az, nx, ny, ok);
        const uint32_t voff = (valid && ok) ? src * (uint32_t)sizeof(R) : lbm::OOB;
#pragma unroll
        for (int k = 0; k < 2; ++k) q.v[k][i] = load3<S>(m, k, i, voff);
    }
}

// Pulled values of one node -> the populations f_i(x, t) (deviations), with
// halfway bounce-back f_i = f*_opp(i)(x, t-1) where the source is
// unavailable; returns false for a solid (or invalid) node.  The densities
// (Eq. 3) follow in the definition's summation order.
template <int S>
__device__ __forceinline__ bool pull3(const KParams3<typename Traits<S>::C> &p, const PopMem3<S> &m, const Axis &ax,
                                      const Axis &ay, const Axis &az, bool valid, const Raw3<S> &q,
                                      typename Traits<S>::C (&f)[2][19], typename Traits<S>::C &r1,
                                      typename Traits<S>::C &r2)
{
    using T = Traits<S>;
    using C = typename T::C;
    using R = typename T::raw_t;
    if (!valid || T::sent(q.v[0][0])) return false;
    C s1 = 0, s2 = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        bool ok;
        (void)src_node3(i, ax, ay, az, p.nx, p.ny, ok);
        f[0][i] = ok ? T::dec(q.v[0][i]) : T::dec(T::sentinel());
        f[1][i] = ok ? T::dec(q.v[1][i]) : T::dec(T::sentinel());
        s1 += f[0][i];
        s2 += f[1][i];
    }
    if (__builtin_isnan(s1 + s2)) {
        // an unavailable source: reflect the node's own post-collision value
        const uint32_t self = (((uint32_t)az.c * (uint32_t)p.ny + (uint32_t)ay.c) * (uint32_t)p.nx + (uint32_t)ax.c) *
                              (uint32_t)sizeof(R);
        s1 = 0;
        s2 = 0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            bool ok;
            (void)src_node3(i, ax, ay, az, p.nx, p.ny, ok);
            if (i > 0 && (!ok || T::sent(q.v[0][i]))) {
                f[0][i] = T::dec(load3<S>(m, 0, opp3(i), self));
                f[1][i] = T::dec(load3<S>(m, 1, opp3(i), self));
            }
            s1 += f[0][i];
            s2 += f[1][i];
        }
    }
    r1 = s1 + p.rho0[0];
    r2 = s2 + p.rho0[1];
    return true;
}

// Reduction accumulators (FP64).
struct RedAcc3 {
    double m1 = 0, m2 = 0, px = 0, py = 0, pz = 0, umax = 0, rmin = __builtin_inf(), rmax = -__builtin_inf(), bad = 0;
};

// Eq. 11 (local adhesion parameter of component 1).
template <class C>
__device__ __forceinline__ C local_G3(const KParams3<C> &p, C re)
{
    if (re > p.delta) return p.Gw1;
    if (re > (C)0) return p.s1 + p.s2 * re + p.s3 * re * re;
    if (re > -p.delta) return p.s1 + p.t2 * re + p.t3 * re * re;
    return p.Gw2;
}

// The stencil again as a table in constant memory, for the near-wall path,
// which walks it in a loop that is not unrolled (it runs only where a wall
// is within two nodes, and unrolled it would take twice the registers of
// everything else).  One 32-bit word per opposite pair (n, n + 1), so that
// the uniform loop index turns each entry into one scalar load (bytes
// would take vector loads, and every such wait would also drain the
// population loads in flight): bits 0-8 the offset e_n (x, y, z, each + 2
// in 3 bits), bit 9 set for a second-layer position, bits 10-18 its
// first-layer partner (same coding).  Position n + 1 and its partner are
// the negations.  The weight W(|e_n|^2) goes beside it.
struct NearTable3 {
    uint32_t code[NS3 / 2];
    double w[NS3 / 2];
};

constexpr NearTable3 make_near3()
{
    NearTable3 t{};
    for (int q = 0; q < NS3 / 2; ++q) {
        const int n = 2 * q, x = kS3.x[n], y = kS3.y[n], z = kS3.z[n], m = kS3.partner[n];
        uint32_t c = (uint32_t)(x + 2) | (uint32_t)(y + 2) << 3 | (uint32_t)(z + 2) << 6;
        if (m >= 0)
            c |= 1u << 9 | (uint32_t)(kS3.x[m] + 2) << 10 | (uint32_t)(kS3.y[m] + 2) << 13 |
                 (uint32_t)(kS3.z[m] + 2) << 16;
        t.code[q] = c;
        t.w[q] = e8w3(x * x + y * y + z * z);
    }
    return t;
}

__constant__ NearTable3 c_near3 = make_near3();

// A brick of BXB x BYB x BZB nodes and its psi tile (2-node halo).
template <int BXB, int BYB, int BZB> struct Brick {
    static constexpr int TX = BXB + 4, TY = BYB + 4, TZ = BZB + 4, NT = BXB * BYB;
    static constexpr int at(int x, int y, int z) { return (z * TY + y) * TX + x; }  // tile coordinates
};

// Stencil value at offset (dx, dy, dz) from tile index c after the wall
// rules (Sec. 2.4): an unavailable first-layer position reads zero (psi(x)
// under WALLPSI_SELF), an unavailable second-layer one what its partner m
// resolves to (zero under E8_COPY_OFF).  `solid` returns the switch s of
// Eq. 9 there.
template <class C>
__device__ __forceinline__ PsiPair<C> resolve3(const PsiPair<C> *tile, int c, int off, bool second, int poff,
                                               PsiPair<C> first, unsigned flags, bool &solid)
{
    const PsiPair<C> v = tile[c + off];
    solid = lds_sent(v.a);
    if (!solid) return v;
    if (!second) return first;
    if (flags & F3_COPY_OFF) {
        PsiPair<C> zero;
        zero.a = 0;
        zero.b = 0;
        return zero;
    }
    const PsiPair<C> w = tile[c + poff];
    return lds_sent(w.a) ? first : w;
}

// Cohesion and adhesion sums at a node with unavailable stencil positions,
// by opposite pairs in the order of the bulk path.
template <class BR, class C>
__device__ __forceinline__ void near_sums3(const PsiPair<C> *tile, int c, C r1, C r2, unsigned flags, C (&s1)[3],
                                           C (&s2)[3], C (&Sv)[3])
{
    PsiPair<C> first;
    first.a = (flags & F3_WALLPSI_SELF) ? r1 : (C)0;
    first.b = (flags & F3_WALLPSI_SELF) ? r2 : (C)0;
    for (int d = 0; d < 3; ++d) {
        s1[d] = 0;
        s2[d] = 0;
        Sv[d] = 0;
    }
#pragma unroll 1
    for (int q = 0; q < NS3 / 2; ++q) {
        const uint32_t code = c_near3.code[q];
        const int ex = (int)(code & 7u) - 2, ey = (int)(code >> 3 & 7u) - 2, ez = (int)(code >> 6 & 7u) - 2;
        const bool second = (code >> 9) & 1u;
        // tile offsets are linear in (x, y, z): the opposite's is the negation
        const int off = BR::at(ex, ey, ez);
        const int poff = BR::at((int)(code >> 10 & 7u) - 2, (int)(code >> 13 & 7u) - 2, (int)(code >> 16 & 7u) - 2);
        bool ua, ub;
        const PsiPair<C> a = resolve3<C>(tile, c, off, second, poff, first, flags, ua);
        const PsiPair<C> b = resolve3<C>(tile, c, -off, second, -poff, first, flags, ub);
        const C w = (C)c_near3.w[q];
        const C d1 = a.a - b.a, d2 = a.b - b.b, ds = (C)(int)ua - (C)(int)ub;
        // the same products and order as the unrolled bulk path (w times
        // +-1 or +-2 is exact, so w e is the bulk path's constant)
        if (ex != 0) { const C wx = w * (C)ex; s1[0] += wx * d1; s2[0] += wx * d2; Sv[0] += wx * ds; }
        if (ey != 0) { const C wy = w * (C)ey; s1[1] += wy * d1; s2[1] += wy * d2; Sv[1] += wy * ds; }
        if (ez != 0) { const C wz = w * (C)ez; s1[2] += wz * d1; s2[2] += wz * d2; Sv[2] += wz * ds; }
    }
}

#ifndef LBM3_PAIRS_PER_FENCE
#define LBM3_PAIRS_PER_FENCE 8
#endif
constexpr int PAIRS_PER_FENCE = LBM3_PAIRS_PER_FENCE;

// Finish node `node` (tile index c): populations from the pull, stencil
// sums from the psi tile, forces (Eq. 8-11 and the body force), velocity
// (Eq. 5), BGK + Guo collision (Eq. 1-2, 6-7), outputs.
template <int S, class BR, int MODE>
__device__ __forceinline__ void finish3(const KParams3<typename Traits<S>::C> &p, const PopMem3<S> &mr,
                                       const PopMem3<S> &mw, const Axis &ax, const Axis &ay, const Axis &az,
                                       const Raw3<S> &q, const PsiPair<typename Traits<S>::C> *tile, int c,
                                       uint32_t node, RedAcc3 &acc)
{
    using T = Traits<S>;
    using C = typename T::C;
    using R = typename T::raw_t;
    const PsiPair<C> ctr = tile[c];
    if (lds_sent(ctr.a)) {  // solid node
        if (MODE & K3_FIELDS) {
            p.out_rho1[node] = 0.0;
            p.out_rho2[node] = 0.0;
            p.out_ux[node] = 0.0;
            p.out_uy[node] = 0.0;
            p.out_uz[node] = 0.0;
        }
        return;
    }
    C f[2][19];
    C pr1, pr2;
    (void)pull3<S>(p, mr, ax, ay, az, true, q, f, pr1, pr2);
    const C r1 = ctr.a, r2 = ctr.b;  // bitwise pr1, pr2: the density pass pulled the same values

    // momenta j_k = sum_i f_i e_i (Eq. 4)
    C j[2][3];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        C a = 0, b = 0, cc = 0;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            if (dx3(i) == 1) a += f[k][i];
            if (dx3(i) == -1) a -= f[k][i];
            if (dy3(i) == 1) b += f[k][i];
            if (dy3(i) == -1) b -= f[k][i];
            if (dz3(i) == 1) cc += f[k][i];
            if (dz3(i) == -1) cc -= f[k][i];
        }
        j[k][0] = a;
        j[k][1] = b;
        j[k][2] = cc;
    }

    // cohesion sums over the 46 opposite pairs; a sentinel turns them into
    // NaN and selects the wall path
    C s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
#pragma unroll
    for (int n = 0; n < NS3; n += 2) {
        // a compiler-only fence every few pairs keeps the LDS reads of the
        // stencil from all being hoisted at once (register pressure)
        if (n % (2 * PAIRS_PER_FENCE) == 0) asm volatile("" ::: "memory");
        const PsiPair<C> a = tile[c + BR::at(s3x(n), s3y(n), s3z(n))];
        const PsiPair<C> b = tile[c + BR::at(s3x(n + 1), s3y(n + 1), s3z(n + 1))];
        const C d1 = a.a - b.a, d2 = a.b - b.b;
        const C wx = (C)(s3w(n) * s3x(n)), wy = (C)(s3w(n) * s3y(n)), wz = (C)(s3w(n) * s3z(n));
        if (s3x(n) != 0) { s1[0] += wx * d1; s2[0] += wx * d2; }
        if (s3y(n) != 0) { s1[1] += wy * d1; s2[1] += wy * d2; }
        if (s3z(n) != 0) { s1[2] += wz * d1; s2[2] += wz * d2; }
    }
    C Sv[3] = {0, 0, 0};
    const bool near = __builtin_isnan(s1[0] + s1[1] + s1[2] + s2[0] + s2[1] + s2[2]);
    if (near) {
        asm volatile("" ::: "memory");
        near_sums3<BR, C>(tile, c, r1, r2, p.flags, s1, s2, Sv);
    }
    // forces: cohesion (Eq. 8) + adhesion (Eq. 9, 11) + body force
    C F[2][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        F[0][d] = (p.negGc * r1) * s2[d];
        F[1][d] = (p.negGc * r2) * s1[d];
    }
    if (near) {
        C G1 = p.Gw1;
        if (!(p.flags & F3_ORIGINAL)) G1 = local_G3<C>(p, (r1 - r2) / (r1 + r2));
        const C a1 = -G1 * r1, a2 = -p.Gw2 * r2;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            F[0][d] += a1 * Sv[d];
            F[1][d] += a2 * Sv[d];
        }
    }
    const bool fdens = p.flags & F3_FORCE_DENSITY;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        F[0][d] += (fdens ? (C)1 : r1) * p.g[0][d];
        F[1][d] += (fdens ? (C)1 : r2) * p.g[1][d];
    }

    // u^eq (Eq. 5 with the half-force shift)
    const C irt = lbm::recip(r1 + r2);
    C u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = ((j[0][d] + p.half * F[0][d]) + (j[1][d] + p.half * F[1][d])) * irt;

    if (MODE & K3_FIELDS) {
        p.out_rho1[node] = (double)r1;
        p.out_rho2[node] = (double)r2;
        p.out_ux[node] = (double)u[0];
        p.out_uy[node] = (double)u[1];
        p.out_uz[node] = (double)u[2];
    }
    if (MODE & K3_REDUCE) {
        const double d1 = r1, d2 = r2, a = u[0], b = u[1], w = u[2];
        if (!__builtin_isfinite(d1) || !__builtin_isfinite(d2) || !__builtin_isfinite(a) || !__builtin_isfinite(b) ||
            !__builtin_isfinite(w)) {
            acc.bad += 1.0;
        } else {
            const double rt = d1 + d2;
            acc.m1 += d1;
            acc.m2 += d2;
            acc.px += rt * a;
            acc.py += rt * b;
            acc.pz += rt * w;
            const double um = __builtin_sqrt(a * a + b * b + w * w);
            acc.umax = um > acc.umax ? um : acc.umax;
            acc.rmin = d1 < acc.rmin ? d1 : acc.rmin;
            acc.rmax = d1 > acc.rmax ? d1 : acc.rmax;
        }
    }

    if (MODE & K3_STORE) {
        // deviation form of BGK + Guo (as in 2-D): g* = (1 - omega) g + w T_i,
        // T_i = c0 + c1 e.u + c2 (e.u)^2 + (e.F)(3 cf + 9 cf e.u), by
        // opposite pairs (i, i+1): T = E +- O
        const C a0 = (C)1 - (C)1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const C rho[2] = {r1, r2};
        C c0[2], c1[2], c2[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const C wr = p.omega * rho[k];
            const C uF = u[0] * F[k][0] + u[1] * F[k][1] + u[2] * F[k][2];
            c0[k] = wr * a0 - p.omega_rho0[k] - p.cf3 * uF;
            c1[k] = (C)3 * wr;
            c2[k] = (C)4.5 * wr;
        }
        constexpr bool sr = (S == lbm::ST_F16 || S == lbm::ST_BF16) && (MODE & K3_SR);
        uint32_t rs = sr ? lbm::sr_seed((int)node, p.tick) : 1u;
        C gs[2][19];
#pragma unroll
        for (int k = 0; k < 2; ++k) gs[k][0] = p.omw * f[k][0] + (C)w3(0) * c0[k];
#pragma unroll
        for (int i = 1; i < 19; i += 2) {
            const int o = i + 1;
            const C w = (C)w3(i);
            const int ex = dx3(i), ey = dy3(i), ez = dz3(i);
            C eu = 0;
            if (ex != 0) eu += (C)ex * u[0];
            if (ey != 0) eu += (C)ey * u[1];
            if (ez != 0) eu += (C)ez * u[2];
            const C eu2 = eu * eu;
            const C h9 = p.cf9 * eu;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                C eF = 0;
                if (ex != 0) eF += (C)ex * F[k][0];
                if (ey != 0) eF += (C)ey * F[k][1];
                if (ez != 0) eF += (C)ez * F[k][2];
                const C E = (c0[k] + c2[k] * eu2) + h9 * eF;
                const C O = c1[k] * eu + p.cf3 * eF;
                gs[k][i] = p.omw * f[k][i] + w * (E + O);
                gs[k][o] = p.omw * f[k][o] + w * (E - O);
            }
        }
        const uint32_t voff = node * (uint32_t)sizeof(R);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            R o0, o1;
            if constexpr (sr) {
                const uint32_t rw = lbm::xorshift32(rs);
                T::enc_sr2(gs[0][i], gs[1][i], rw, o0, o1);
            } else {
                o0 = T::enc(gs[0][i]);
                o1 = T::enc(gs[1][i]);
            }
            store3<S>(mw, 0, i, voff, o0);
            store3<S>(mw, 1, i, voff, o1);
        }
    }
}

template <int NT>
__device__ void block_reduce3(const RedAcc3 &acc, double *out)
{
    constexpr int NW = NT / 64;
    __shared__ double red[9][NW];
    auto wsum = [](double v) {
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
        return v;
    };
    auto wmax = [](double v) {
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            const double o = __shfl_xor(v, m, 64);
            v = o > v ? o : v;
        }
        return v;
    };
    auto wmin = [](double v) {
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            const double o = __shfl_xor(v, m, 64);
            v = o < v ? o : v;
        }
        return v;
    };
    const double r[9] = {wsum(acc.m1), wsum(acc.m2), wsum(acc.px), wsum(acc.py), wsum(acc.pz),
                         wmax(acc.umax), wmin(acc.rmin), wmax(acc.rmax), wsum(acc.bad)};
    const int t = threadIdx.x;
    if ((t & 63) == 0)
        for (int q = 0; q < 9; ++q) red[q][t >> 6] = r[q];
    __syncthreads();
    if (t == 0) {
        double v[9];
        for (int q = 0; q < 9; ++q) v[q] = red[q][0];
        for (int w = 1; w < NW; ++w) {
            for (int q = 0; q < 5; ++q) v[q] += red[q][w];
            v[5] = red[5][w] > v[5] ? red[5][w] : v[5];
            v[6] = red[6][w] < v[6] ? red[6][w] : v[6];
            v[7] = red[7][w] > v[7] ? red[7][w] : v[7];
            v[8] += red[8][w];
        }
        for (int q = 0; q < 9; ++q) out[q] = v[q];
    }
}

// Density pass: psi = rho of both components at every node (Eq. 3 on the
// pulled populations, Eq. 1 streaming with halfway bounce-back), the
// all-ones sentinel at solid nodes.  One thread per node.
template <int S>
__global__ void __launch_bounds__(256) k_density3(const KParams3<typename Traits<S>::C> p)
{
    using C = typename Traits<S>::C;
    // 32-bit index arithmetic: a lattice has fewer than 2^31 nodes
    const uint32_t id = blockIdx.x * 256u + threadIdx.x;
    if (id >= (uint32_t)p.N) return;
    const uint32_t plane = (uint32_t)p.nx * (uint32_t)p.ny;
    const uint32_t zu = id / plane, rem = id - zu * plane, yu = rem / (uint32_t)p.nx;
    const int z = (int)zu, y = (int)yu, x = (int)(rem - yu * (uint32_t)p.nx);
    // coordinates inside the lattice: wrapping needs no division
    const Axis ax = make_axis_near(x, p.nx, p.flags & F3_PERIODIC_X);
    const Axis ay = make_axis_near(y, p.ny, p.flags & F3_PERIODIC_Y);
    const Axis az = make_axis_near(z, p.nz, p.flags & F3_PERIODIC_Z);
    const PopMem3<S> m = make_mem3<S>(p.A, p.N);
    Raw3<S> q;
    issue3<S>(m, p.nx, p.ny, ax, ay, az, true, q);
    C f[2][19], r1 = 0, r2 = 0;
    const bool fluid = pull3<S>(p, m, ax, ay, az, true, q, f, r1, r2);
    PsiPair<C> ps;
    ps.a = fluid ? r1 : lds_sentinel<C>();
    ps.b = fluid ? r2 : lds_sentinel<C>();
    p.psi[id] = ps;
}

// Collide pass over bricks of BXB x BYB x BZB nodes.  The workgroup has
// BXB x BYB x TZ threads: thread (x, y, t) finishes planes t, t + TZ, ...
// of its column (TZ = BZB: one node per thread; TZ < BZB: a short march,
// the next node's loads issued before the current one is finished).  The
// FP32 stepping instances are held to 128 registers (four waves per SIMD,
// a few values spilled), which lets two 512-thread workgroups share a CU.
// Grid: 8 * per_xcd workgroups; workgroup b takes brick (b % 8) * per_xcd
// + b / 8, so each XCD works on a contiguous run of bricks (numbered x
// fastest, then y, then z), whose psi halos meet in that XCD's L2.
template <int S, int BXB, int BYB, int BZB, int TZ, int MODE>
__global__ void __launch_bounds__(BXB * BYB * TZ)
__attribute__((amdgpu_waves_per_eu((S == lbm::ST_F32 && !(MODE & K3_REDUCE)) ? 4 : 1))) k_collide3(const KParams3<typename Traits<S>::C> p, int per_xcd)
{
    using C = typename Traits<S>::C;
    using BR = Brick<BXB, BYB, BZB>;
    constexpr int NTH = BXB * BYB * TZ;
    static_assert(BZB % TZ == 0, "the brick depth must be a multiple of the threads in z");
    __shared__ PsiPair<C> tile[BR::TX * BR::TY * BR::TZ];
    const int b = blockIdx.x;
    const int unit = (b & 7) * per_xcd + (b >> 3);
    const int tid = threadIdx.x;
    RedAcc3 acc;
    if (unit < p.n_units) {
        const int bxi = unit % p.bricks_x, rest = unit / p.bricks_x;
        const int byi = rest % p.bricks_y, bzi = rest / p.bricks_y;
        const int x0 = bxi * BXB, y0 = byi * BYB, z0 = bzi * BZB;
        const bool wx = p.flags & F3_PERIODIC_X, wy = p.flags & F3_PERIODIC_Y, wz = p.flags & F3_PERIODIC_Z;
        // psi of the brick and its halo (outside a closed face: the sentinel)
        for (int t = tid; t < BR::TX * BR::TY * BR::TZ; t += NTH) {
            const int lx = t % BR::TX, r = t / BR::TX;
            const int ly = r % BR::TY, lz = r / BR::TY;
            // (a brick may be wider than a small periodic lattice: full wrap)
            const Axis gx = make_axis(x0 - 2 + lx, p.nx, wx);
            const Axis gy = make_axis(y0 - 2 + ly, p.ny, wy);
            const Axis gz = make_axis(z0 - 2 + lz, p.nz, wz);
            PsiPair<C> v;
            if (gx.ok && gy.ok && gz.ok) {
                v = p.psi[((long long)gz.c * p.ny + gy.c) * p.nx + gx.c];
            } else {
                v.a = lds_sentinel<C>();
                v.b = lds_sentinel<C>();
            }
            tile[t] = v;
        }
        __syncthreads();
        const int lx = tid % BXB, ly = (tid / BXB) % BYB, lt = tid / (BXB * BYB);
        const int x = x0 + lx, y = y0 + ly;
        if (x < p.nx && y < p.ny) {
            const PopMem3<S> mr = make_mem3<S>(p.A, p.N);
            const PopMem3<S> mw = make_mem3<S>(p.B, p.N);
            // the thread's own node lies inside the lattice: no division
            const Axis ax = make_axis_near(x, p.nx, wx);
            const Axis ay = make_axis_near(y, p.ny, wy);
            const int zend = z0 + BZB < p.nz ? z0 + BZB : p.nz;
            const int zs = z0 + lt;
            Raw3<S> q;
            if (zs < zend) {
                const Axis az = make_axis_near(zs, p.nz, wz);
                const bool solid = lds_sent(tile[BR::at(lx + 2, ly + 2, lt + 2)].a);
                issue3<S>(mr, p.nx, p.ny, ax, ay, az, !solid, q);
            }
            for (int z = zs; z < zend; z += TZ) {
                const Axis az = make_axis_near(z, p.nz, wz);
                const int c = BR::at(lx + 2, ly + 2, z - z0 + 2);
                const uint32_t node = ((uint32_t)z * (uint32_t)p.ny + (uint32_t)y) * (uint32_t)p.nx + (uint32_t)x;
                Raw3<S> cur = q;
                // the next node's loads go out before this one is finished
                if constexpr (TZ < BZB) {
                    if (z + TZ < zend) {
                        const Axis azn = make_axis_near(z + TZ, p.nz, wz);
                        const bool solid = lds_sent(tile[c + BR::at(0, 0, TZ)].a);
                        issue3<S>(mr, p.nx, p.ny, ax, ay, azn, !solid, q);
                    }
                }
                finish3<S, BR, MODE>(p, mr, mw, ax, ay, az, cur, tile, c, node, acc);
            }
        }
    }
    if (MODE & K3_REDUCE) {
        __syncthreads();
        block_reduce3<NTH>(acc, p.partials + (long long)b * 9);
    }
}

// Deterministic compensated (Neumaier) sums of the workgroup partials in a
// fixed order; one workgroup of 256 threads.
static __global__ void __launch_bounds__(256) k_reduce3_final(const double *__restrict__ partials, int nparts, double *out)
{
    __shared__ double s[6][256], cmp[6][256], mx[3][256];
    const int t = threadIdx.x;
    const int idx[6] = {0, 1, 2, 3, 4, 8};
    double sum[6] = {0, 0, 0, 0, 0, 0}, c[6] = {0, 0, 0, 0, 0, 0};
    double umax = 0, rmin = __builtin_inf(), rmax = -__builtin_inf();
    for (int j = t; j < nparts; j += 256) {
        const double *q = partials + (long long)j * 9;
        for (int a = 0; a < 6; ++a) {
            const double v = q[idx[a]], tt = sum[a] + v;
            c[a] += (__builtin_fabs(sum[a]) >= __builtin_fabs(v)) ? (sum[a] - tt) + v : (v - tt) + sum[a];
            sum[a] = tt;
        }
        umax = q[5] > umax ? q[5] : umax;
        rmin = q[6] < rmin ? q[6] : rmin;
        rmax = q[7] > rmax ? q[7] : rmax;
    }
    for (int a = 0; a < 6; ++a) {
        s[a][t] = sum[a];
        cmp[a][t] = c[a];
    }
    mx[0][t] = umax;
    mx[1][t] = rmin;
    mx[2][t] = rmax;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            for (int a = 0; a < 6; ++a) {
                const double x = s[a][t], v = s[a][t + h], tt = x + v;
                cmp[a][t] += cmp[a][t + h] + ((__builtin_fabs(x) >= __builtin_fabs(v)) ? (x - tt) + v : (v - tt) + x);
                s[a][t] = tt;
            }
            mx[0][t] = mx[0][t] > mx[0][t + h] ? mx[0][t] : mx[0][t + h];
            mx[1][t] = mx[1][t] < mx[1][t + h] ? mx[1][t] : mx[1][t + h];
            mx[2][t] = mx[2][t] > mx[2][t + h] ? mx[2][t] : mx[2][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int a = 0; a < 5; ++a) out[a] = s[a][0] + cmp[a][0];
        out[5] = mx[0][0];
        out[6] = mx[1][0];
        out[7] = mx[2][0];
        out[8] = s[5][0] + cmp[5][0];
    }
}

// Post-collision set whose streaming gives f(t): slot (z, j) is pulled by
// z + e_j when that position is available, else by z itself as the
// bounce-back of opp(j); so f*_j(z) = f_j(z + e_j) or f_opp(j)(z).  From
// FP64 f [2][19][N], or with `rho` [2][N] from f_i = w_i rho_k.
template <int S>
__global__ void __launch_bounds__(256)
k_inverse3(const KParams3<typename Traits<S>::C> p, const uint8_t *__restrict__ solid, const double *__restrict__ fsrc,
           const double *__restrict__ rho)
{
    using T = Traits<S>;
    using C = typename T::C;
    const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
    if (id >= p.N || solid[id]) return;
    const PopMem3<S> m = make_mem3<S>(p.B, p.N);
    const int x = (int)(id % p.nx), y = (int)((id / p.nx) % p.ny), z = (int)(id / ((long long)p.nx * p.ny));
#pragma unroll
    for (int j = 0; j < 19; ++j) {
        const Axis ax = make_axis(x + dx3(j), p.nx, p.flags & F3_PERIODIC_X);
        const Axis ay = make_axis(y + dy3(j), p.ny, p.flags & F3_PERIODIC_Y);
        const Axis az = make_axis(z + dz3(j), p.nz, p.flags & F3_PERIODIC_Z);
        const long long nb = ((long long)az.c * p.ny + ay.c) * p.nx + ax.c;
        const bool avail = ax.ok && ay.ok && az.ok && !solid[nb];
        for (int k = 0; k < 2; ++k) {
            double v;
            if (rho) v = w3(j) * rho[(long long)k * p.N + (avail ? nb : id)];
            else v = avail ? fsrc[(long long)(k * 19 + j) * p.N + nb] : fsrc[(long long)(k * 19 + opp3(j)) * p.N + id];
            const double base = T::deviation ? w3(j) * (double)p.rho0[k] : 0.0;
            store3<S>(m, k, j, (uint32_t)id * (uint32_t)sizeof(typename T::raw_t), T::enc((C)(v - base)));
        }
    }
}

// Pre-collision populations f(x, t) = g + w_i rho0 (FP64, solid -> 0) of
// every node, [2][19][N], by the step's own pull.
template <int S>
__global__ void __launch_bounds__(256)
k_pull3_all(const KParams3<typename Traits<S>::C> p, double *__restrict__ out)
{
    using T = Traits<S>;
    using C = typename T::C;
    const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
    if (id >= p.N) return;
    const int x = (int)(id % p.nx), y = (int)((id / p.nx) % p.ny), z = (int)(id / ((long long)p.nx * p.ny));
    const Axis ax = make_axis(x, p.nx, p.flags & F3_PERIODIC_X);
    const Axis ay = make_axis(y, p.ny, p.flags & F3_PERIODIC_Y);
    const Axis az = make_axis(z, p.nz, p.flags & F3_PERIODIC_Z);
    const PopMem3<S> m = make_mem3<S>(p.A, p.N);
    Raw3<S> q;
    issue3<S>(m, p.nx, p.ny, ax, ay, az, true, q);
    C f[2][19], r1, r2;
    const bool fluid = pull3<S>(p, m, ax, ay, az, true, q, f, r1, r2);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double base = T::deviation ? w3(i) * (double)p.rho0[k] : 0.0;
            out[(long long)(k * 19 + i) * p.N + id] = fluid ? (double)f[k][i] + base : 0.0;
        }
}

}  // namespace lbm3
