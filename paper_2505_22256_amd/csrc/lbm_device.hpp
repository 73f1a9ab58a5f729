// Device building blocks of the fused two-component pseudopotential LBM
// step for gfx950 (arXiv 2505.22256, Sec. 2.1-2.4, Eq. 1-12, Table 1).
//
// Data layout in HBM: one population set per buffer, structure of arrays
// [component k][direction i][node], node = y*nx + x.  Solid nodes carry an
// all-ones bit pattern (a NaN that arithmetic never produces) in every
// population slot, so the step kernel reads no geometry array: a pulled
// sentinel marks a solid source (bounce-back), a sentinel at the node's own
// rest slot marks a solid node, and a sentinel psi in the LDS tile marks an
// unavailable stencil position.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum Storage : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

enum : unsigned {
    FL_PERIODIC_X = 1u,
    FL_PERIODIC_Y = 2u,
    FL_ORIGINAL = 4u,
    FL_COPY_OFF = 8u,
    FL_WALLPSI_SELF = 16u,
    FL_VEL_LITERAL = 32u,
    FL_FORCE_DENSITY = 64u,
    FL_ROUND_STOCHASTIC = 128u,
    FL_INLET = 256u,    // Zou-He velocity inlet at x = 0 (Sec. 3.3)
    FL_OUTFLOW = 512u,  // zero-gradient outflow at x = nx - 1 (Sec. 3.3)
    FL_ROUND_NEAREST = 1024u,  // 16-bit storage rounds to nearest even (resolved on the host)
    FL_ALL = 2047u
};

// Kernel modes (bit set).
enum : int {
    M_STORE = 1,   // collide and write the post-collision set
    M_REDUCE = 2,  // per-workgroup diagnostic partial sums
    M_FIELDS = 4,  // write rho_1, rho_2, u (FP64)
    M_TABLES = 8,  // write link bits and resolved stencil sources
    M_SR = 16,     // stochastic rounding of FP16 / BF16 stores (compile-time)
    M_LDS = 32,    // first of two fused steps: post-collision values to the LDS ring
    M_TWO = 64,    // kernel advances two steps per launch
    M_DIAG_FIRST = 128,  // two steps: M_REDUCE records the first step (else the second)
    M_BND = 256,         // open and moving boundaries compiled in (else plain walls only)
    M_REPULL = 512       // two steps: the first step pulls a row again when it finishes it
};

// ---------------------------------------------------------------------------
// D2Q9 and E8 constants
// ---------------------------------------------------------------------------
// D2Q9: e_0 = 0, e_1..4 axis links, e_5..8 diagonals.
__host__ __device__ constexpr int qx(int i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); }
__host__ __device__ constexpr int qy(int i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); }
// opposite direction: 1<->3, 2<->4, 5<->7, 6<->8
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
__host__ __device__ constexpr double qw(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

// E8 stencil position n = 0..23 (0-based): n < 8 the D2Q9 links e_1..e_8,
// 8..15 the same links doubled, 16..23 the knight moves.  Within every
// group of four, n and n+2 are opposite.
__host__ __device__ constexpr int sx(int n)
{
    return n < 8 ? qx(n + 1) : n < 16 ? 2 * qx(n - 7)
         : (n == 16 ? 2 : n == 17 ? -1 : n == 18 ? -2 : n == 19 ? 1 : n == 20 ? 1 : n == 21 ? -2 : n == 22 ? -1 : 2);
}
__host__ __device__ constexpr int sy(int n)
{
    return n < 8 ? qy(n + 1) : n < 16 ? 2 * qy(n - 7)
         : (n == 16 ? 1 : n == 17 ? 2 : n == 18 ? -1 : n == 19 ? -2 : n == 20 ? 2 : n == 21 ? 1 : n == 22 ? -2 : -1);
}
// Table 1: second-layer position copies first-layer position n-8 (n=9..16),
// n-12 (17..20) or n-16 (21..24), in 1-based numbering.
__host__ __device__ constexpr int table1(int n) { return n < 8 ? -1 : n < 16 ? n - 8 : n < 20 ? n - 12 : n - 16; }
// Eighth-order isotropic weight by |e|^2, normalised to sum W e_x^2 = 1.
__host__ __device__ constexpr double e8w(int e2)
{
    return e2 == 1 ? 4.0 / 21.0 : e2 == 2 ? 4.0 / 45.0 : e2 == 4 ? 1.0 / 60.0 : e2 == 5 ? 2.0 / 315.0 : e2 == 8 ? 1.0 / 5040.0 : 0.0;
}
__host__ __device__ constexpr double e8wn(int n) { return e8w(sx(n) * sx(n) + sy(n) * sy(n)); }

// Reciprocal in the compute type: exact division in FP64; the hardware
// reciprocal (1 ulp) in FP32.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Storage traits: raw element type, compute type, sentinel, codec
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN -> canonical quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int S> struct Traits;

// dec/enc convert between the stored element and the compute type; the
// stored value is the deviation g = f - w_i rho0_k (rho0 = 0 for FP64), and
// the step works on deviations directly.
template <> struct Traits<ST_F64> {
    using raw_t = double;
    using C = double;
    static constexpr bool deviation = false;
    __device__ static bool sent(raw_t v) { return __double_as_longlong(v) == -1LL; }
    __device__ static C dec(raw_t v) { return v; }
    __device__ static raw_t enc(C g) { return g; }
    __device__ static void enc_sr2(C g0, C g1, uint32_t, raw_t &o0, raw_t &o1)
    {
        o0 = g0;
        o1 = g1;
    }
    __device__ static raw_t sentinel() { return __longlong_as_double(-1LL); }
};
template <> struct Traits<ST_F32> {
    using raw_t = float;
    using C = float;
    static constexpr bool deviation = true;
    __device__ static bool sent(raw_t v) { return __float_as_uint(v) == 0xffffffffu; }
    __device__ static C dec(raw_t v) { return v; }
    __device__ static raw_t enc(C g) { return g; }
    __device__ static void enc_sr2(C g0, C g1, uint32_t, raw_t &o0, raw_t &o1)
    {
        o0 = g0;
        o1 = g1;
    }
    __device__ static raw_t sentinel() { return __uint_as_float(0xffffffffu); }
};
template <> struct Traits<ST_F16> {
    using raw_t = uint16_t;
    using C = float;
    static constexpr bool deviation = true;
    __device__ static bool sent(raw_t v) { return v == 0xffffu; }
    __device__ static C dec(raw_t v) { return (float)__builtin_bit_cast(_Float16, v); }
    __device__ static raw_t enc(C g) { return __builtin_bit_cast(uint16_t, (_Float16)g); }
    // Stochastic rounding of both components of one direction from one
    // 32-bit random word: add 13 random bits below the FP16 mantissa of the
    // FP32 value and truncate them (component 1 takes bits 0-12 of the
    // word, component 2 bits 16-28).  gfx950's conversion instruction does
    // this with the top 13 bits of its random operand, hence the shifts;
    // for results in FP16's normal range it gives exactly the add-and-
    // truncate rule (checked on 4 M values), and it also rounds results in
    // the subnormal range stochastically at their own precision.
    __device__ static void enc_sr2(C g0, C g1, uint32_t r, raw_t &o0, raw_t &o1)
    {
        // (the instruction keeps the other half of its destination; only the
        // written half is read, so the value being converted fills the rest
        // and no register needs clearing)
        typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
        const h2_t v0 = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(h2_t, g0), g0, r << 19, false);
        const h2_t v1 = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(h2_t, g1), g1, r << 3, false);
        o0 = __builtin_bit_cast(uint16_t, v0[0]);
        o1 = __builtin_bit_cast(uint16_t, v1[0]);
    }
    __device__ static raw_t sentinel() { return 0xffffu; }
};
template <> struct Traits<ST_BF16> {
    using raw_t = uint16_t;
    using C = float;
    static constexpr bool deviation = true;
    __device__ static bool sent(raw_t v) { return v == 0xffffu; }
    __device__ static C dec(raw_t v) { return __uint_as_float((uint32_t)v << 16); }
    __device__ static raw_t enc(C g) { return f32_to_bf16_rne(g); }
    // Stochastic rounding of both components of one direction: add 16
    // random bits below the BF16 mantissa and truncate (component 1 takes
    // bits 0-15 of the word, component 2 bits 16-31).  gfx950's conversion
    // instruction does exactly this with the top 16 bits of its random
    // operand (checked on 4 M values of every magnitude).
    __device__ static void enc_sr2(C g0, C g1, uint32_t r, raw_t &o0, raw_t &o1)
    {
        // the builtin returns two BF16 values: reinterpret, never convert
        typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
        const b2_t v0 = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(b2_t, g0), g0, r << 16, false);
        const b2_t v1 = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(b2_t, g1), g1, r, false);
        o0 = __builtin_bit_cast(uint16_t, v0[0]);
        o1 = __builtin_bit_cast(uint16_t, v1[0]);
    }
    __device__ static raw_t sentinel() { return 0xffffu; }
};

// ---------------------------------------------------------------------------
// Population memory through buffer resources: one resource per component
// (its 9 direction arrays, at most 4 GiB), the direction selected by a
// scalar offset, the node by a 32-bit vector offset.  Accesses beyond the
// resource return 0 / are dropped instead of faulting.
// ---------------------------------------------------------------------------
static constexpr int BUF_RSRC_WORD3 = 0x00020000;

template <int S> struct PopMem {
    __amdgpu_buffer_rsrc_t r[2];
    uint32_t dstride;  // bytes between direction arrays
};

template <int S>
__device__ __forceinline__ PopMem<S> make_mem(const void *base, long long N)
{
    using R = typename Traits<S>::raw_t;
    PopMem<S> m;
    const uint32_t ds = (uint32_t)(N * (long long)sizeof(R));
    for (int k = 0; k < 2; ++k)
        m.r[k] = __builtin_amdgcn_make_buffer_rsrc((char *)base + (long long)k * 9 * N * (long long)sizeof(R),
                                                   (short)0, (int)(9u * ds), BUF_RSRC_WORD3);
    m.dstride = ds;
    return m;
}

// Vector offset that lies outside every resource (the load returns 0).
static constexpr uint32_t OOB = 0xffffffffu;

// Cache-policy bits of the population loads and stores (bit 1: nt).
#ifndef LBM_LOAD_AUX
#define LBM_LOAD_AUX 0
#endif
#ifndef LBM_STORE_AUX
#define LBM_STORE_AUX 0
#endif

template <int S>
__device__ __forceinline__ typename Traits<S>::raw_t pop_load(const PopMem<S> &m, int k, int i, uint32_t voff)
{
    using R = typename Traits<S>::raw_t;
    if constexpr (sizeof(R) == 8) {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(m.r[k], voff, (int)((uint32_t)i * m.dstride), LBM_LOAD_AUX);
        return __builtin_bit_cast(R, v);
    } else if constexpr (sizeof(R) == 4) {
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(m.r[k], voff, (int)((uint32_t)i * m.dstride), LBM_LOAD_AUX));
    } else {
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b16(m.r[k], voff, (int)((uint32_t)i * m.dstride), LBM_LOAD_AUX));
    }
}

template <int S>
__device__ __forceinline__ void pop_store(const PopMem<S> &m, int k, int i, uint32_t voff, typename Traits<S>::raw_t v)
{
    using R = typename Traits<S>::raw_t;
    if constexpr (sizeof(R) == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v),
                                              m.r[k], voff, (int)((uint32_t)i * m.dstride), LBM_STORE_AUX);
    } else if constexpr (sizeof(R) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), m.r[k], voff,
                                              (int)((uint32_t)i * m.dstride), LBM_STORE_AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), m.r[k], voff,
                                              (int)((uint32_t)i * m.dstride), LBM_STORE_AUX);
    }
}

// Sentinel psi in the LDS tile (same all-ones pattern in the compute type).
__device__ __forceinline__ bool lds_sent(float v) { return __float_as_uint(v) == 0xffffffffu; }
__device__ __forceinline__ bool lds_sent(double v) { return __double_as_longlong(v) == -1LL; }
template <class C> __device__ __forceinline__ C lds_sentinel();
template <> __device__ __forceinline__ float lds_sentinel<float>() { return __uint_as_float(0xffffffffu); }
template <> __device__ __forceinline__ double lds_sentinel<double>() { return __longlong_as_double(-1LL); }

template <class C> struct alignas(2 * sizeof(C)) PsiPair {
    C a, b;  // psi_1, psi_2
};

// ---------------------------------------------------------------------------
// Per-run parameters (kernel argument, or a device array for batches)
// ---------------------------------------------------------------------------
template <class C> struct KParams {
    const void *A;  // post-collision set at t-1 (read)
    void *B;        // post-collision set at t   (written)
    int nx, ny;
    unsigned flags;
    int n_strips, n_segs;
    int n_units;    // work units of the run (strips * segs, or the resident workgroup count)
    int strip_w;    // > 0: strips of this width from x = 0 (the last one ragged); 0: balanced
    int band_order; // 1: units run across strips first (row bands), 0: down each strip
    int xcd_slabs;  // 1: unit b = (strip b / 8, row slab b % 8): XCD j marches slab j
    int item0;      // first work item of this run in a batch work list
    unsigned tick;  // time step index (stochastic-rounding counter)
    long long N;    // nodes = array stride
    C omega, cforce, half, negGc, Gw1, Gw2, s1, s2, s3, t2, t3, delta;
    C omw, cf3, cf9;     // 1 - omega, 3 (1 - omega/2), 9 (1 - omega/2)
    C omega_rho0[2];     // omega * rho0_k
    C g[2][2];
    C rho0[2];      // deviation base density per component (zero for FP64)
    // open and moving boundaries (Sec. 3.1 sliding walls, Sec. 3.3 inlet and
    // outflow): wall velocity of rows y < ny/2 ([0]) and of the others ([1]);
    // inlet velocity per row [2][ny]; `plain` pulls without these boundary
    // conditions (the state right after it was set, which the populations
    // themselves define)
    C uw[2][2];
    int moving;
    int plain;
    const double *inlet;
    // mode outputs
    double *out_rho1, *out_rho2, *out_ux, *out_uy;
    double *partials;
    uint8_t *tab_link, *tab_nw;
    int32_t *tab_src;
};

// Counter-based random bits for stochastic rounding: a murmur3-style
// finaliser of (node, step) seeds Marsaglia's xorshift32 (shifts 13, 17,
// 5), whose every 32-bit word feeds the two components of one direction
// (low and high half).  Shifts and xors only: no multiply per draw.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t sr_seed(int node, unsigned tick)
{
    return mix32((uint32_t)node ^ mix32(tick * 0x9e3779b9u + 0x632be5abu)) | 1u;  // xorshift state != 0
}
__device__ __forceinline__ uint32_t xorshift32(uint32_t &s)
{
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    return s;
}

// Position along one axis with its two neighbours, after periodic wrapping;
// ok* false when the position falls outside a non-periodic domain.
struct Axis {
    int c, m, p;
    bool ok, okm, okp;
};

// Same as make_axis for a position at most one period outside [0, n).
__device__ __forceinline__ Axis make_axis_near(int v, int n, bool periodic)
{
    Axis a;
    if (periodic) {
        const int w = v < 0 ? v + n : (v >= n ? v - n : v);
        a.c = w;
        a.m = (w == 0) ? n - 1 : w - 1;
        a.p = (w == n - 1) ? 0 : w + 1;
        a.ok = a.okm = a.okp = true;
    } else {
        a.c = v;
        a.m = v - 1;
        a.p = v + 1;
        a.ok = v >= 0 && v < n;
        a.okm = v - 1 >= 0 && v - 1 < n;
        a.okp = v + 1 >= 0 && v + 1 < n;
    }
    return a;
}

// The column axis of the outflow column pulls the populations that enter
// from outside (directions 3, 6, 7) from its own column, rows y - e_iy:
// what the upstream neighbour receives (zero normal gradient).
template <class P>
__device__ __forceinline__ Axis open_axis(Axis a, const P &p)
{
    if ((p.flags & FL_OUTFLOW) && !p.plain && a.c == p.nx - 1) {
        a.p = p.nx - 1;
        a.okp = true;
    }
    return a;
}

__device__ __forceinline__ Axis make_axis(int v, int n, bool periodic)
{
    Axis a;
    if (periodic) {
        int w = v % n;
        if (w < 0) w += n;
        a.c = w;
        a.m = (w == 0) ? n - 1 : w - 1;
        a.p = (w == n - 1) ? 0 : w + 1;
        a.ok = a.okm = a.okp = true;
    } else {
        a.c = v;
        a.m = v - 1;
        a.p = v + 1;
        a.ok = v >= 0 && v < n;
        a.okm = v - 1 >= 0 && v - 1 < n;
        a.okp = v + 1 >= 0 && v + 1 < n;
    }
    return a;
}

// State of a pulled node between its moments and its collision: the
// populations f_i(x, t) as deviations and the link bits (bit 8: solid or
// outside; bits 0-7: bounced-back directions).  get(k, i) gives the value;
// put_raw stores the two components' pulled elements of direction i.
template <int S, bool PACK = false> struct RowState {
    using C = typename Traits<S>::C;
    using R = typename Traits<S>::raw_t;
    C f[2][9];
    int info;
    __device__ __forceinline__ C get(int k, int i) const { return f[k][i]; }
    __device__ __forceinline__ void put_raw(int i, R a, R b)
    {
        f[0][i] = Traits<S>::dec(a);
        f[1][i] = Traits<S>::dec(b);
    }
};

// 16-bit storage: the pulled elements as loaded, two to a register
// (component 1 in the low half), decoded where they are used.  Decoding is
// exact, so the arithmetic is that of the decoded state, in half the
// registers (a thread holds two or six row states).  Only for states that
// hold pulled values alone: sliding-wall and inlet corrections give values
// a 16-bit element cannot hold, so the boundary kernels keep them decoded.
template <int S> struct RowState<S, true> {
    using C = typename Traits<S>::C;
    using R = typename Traits<S>::raw_t;
    static_assert(sizeof(R) == 2, "a packed state holds 16-bit elements");
    uint32_t h[9];
    int info;
    __device__ __forceinline__ C get(int k, int i) const
    {
        return Traits<S>::dec((R)(k ? h[i] >> 16 : h[i] & 0xffffu));
    }
    __device__ __forceinline__ void put_raw(int i, R a, R b) { h[i] = (uint32_t)a | (uint32_t)b << 16; }
};

// The state type of a kernel: packed for 16-bit storage without boundary code.
template <int S, bool BND>
using StateOf = RowState<S, (S == ST_F16 || S == ST_BF16) && !BND>;

// Cohesion sums sum_n W_n e_n Psi_n over the 24 positions, by opposite
// pairs (n, n+2) in each group of four (Eq. 8 on the E8 stencil).
// s1 sums psi_1 values, s2 psi_2 values.
template <class C>
__device__ __forceinline__ void cohesion_sums(const PsiPair<C> P[24], C &s1x, C &s1y, C &s2x, C &s2y)
{
    s1x = 0; s1y = 0; s2x = 0; s2y = 0;
#pragma unroll
    for (int g = 0; g < 6; ++g) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = 4 * g + h, o = n + 2;
            const C cx = (C)(e8wn(n) * sx(n));
            const C cy = (C)(e8wn(n) * sy(n));
            const C d1 = P[n].a - P[o].a;
            const C d2 = P[n].b - P[o].b;
            if (sx(n) != 0) { s1x += cx * d1; s2x += cx * d2; }
            if (sy(n) != 0) { s1y += cy * d1; s2y += cy * d2; }
        }
    }
}

// Wall rules for stencil positions (Sec. 2.4, Table 1): an unavailable
// first-layer position reads `zero` (or `self` under WALLPSI_SELF); an
// unavailable second-layer position reads whatever its Table 1 partner
// resolved to (or `zero` under E8_COPY_OFF).  Shared by the step (psi
// values) and the table export (node indices).
template <class V>
__device__ __forceinline__ void apply_wall_rules(V P[24], uint32_t unav, V self, V zero, unsigned flags)
{
#pragma unroll
    for (int n = 0; n < 8; ++n)
        if ((unav >> n) & 1u) P[n] = (flags & FL_WALLPSI_SELF) ? self : zero;
#pragma unroll
    for (int n = 8; n < 24; ++n)
        if ((unav >> n) & 1u) P[n] = (flags & FL_COPY_OFF) ? zero : P[table1(n)];
}

// S(x) = sum_n W_n s(x + e_n) e_n from the unavailable-position mask
// (Eq. 9 on the E8 stencil), by opposite pairs.
template <class C>
__device__ __forceinline__ void adhesion_vector(uint32_t unav, C &Sx, C &Sy)
{
    Sx = 0;
    Sy = 0;
#pragma unroll
    for (int g = 0; g < 6; ++g) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = 4 * g + h, o = n + 2;
            const C d = (C)(int)(((unav >> n) & 1u)) - (C)(int)(((unav >> o) & 1u));
            if (sx(n) != 0) Sx += (C)(e8wn(n) * sx(n)) * d;
            if (sy(n) != 0) Sy += (C)(e8wn(n) * sy(n)) * d;
        }
    }
}

// Eq. 11: local adhesion parameter of component 1 from rho^e (Eq. 10).
template <class C>
__device__ __forceinline__ C local_G(const KParams<C> &p, C re)
{
    if (re > p.delta) return p.Gw1;
    if (re > (C)0) return p.s1 + p.s2 * re + p.s3 * re * re;
    if (re > -p.delta) return p.s1 + p.t2 * re + p.t3 * re * re;
    return p.Gw2;
}

}  // namespace lbm
