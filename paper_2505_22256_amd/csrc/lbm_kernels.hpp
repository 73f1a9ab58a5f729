// Kernels of the two-component pseudopotential LBM hot path for gfx950
// (arXiv 2505.22256).  See lbm_device.hpp for the data layout.
//
// Step kernel: pull scheme.  The buffer read holds the post-collision set
// f*(t-1); pulling gives f(x, t), from which the densities at time t, the
// forces (Eq. 8-9, 11) and the collision (Eq. 1-2, 6-7) follow, and f*(t)
// is written to the other buffer.  The cohesion at x needs psi = rho(t) at
// the 24 E8 positions around x, so each workgroup also pulls a 2-node halo
// of rows and columns and keeps psi in an LDS ring of rows.
//
// Work decomposition: a workgroup of BLOCK threads owns a strip of at most
// BLOCK-4 columns (one thread per column plus two halo columns on each
// side) and marches down a segment of rows.  Each iteration pulls row y+2
// into registers and the LDS ring, synchronises once, and finishes row y,
// whose populations were pulled two iterations earlier and stayed in
// registers.  HBM traffic is one read and one write of every population;
// halo re-reads hit L2.  Work items are dealt to the 8 XCDs in contiguous
// chunks so that neighbouring segments share an L2.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

// Slot of row r in an LDS ring of RS rows (rows may be a few below zero in
// the halo of a segment).
template <int RS = 8> __device__ __forceinline__ int ring_slot(int r)
{
    if constexpr ((RS & (RS - 1)) == 0) return r & (RS - 1);
    else return (r + 64 * RS) % RS;
}

// Post-collision values of the first of two fused steps, kept in LDS for
// the second.  They are grouped by how long the second step needs them: the
// downward directions (4, 7, 8) of a row are pulled by the row below in the
// same iteration that writes them, the upward ones (2, 5, 6) by the row
// above one iteration later, and the rest and horizontal directions
// (0, 1, 3) only by the row itself.  Writing the last two groups only after
// the second step has read the row before lets the downward and upward
// groups live in two row slots and the rest/horizontal group in one.
__host__ __device__ constexpr int fr_gidx(int i) { return i == 0 || i == 2 || i == 4 ? 0 : (i == 1 || i == 5 || i == 7 ? 1 : 2); }

template <int S, int BLOCK> struct FRingMem {
    typename Traits<S>::raw_t h[2][3][BLOCK];     // directions 0, 1, 3 of one row
    typename Traits<S>::raw_t d[2][2][3][BLOCK];  // 4, 7, 8 of two rows (slot = row & 1)
    typename Traits<S>::raw_t u[2][2][3][BLOCK];  // 2, 5, 6 of two rows (slot = row & 1)
};

// Slot of direction i, component k, of row `row` at column `lane`.
template <int S, int BLOCK>
__device__ __forceinline__ typename Traits<S>::raw_t &fr_at(FRingMem<S, BLOCK> *m, int k, int i, int row, int lane)
{
    if (qy(i) == 0) return m->h[k][fr_gidx(i)][lane];
    if (qy(i) < 0) return m->d[row & 1][k][fr_gidx(i)][lane];
    return m->u[row & 1][k][fr_gidx(i)][lane];
}

// The rest/horizontal and upward values of the row just finished by the
// first step, held in registers until the second step has read the
// previous row.
template <int S> struct FPending {
    typename Traits<S>::raw_t h[2][3];
    typename Traits<S>::raw_t u[2][3];
};

// Reduction accumulators of one thread (FP64).
struct RedAcc {
    double m1 = 0, m2 = 0, px = 0, py = 0, umax = 0, rmin = __builtin_inf(), rmax = -__builtin_inf(), bad = 0;
};

// The 18 stored values pulled towards one node (prefetch unit).
template <int S> struct RawRow {
    typename Traits<S>::raw_t v[2][9];
};

// Source of direction i for a node at (cx, ry): the position x - e_i and
// whether it lies inside the domain.
__device__ __forceinline__ void pull_source(int i, const Axis &cx, const Axis &ry, int &col, int &row, bool &ok)
{
    const int ex = qx(i), ey = qy(i);
    col = ex == 1 ? cx.m : (ex == -1 ? cx.p : cx.c);
    row = ey == 1 ? ry.m : (ey == -1 ? ry.p : ry.c);
    ok = (ex == 1 ? cx.okm : (ex == -1 ? cx.okp : true)) && (ey == 1 ? ry.okm : (ey == -1 ? ry.okp : true));
}

// Issue the loads of f*_i(x - e_i, t-1) for every direction (pull
// streaming, Eq. 1).  Sources outside the domain and nodes that are not
// valid get an out-of-range offset (the load returns 0 without traffic);
// process_node substitutes the sentinel for them.
template <int S>
__device__ __forceinline__ void issue_node(const PopMem<S> &m, int nx, const Axis &cx, const Axis &ry, bool valid,
                                           RawRow<S> &q)
{
    using R = typename Traits<S>::raw_t;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int col, row;
        bool ok;
        pull_source(i, cx, ry, col, row, ok);
        const uint32_t voff = (valid && ok) ? (uint32_t)(row * nx + col) * (uint32_t)sizeof(R) : OOB;
#pragma unroll
        for (int k = 0; k < 2; ++k) q.v[k][i] = pop_load<S>(m, k, i, voff);
    }
}

// Where the bounce-back path reads f*_opp(i)(x, t-1) of the node itself:
// the post-collision set in HBM (one step per launch) or the LDS ring of
// the first of two fused steps.
template <int S> struct GlobalReload {
    const PopMem<S> &m;
    uint32_t off;  // byte offset of the node
    __device__ __forceinline__ typename Traits<S>::raw_t operator()(int k, int i) const
    {
        return pop_load<S>(m, k, i, off);
    }
};

// Turn the pulled values of one node into its state: deviations g_i of
// f_i(x, t), with halfway bounce-back f_i(x, t) = f*_opp(i)(x, t-1) where
// the source is unavailable (a sentinel or outside the domain), and the
// densities rho_k = sum_i f_i (Eq. 3) in the definition's summation order.
template <int S, bool BND, class Reload>
__device__ __forceinline__ void process_node_src(const KParams<typename Traits<S>::C> &p, const Reload &reload,
                                                 const Axis &cx, const Axis &ry, bool valid, const RawRow<S> &q,
                                                 StateOf<S, BND> &st, typename Traits<S>::C &r1,
                                                 typename Traits<S>::C &r2)
{
    using T = Traits<S>;
    using C = typename T::C;
    st.info = 256;
    if (!valid) return;
    // the node's own rest slot is always inside the domain
    if (T::sent(q.v[0][0])) return;  // solid node
    C s1 = 0, s2 = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int col, row;
        bool ok;
        pull_source(i, cx, ry, col, row, ok);
        // a source outside a non-periodic domain reads as the sentinel
        st.put_raw(i, ok ? q.v[0][i] : T::sentinel(), ok ? q.v[1][i] : T::sentinel());
        s1 += st.get(0, i);
        s2 += st.get(1, i);
    }
    s1 += p.rho0[0];
    s2 += p.rho0[1];
    st.info = 0;
    if constexpr (!BND) {
        if (__builtin_isnan(s1 + s2)) {
            // an unavailable source (or a non-finite state): reflect
            int info = 0;
            s1 = 0;
            s2 = 0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                int col, row;
                bool ok;
                pull_source(i, cx, ry, col, row, ok);
                if (i > 0 && (!ok || T::sent(q.v[0][i]))) {
                    info |= 1 << (i - 1);
                    st.put_raw(i, reload(0, opp(i)), reload(1, opp(i)));
                }
                s1 += st.get(0, i);
                s2 += st.get(1, i);
            }
            st.info = info;
            s1 += p.rho0[0];
            s2 += p.rho0[1];
        }
    } else if (__builtin_isnan(s1 + s2)) {
        // an unavailable source (or a non-finite state): reflect, from a
        // moving wall with Ladd's momentum term 6 w_i rho*_k (e_i . u_w)
        // (rho*_k: the node's own post-collision density); a source left of
        // the inlet is a Zou-He unknown
        const bool inlet = (p.flags & FL_INLET) && !p.plain && cx.c == 0;
        const bool moving = p.moving && !p.plain;
        C rp[2] = {0, 0};
        if (moving) {
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                rp[0] += T::dec(reload(0, j));
                rp[1] += T::dec(reload(1, j));
            }
            rp[0] += p.rho0[0];
            rp[1] += p.rho0[1];
        }
        int info = 0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            int col, row;
            bool ok;
            pull_source(i, cx, ry, col, row, ok);
            if (!ok || T::sent(q.v[0][i])) {
                info |= 1 << (i - 1);
                if (inlet && qx(i) == 1) continue;  // rebuilt below
                st.f[0][i] = T::dec(reload(0, opp(i)));
                st.f[1][i] = T::dec(reload(1, opp(i)));
                if (moving) {
                    // no fused multiply-adds: the same rounding in every
                    // kernel that inlines this (one or two steps per launch)
#pragma clang fp contract(off)
                    const int sy_row = ry.c - qy(i);
                    const C ux = sy_row < p.ny / 2 ? p.uw[0][0] : p.uw[1][0];
                    const C uy = sy_row < p.ny / 2 ? p.uw[0][1] : p.uw[1][1];
                    const C eu = (C)qx(i) * ux + (C)qy(i) * uy;
                    st.f[0][i] += (C)(6.0 * qw(i)) * rp[0] * eu;
                    st.f[1][i] += (C)(6.0 * qw(i)) * rp[1] * eu;
                }
            }
        }
        if (inlet) {
            // Zou-He on the west edge with the row's velocity (U, V):
            // rho = [f0 + f2 + f4 + 2 (f3 + f6 + f7)] / (1 - U),
            // f1 = f3 + 2/3 rho U, f5 = f7 - (f2 - f4)/2 + rho U/6 + rho V/2,
            // f8 = f6 + (f2 - f4)/2 + rho U/6 - rho V/2 (full populations;
            // deviations add back w_i rho0)
#pragma clang fp contract(off)
            const C U = (C)p.inlet[ry.c], V = (C)p.inlet[p.ny + ry.c];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                C F[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) F[i] = st.f[k][i] + (C)qw(i) * p.rho0[k];
                const C rho = (((F[0] + F[2]) + F[4]) + (C)2 * ((F[3] + F[6]) + F[7])) / ((C)1 - U);
                const C d24 = F[2] - F[4];
                F[1] = F[3] + (C)(2.0 / 3.0) * rho * U;
                F[5] = ((F[7] - (C)0.5 * d24) + (C)(1.0 / 6.0) * rho * U) + (C)0.5 * rho * V;
                F[8] = ((F[6] + (C)0.5 * d24) + (C)(1.0 / 6.0) * rho * U) - (C)0.5 * rho * V;
                st.f[k][1] = F[1] - (C)qw(1) * p.rho0[k];
                st.f[k][5] = F[5] - (C)qw(5) * p.rho0[k];
                st.f[k][8] = F[8] - (C)qw(8) * p.rho0[k];
            }
        }
        s1 = 0;
        s2 = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            s1 += st.f[0][i];
            s2 += st.f[1][i];
        }
        st.info = info;
        s1 += p.rho0[0];
        s2 += p.rho0[1];
    }
    r1 = s1;
    r2 = s2;
}

template <int S, bool BND>
__device__ __forceinline__ void process_node(const KParams<typename Traits<S>::C> &p, const PopMem<S> &m,
                                             const Axis &cx, const Axis &ry, bool valid, const RawRow<S> &q,
                                             StateOf<S, BND> &st, typename Traits<S>::C &r1,
                                             typename Traits<S>::C &r2)
{
    const GlobalReload<S> reload{m, (uint32_t)(ry.c * p.nx + cx.c) * (uint32_t)sizeof(typename Traits<S>::raw_t)};
    process_node_src<S, BND>(p, reload, cx, ry, valid, q, st, r1, r2);
}

// Process a prefetched row: node state into `st`, psi into the LDS ring.
template <int S, int BLOCK, int RS, bool BND>
__device__ __forceinline__ void process_row(const KParams<typename Traits<S>::C> &p, const PopMem<S> &m,
                                            const Axis &cx, bool col_ok, int r, const RawRow<S> &q,
                                            PsiPair<typename Traits<S>::C> (*ring)[BLOCK],
                                            StateOf<S, BND> &st)
{
    using C = typename Traits<S>::C;
    const Axis ry = make_axis_near(r, p.ny, p.flags & FL_PERIODIC_Y);
    C r1 = 0, r2 = 0;
    process_node<S, BND>(p, m, cx, ry, col_ok && ry.ok, q, st, r1, r2);
    PsiPair<C> ps;
    ps.a = (st.info & 256) ? lds_sentinel<C>() : r1;
    ps.b = (st.info & 256) ? lds_sentinel<C>() : r2;
    ring[ring_slot<RS>(r)][threadIdx.x] = ps;
}

template <int S>
__device__ __forceinline__ void issue_row(const KParams<typename Traits<S>::C> &p, const PopMem<S> &m,
                                          const Axis &cx, bool col_ok, int r, RawRow<S> &q)
{
    const Axis ry = make_axis_near(r, p.ny, p.flags & FL_PERIODIC_Y);
    issue_node<S>(m, p.nx, cx, ry, col_ok && ry.ok, q);
}

// Bulk cohesion sums straight from the LDS ring, pair by pair (the same
// order and operations as cohesion_sums on a gathered stencil).
template <class C, int BLOCK, int RS = 8>
__device__ __forceinline__ void cohesion_sums_lds(PsiPair<C> (*ring)[BLOCK], int y, int tid, C &s1x, C &s1y, C &s2x,
                                                  C &s2y)
{
    s1x = 0; s1y = 0; s2x = 0; s2y = 0;
#pragma unroll
    for (int g = 0; g < 6; ++g) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = 4 * g + h, o = n + 2;
            const PsiPair<C> a = ring[ring_slot<RS>(y + sy(n))][tid + sx(n)];
            const PsiPair<C> b = ring[ring_slot<RS>(y + sy(o))][tid + sx(o)];
            const C cx = (C)(e8wn(n) * sx(n));
            const C cy = (C)(e8wn(n) * sy(n));
            const C d1 = a.a - b.a;
            const C d2 = a.b - b.b;
            if (sx(n) != 0) { s1x += cx * d1; s2x += cx * d2; }
            if (sy(n) != 0) { s1y += cy * d1; s2y += cy * d2; }
        }
    }
}

// Lane of stencil position n, or of its ghost when the position lies
// beyond an open x edge (left of the inlet, right of the outflow): the node
// of the same row clamped into the domain.  `open` says which.
template <bool BND>
__device__ __forceinline__ int stencil_lane(int n, int tid, int col, int nx, unsigned flags, bool &open)
{
    open = false;
    if constexpr (!BND) return tid + sx(n);
    const int pc = col + sx(n);
    open = ((flags & FL_INLET) && pc < 0) || ((flags & FL_OUTFLOW) && pc >= nx);
    return tid + sx(n) + (!open ? 0 : pc < 0 ? -pc : nx - 1 - pc);
}

// Stencil value at position n after the wall rules of Sec. 2.4 / Table 1,
// resolved on the fly from the ring (at most two LDS reads): an unavailable
// first-layer position reads zero (or psi(x) under WALLPSI_SELF); an
// unavailable second-layer position reads what its Table 1 partner
// resolves to (zero under E8_COPY_OFF).  Beyond an open edge a first-layer
// position reads its ghost (when fluid) and a second-layer one takes the
// Table 1 copy.  `solid` is the switch s of Eq. 9 at the position (beyond
// an open edge: at its ghost).  Same rules as apply_wall_rules.
template <class C, int BLOCK, int RS, bool BND>
__device__ __forceinline__ PsiPair<C> resolve_position(PsiPair<C> (*vr)[BLOCK], int n, int y, int tid,
                                                       int col, int nx, C r1, C r2, unsigned flags, bool &solid)
{
    bool open;
    const int lane = stencil_lane<BND>(n, tid, col, nx, flags, open);
    const PsiPair<C> v = vr[ring_slot<RS>(y + sy(n))][lane];
    solid = lds_sent(v.a);
    if (!solid && (!open || n < 8)) return v;
    PsiPair<C> self, zero;
    self.a = r1;
    self.b = r2;
    zero.a = 0;
    zero.b = 0;
    const PsiPair<C> first_rule = (flags & FL_WALLPSI_SELF) ? self : zero;
    if (n < 8) return first_rule;
    if (flags & FL_COPY_OFF) return zero;
    const int m = table1(n);
    bool open_m;
    const int lane_m = stencil_lane<BND>(m, tid, col, nx, flags, open_m);
    const PsiPair<C> w = vr[ring_slot<RS>(y + sy(m))][lane_m];
    return lds_sent(w.a) ? first_rule : w;
}

// Cohesion and adhesion sums at a node with unavailable stencil positions:
// the same pair order as cohesion_sums / adhesion_vector, positions
// resolved by the wall rules, S(x) from the solid switches.
template <class C, int BLOCK, int RS, bool BND>
__device__ __forceinline__ void wall_sums(PsiPair<C> (*vr)[BLOCK], int y, int tid, int col, int nx, C r1, C r2,
                                          unsigned flags, C &s1x, C &s1y, C &s2x, C &s2y, C &Sx, C &Sy)
{
    // read the stencil afresh rather than keeping the bulk path's values
    // alive across the branch (a compiler-only memory clobber, no code)
    asm volatile("" ::: "memory");
    s1x = 0; s1y = 0; s2x = 0; s2y = 0;
    Sx = 0; Sy = 0;
#pragma unroll
    for (int g = 0; g < 6; ++g) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = 4 * g + h, o = n + 2;
            bool un, uo;
            const PsiPair<C> a = resolve_position<C, BLOCK, RS, BND>(vr, n, y, tid, col, nx, r1, r2, flags, un);
            const PsiPair<C> b = resolve_position<C, BLOCK, RS, BND>(vr, o, y, tid, col, nx, r1, r2, flags, uo);
            const C cx = (C)(e8wn(n) * sx(n));
            const C cy = (C)(e8wn(n) * sy(n));
            const C d1 = a.a - b.a;
            const C d2 = a.b - b.b;
            const C ds = (C)(int)un - (C)(int)uo;
            if (sx(n) != 0) { s1x += cx * d1; s2x += cx * d2; Sx += cx * ds; }
            if (sy(n) != 0) { s1y += cy * d1; s2y += cy * d2; Sy += cy * ds; }
        }
    }
}

// Finish node (x, y) of an interior column: stencil, forces, velocity,
// collision and the selected outputs.
template <int S, int BLOCK, int MODE, int RS = 8, class St>
__device__ __forceinline__ void finish_node(const KParams<typename Traits<S>::C> &p, const PopMem<S> &mw,
                                            const Axis &cx, int y, int yw, const St &st,
                                            PsiPair<typename Traits<S>::C> (*ring)[BLOCK], RedAcc &acc,
                                            FRingMem<S, BLOCK> *fring = nullptr, unsigned dtick = 0,
                                            FPending<S> *pend = nullptr, bool count = true)
{
    using T = Traits<S>;
    using C = typename T::C;
    using R = typename T::raw_t;
    // y numbers the LDS ring rows (it may lie outside the lattice in a halo
    // of the fused two-step kernel); yw is the lattice row after wrapping
    const int node = yw * p.nx + cx.c;
    const int tid = threadIdx.x;

    if (st.info & 256) {  // solid node (or outside the domain)
        if constexpr (MODE & M_LDS) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    if (qy(i) < 0) fr_at<S, BLOCK>(fring, k, i, y, tid) = T::sentinel();
                    else if (qy(i) == 0) pend->h[k][fr_gidx(i)] = T::sentinel();
                    else pend->u[k][fr_gidx(i)] = T::sentinel();
                }
        }
        if (MODE & M_FIELDS) {
            p.out_rho1[node] = 0.0;
            p.out_rho2[node] = 0.0;
            p.out_ux[node] = 0.0;
            p.out_uy[node] = 0.0;
        }
        if (MODE & M_TABLES) {
            p.tab_link[node] = 0;
            p.tab_nw[node] = 0;
        }
        return;
    }

    const PsiPair<C> ctr = ring[ring_slot<RS>(y)][tid];
    const C r1 = ctr.a, r2 = ctr.b;

    // first moments j_k = sum_i f_i e_i (Eq. 4), definition order; the
    // deviation base w_i rho0 has zero first moment
    C jx[2], jy[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        C ax = st.get(k, 1);
        ax -= st.get(k, 3);
        ax += st.get(k, 5);
        ax -= st.get(k, 6);
        ax -= st.get(k, 7);
        ax += st.get(k, 8);
        C ay = st.get(k, 2);
        ay -= st.get(k, 4);
        ay += st.get(k, 5);
        ay += st.get(k, 6);
        ay -= st.get(k, 7);
        ay -= st.get(k, 8);
        jx[k] = ax;
        jy[k] = ay;
    }

    // E8 cohesion sums (Eq. 8); a sentinel (unavailable position) turns
    // them into NaN and selects the wall path
    C s1x, s1y, s2x, s2y;
    cohesion_sums_lds<C, BLOCK, RS>(ring, y, tid, s1x, s1y, s2x, s2y);
    C Sx = 0, Sy = 0;
    const bool near = __builtin_isnan(s1x + s1y + s2x + s2y);
    if (near) {
        wall_sums<C, BLOCK, RS, (MODE & M_BND) != 0>(ring, y, tid, cx.c, p.nx, r1, r2, p.flags, s1x, s1y, s2x, s2y,
                                                    Sx, Sy);
    }

    if (MODE & M_TABLES) {
        uint32_t unav = 0;
#pragma unroll
        for (int n = 0; n < 24; ++n) unav |= (uint32_t)lds_sent(ring[ring_slot<RS>(y + sy(n))][tid + sx(n)].a) << n;
        p.tab_link[node] = (uint8_t)(st.info & 255);
        p.tab_nw[node] = unav ? 1 : 0;
        if (unav) {
            int idx[24];
            uint32_t rule = unav;  // positions the wall rules resolve
#pragma unroll
            for (int n = 0; n < 24; ++n) {
                const Axis ax = make_axis(cx.c + sx(n), p.nx, p.flags & FL_PERIODIC_X);
                const Axis ay = make_axis(y + sy(n), p.ny, p.flags & FL_PERIODIC_Y);
                idx[n] = (ax.ok && ay.ok) ? ay.c * p.nx + ax.c : -1;
                bool open;
                const int gl = stencil_lane<(MODE & M_BND) != 0>(n, tid, cx.c, p.nx, p.flags, open);
                if (open && n < 8 && ay.ok && !lds_sent(ring[ring_slot<RS>(y + sy(n))][gl].a)) {
                    // first layer beyond an open edge: the fluid ghost
                    idx[n] = ay.c * p.nx + (cx.c + sx(n) < 0 ? 0 : p.nx - 1);
                    rule &= ~(1u << n);
                }
            }
            apply_wall_rules<int>(idx, rule, node, -1, p.flags);
#pragma unroll
            for (int n = 0; n < 24; ++n) p.tab_src[(long long)node * 24 + n] = idx[n];
        }
        if (!(MODE & (M_STORE | M_FIELDS | M_REDUCE))) return;
    }

    // forces: cohesion (Eq. 8) + adhesion (Eq. 9, 11) + body force
    C Fx[2], Fy[2];
    Fx[0] = (p.negGc * r1) * s2x;
    Fy[0] = (p.negGc * r1) * s2y;
    Fx[1] = (p.negGc * r2) * s1x;
    Fy[1] = (p.negGc * r2) * s1y;
    if (near) {
        C G1 = p.Gw1;
        if (!(p.flags & FL_ORIGINAL)) G1 = local_G<C>(p, (r1 - r2) / (r1 + r2));
        const C a1 = -G1 * r1, a2 = -p.Gw2 * r2;
        Fx[0] += a1 * Sx;
        Fy[0] += a1 * Sy;
        Fx[1] += a2 * Sx;
        Fy[1] += a2 * Sy;
    }
    const bool fdens = p.flags & FL_FORCE_DENSITY;
    Fx[0] += (fdens ? (C)1 : r1) * p.g[0][0];
    Fy[0] += (fdens ? (C)1 : r1) * p.g[0][1];
    Fx[1] += (fdens ? (C)1 : r2) * p.g[1][0];
    Fy[1] += (fdens ? (C)1 : r2) * p.g[1][1];

    // common velocity (Eq. 5 with the half-force shift of Guo's scheme);
    // one reciprocal of the total density serves both components
    const C rt = r1 + r2;
    const C irt = recip(rt);
    const C ux = ((jx[0] + p.half * Fx[0]) + (jx[1] + p.half * Fx[1])) * irt;
    const C uy = ((jy[0] + p.half * Fy[0]) + (jy[1] + p.half * Fy[1])) * irt;

    if (MODE & M_FIELDS) {
        p.out_rho1[node] = (double)r1;
        p.out_rho2[node] = (double)r2;
        p.out_ux[node] = (double)ux;
        p.out_uy[node] = (double)uy;
    }
    if ((MODE & M_REDUCE) && count) {
        const double d1 = r1, d2 = r2, dux = ux, duy = uy;
        if (!__builtin_isfinite(d1) || !__builtin_isfinite(d2) || !__builtin_isfinite(dux) ||
            !__builtin_isfinite(duy)) {
            acc.bad += 1.0;
        } else {
            const double drt = d1 + d2;
            acc.m1 += d1;
            acc.m2 += d2;
            acc.px += drt * dux;
            acc.py += drt * duy;
            const double um = __builtin_sqrt(dux * dux + duy * duy);
            acc.umax = um > acc.umax ? um : acc.umax;
            acc.rmin = d1 < acc.rmin ? d1 : acc.rmin;
            acc.rmax = d1 > acc.rmax ? d1 : acc.rmax;
        }
    }

    if (MODE & M_STORE) {
        // BGK with Guo forcing (Eq. 1, 2, 6, 7) on deviations g = f - w rho0:
        //   g* = g + omega (f^eq - w rho0 - g) + (1 - omega/2) F_i,
        //   f^eq = w rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u],
        //   F_i  = w [3 (e.F - u.F) + 9 (e.u)(e.F)],
        // collected as g* = (1 - omega) g + w T_i with
        //   T_i = c0 + c1 e.u + c2 (e.u)^2 + (e.F)(3 cf + 9 cf e.u),
        //   c0 = omega rho (1 - 1.5 u.u) - omega rho0 - 3 cf u.F,
        //   c1 = 3 omega rho, c2 = 4.5 omega rho, cf = 1 - omega/2.
        // Opposite directions share e.u and e.F up to sign, so each pair
        // (i, opp(i)) evaluates the even part E = c0 + c2 (e.u)^2 + 9 cf
        // (e.u)(e.F) and the odd part O = c1 e.u + 3 cf e.F once:
        // T_i = E + O, T_opp(i) = E - O.
        const C a0 = (C)1 - (C)1.5 * (ux * ux + uy * uy);
        const C rho[2] = {r1, r2};
        C c0[2], c1[2], c2[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const C wr = p.omega * rho[k];
            const C uF = ux * Fx[k] + uy * Fy[k];
            c0[k] = wr * a0 - p.omega_rho0[k] - p.cf3 * uF;
            c1[k] = (C)3 * wr;
            c2[k] = (C)4.5 * wr;
        }
        constexpr bool sr = (S == ST_F16 || S == ST_BF16) && (MODE & M_SR);
        uint32_t rs = sr ? sr_seed(node, p.tick + dtick) : 1u;
        const uint32_t voff = (uint32_t)node * (uint32_t)sizeof(R);
        C gs[2][9];
#pragma unroll
        for (int k = 0; k < 2; ++k) gs[k][0] = p.omw * st.get(k, 0) + (C)qw(0) * c0[k];
#pragma unroll
        for (int pair = 0; pair < 4; ++pair) {
            const int i = pair < 2 ? pair + 1 : pair + 3;  // 1, 2, 5, 6; partners 3, 4, 7, 8
            const int o = opp(i);
            const C w = (C)qw(i);
            const int ex = qx(i), ey = qy(i);
            const C eu = ex == 0 ? (C)ey * uy : (ey == 0 ? (C)ex * ux : (C)ex * ux + (C)ey * uy);
            const C eu2 = eu * eu;
            const C h9 = p.cf9 * eu;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const C eF = ex == 0 ? (C)ey * Fy[k] : (ey == 0 ? (C)ex * Fx[k] : (C)ex * Fx[k] + (C)ey * Fy[k]);
                const C E = (c0[k] + c2[k] * eu2) + h9 * eF;
                const C O = c1[k] * eu + p.cf3 * eF;
                gs[k][i] = p.omw * st.get(k, i) + w * (E + O);
                gs[k][o] = p.omw * st.get(k, o) + w * (E - O);
            }
        }
        // encode (with stochastic rounding: one random word per direction,
        // low half for component 1, high half for component 2), then store;
        // the rounding mode is a compile-time mode bit, so each kernel
        // carries only its own encoder
        R out[2][9];
        if constexpr (sr) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint32_t rw = xorshift32(rs);
                T::enc_sr2(gs[0][i], gs[1][i], rw, out[0][i], out[1][i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                out[0][i] = T::enc(gs[0][i]);
                out[1][i] = T::enc(gs[1][i]);
            }
        }
        if constexpr (MODE & M_LDS) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    if (qy(i) < 0) fr_at<S, BLOCK>(fring, k, i, y, tid) = out[k][i];
                    else if (qy(i) == 0) pend->h[k][fr_gidx(i)] = out[k][i];
                    else pend->u[k][fr_gidx(i)] = out[k][i];
                }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                pop_store<S>(mw, 0, i, voff, out[0][i]);
                pop_store<S>(mw, 1, i, voff, out[1][i]);
            }
        }
    }
}

// Block-wide deterministic reduction of the 8 accumulators: a fixed
// butterfly of cross-lane exchanges inside each 64-lane wavefront (every
// lane ends with the same value, since a + b == b + a exactly), then the
// wavefront results in wavefront order; thread 0 writes the workgroup's
// partial record.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const double o = __shfl_xor(v, m, 64);
        v = o > v ? o : v;
    }
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const double o = __shfl_xor(v, m, 64);
        v = o < v ? o : v;
    }
    return v;
}

template <int BLOCK>
__device__ void block_reduce_write(RedAcc acc, double *out)
{
    constexpr int NW = BLOCK / 64;
    __shared__ double red[8][NW];
    const double r[8] = {wave_sum(acc.m1), wave_sum(acc.m2), wave_sum(acc.px),   wave_sum(acc.py),
                         wave_max(acc.umax), wave_min(acc.rmin), wave_max(acc.rmax), wave_sum(acc.bad)};
    const int t = threadIdx.x;
    if ((t & 63) == 0)
        for (int q = 0; q < 8; ++q) red[q][t >> 6] = r[q];
    __syncthreads();
    if (t == 0) {
        double v[8];
        for (int q = 0; q < 8; ++q) v[q] = red[q][0];
        for (int w = 1; w < NW; ++w) {
            v[0] += red[0][w];
            v[1] += red[1][w];
            v[2] += red[2][w];
            v[3] += red[3][w];
            v[4] = red[4][w] > v[4] ? red[4][w] : v[4];
            v[5] = red[5][w] < v[5] ? red[5][w] : v[5];
            v[6] = red[6][w] > v[6] ? red[6][w] : v[6];
            v[7] += red[7][w];
        }
        for (int q = 0; q < 8; ++q) out[q] = v[q];
    }
}

// One segment: rows [y0, y1) of a strip.  The psi of rows y0-2 .. y1+1
// passes through the LDS ring; each iteration processes row y+2 (moments,
// psi), issues the loads of row y+3, synchronises once and finishes row y;
// the populations of rows y, y+1 and y+2 stay in registers.  Rows past y1+1
// are never loaded.  (Deeper prefetch, three raw rows in flight, measured
// slower for every storage: the extra registers cost more occupancy than
// the latency it hides.)
template <int S, int BLOCK, int MODE>
__device__ __forceinline__ void process_segment(const KParams<typename Traits<S>::C> &p, const PopMem<S> &mr,
                                                const PopMem<S> &mw, int strip, int y0, int y1,
                                                PsiPair<typename Traits<S>::C> (*ring)[BLOCK], RedAcc &acc)
{
    using C = typename Traits<S>::C;
    const int tid = threadIdx.x;
    int x0, x1;
    if (p.strip_w > 0) {
        x0 = strip * p.strip_w;
        x1 = x0 + p.strip_w < p.nx ? x0 + p.strip_w : p.nx;
    } else {
        x0 = (int)(((long long)strip * p.nx) / p.n_strips);
        x1 = (int)(((long long)(strip + 1) * p.nx) / p.n_strips);
    }
    const int w = x1 - x0;
    const bool active = tid < w + 4;
    const bool interior = tid >= 2 && tid < w + 2;
    constexpr bool BND = (MODE & M_BND) != 0;
    const Axis cx0 = make_axis(x0 - 2 + tid, p.nx, p.flags & FL_PERIODIC_X);
    const Axis cx = BND ? open_axis(cx0, p) : cx0;
    const bool col_ok = active && cx.ok;
    const int last = y1 + 1;  // last row whose psi is needed

    StateOf<S, BND> ra, rb, rc;
    RawRow<S> q;
    issue_row<S>(p, mr, cx, col_ok, y0 - 2, q);
    process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y0 - 2, q, ring, ra);
    issue_row<S>(p, mr, cx, col_ok, y0 - 1, q);
    process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y0 - 1, q, ring, ra);
    issue_row<S>(p, mr, cx, col_ok, y0, q);
    process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y0, q, ring, ra);
    issue_row<S>(p, mr, cx, col_ok, y0 + 1, q);
    process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y0 + 1, q, ring, rb);
    issue_row<S>(p, mr, cx, col_ok, y0 + 2, q);
    int y = y0;
    for (;;) {
        if (y >= y1) break;
        process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y + 2, q, ring, rc);
        if (y + 3 <= last) issue_row<S>(p, mr, cx, col_ok, y + 3, q);
        __syncthreads();
        if (interior) finish_node<S, BLOCK, MODE>(p, mw, cx, y, y, ra, ring, acc);
        ++y;
        if (y >= y1) break;
        process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y + 2, q, ring, ra);
        if (y + 3 <= last) issue_row<S>(p, mr, cx, col_ok, y + 3, q);
        __syncthreads();
        if (interior) finish_node<S, BLOCK, MODE>(p, mw, cx, y, y, rb, ring, acc);
        ++y;
        if (y >= y1) break;
        process_row<S, BLOCK, 8, BND>(p, mr, cx, col_ok, y + 2, q, ring, rb);
        if (y + 3 <= last) issue_row<S>(p, mr, cx, col_ok, y + 3, q);
        __syncthreads();
        if (interior) finish_node<S, BLOCK, MODE>(p, mw, cx, y, y, rc, ring, acc);
        ++y;
    }
}

// Rows of a run are numbered strip-major (strip * ny + y).  Work unit u of
// n_units covers rows [u * R / n_units, (u + 1) * R / n_units) of the R =
// strips * ny rows, split where it crosses a strip boundary.  With
// band_order the units of a fixed-segment tiling are taken across the
// strips first, so that workgroups running at the same time cover whole
// rows of the lattice.
template <class Seg>
__device__ __forceinline__ void for_unit_segments(int n_strips, int n_segs, int ny, int xcd_slabs, int band_order,
                                                  int u, int n_units, Seg &&seg)
{
    if (xcd_slabs) {
        // workgroup b runs on XCD b % 8: slab b % 8 of the rows, strip b / 8
        const int strip = u >> 3, slab = u & 7;
        const int y0 = (int)(((long long)slab * ny) >> 3);
        const int y1 = (int)(((long long)(slab + 1) * ny) >> 3);
        if (strip < n_strips && y1 > y0) seg(strip, y0, y1);
        return;
    }
    if (band_order && n_units == n_strips * n_segs) {
        const int strip = u % n_strips, sg = u / n_strips;
        const int y0 = (int)(((long long)sg * ny) / n_segs);
        const int y1 = (int)(((long long)(sg + 1) * ny) / n_segs);
        seg(strip, y0, y1);
        return;
    }
    const long long R = (long long)n_strips * ny;
    long long q0 = (long long)u * R / n_units;
    const long long q1 = (long long)(u + 1) * R / n_units;
    bool first = true;
    while (q0 < q1) {
        const int strip = (int)(q0 / ny);
        const int y0 = (int)(q0 - (long long)strip * ny);
        const long long end = (long long)(strip + 1) * ny < q1 ? (long long)(strip + 1) * ny : q1;
        const int y1 = (int)(end - (long long)strip * ny);
        if (!first) __syncthreads();  // the LDS rings are reused
        seg(strip, y0, y1);
        first = false;
        q0 = end;
    }
}

template <int S, int BLOCK, int MODE>
__device__ __forceinline__ void process_unit(const KParams<typename Traits<S>::C> &p, int u, int n_units,
                                             PsiPair<typename Traits<S>::C> (*ring)[BLOCK], RedAcc &acc)
{
    const PopMem<S> mr = make_mem<S>(p.A, p.N);
    const PopMem<S> mw = make_mem<S>(p.B, p.N);
    for_unit_segments(p.n_strips, p.n_segs, p.ny, p.xcd_slabs, p.band_order, u, n_units,
                      [&](int strip, int y0, int y1) {
                          process_segment<S, BLOCK, MODE>(p, mr, mw, strip, y0, y1, ring, acc);
                      });
}

// ---------------------------------------------------------------------------
// Two fused time steps per launch (temporal blocking).  The first step runs
// exactly the code of the single step but keeps its post-collision rows in
// LDS (FRingMem) instead of HBM; the second step pulls from there and
// writes HBM.  HBM then sees one read and one write of the populations per
// two steps (plus a wider halo: 5 columns and 5 rows on each side instead of
// 2), and the result is bitwise that of two single steps.  The LDS holds
// 5 rows' worth of post-collision values (two rows of the downward and
// upward groups, one of the rest) and 5 rows of psi per step, so that six
// 128-thread FP32 workgroups fit a CU's LDS.
// ---------------------------------------------------------------------------
constexpr int TWO_PR = 5;  // rows in each psi ring

// Pull f(x, t+1) = f*(x - e_i, t) of row r from the LDS (lane = column);
// the outflow column pulls the directions entering from outside from its
// own lane (zero normal gradient, as open_axis does for HBM pulls).
template <int S, int BLOCK>
__device__ __forceinline__ void issue_row_lds(FRingMem<S, BLOCK> *fring, int r, RawRow<S> &q, bool outflow_col)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int src = (qx(i) == -1 && outflow_col) ? tid : tid - qx(i);
        const bool in = src >= 0 && src < BLOCK;
        const int lane = in ? src : tid;
        q.v[0][i] = in ? fr_at<S, BLOCK>(fring, 0, i, r - qy(i), lane) : Traits<S>::sentinel();
        q.v[1][i] = in ? fr_at<S, BLOCK>(fring, 1, i, r - qy(i), lane) : Traits<S>::sentinel();
    }
}

template <int S, int BLOCK> struct LdsReload {
    FRingMem<S, BLOCK> *fring;
    int row, lane;
    __device__ __forceinline__ typename Traits<S>::raw_t operator()(int k, int i) const
    {
        return fr_at<S, BLOCK>(fring, k, i, row, lane);
    }
};

template <int S, int BLOCK, bool BND>
__device__ __forceinline__ void process_row_lds(const KParams<typename Traits<S>::C> &p, FRingMem<S, BLOCK> *fring,
                                                const Axis &cx, bool col_ok, int r,
                                                PsiPair<typename Traits<S>::C> (*ring)[BLOCK],
                                                StateOf<S, BND> &st)
{
    using C = typename Traits<S>::C;
    const Axis ry = make_axis_near(r, p.ny, p.flags & FL_PERIODIC_Y);
    RawRow<S> q;
    issue_row_lds<S, BLOCK>(fring, r, q, BND && cx.okp && cx.p == cx.c);
    const LdsReload<S, BLOCK> reload{fring, r, (int)threadIdx.x};
    C r1 = 0, r2 = 0;
    process_node_src<S, BND>(p, reload, cx, ry, col_ok && ry.ok, q, st, r1, r2);
    PsiPair<C> ps;
    ps.a = (st.info & 256) ? lds_sentinel<C>() : r1;
    ps.b = (st.info & 256) ? lds_sentinel<C>() : r2;
    ring[ring_slot<TWO_PR>(r)][threadIdx.x] = ps;
}

// Rows [y0, y1) of a strip, two steps.  Iteration p (two barriers):
//   1. step 1 processes row p (pulled from HBM), the loads of row p + 1 go out;
//   -- barrier --
//   2. the held directions of row p - 3 go to LDS; step 2 finishes row
//      p - 6 into HBM (its psi(t+1) rows p - 8 .. p - 4 are complete);
//      step 1 finishes row p - 2: its downward directions go to LDS, the
//      others to registers;
//   -- barrier --
//   3. step 2 processes row p - 3 (pulled from LDS).
// Each barrier separates every LDS write from the reads of what it
// replaces: ring slots are rewritten only one iteration after their last
// reader, and the held group of a row is written between the second-step
// pull of the row above (previous iteration) and its own (this one).
// Lanes cover columns x0-5 .. x1+4: step 1 needs psi(t) there and finishes
// x0-3 .. x1+2; step 2 needs psi(t+1) on x0-2 .. x1+1 and finishes
// x0 .. x1-1.  Rows: step 1 pulls y0-5 .. y1+4 and finishes y0-3 .. y1+2;
// step 2 processes y0-2 .. y1+1 and finishes y0 .. y1-1.
template <int S, int BLOCK, int MODE>
__device__ __forceinline__ void process_segment2(const KParams<typename Traits<S>::C> &p, const PopMem<S> &mr,
                                                 const PopMem<S> &mw, int strip, int y0, int y1,
                                                 PsiPair<typename Traits<S>::C> (*ring1)[BLOCK],
                                                 PsiPair<typename Traits<S>::C> (*ring2)[BLOCK],
                                                 FRingMem<S, BLOCK> *fring, RedAcc &acc)
{
    using C = typename Traits<S>::C;
    // diagnostics of step t come from the first step (core nodes only: the
    // halo is computed twice), those of step t+1 from the second
    constexpr bool red1 = (MODE & M_REDUCE) && (MODE & M_DIAG_FIRST);
    constexpr bool red2 = (MODE & M_REDUCE) && !(MODE & M_DIAG_FIRST);
    constexpr int M1 = (MODE & (M_SR | M_BND)) | M_STORE | M_LDS | (red1 ? M_REDUCE : 0);
    constexpr int M2 = (MODE & (M_SR | M_BND)) | M_STORE | (red2 ? M_REDUCE : 0);
    // with M_REPULL the first step keeps no pulled rows in registers: it
    // pulls the row it finishes again (the second read of addresses read
    // two iterations earlier, served by the caches), which frees the
    // registers of two row states
    constexpr bool REPULL = (MODE & M_REPULL) != 0;
    const int tid = threadIdx.x;
    int x0, x1;
    if (p.strip_w > 0) {
        x0 = strip * p.strip_w;
        x1 = x0 + p.strip_w < p.nx ? x0 + p.strip_w : p.nx;
    } else {
        x0 = (int)(((long long)strip * p.nx) / p.n_strips);
        x1 = (int)(((long long)(strip + 1) * p.nx) / p.n_strips);
    }
    const int w = x1 - x0;
    constexpr bool BND = (MODE & M_BND) != 0;
    const Axis cx0 = make_axis(x0 - 5 + tid, p.nx, p.flags & FL_PERIODIC_X);
    const Axis cx = BND ? open_axis(cx0, p) : cx0;
    const bool act1 = tid < w + 10 && cx.ok;
    const bool in1 = tid >= 2 && tid < w + 8;
    const bool act2 = tid >= 3 && tid < w + 7 && cx.ok;
    const bool in2 = tid >= 5 && tid < w + 5;
    const int p_first = y0 - 5, p_pull_last = y1 + 4, p_last = y1 + 4;
    const bool wrap_y = p.flags & FL_PERIODIC_Y;
    const bool core_col = tid >= 5 && tid < w + 5;

    using St = StateOf<S, BND>;
    St a1, b1, c1, a2, b2, c2;
    RawRow<S> q;
    FPending<S> pend;  // held group of the row step 1 finished last
    issue_row<S>(p, mr, cx, act1, p_first, q);
    auto iter = [&](int pp, St &s1w, St &s1f, St &s2) {
        const bool fin1 = in1 && pp - 2 >= y0 - 3 && pp - 2 <= y1 + 2;
        const bool held = in1 && pp - 3 >= y0 - 3 && pp - 3 <= y1 + 2;
        RawRow<S> qf;
        if constexpr (REPULL) {
            if (fin1) issue_row<S>(p, mr, cx, act1, pp - 2, qf);
        }
        if (pp <= p_pull_last) process_row<S, BLOCK, TWO_PR, BND>(p, mr, cx, act1, pp, q, ring1, s1w);
        if (pp + 1 <= p_pull_last) issue_row<S>(p, mr, cx, act1, pp + 1, q);
        __syncthreads();
        if (held) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    fring->h[k][j][tid] = pend.h[k][j];
                    fring->u[(pp - 3) & 1][k][j][tid] = pend.u[k][j];
                }
        }
        // s2 holds row p - 6 (written three iterations ago) until the pull
        // of row p - 3 below replaces it
        if (in2 && pp - 6 >= y0 && pp - 6 < y1)
            finish_node<S, BLOCK, M2, TWO_PR>(p, mw, cx, pp - 6, pp - 6, s2, ring2, acc, nullptr, 1u);
        if (fin1) {
            const Axis ry = make_axis_near(pp - 2, p.ny, wrap_y);
            const bool core = core_col && pp - 2 >= y0 && pp - 2 < y1;
            if constexpr (REPULL) {
                St st;
                C r1 = 0, r2 = 0;
                process_node<S, BND>(p, mr, cx, ry, act1 && ry.ok, qf, st, r1, r2);
                finish_node<S, BLOCK, M1, TWO_PR>(p, mw, cx, pp - 2, ry.c, st, ring1, acc, fring, 0u, &pend, core);
            } else {
                finish_node<S, BLOCK, M1, TWO_PR>(p, mw, cx, pp - 2, ry.c, s1f, ring1, acc, fring, 0u, &pend, core);
            }
        }
        __syncthreads();
        if (pp - 3 >= y0 - 2 && pp - 3 <= y1 + 1) process_row_lds<S, BLOCK, BND>(p, fring, cx, act2, pp - 3, ring2, s2);
    };
    // state of row r: step 1 in {a1, b1, c1}, step 2 in {a2, b2, c2}, both by
    // (r - p_first) mod 3; iteration p writes rows p (step 1) and p - 3
    // (step 2) and finishes rows p - 2 and p - 6; one iteration past the
    // last pull finishes the last row of step 2
    for (int pp = p_first;;) {
        iter(pp, a1, b1, a2);
        if (++pp > p_last + 1) break;
        iter(pp, b1, c1, b2);
        if (++pp > p_last + 1) break;
        iter(pp, c1, a1, c2);
        if (++pp > p_last + 1) break;
    }
}

template <int S, int BLOCK, int MODE>
__global__ void __launch_bounds__(BLOCK) k_step2(const KParams<typename Traits<S>::C> p, int per_xcd)
{
    using C = typename Traits<S>::C;
    __shared__ PsiPair<C> ring1[TWO_PR][BLOCK];
    __shared__ PsiPair<C> ring2[TWO_PR][BLOCK];
    __shared__ FRingMem<S, BLOCK> fring;
    const int b = blockIdx.x;
    const int unit = p.xcd_slabs ? b : (b & 7) * per_xcd + (b >> 3);
    RedAcc acc;
    if (unit < p.n_units) {
        const PopMem<S> mr = make_mem<S>(p.A, p.N);
        const PopMem<S> mw = make_mem<S>(p.B, p.N);
        for_unit_segments(p.n_strips, p.n_segs, p.ny, p.xcd_slabs, p.band_order, unit, p.n_units,
                          [&](int strip, int y0, int y1) {
                              process_segment2<S, BLOCK, MODE>(p, mr, mw, strip, y0, y1, ring1, ring2, &fring, acc);
                          });
    }
    if (MODE & M_REDUCE) {
        __syncthreads();
        block_reduce_write<BLOCK>(acc, p.partials + (long long)b * 8);
    }
}

// One time step (or one field/diagnostic/table pass) of a single run.
// Grid: 8 * per_xcd workgroups over the run's n_units units;
// workgroup b takes unit (b % 8) * per_xcd + b / 8, so each XCD works on a
// contiguous part of the lattice.
template <int S, int BLOCK, int MODE>
__global__ void __launch_bounds__(BLOCK) k_step(const KParams<typename Traits<S>::C> p, int per_xcd)
{
    using C = typename Traits<S>::C;
    __shared__ PsiPair<C> ring[8][BLOCK];
    const int b = blockIdx.x;
    const int unit = p.xcd_slabs ? b : (b & 7) * per_xcd + (b >> 3);
    RedAcc acc;
    if (unit < p.n_units) process_unit<S, BLOCK, MODE>(p, unit, p.n_units, ring, acc);
    if (MODE & M_REDUCE) {
        __syncthreads();
        block_reduce_write<BLOCK>(acc, p.partials + (long long)b * 8);
    }
}

// Batched step: the work list concatenates the units of all runs; run r
// owns units [item0_r, item0_r + strips_r * segs_r).
template <int S, int BLOCK, int MODE>
__global__ void __launch_bounds__(BLOCK)
k_step_batch(const KParams<typename Traits<S>::C> *__restrict__ runs, int nruns, int n_items, int per_xcd, int flip,
             const unsigned *__restrict__ tick)
{
    using C = typename Traits<S>::C;
    __shared__ PsiPair<C> ring[8][BLOCK];
    const int b = blockIdx.x;
    const int item = (b & 7) * per_xcd + (b >> 3);
    if (item >= n_items) return;
    int lo = 0, hi = nruns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (runs[mid].item0 <= item) lo = mid; else hi = mid - 1;
    }
    KParams<C> p = runs[lo];
    p.tick = *tick;
    if (flip) {
        const void *t = p.A;
        p.A = p.B;
        p.B = (void *)t;
    }
    RedAcc acc;
    process_unit<S, BLOCK, MODE>(p, item - p.item0, p.n_units, ring, acc);
}

// Two fused steps of every run of a batch (see k_step2).
template <int S, int BLOCK, int MODE>
__global__ void __launch_bounds__(BLOCK)
k_step2_batch(const KParams<typename Traits<S>::C> *__restrict__ runs, int nruns, int n_items, int per_xcd, int flip,
              const unsigned *__restrict__ tick)
{
    using C = typename Traits<S>::C;
    __shared__ PsiPair<C> ring1[TWO_PR][BLOCK];
    __shared__ PsiPair<C> ring2[TWO_PR][BLOCK];
    __shared__ FRingMem<S, BLOCK> fring;
    const int b = blockIdx.x;
    const int item = (b & 7) * per_xcd + (b >> 3);
    if (item >= n_items) return;
    int lo = 0, hi = nruns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (runs[mid].item0 <= item) lo = mid; else hi = mid - 1;
    }
    KParams<C> p = runs[lo];
    p.tick = *tick;
    if (flip) {
        const void *t = p.A;
        p.A = p.B;
        p.B = (void *)t;
    }
    const PopMem<S> mr = make_mem<S>(p.A, p.N);
    const PopMem<S> mw = make_mem<S>(p.B, p.N);
    RedAcc acc;
    for_unit_segments(p.n_strips, p.n_segs, p.ny, p.xcd_slabs, p.band_order, item - p.item0, p.n_units,
                      [&](int strip, int y0, int y1) {
                          process_segment2<S, BLOCK, MODE>(p, mr, mw, strip, y0, y1, ring1, ring2, &fring, acc);
                      });
}

// Advance the batch step counter (one thread; graph-capturable).
static __global__ void k_tick(unsigned *tick, unsigned n) { tick[0] += n; }

// Finalise diagnostics: deterministic compensated (Neumaier) sums over the
// workgroup partials in a fixed order; one workgroup of 256 threads.
static __global__ void __launch_bounds__(256) k_reduce_final(const double *__restrict__ partials, int nparts, double *out)
{
    __shared__ double s[5][256], cmp[5][256], mx[3][256];
    const int t = threadIdx.x;
    double sum[5] = {0, 0, 0, 0, 0}, c[5] = {0, 0, 0, 0, 0};
    double umax = 0, rmin = __builtin_inf(), rmax = -__builtin_inf();
    const int idx[5] = {0, 1, 2, 3, 7};
    for (int j = t; j < nparts; j += 256) {
        const double *q = partials + (long long)j * 8;
        for (int a = 0; a < 5; ++a) {
            const double v = q[idx[a]], tt = sum[a] + v;
            c[a] += (__builtin_fabs(sum[a]) >= __builtin_fabs(v)) ? (sum[a] - tt) + v : (v - tt) + sum[a];
            sum[a] = tt;
        }
        umax = q[4] > umax ? q[4] : umax;
        rmin = q[5] < rmin ? q[5] : rmin;
        rmax = q[6] > rmax ? q[6] : rmax;
    }
    for (int a = 0; a < 5; ++a) {
        s[a][t] = sum[a];
        cmp[a][t] = c[a];
    }
    mx[0][t] = umax;
    mx[1][t] = rmin;
    mx[2][t] = rmax;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            for (int a = 0; a < 5; ++a) {
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
        out[0] = s[0][0] + cmp[0][0];
        out[1] = s[1][0] + cmp[1][0];
        out[2] = s[2][0] + cmp[2][0];
        out[3] = s[3][0] + cmp[3][0];
        out[4] = mx[0][0];
        out[5] = mx[1][0];
        out[6] = mx[2][0];
        out[7] = s[4][0] + cmp[4][0];
    }
}

// Post-collision set whose streaming gives the pre-collision set f(t):
// slot (z, j) is pulled by z + e_j when that position is available, else by
// z itself as the bounce-back of direction opp(j).  So
// f*_j(z) = f_j(z + e_j) or f_opp(j)(z).  Source f is FP64 [2][9][N]; when
// `rho` is given instead, f_i = w_i rho_k (equilibrium at rest).  Stored as
// the deviation f - w_j rho0_k.
template <int S>
__global__ void __launch_bounds__(256)
k_inverse_stream(const KParams<typename Traits<S>::C> p, const uint8_t *__restrict__ solid,
                 const double *__restrict__ fsrc, const double *__restrict__ rho)
{
    using T = Traits<S>;
    using C = typename T::C;
    const long long z = (long long)blockIdx.x * 256 + threadIdx.x;
    if (z >= p.N) return;
    if (solid[z]) return;  // slots stay at the sentinel
    const PopMem<S> m = make_mem<S>(p.B, p.N);
    const int x = (int)(z % p.nx), y = (int)(z / p.nx);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const Axis ax = make_axis(x + qx(j), p.nx, p.flags & FL_PERIODIC_X);
        const Axis ay = make_axis(y + qy(j), p.ny, p.flags & FL_PERIODIC_Y);
        const long long nb = (long long)ay.c * p.nx + ax.c;
        const bool avail = ax.ok && ay.ok && !solid[nb];
        for (int k = 0; k < 2; ++k) {
            double v;
            if (rho) {
                v = qw(j) * rho[(long long)k * p.N + (avail ? nb : z)];
            } else {
                v = avail ? fsrc[(long long)(k * 9 + j) * p.N + nb] : fsrc[(long long)(k * 9 + opp(j)) * p.N + z];
            }
            const double base = T::deviation ? qw(j) * (double)p.rho0[k] : 0.0;
            pop_store<S>(m, k, j, (uint32_t)z * (uint32_t)sizeof(typename T::raw_t), T::enc((C)(v - base)));
        }
    }
}

// Pre-collision populations f(x, t) = g + w_i rho0 as FP64 (solid -> 0) of
// the w x h window at (x0, y0) (periodic wrap), out [2][9][h][w], by the
// same pull as the step kernel.
template <int S>
__global__ void __launch_bounds__(256)
k_pull_window(const KParams<typename Traits<S>::C> p, int x0, int y0, int w, int h, double *__restrict__ out)
{
    using T = Traits<S>;
    using C = typename T::C;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long M = (long long)w * h;
    if (q >= M) return;
    const int wx = (int)(q % w), wy = (int)(q / w);
    const Axis cx = open_axis(make_axis(x0 + wx, p.nx, p.flags & FL_PERIODIC_X), p);
    const Axis ry = make_axis(y0 + wy, p.ny, p.flags & FL_PERIODIC_Y);
    const PopMem<S> m = make_mem<S>(p.A, p.N);
    RawRow<S> raw;
    issue_node<S>(m, p.nx, cx, ry, true, raw);
    StateOf<S, true> st;
    C r1, r2;
    process_node<S, true>(p, m, cx, ry, true, raw, st, r1, r2);
    const bool solid = st.info & 256;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double base = T::deviation ? qw(i) * (double)p.rho0[k] : 0.0;
            out[(long long)(k * 9 + i) * M + q] = solid ? 0.0 : (double)st.f[k][i] + base;
        }
}

}  // namespace lbm
