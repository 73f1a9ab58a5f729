// Host-side parameter mapping shared by the single-run and batched paths.
#pragma once

#include "lbm.h"
#include "lbm_device.hpp"

#include <algorithm>

namespace lbm_host {

using lbm::KParams;
using lbm::qw;

// Schedule bits of a tile (lbm_set_tile).
enum : unsigned { SCHED_ALIGN = 1u, SCHED_BANDS = 2u, SCHED_XCD_SLABS = 4u, SCHED_TWO_STEP = 8u, SCHED_REPULL = 16u };

// Rounding of the stores in effect for a storage type: F16 and BF16 round
// stochastically unless LBM_ROUND_NEAREST asks for round-to-nearest-even;
// F64 and F32 carry neither bit.
inline unsigned resolve_rounding(unsigned flags, int storage)
{
    const bool narrow = storage == LBM_F16 || storage == LBM_BF16;
    flags &= ~(unsigned)LBM_ROUND_STOCHASTIC;
    if (narrow && !(flags & LBM_ROUND_NEAREST)) flags |= LBM_ROUND_STOCHASTIC;
    if (!narrow) flags &= ~(unsigned)LBM_ROUND_NEAREST;
    return flags;
}

// Strips are block - 4 columns wide (balanced over nx), or, with
// SCHED_ALIGN, the widest multiple of `align_cols` columns that fits, from
// x = 0, so that every strip's stores start on a 128-byte boundary.
inline void tile_counts(int block, int seg_rows, int nx, int ny, int *strips, int *segs, unsigned sched = 0,
                        int align_cols = 32, int *strip_w = nullptr, int halo = 2)
{
    int w = block - 2 * halo;
    if ((sched & SCHED_ALIGN) && w >= align_cols) w = (w / align_cols) * align_cols;
    else if (sched & SCHED_ALIGN) w = block - 2 * halo;
    *strips = (nx + w - 1) / w;
    if (strip_w) *strip_w = (sched & SCHED_ALIGN) ? w : 0;
    const int s = (ny + seg_rows - 1) / seg_rows;
    *segs = std::max(1, std::min(s, ny));
}

template <class C>
inline void fill_physics(KParams<C> &p, unsigned flags, double Gc, double Gw1, double Gw2, double delta, double tau,
                  const double acc[2][2], const double rho0[2], bool deviation)
{
    p.omega = (C)(1.0 / tau);
    p.cforce = (C)(1.0 - 1.0 / (2.0 * tau));
    p.omw = (C)(1.0 - 1.0 / tau);
    p.cf3 = (C)(3.0 * (1.0 - 1.0 / (2.0 * tau)));
    p.cf9 = (C)(9.0 * (1.0 - 1.0 / (2.0 * tau)));
    p.half = (flags & LBM_VEL_LITERAL) ? (C)0 : (C)0.5;
    p.negGc = (C)(-Gc);
    p.Gw1 = (C)Gw1;
    p.Gw2 = (C)Gw2;
    p.delta = (C)delta;
    // Eq. 11 coefficients (s1 = t1 = harmonic mean); unused by the original scheme
    double s1 = 0, s2 = 0, s3 = 0, t2 = 0, t3 = 0;
    if (!(flags & LBM_SCHEME_ORIGINAL)) {
        s1 = 2.0 * Gw1 * Gw2 / (Gw1 + Gw2);
        s2 = 2.0 * (Gw1 - s1) / delta;
        s3 = -s2 / (2.0 * delta);
        t2 = 2.0 * (s1 - Gw2) / delta;
        t3 = t2 / (2.0 * delta);
    }
    p.s1 = (C)s1;
    p.s2 = (C)s2;
    p.s3 = (C)s3;
    p.t2 = (C)t2;
    p.t3 = (C)t3;
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 2; ++a) p.g[k][a] = (C)acc[k][a];
    for (int k = 0; k < 2; ++k) {
        p.rho0[k] = deviation ? (C)rho0[k] : (C)0;
        p.omega_rho0[k] = deviation ? (C)(rho0[k] / tau) : (C)0;
    }
}

}  // namespace lbm_host
