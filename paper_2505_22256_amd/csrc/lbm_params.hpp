// Host-side parameter mapping shared by the single-run and batched paths.
#pragma once

#include "lbm.h"
#include "lbm_device.hpp"

#include <algorithm>

namespace lbm_host {

using lbm::KParams;
using lbm::qw;

inline void tile_counts(int block, int seg_rows, int nx, int ny, int *strips, int *segs)
{
    *strips = (nx + (block - 4) - 1) / (block - 4);
    const int s = (ny + seg_rows - 1) / seg_rows;
    *segs = std::max(1, std::min(s, ny));
}

template <class C>
inline void fill_physics(KParams<C> &p, unsigned flags, double Gc, double Gw1, double Gw2, double delta, double tau,
                  const double acc[2][2], const double rho0[2], bool deviation)
{
    p.omega = (C)(1.0 / tau);
    p.cforce = (C)(1.0 - 1.0 / (2.0 * tau));
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
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) p.base[k][i] = deviation ? (C)(qw(i) * rho0[k]) : (C)0;
}

}  // namespace lbm_host
