// Definitions behind lbm3d_launch.hpp; included only by the per-storage
// translation units lbm3d_launch_<storage>.hip.
#pragma once

#include "lbm3d_launch.hpp"

namespace lbm3_host {

using namespace lbm3;

template <int S, int BX, int BY, int BZ, int TZ, int MODE>
hipError_t launch3_t(const KParams3<typename lbm::Traits<S>::C> &p, hipStream_t st)
{
    const long long blocks = (p.N + 255) / 256;
    hipLaunchKernelGGL((k_density3<S>), dim3((unsigned)blocks), dim3(256), 0, st, p);
    const int per_xcd = (p.n_units + 7) / 8;
    hipLaunchKernelGGL((k_collide3<S, BX, BY, BZ, TZ, MODE>), dim3(per_xcd * 8), dim3(BX * BY * TZ), 0, st, p,
                       per_xcd);
    return hipGetLastError();
}

// bricks bx x by x bz with tz threads in z: 32 x 8 x 4 x 1 (the default),
// 32 x 8 x 4 x 2, 32 x 8 x 4 x 4, 32 x 8 x 8 x 1, 32 x 8 x 8 x 2, 64 x 4 x 4 x 2
template <int S, int MODE>
hipError_t launch3_tile(const KParams3<typename lbm::Traits<S>::C> &p, int bx, int by, int bz, int tz, hipStream_t st)
{
    if (bx == 32 && by == 8 && bz == 4 && tz == 1) return launch3_t<S, 32, 8, 4, 1, MODE>(p, st);
    if (bx == 32 && by == 8 && bz == 4 && tz == 2) return launch3_t<S, 32, 8, 4, 2, MODE>(p, st);
    if (bx == 32 && by == 8 && bz == 4 && tz == 4) return launch3_t<S, 32, 8, 4, 4, MODE>(p, st);
    if (bx == 32 && by == 8 && bz == 8 && tz == 1) return launch3_t<S, 32, 8, 8, 1, MODE>(p, st);
    if (bx == 32 && by == 8 && bz == 8 && tz == 2) return launch3_t<S, 32, 8, 8, 2, MODE>(p, st);
    if (bx == 64 && by == 4 && bz == 4 && tz == 2) return launch3_t<S, 64, 4, 4, 2, MODE>(p, st);
    return hipErrorInvalidValue;
}

template <int S>
hipError_t launch3(const KParams3<typename lbm::Traits<S>::C> &p, Pass3 pass, int bx, int by, int bz, int tz, bool sr,
                   hipStream_t st)
{
    if (pass == P3_FIELDS_REDUCE) return launch3_t<S, 32, 8, 4, 1, K3_FIELDS | K3_REDUCE>(p, st);
    if constexpr (S == lbm::ST_F16 || S == lbm::ST_BF16) {
        if (sr)
            return pass == P3_STEP ? launch3_tile<S, K3_STORE | K3_SR>(p, bx, by, bz, tz, st)
                                   : launch3_tile<S, K3_STORE | K3_REDUCE | K3_SR>(p, bx, by, bz, tz, st);
    }
    return pass == P3_STEP ? launch3_tile<S, K3_STORE>(p, bx, by, bz, tz, st)
                           : launch3_tile<S, K3_STORE | K3_REDUCE>(p, bx, by, bz, tz, st);
}

}  // namespace lbm3_host
