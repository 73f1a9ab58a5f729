// Definitions behind lbm3d_launch.hpp; included only by the per-storage
// translation units lbm3d_launch_<storage>.hip.
#pragma once

#include "lbm3d_launch.hpp"

namespace lbm3_host {

using namespace lbm3;

template <int S, int BX, int BY, int MODE>
hipError_t launch3_t(const KParams3<typename lbm::Traits<S>::C> &p, hipStream_t st)
{
    const int per_xcd = (p.n_units + 7) / 8;
    hipLaunchKernelGGL((k_step3<S, BX, BY, MODE>), dim3(per_xcd * 8), dim3(BX * BY), 0, st, p, per_xcd);
    return hipGetLastError();
}

template <int S, int MODE>
hipError_t launch3_tile(const KParams3<typename lbm::Traits<S>::C> &p, int bx, int by, hipStream_t st)
{
    if (bx == 32 && by == 8) return launch3_t<S, 32, 8, MODE>(p, st);
    if (bx == 32 && by == 16) return launch3_t<S, 32, 16, MODE>(p, st);
    if (bx == 64 && by == 8) return launch3_t<S, 64, 8, MODE>(p, st);
    return hipErrorInvalidValue;
}

template <int S>
hipError_t launch3(const KParams3<typename lbm::Traits<S>::C> &p, Pass3 pass, int bx, int by, bool sr, hipStream_t st)
{
    if (pass == P3_FIELDS_REDUCE) return launch3_t<S, 32, 8, K3_FIELDS | K3_REDUCE>(p, st);
    if constexpr (S == lbm::ST_F16 || S == lbm::ST_BF16) {
        if (sr)
            return pass == P3_STEP ? launch3_tile<S, K3_STORE | K3_SR>(p, bx, by, st)
                                   : launch3_tile<S, K3_STORE | K3_REDUCE | K3_SR>(p, bx, by, st);
    }
    return pass == P3_STEP ? launch3_tile<S, K3_STORE>(p, bx, by, st)
                           : launch3_tile<S, K3_STORE | K3_REDUCE>(p, bx, by, st);
}

}  // namespace lbm3_host
