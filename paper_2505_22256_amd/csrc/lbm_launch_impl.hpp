// Definitions behind lbm_launch.hpp; included only by the per-storage
// translation units lbm_launch_<storage>.hip.
#pragma once

#include "lbm_launch.hpp"

#include <algorithm>

namespace lbm_host {

using namespace lbm;

template <int S, int BLOCK, int MODE>
hipError_t launch_step_t(const KParams<typename Traits<S>::C> &p, hipStream_t st)
{
    const int per_xcd = (p.n_units + 7) / 8;
    hipLaunchKernelGGL((k_step<S, BLOCK, MODE>), dim3(per_xcd * 8), dim3(BLOCK), 0, st, p, per_xcd);
    return hipGetLastError();
}

template <int S, int MODE>
hipError_t launch_step_b(const KParams<typename Traits<S>::C> &p, int block, hipStream_t st)
{
    switch (block) {
    case 64: return launch_step_t<S, 64, MODE>(p, st);
    case 128: return launch_step_t<S, 128, MODE>(p, st);
    default: return launch_step_t<S, 256, MODE>(p, st);
    }
}

template <int S, int BLOCK, int MODE>
hipError_t launch_step2_t(const KParams<typename Traits<S>::C> &p, hipStream_t st)
{
    const int per_xcd = (p.n_units + 7) / 8;
    hipLaunchKernelGGL((k_step2<S, BLOCK, MODE>), dim3(per_xcd * 8), dim3(BLOCK), 0, st, p, per_xcd);
    return hipGetLastError();
}

template <int S, int MODE>
hipError_t launch_step2_b(const KParams<typename Traits<S>::C> &p, int block, hipStream_t st)
{
    switch (block) {
    case 64: return launch_step2_t<S, 64, MODE>(p, st);
    case 128: return launch_step2_t<S, 128, MODE>(p, st);
    default: return launch_step2_t<S, 256, MODE>(p, st);
    }
}

template <int S, int B>
hipError_t launch_pass_b(const KParams<typename Traits<S>::C> &p, Pass pass, int block, bool sr, hipStream_t st,
                         bool repull)
{
    constexpr bool narrow = S == ST_F16 || S == ST_BF16;
    constexpr int R1 = M_REDUCE | M_DIAG_FIRST, R2 = M_REDUCE;
    if constexpr (S != ST_F64 && B == 0) {
        // the re-pull variant of the plain two-step pass (the 1-in-K
        // diagnostic passes keep the other: the results are the same)
        if (repull && pass == P_STEP2 && block != 256) {
            if (narrow && sr) return launch_step2_b<S, M_STORE | M_SR | M_REPULL>(p, block, st);
            return launch_step2_b<S, M_STORE | M_REPULL>(p, block, st);
        }
    }
    if constexpr (narrow) {
        if (sr) {
            switch (pass) {
            case P_STEP: return launch_step_b<S, B | M_STORE | M_SR>(p, block, st);
            case P_STEP_REDUCE: return launch_step_b<S, B | M_STORE | M_REDUCE | M_SR>(p, block, st);
            case P_STEP2: return launch_step2_b<S, B | M_STORE | M_SR>(p, block, st);
            case P_STEP2_RED1: return launch_step2_b<S, B | M_STORE | M_SR | R1>(p, block, st);
            case P_STEP2_RED2: return launch_step2_b<S, B | M_STORE | M_SR | R2>(p, block, st);
            default: break;  // field and table passes do not store
            }
        }
    }
    switch (pass) {
    case P_STEP: return launch_step_b<S, B | M_STORE>(p, block, st);
    case P_STEP_REDUCE: return launch_step_b<S, B | M_STORE | M_REDUCE>(p, block, st);
    case P_FIELDS_REDUCE:
    case P_TABLES:
    case P_REDUCE: return hipErrorInvalidValue;  // launched by launch_pass
    case P_STEP2:
    case P_STEP2_RED1:
    case P_STEP2_RED2:
        if constexpr (S == ST_F64) {
            // FP64: one wavefront per SIMD at any block; 64- and 128-thread strips
            const bool b128 = block == 128;
            if (pass == P_STEP2)
                return b128 ? launch_step2_t<S, 128, B | M_STORE>(p, st) : launch_step2_t<S, 64, B | M_STORE>(p, st);
            if (pass == P_STEP2_RED1)
                return b128 ? launch_step2_t<S, 128, B | M_STORE | R1>(p, st)
                            : launch_step2_t<S, 64, B | M_STORE | R1>(p, st);
            return b128 ? launch_step2_t<S, 128, B | M_STORE | R2>(p, st) : launch_step2_t<S, 64, B | M_STORE | R2>(p, st);
        } else {
            return pass == P_STEP2 ? launch_step2_b<S, B | M_STORE>(p, block, st)
                 : pass == P_STEP2_RED1 ? launch_step2_b<S, B | M_STORE | R1>(p, block, st)
                                        : launch_step2_b<S, B | M_STORE | R2>(p, block, st);
        }
    }
    return hipErrorInvalidValue;
}

// Stepping passes take the instance without boundary code unless open or
// moving boundaries are on; the (rare) field and table passes always have it.
template <int S>
hipError_t launch_pass(const KParams<typename Traits<S>::C> &p, Pass pass, int block, bool sr, bool bnd, hipStream_t st,
                       bool repull)
{
    if (pass == P_FIELDS_REDUCE) return launch_step_t<S, 256, M_BND | M_FIELDS | M_REDUCE>(p, st);
    if (pass == P_REDUCE) return launch_step_t<S, 256, M_BND | M_REDUCE>(p, st);
    if (pass == P_TABLES) return launch_step_t<S, 256, M_BND | M_TABLES>(p, st);
    return bnd ? launch_pass_b<S, M_BND>(p, pass, block, sr, st, false)
               : launch_pass_b<S, 0>(p, pass, block, sr, st, repull);
}

template <int S, int BLOCK>
int occupancy_of()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_step<S, BLOCK, M_STORE>, BLOCK, 0) !=
        hipSuccess)
        nb = 1;
    return std::max(nb, 1);
}

template <int S>
int step_occupancy(int block)
{
    return block == 64 ? occupancy_of<S, 64>() : block == 128 ? occupancy_of<S, 128>() : occupancy_of<S, 256>();
}

}  // namespace lbm_host
