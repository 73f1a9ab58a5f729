// Launches of the step kernels, one translation unit per storage type
// (lbm_launch_<storage>.hip) so that their many template instances compile
// in parallel; the host side (lbm_api.hip) calls them through these
// declarations.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm_host {

// Kinds of pass over the lattice.  P_STEP2* advance two steps; RED1 / RED2
// record the diagnostics of the first / second of them.
// P_REDUCE records the diagnostics of the current state without writing
// anything else.
enum Pass { P_STEP, P_STEP_REDUCE, P_FIELDS_REDUCE, P_TABLES, P_STEP2, P_STEP2_RED1, P_STEP2_RED2, P_REDUCE };

// Launch one pass on `st` with the kernel instance that `pass`, `block`,
// the rounding mode, `bnd` (open or moving boundaries on: the instance
// that has them compiled in) and `repull` (two-step passes: the variant
// that pulls the first step's rows again instead of holding them) select;
// returns the launch status.
template <int S>
hipError_t launch_pass(const lbm::KParams<typename lbm::Traits<S>::C> &p, Pass pass, int block, bool sr, bool bnd,
                       hipStream_t st, bool repull = false);

// Resident workgroups per CU of the one-step kernel at this block size.
template <int S>
int step_occupancy(int block);

extern template hipError_t launch_pass<lbm::ST_F64>(const lbm::KParams<double> &, Pass, int, bool, bool,
                                                     hipStream_t, bool);
extern template hipError_t launch_pass<lbm::ST_F32>(const lbm::KParams<float> &, Pass, int, bool, bool,
                                                     hipStream_t, bool);
extern template hipError_t launch_pass<lbm::ST_F16>(const lbm::KParams<float> &, Pass, int, bool, bool,
                                                     hipStream_t, bool);
extern template hipError_t launch_pass<lbm::ST_BF16>(const lbm::KParams<float> &, Pass, int, bool, bool,
                                                     hipStream_t, bool);
extern template int step_occupancy<lbm::ST_F64>(int);
extern template int step_occupancy<lbm::ST_F32>(int);
extern template int step_occupancy<lbm::ST_F16>(int);
extern template int step_occupancy<lbm::ST_BF16>(int);

}  // namespace lbm_host
