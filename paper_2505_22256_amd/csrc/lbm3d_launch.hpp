// Launches of the 3-D step kernels, one translation unit per storage type
// (lbm3d_launch_<storage>.hip), called by lbm3d_api.hip through these
// declarations.
#pragma once

#include "lbm3d_kernels.hpp"

namespace lbm3_host {

// Kinds of pass: one step (optionally with the diagnostics), or the
// fields + diagnostics pass.
enum Pass3 { P3_STEP, P3_STEP_REDUCE, P3_FIELDS_REDUCE };

// Launch one pass (the density pass, then the collide pass with the
// instance selected by the brick bx x by x bz with tz threads in z, the
// rounding mode and the
// pass); returns the launch status.
template <int S>
hipError_t launch3(const lbm3::KParams3<typename lbm::Traits<S>::C> &p, Pass3 pass, int bx, int by, int bz, int tz,
                   bool sr, hipStream_t st);

extern template hipError_t launch3<lbm::ST_F64>(const lbm3::KParams3<double> &, Pass3, int, int, int, int, bool,
                                                  hipStream_t);
extern template hipError_t launch3<lbm::ST_F32>(const lbm3::KParams3<float> &, Pass3, int, int, int, int, bool,
                                                  hipStream_t);
extern template hipError_t launch3<lbm::ST_F16>(const lbm3::KParams3<float> &, Pass3, int, int, int, int, bool,
                                                  hipStream_t);
extern template hipError_t launch3<lbm::ST_BF16>(const lbm3::KParams3<float> &, Pass3, int, int, int, int, bool,
                                                  hipStream_t);

}  // namespace lbm3_host
