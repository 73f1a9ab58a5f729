// Step-kernel instances for F32 storage (see lbm_launch.hpp).
#include "lbm_launch_impl.hpp"

namespace lbm_host {
template hipError_t launch_pass<lbm::ST_F32>(const lbm::KParams<float> &, Pass, int, bool, bool, hipStream_t, bool);
template int step_occupancy<lbm::ST_F32>(int);
}  // namespace lbm_host
