// Step-kernel instances for F64 storage (see lbm_launch.hpp).
#include "lbm_launch_impl.hpp"

namespace lbm_host {
template hipError_t launch_pass<lbm::ST_F64>(const lbm::KParams<double> &, Pass, int, bool, bool, hipStream_t, bool);
template int step_occupancy<lbm::ST_F64>(int);
}  // namespace lbm_host
