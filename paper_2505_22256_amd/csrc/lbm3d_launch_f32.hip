// 3-D step-kernel instances for one storage type (compiled on their own).
#include "lbm3d_launch_impl.hpp"

namespace lbm3_host {
template hipError_t launch3<lbm::ST_F32>(const lbm3::KParams3<typename lbm::Traits<lbm::ST_F32>::C> &, Pass3, int, int, int, int, bool,
                                    hipStream_t);
}  // namespace lbm3_host
