// Fused apply kernels for 3 nodes per direction (degree 2).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<3>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
