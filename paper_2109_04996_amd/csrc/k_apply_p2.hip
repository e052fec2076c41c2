// Fused apply kernels for 2 nodes per direction (degree 1).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<2>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
