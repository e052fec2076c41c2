// Fused apply kernels for 4 nodes per direction (degree 3).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<4>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
