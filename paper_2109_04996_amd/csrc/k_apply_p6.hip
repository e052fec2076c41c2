// Fused apply kernels for 6 nodes per direction (degree 5).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<6>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
