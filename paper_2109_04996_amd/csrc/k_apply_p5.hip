// Fused apply kernels for 5 nodes per direction (degree 4).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<5>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
