// Fused apply kernels for 7 nodes per direction (degree 6).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<7>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
