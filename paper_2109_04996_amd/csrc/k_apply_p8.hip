// Fused apply kernels for 8 nodes per direction (degree 7).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<8>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
