// Fused apply kernels for 9 nodes per direction (degree 8).
#include "apply_launch.h"

namespace hx {
template hx_status launch_apply_P<9>(const hx_op_s &, Prec, bool, const ApplyArgs &, hipStream_t);
}  // namespace hx
