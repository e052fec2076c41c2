// Scalar diffusion apply with the basis contractions on bf16 matrix cores.
// (Filled in below by the matrix-core kernel; until then the entry point reports
// HX_EUNSUPPORTED.)
#include "hx_internal.h"

namespace hx {

hx_status launch_apply_bf16(hx_op_s &op, const float *x, float *y, hipStream_t s) {
  (void)op;
  (void)x;
  (void)y;
  (void)s;
  return fail(HX_EUNSUPPORTED, "the bf16 matrix-core operator is not built yet");
}

}  // namespace hx
