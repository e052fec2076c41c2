// Internal declarations of the two-layer network (not part of the ABI).
#pragma once

#include "bf16_util.h"
#include "hx_internal.h"

struct hx_mlp_s {
  int n_in = 0, n_hid = 0, n_out = 0;
  int64_t nparam = 0, off_W1 = 0, off_b1 = 0, off_W2 = 0, off_b2 = 0;  // offsets into p / g
  hx::DevBuf<float> p;   // W1 (n_hid x n_in), b1, W2 (n_out x n_hid), b2: FP32
  hx::DevBuf<float> g;   // gradients, same layout
  hx::DevBuf<uint16_t> W1b, W2b;  // bf16 copies for inference
  bool bf16_valid = false;
  int64_t adam_t = 0;
  // work buffers
  hx::DevBuf<float> hact, yout, dy, dz;
  hx::DevBuf<uint16_t> act16;
  hx::DevBuf<double> part;
};

namespace hx {
hx_status mlp_refresh_bf16(hx_mlp_s &net, hipStream_t s);
hx_status mlp_forward_bf16(hx_mlp_s &net, const float *X, int64_t batch, float *Y, hipStream_t s);
// both layers on bf16 inputs (rows of n_in), bf16 hidden activations H16 (rows of n_hidden), FP32 output
// row_scale (optional, [batch]) multiplies each row of the output layer
hx_status mlp_layers_bf16(hx_mlp_s &net, const uint16_t *X16, int64_t batch, uint16_t *H16, float *Y, hipStream_t s,
                          const float *row_scale = nullptr);
// per-operator set-up of the learned preconditioner (node log kappa, element features and scales,
// partition-of-unity weights); done once, on first use
hx_status mlp_prepare(hx_op_s &op, hipStream_t s);
// learned preconditioner z = D^-1/2 G^T (w * |r~_e| * net(features_e(r))), FP64 L-vectors; mode 1 adds the
// Jacobi step D^-1 r (0 on constrained nodes)
hx_status mlp_precond_apply(hx_op_s &op, hx_mlp_s &net, int mode, const double *r, double *z, hipStream_t s);
}  // namespace hx
