// Learned element-local preconditioner (not in the paper): an approximate inverse of the
// operator's element blocks, in Jacobi-scaled variables.
//
// With D the assembled diagonal and r~ = D^-1/2 r (zero on constrained nodes), element e sees
//   x_e = [ r~_e / |r~_e| , f_e ]                                  (2 (p+1)^3 values)
// where r~_e = G_e r~ is the element restriction (libCEED section: G) and f_e the element's
// log kappa at its nodes minus its mean, with the marker value kConstrained on constrained
// nodes. The network's output, scaled back by |r~_e|, is an element correction c_e in the
// scaled variables; the corrections are averaged at shared nodes (w = 1/multiplicity, a
// partition of unity, 0 on constrained nodes), summed over the elements of each node in a fixed
// order (G^T as a node-wise gather, no atomics), and mapped back: z = D^-1/2 G^T (w |r~_e| net(x_e)).
// In scaled variables the element block D_e^-1/2 A_ee D_e^-1/2 no longer depends on the size of
// kappa or of the element, so one network serves all elements and mesh sizes; trained on
// c_e = D_e^1/2 e_e - r~_e with e_e = A_ee^-1 r_e, z + D^-1 r is a restricted additive
// Schwarz step over element blocks.
//
// Hot path: k_mlp_in (gather + scale + norm into bf16 rows, a wavefront per element), two bf16 matrix-core layers over all
// elements (mlp.hip), k_mlp_gather_out (the node-wise sum over each node's element slots, with the
// D^-1 r term of mode 1).
#include <algorithm>
#include <cmath>

#include "mlp_internal.h"

namespace hx {

namespace {

constexpr int kThreads = 256;
constexpr float kConstrained = 3.0f;  // feature marker of a constrained node (|f| < 3 on free nodes)

__device__ __forceinline__ double block_sum_d(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// log kappa at every node: s * sqrt(2/M) sum_m cos(omega_m . x + b_m) + t
__global__ void k_node_logkappa(int64_t n, const double *__restrict__ xyz, int M, const double *__restrict__ om,
                                const double *__restrict__ ph, double scale, double shift, float *__restrict__ logk) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    if (M == 0) {
      logk[t] = 0.f;
      continue;
    }
    const double x = xyz[3 * t], y = xyz[3 * t + 1], z = xyz[3 * t + 2];
    double g = 0.0;
    for (int m = 0; m < M; ++m) g += cos(om[3 * m] * x + om[3 * m + 1] * y + om[3 * m + 2] * z + ph[m]);
    logk[t] = (float)(scale * sqrt(2.0 / M) * g + shift);
  }
}

// per element (internal order): log kappa minus its element mean, kConstrained on constrained nodes (bf16)
__global__ void __launch_bounds__(kThreads)
    k_elem_prep(int P, const int32_t *__restrict__ idx, const float *__restrict__ logk, const uint8_t *__restrict__ fm,
                uint16_t *__restrict__ feat) {
  __shared__ double sh[kThreads];
  const int64_t e = blockIdx.x;
  const int P3 = P * P * P;
  double sl = 0.0;
  for (int l = threadIdx.x; l < P3; l += kThreads) sl += logk[idx[e * P3 + l]];
  const double mean_l = block_sum_d(sl, sh) / P3;
  for (int l = threadIdx.x; l < P3; l += kThreads) {
    const int64_t nd = idx[e * P3 + l];
    feat[e * P3 + l] = f32_to_bf16_bits(fm[nd] ? (float)(logk[nd] - mean_l) : kConstrained);
  }
}

// D^-1/2 on free nodes, 0 on constrained ones
__global__ void k_dis(int64_t n, const double *__restrict__ diag, const uint8_t *__restrict__ fm,
                      float *__restrict__ dis) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dis[t] = (fm[t] && diag[t] > 0.0) ? (float)(1.0 / sqrt(diag[t])) : 0.f;
}

// multiplicity: colored scatter of ones (store by the first element, add by later ones)
__global__ void __launch_bounds__(kThreads)
    k_count(int P, const int32_t *__restrict__ idx, const uint16_t *__restrict__ own, float *__restrict__ cnt,
            int64_t e_begin) {
  const int64_t e = e_begin + blockIdx.x;
  const int P2 = P * P, P3 = P2 * P;
  for (int l = threadIdx.x; l < P3; l += kThreads) {
    const int k = l / P2;
    float *dst = cnt + idx[e * P3 + l];
    if ((own[e * P2 + (l % P2)] >> k) & 1u)
      *dst = 1.f;
    else
      *dst += 1.f;
  }
}

__global__ void k_wmult(int64_t n, const uint8_t *__restrict__ fm, float *__restrict__ w) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    w[t] = (fm[t] && w[t] > 0.f) ? 1.f / w[t] : 0.f;
}

// network input of each element: r~_e / |r~_e| into the first half of its bf16 row (internal order; the
// second half, the element's coefficient feature, is written once per operator by k_mlp_feat) and
// |r~_e|. One wavefront per element: each lane keeps its (at most kMaxInW) values in registers while
// the wavefront sums the squares with shuffles (no LDS, no barrier).
// AFF: node ids from the element's affine numbering {base, s_j, s_k} (read with scalar loads) instead of
// the full element restriction, so the gathers do not wait on an index load.
constexpr int kMaxInW = (kMaxP * kMaxP * kMaxP + 63) / 64;
template <bool AFF>
__global__ void __launch_bounds__(kThreads)
    k_mlp_in(int64_t E, int P, const int32_t *__restrict__ idx, const double *__restrict__ r,
             const float *__restrict__ dis, uint16_t *__restrict__ X16, float *__restrict__ rnorm) {
  const int lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (e >= E) return;  // the whole wavefront
  const int P2 = P * P, P3 = P2 * P;
  int32_t base = 0, sj = 0, sk = 0;
  if constexpr (AFF) {
    base = idx[e * 4];
    sj = idx[e * 4 + 1];
    sk = idx[e * 4 + 2];
  }
  double v[kMaxInW];
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kMaxInW; ++q) {
    const int l = lane + 64 * q;
    v[q] = 0.0;
    if (l < P3) {
      const int64_t nd = AFF ? (int64_t)base + l % P + (l / P) % P * sj + l / P2 * sk : idx[e * P3 + l];
      v[q] = (double)dis[nd] * r[nd];
      s += v[q] * v[q];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const double nrm = sqrt(s);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  uint16_t *row = X16 + e * (int64_t)(2 * P3);
#pragma unroll
  for (int q = 0; q < kMaxInW; ++q) {
    const int l = lane + 64 * q;
    if (l < P3) row[l] = f32_to_bf16_bits((float)(v[q] * inv));
  }
  if (lane == 0) rnorm[e] = (float)nrm;
}

// the coefficient half of every element's network input row (constant for an operator)
__global__ void k_mlp_feat(int64_t E, int P3, const uint16_t *__restrict__ feat, uint16_t *__restrict__ X16) {
  const int64_t total = E * P3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / P3, l = t - e * P3;
    X16[e * 2 * P3 + P3 + l] = feat[t];
  }
}

// z[t] = (D^-1/2 w)[t] sum over the element slots of t (ascending) of |r~_e| y_e[l] (Ys holds the output rows
// already scaled by |r~_e|), plus D^-1 r in mode 1 (dinv 0 on constrained nodes): one thread per node, the
// corrections summed in a fixed order (no colors, no atomics).
__global__ void __launch_bounds__(256)
    k_mlp_gather_out(int64_t n, const int32_t *__restrict__ sptr, const int32_t *__restrict__ sslot,
                     const float *__restrict__ Ys, const float *__restrict__ dw, int mode, const double *__restrict__ dinv,
                     const double *__restrict__ r, double *__restrict__ z) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int32_t k = sptr[t]; k < sptr[t + 1]; ++k) s += (double)Ys[sslot[k]];
    double v = (double)dw[t] * s;
    if (mode == 1) v += dinv[t] * r[t];
    z[t] = v;
  }
}

// (D^-1/2 w)[t] and D^-1[t] on free nodes (1 / diag), 0 on constrained ones
__global__ void k_mlp_factors(int64_t n, const float *__restrict__ dis, const float *__restrict__ w,
                              const double *__restrict__ diag, const uint8_t *__restrict__ fm, float *__restrict__ dw,
                              double *__restrict__ dinv) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    dw[t] = (float)((double)dis[t] * (double)w[t]);
    dinv[t] = fm[t] ? 1.0 / diag[t] : 0.0;
  }
}


// training features in caller element order (FP32): [r~_e / |r~_e|, feature]; |r~_e|
__global__ void __launch_bounds__(kThreads)
    k_features_f32(int P, const int32_t *__restrict__ idx, const int32_t *__restrict__ order,
                   const double *__restrict__ r, const float *__restrict__ dis, const uint16_t *__restrict__ feat,
                   float *__restrict__ X, float *__restrict__ rnorm) {
  __shared__ double sh[kThreads];
  const int64_t e = blockIdx.x;
  const int P3 = P * P * P;
  double s = 0.0;
  for (int l = threadIdx.x; l < P3; l += kThreads) {
    const int64_t nd = idx[e * P3 + l];
    const double v = (double)dis[nd] * r[nd];
    s += v * v;
  }
  const double nrm = sqrt(block_sum_d(s, sh));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  float *row = X + (int64_t)order[e] * (2 * P3);
  for (int l = threadIdx.x; l < P3; l += kThreads) {
    const int64_t nd = idx[e * P3 + l];
    row[l] = (float)((double)dis[nd] * r[nd] * inv);
    row[P3 + l] = bf16_bits_to_f32(feat[e * P3 + l]);
  }
  if (threadIdx.x == 0) rnorm[order[e]] = (float)nrm;
}

// training targets in caller element order: D^1/2 err_e / |r~_e| (0 on constrained nodes)
__global__ void __launch_bounds__(kThreads)
    k_targets_f32(int P, const int32_t *__restrict__ idx, const int32_t *__restrict__ order,
                  const double *__restrict__ err, const float *__restrict__ rnorm, const float *__restrict__ dis,
                  float *__restrict__ T) {
  const int64_t e = blockIdx.x;
  const int P3 = P * P * P;
  const int64_t oe = order[e];
  const double d = (double)rnorm[oe];
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  for (int l = threadIdx.x; l < P3; l += kThreads) {
    const int64_t nd = idx[e * P3 + l];
    const double ds = (double)dis[nd];
    T[oe * P3 + l] = ds > 0.0 ? (float)(err[nd] / ds * inv) : 0.f;
  }
}

}  // namespace

hx_status mlp_prepare(hx_op_s &op, hipStream_t s) {
  if (op.mlp_ready) return HX_OK;
  const hx_mesh_s &m = *op.mesh;
  if (op.ncomp != 1 || op.kind != HX_DIFFUSION)
    return fail(HX_EUNSUPPORTED, "the learned preconditioner supports scalar diffusion only");
  const int64_t E = m.nelem, n = m.nnodes;
  const int P3 = op.P * op.P * op.P;
  DevBuf<double> om, ph;
  if (op.kappa_M > 0) {
    HX_HIP(om.upload(op.kappa_omega.data(), op.kappa_omega.size()));
    HX_HIP(ph.upload(op.kappa_phase.data(), op.kappa_phase.size()));
  }
  HX_HIP(op.mlp_logk.alloc(n));
  HX_HIP(op.mlp_feat16.alloc((size_t)E * P3));
  HX_HIP(op.mlp_dis.alloc(n));
  HX_HIP(op.mlp_wmult.alloc(n));
  HX_HIP(op.mlp_rnorm.alloc(E));
  if (!op.diag_valid) {
    if (op.diag.count < (size_t)n) HX_HIP(op.diag.alloc(n));
    if (hx_status st = hx_op_diagonal(&op, op.diag.ptr, s)) return st;
    op.diag_valid = true;
  }
  hipLaunchKernelGGL(k_dis, dim3(2048), dim3(256), 0, s, n, op.diag.ptr, m.freemask.ptr, op.mlp_dis.ptr);
  hipLaunchKernelGGL(k_node_logkappa, dim3(2048), dim3(256), 0, s, n, m.xyz.ptr, op.kappa_M, om.ptr, ph.ptr,
                     op.kappa_scale, op.kappa_shift, op.mlp_logk.ptr);
  hipLaunchKernelGGL(k_elem_prep, dim3((unsigned)E), dim3(kThreads), 0, s, op.P, m.idx.ptr, op.mlp_logk.ptr,
                     m.freemask.ptr, op.mlp_feat16.ptr);
  HX_HIP(hipMemsetAsync(op.mlp_wmult.ptr, 0, sizeof(float) * n, s));
  for (int c = 0; c < m.ncolors; ++c) {
    const int64_t e0 = m.color_start[c], e1 = m.color_start[c + 1];
    if (e1 > e0)
      hipLaunchKernelGGL(k_count, dim3((unsigned)(e1 - e0)), dim3(kThreads), 0, s, op.P, m.idx.ptr, m.own.ptr,
                         op.mlp_wmult.ptr, e0);
  }
  hipLaunchKernelGGL(k_wmult, dim3(2048), dim3(256), 0, s, n, m.freemask.ptr, op.mlp_wmult.ptr);
  if (hx_status st = mesh_slots(*op.mesh)) return st;  // the node -> element slot table of the output gather
  HX_HIP(op.mlp_dw.alloc(n));
  HX_HIP(op.mlp_dinv.alloc(n));
  hipLaunchKernelGGL(k_mlp_factors, dim3(2048), dim3(256), 0, s, n, op.mlp_dis.ptr, op.mlp_wmult.ptr, op.diag.ptr,
                     m.freemask.ptr, op.mlp_dw.ptr, op.mlp_dinv.ptr);
  HX_HIP(hipGetLastError());
  HX_HIP(hipStreamSynchronize(s));  // om/ph are freed on return
  op.mlp_ready = true;
  return HX_OK;
}

hx_status mlp_precond_apply(hx_op_s &op, hx_mlp_s &net, int mode, const double *r, double *z, hipStream_t s) {
  if (mode != 0 && mode != 1) return fail(HX_EINVAL, "mode must be 0 (network correction) or 1 (plus D^-1 r)");
  const int P3 = op.P * op.P * op.P;
  if (net.n_in != 2 * P3 || net.n_out != P3)
    return fail(HX_EINVAL, "network shape must be (2 (p+1)^3 inputs, (p+1)^3 outputs) for this operator");
  if (hx_status st = mlp_prepare(op, s)) return st;
  const hx_mesh_s &m = *op.mesh;
  const int64_t E = m.nelem;
  if (op.mlp_x16.count < (size_t)(E * 2 * P3)) {
    HX_HIP(op.mlp_x16.alloc((size_t)E * 2 * P3));
    op.mlp_x16_feat = false;
    HX_HIP(op.mlp_h16.alloc((size_t)E * net.n_hid));
    HX_HIP(op.mlp_y.alloc((size_t)E * P3));
  }
  if (op.mlp_h16.count < (size_t)(E * net.n_hid)) HX_HIP(op.mlp_h16.alloc((size_t)E * net.n_hid));
  if (!op.mlp_x16_feat) {
    hipLaunchKernelGGL(k_mlp_feat, dim3(2048), dim3(256), 0, s, E, P3, op.mlp_feat16.ptr, op.mlp_x16.ptr);
    op.mlp_x16_feat = true;
  }
  const dim3 gin((unsigned)((E + kThreads / 64 - 1) / (kThreads / 64)));
  if (m.idx_affine.ptr)
    hipLaunchKernelGGL(k_mlp_in<true>, gin, dim3(kThreads), 0, s, E, op.P, m.idx_affine.ptr, r, op.mlp_dis.ptr,
                       op.mlp_x16.ptr, op.mlp_rnorm.ptr);
  else
    hipLaunchKernelGGL(k_mlp_in<false>, gin, dim3(kThreads), 0, s, E, op.P, m.idx.ptr, r, op.mlp_dis.ptr,
                       op.mlp_x16.ptr, op.mlp_rnorm.ptr);
  // the output rows come out scaled by |r~_e|
  if (hx_status st = mlp_layers_bf16(net, op.mlp_x16.ptr, E, op.mlp_h16.ptr, op.mlp_y.ptr, s, op.mlp_rnorm.ptr))
    return st;
  const int64_t n = m.nnodes;
  hipLaunchKernelGGL(k_mlp_gather_out, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s, n,
                     m.slot_ptr.ptr, m.slot_idx.ptr, op.mlp_y.ptr, op.mlp_dw.ptr, mode, op.mlp_dinv.ptr, r, z);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace hx

using namespace hx;

extern "C" hx_status hx_op_mlp_features(hx_op op, const double *r, float *X, float *rnorm, hx_stream stream) {
  if (!op || !r || !X || !rnorm) return fail(HX_EINVAL, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hx_status st = mlp_prepare(*op, s)) return st;
  const hx_mesh_s &m = *op->mesh;
  hipLaunchKernelGGL(k_features_f32, dim3((unsigned)m.nelem), dim3(kThreads), 0, s, op->P, m.idx.ptr,
                     m.order_d.ptr, r, op->mlp_dis.ptr, op->mlp_feat16.ptr, X, rnorm);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

extern "C" hx_status hx_op_mlp_targets(hx_op op, const double *err, const float *rnorm, float *T, hx_stream stream) {
  if (!op || !err || !rnorm || !T) return fail(HX_EINVAL, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hx_status st = mlp_prepare(*op, s)) return st;
  const hx_mesh_s &m = *op->mesh;
  hipLaunchKernelGGL(k_targets_f32, dim3((unsigned)m.nelem), dim3(kThreads), 0, s, op->P, m.idx.ptr, m.order_d.ptr,
                     err, rnorm, op->mlp_dis.ptr, T);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

extern "C" hx_status hx_op_mlp_precond(hx_op op, hx_mlp net, int mode, const double *r, double *z,
                                       hx_stream stream) {
  if (!op || !net || !r || !z) return fail(HX_EINVAL, "null argument");
  if (r == z) return fail(HX_EINVAL, "z must not alias r");
  return mlp_precond_apply(*op, *net, mode, r, z, static_cast<hipStream_t>(stream));
}
