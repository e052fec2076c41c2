// Scalar diffusion apply with the basis contractions on bf16 matrix cores, for the
// Chebyshev preconditioner. Not in the paper (its operators are FP64); the structure is
// the same fused G^T B^T D B G (libCEED section) on an element, with every 1D contraction
// (Benchmarks section: tensor-product sum factorization) done as a small matrix product on
// V_MFMA_F32_16X16X16_BF16: operands rounded to bfloat16, products accumulated in FP32.
//
// Work decomposition: one element per wavefront. A contraction of dimension d of a 3-D
// array X (held in LDS as FP32) with a 1D table T (m_out x n_d) is the product
// T (m_out x n_d) * X_d (n_d x columns), the columns being the pairs of the two other
// indices (at most 64 for q <= 8), taken 16 at a time: one MFMA per 16 columns, with T
// and the column block zero-padded to 16 x 16. Lane l supplies T[l%16][4(l/16)..+3] (A
// operand) and X[4(l/16)..+3][column l%16] (B operand), and receives
// Y[4(l/16)..+3][column l%16] (accumulator).
//
// The pointwise operator runs in FP32 on a bfloat16 copy of the stored FP64 qdata. The
// scatter is the atomic-free colored scatter of the FP64 kernels.
#include "bf16_util.h"
#include "hx_internal.h"

namespace hx {

namespace {

__device__ __forceinline__ short to_bf16(float f) { return (short)f32_to_bf16_bits(f); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return bf16_bits_to_f32(h); }

// A operand of a table T (rows x cols, row-major, FP32 in LDS), optionally transposed:
// lane l holds T[l%16][4(l/16)+t] (or T^T), zero outside the table.
__device__ __forceinline__ bf16x4 table_operand(const float *T, int rows, int cols, bool transpose) {
  const int l = threadIdx.x & 63, m = l & 15, kb = 4 * (l >> 4);
  bf16x4 a;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kb + t;
    float v = 0.f;
    if (!transpose) {
      if (m < rows && k < cols) v = T[m * cols + k];
    } else {
      // (T^T)[m][k] = T[k][m]; T^T has cols rows and rows cols
      if (m < cols && k < rows) v = T[k * cols + m];
    }
    a[t] = to_bf16(v);
  }
  return a;
}

// Y = A x_d X: contract dimension DIM (0 fastest) of X (sizes n0, n1, n2 along dims 0, 1, 2, strides
// 1, n0, n0*n1) with the operand A (m_out rows, n_d columns); Y has dimension DIM replaced by m_out
// and the same stride convention. ACC: add into Y instead of overwriting.
template <int DIM, bool ACC>
__device__ __forceinline__ void contract(const float *X, int n0, int n1, int n2, float *Y, int m_out, bf16x4 A) {
  const int l = threadIdx.x & 63, col = l & 15, kb = 4 * (l >> 4);
  const int nd = DIM == 0 ? n0 : DIM == 1 ? n1 : n2;
  // the two other dimensions, in increasing order: (u, v) with sizes (nu, nv)
  const int nu = DIM == 0 ? n1 : n0, nv = DIM == 2 ? n1 : n2;
  // input strides
  const int sx0 = 1, sx1 = n0, sx2 = n0 * n1;
  const int sxd = DIM == 0 ? sx0 : DIM == 1 ? sx1 : sx2;
  const int sxu = DIM == 0 ? sx1 : sx0, sxv = DIM == 2 ? sx1 : sx2;
  // output sizes and strides (dimension DIM has m_out entries)
  const int y0 = DIM == 0 ? m_out : n0, y1 = DIM == 1 ? m_out : n1;
  const int sy1 = y0, sy2 = y0 * y1;
  const int syd = DIM == 0 ? 1 : DIM == 1 ? sy1 : sy2;
  const int syu = DIM == 0 ? sy1 : 1, syv = DIM == 2 ? sy1 : sy2;
  const int ncols = nu * nv;
  for (int c0 = 0; c0 < ncols; c0 += 16) {
    const int c = c0 + col;
    const bool cv = c < ncols;
    const int u = cv ? c % nu : 0, v = cv ? c / nu : 0;
    bf16x4 b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = kb + t;
      b[t] = to_bf16((cv && k < nd) ? X[k * sxd + u * sxu + v * sxv] : 0.f);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, b, acc, 0, 0, 0);
    if (cv) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = kb + t;
        if (r < m_out) {
          float *dst = Y + r * syd + u * syu + v * syv;
          if (ACC)
            *dst += acc[t];
          else
            *dst = acc[t];
        }
      }
    }
  }
}

constexpr int kBfMaxQ = 8;
constexpr int kBfBuf = kBfMaxQ * kBfMaxQ * kBfMaxQ;

__global__ void __launch_bounds__(64)
    k_diff_bf16(int P, int Q, const int32_t *__restrict__ idx, const uint16_t *__restrict__ own,
                const uint16_t *__restrict__ qd16, const float *__restrict__ tab, const float *__restrict__ x,
                float *__restrict__ y, int64_t e_begin) {
  __shared__ float X0[kBfBuf], X1[kBfBuf], X2[kBfBuf], X3[kBfBuf];
  __shared__ float sI[kBfMaxQ * kBfMaxQ], sD[kBfMaxQ * kBfMaxQ];
  const int l = threadIdx.x;
  const int64_t e = e_begin + blockIdx.x;
  const int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
  for (int t = l; t < Q * P; t += 64) sI[t] = tab[t];
  for (int t = l; t < Q * Q; t += 64) sD[t] = tab[Q * P + t];
  // gather u into X0 [k][j][i]
  for (int t = l; t < P3; t += 64) X0[t] = x[idx[e * P3 + t]];
  __syncthreads();
  const bf16x4 aI = table_operand(sI, Q, P, false);   // interp: Q x P
  const bf16x4 aIt = table_operand(sI, Q, P, true);   // transposed interp: P x Q
  const bf16x4 aD = table_operand(sD, Q, Q, false);   // derivative on the q points: Q x Q
  const bf16x4 aDt = table_operand(sD, Q, Q, true);   // its transpose
  // interpolate to the q^3 points
  contract<0, false>(X0, P, P, P, X1, Q, aI);  // X1: (Q, P, P)
  __syncthreads();
  contract<1, false>(X1, Q, P, P, X2, Q, aI);  // X2: (Q, Q, P)
  __syncthreads();
  contract<2, false>(X2, Q, Q, P, X3, Q, aI);  // X3: (Q, Q, Q) = u at the points
  __syncthreads();
  // reference gradient at the points
  contract<0, false>(X3, Q, Q, Q, X0, Q, aD);
  contract<1, false>(X3, Q, Q, Q, X1, Q, aD);
  contract<2, false>(X3, Q, Q, Q, X2, Q, aD);
  __syncthreads();
  // pointwise: (vr, vs, vt) = G (ur, us, ut), qdata layout [e][qc][m][qb][qa]
  const uint16_t *qe = qd16 + e * (int64_t)(6 * Q3);
  for (int pt = l; pt < Q3; pt += 64) {
    const int qc = pt / Q2, ab = pt - qc * Q2;
    const uint16_t *g = qe + qc * 6 * Q2 + ab;
    const float g0 = from_bf16(g[0]), g1 = from_bf16(g[Q2]), g2 = from_bf16(g[2 * Q2]);
    const float g3 = from_bf16(g[3 * Q2]), g4 = from_bf16(g[4 * Q2]), g5 = from_bf16(g[5 * Q2]);
    const float ur = X0[pt], us = X1[pt], ut = X2[pt];
    X0[pt] = g0 * ur + g1 * us + g2 * ut;
    X1[pt] = g1 * ur + g3 * us + g4 * ut;
    X2[pt] = g2 * ur + g4 * us + g5 * ut;
  }
  __syncthreads();
  // transposed gradient, summed into X3
  contract<0, false>(X0, Q, Q, Q, X3, Q, aDt);
  __syncthreads();
  contract<1, true>(X1, Q, Q, Q, X3, Q, aDt);
  __syncthreads();
  contract<2, true>(X2, Q, Q, Q, X3, Q, aDt);
  __syncthreads();
  // transposed interpolation back to the nodes
  contract<2, false>(X3, Q, Q, Q, X0, P, aIt);  // (Q, Q, P)
  __syncthreads();
  contract<1, false>(X0, Q, Q, P, X1, P, aIt);  // (Q, P, P)
  __syncthreads();
  contract<0, false>(X1, Q, P, P, X2, P, aIt);  // (P, P, P)
  __syncthreads();
  // colored scatter: thread (i, j) walks the column k
  if (l < P2) {
    const uint32_t ob = own[e * P2 + l];
    for (int k = 0; k < P; ++k) {
      const int t = l + k * P2;
      float *dst = y + idx[e * P3 + t];
      const float v = X2[t];
      if (ob & (1u << k))
        *dst = v;
      else
        *dst += v;
    }
  }
}

__global__ void k_qdata_bf16(int64_t n, const double *__restrict__ a, uint16_t *__restrict__ b) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = f32_to_bf16_bits((float)a[t]);
}

}  // namespace

hx_status launch_apply_bf16(hx_op_s &op, const float *x, float *y, hipStream_t s) {
  if (op.kind != HX_DIFFUSION || op.ncomp != 1) return fail(HX_EUNSUPPORTED, "the bf16 operator supports scalar diffusion only");
  if (op.P > kBfMaxQ || op.Q > kBfMaxQ) return fail(HX_EUNSUPPORTED, "the bf16 operator supports p+1 <= 8 and q <= 8");
  if (!op.qdata_bf16.ptr) {
    HX_HIP(op.qdata_bf16.alloc(op.qdata.count));
    hipLaunchKernelGGL(k_qdata_bf16, dim3(1024), dim3(256), 0, s, (int64_t)op.qdata.count, op.qdata.ptr,
                       op.qdata_bf16.ptr);
    // tables: interp [Q][P] then the q-point derivative [Q][Q] (for the collocated rule: identity, D)
    std::vector<float> t;
    if (op.colloc) {
      t.assign((size_t)op.Q * op.P, 0.f);
      for (int a = 0; a < op.Q; ++a) t[(size_t)a * op.P + a] = 1.f;
      for (double v : op.b.grad) t.push_back((float)v);
    } else {
      for (double v : op.b.interp) t.push_back((float)v);
      for (double v : op.b.colloc) t.push_back((float)v);
    }
    HX_HIP(op.tab_bf16.upload(t.data(), t.size()));
  }
  const hx_mesh_s &m = *op.mesh;
  if (m.nuntouched > 0) HX_HIP(hipMemsetAsync(y, 0, sizeof(float) * m.nnodes, s));
  for (int c = 0; c < m.ncolors; ++c) {
    const int64_t e0 = m.color_start[c], e1 = m.color_start[c + 1];
    if (e1 <= e0) continue;
    hipLaunchKernelGGL(k_diff_bf16, dim3((unsigned)(e1 - e0)), dim3(64), 0, s, op.P, op.Q, m.idx.ptr, m.own.ptr,
                       op.qdata_bf16.ptr, op.tab_bf16.ptr, x, y, e0);
  }
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace hx
