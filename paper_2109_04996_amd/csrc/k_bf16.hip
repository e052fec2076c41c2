// Scalar diffusion apply with the basis contractions on bf16 matrix cores, for the
// Chebyshev preconditioner. Not in the paper (its operators are FP64); the structure is
// the same fused G^T B^T D B G (libCEED section) on an element, with every 1D contraction
// (Benchmarks section: tensor-product sum factorization) done as a small matrix product on
// V_MFMA_F32_16X16X16_BF16: operands rounded to bfloat16, products accumulated in FP32.
//
// Work decomposition: one element per wavefront, four per workgroup, each wavefront with its
// own LDS buffers (so the steps synchronise the wavefront only). Every element is padded to
// 8 x 8 x 8 (nodes and points beyond P or Q are zero; the tables are zero-padded to 8 x 8),
// so one kernel serves every P, Q <= 8. A contraction of dimension d with a table T (8 x 8)
// is T * X_d, X_d the 8 x 64 matrix whose columns are the pairs of the two other indices.
// Two 16-column groups share one MFMA: the A operand is diag(T, T) and the B operand stacks
// the first group's 8 rows over the second's, so the 16 x 16 x 16 product has no zero
// padding and a contraction is two MFMAs. Lane l supplies A[l%16][4(l/16)..+3] and
// B[4(l/16)..+3][l%16] and receives D[4(l/16)..+3][l%16]: its 4 inputs and 4 outputs are the
// same column, entries kb..kb+3 (kb = 0 or 4) along d, of group (l/32) of the pair.
//
// The pointwise operator runs in FP32 on a bfloat16 copy of the stored FP64 qdata. The
// scatter is the atomic-free colored scatter of the FP64 kernels.
#include "bf16_util.h"
#include "hx_internal.h"

namespace hx {

namespace {

__device__ __forceinline__ short to_bf16(float f) { return (short)f32_to_bf16_bits(f); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return bf16_bits_to_f32(h); }

constexpr int kBfMaxQ = 8;
constexpr int kBfWpb = 4;                 // elements (wavefronts) per workgroup
constexpr int kSJ = 10, kSK = 80;         // LDS strides of j and k (i unit stride), padded against bank conflicts
constexpr int kBuf = kSK * 8;             // floats per 8 x 8 x 8 buffer
constexpr int kQdBf16 = 6 * 512;          // bf16 qdata values per element (padded to 8 x 8 x 8 points)

__device__ __forceinline__ int at8(int i, int j, int k) { return i + kSJ * j + kSK * k; }

// An operand carried as hi + lo, both bfloat16 (lo = the rounding error of hi): products of
// such pairs, hi*hi + hi*lo + lo*hi accumulated in FP32, carry about 16 significant bits.
struct Opnd {
  bf16x4 hi, lo;
};

__device__ __forceinline__ short bf16_hi(float v) { return (short)f32_to_bf16_bits(v); }
__device__ __forceinline__ short bf16_lo(float v, short hi) { return to_bf16(v - bf16_bits_to_f32((uint16_t)hi)); }

// A operand diag(T, T) of a table T (rows x cols, row-major FP32, zero-padded to 8 x 8), or of
// its transpose: lane l holds A[l%16][4(l/16)+t].
__device__ __forceinline__ Opnd diag_operand(const float *__restrict__ T, int rows, int cols, bool transpose,
                                             int l) {
  const int m = l & 15, kb = 4 * (l >> 4);
  Opnd a;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int kk = kb + t;
    float v = 0.f;
    if ((m >> 3) == (kk >> 3)) {
      const int r = m & 7, c = kk & 7;
      if (!transpose) {
        if (r < rows && c < cols) v = T[r * cols + c];
      } else if (c < rows && r < cols) {
        v = T[c * cols + r];  // (T^T)[r][c] = T[c][r]
      }
    }
    const short h = bf16_hi(v);
    a.hi[t] = h;
    a.lo[t] = bf16_lo(v, h);
  }
  return a;
}

// Y = T x_DIM X on 8 x 8 x 8 buffers (A = diag(T, T)); ACC adds into Y. X and Y may not be the
// same buffer unless every lane's column is its own (it is: a lane reads and writes one column).
template <int DIM, bool ACC, bool SPLIT>
__device__ __forceinline__ void contract8(const float *X, float *Y, const Opnd &A, int l) {
  constexpr int sd = DIM == 0 ? 1 : DIM == 1 ? kSJ : kSK;  // stride of the contracted index
  constexpr int su = DIM == 0 ? kSJ : 1;                   // the two other indices (u, v), u first
  constexpr int sv = DIM == 2 ? kSJ : kSK;
  const int col = l & 15, kq = l >> 4, grp = kq >> 1, kb = 4 * (kq & 1);
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const int c = (2 * pair + grp) * 16 + col;  // column 0..63 = u + 8 v
    const int base = (c & 7) * su + (c >> 3) * sv + kb * sd;
    bf16x4 b, blo;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float v = X[base + t * sd];
      const short h = bf16_hi(v);
      b[t] = h;
      if (SPLIT) blo[t] = bf16_lo(v, h);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.hi, b, acc, 0, 0, 0);
    if (SPLIT) {
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.hi, blo, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.lo, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (ACC)
        Y[base + t * sd] += acc[t];
      else
        Y[base + t * sd] = acc[t];
    }
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// idx: one node id per element node, or (AFF) {base, s_j, s_k} per element (node (i, j, k) =
// base + i + j s_j + k s_k). Every global load the element needs -- its x, the old y of the
// nodes it read-modify-writes (no other element of this launch touches them) and its qdata --
// is issued before the first contraction, so their latencies overlap the matrix-core chain.
template <bool AFF, bool SPLIT>
__global__ void __launch_bounds__(kBfWpb * 64)
    k_diff_bf16(int P, int Q, const int32_t *__restrict__ idx, const uint16_t *__restrict__ own,
                const uint16_t *__restrict__ qd16, const float *__restrict__ tab, const float *__restrict__ x,
                float *__restrict__ y, int64_t e_begin, int64_t e_end, const float *__restrict__ zero) {
  __shared__ float sbuf[kBfWpb][3][kBuf];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int64_t e = e_begin + (int64_t)blockIdx.x * kBfWpb + w;
  const bool live = e < e_end;
  const int64_t ee = live ? e : e_begin;
  float *const U = sbuf[w][0];
  float *const G0 = sbuf[w][1];
  float *const G1 = sbuf[w][2];
  const int P2 = P * P, P3 = P2 * P;
  // node lane (i, j) walks its column k; point lane (a, b) walks its column c
  const int gi = l & 7, gj = l >> 3;
  const bool node_lane = live && gi < P && gj < P;
  int32_t nid[8];
  if constexpr (AFF) {
    const int32_t *af = idx + ee * 4;
    const int32_t base = af[0] + gi + gj * af[1], sk = af[2];
#pragma unroll
    for (int k = 0; k < 8; ++k) nid[k] = base + k * sk;
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) nid[k] = (node_lane && k < P) ? idx[ee * P3 + gi + P * gj + P2 * k] : 0;
  }
  const uint32_t ob = node_lane ? (uint32_t)own[ee * P2 + gj * P + gi] : 0xffffu;
  float u[8], old[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bool in = node_lane && k < P;
    const float xv = x[in ? nid[k] : 0];  // lanes off the element read a valid address and drop it
    u[k] = in ? xv : 0.f;
    old[k] = *((in && !(ob & (1u << k))) ? y + nid[k] : zero);
  }
  // qdata of this lane's point row (qa = 0..7 at qb = l % 8, qc = l / 8): six 16-byte loads from
  // the padded bf16 copy [e][qc][m][qb][qa] (8 x 6 x 8 x 8 per element, zero past Q)
  const int pb = l & 7, pc = l >> 3;
  uint4 g[6];
  {
    const uint4 *qv = reinterpret_cast<const uint4 *>(qd16 + ee * (int64_t)kQdBf16 + (pc * 6) * 64 + pb * 8);
#pragma unroll
    for (int m = 0; m < 6; ++m) g[m] = qv[m * 8];  // planes (pc, m) are 64 values = 8 uint4 apart
  }

  const float *tI = tab, *tD = tab + Q * P;                 // interp [Q][P], q-point derivative [Q][Q]
  const Opnd aI = diag_operand(tI, Q, P, false, l);   // nodes -> points
  const Opnd aIt = diag_operand(tI, Q, P, true, l);   // points -> nodes
  const Opnd aD = diag_operand(tD, Q, Q, false, l);
  const Opnd aDt = diag_operand(tD, Q, Q, true, l);
#pragma unroll
  for (int k = 0; k < 8; ++k) U[at8(gi, gj, k)] = u[k];
  wave_lds_sync();
  // interpolate to the points: (a, j, k) -> (a, b, k) -> (a, b, c)
  contract8<0, false, SPLIT>(U, G0, aI, l);
  wave_lds_sync();
  contract8<1, false, SPLIT>(G0, G1, aI, l);
  wave_lds_sync();
  contract8<2, false, SPLIT>(G1, U, aI, l);
  wave_lds_sync();
  // reference gradient at the points: ur -> G0, us -> G1, ut -> U (in place: a lane reads and
  // writes only its own column)
  contract8<0, false, SPLIT>(U, G0, aD, l);
  contract8<1, false, SPLIT>(U, G1, aD, l);
  wave_lds_sync();
  contract8<2, false, SPLIT>(U, U, aD, l);
  wave_lds_sync();
  // pointwise: (vr, vs, vt) = G (ur, us, ut) on the lane's point row; padded points have G = 0
#pragma unroll
  for (int qa = 0; qa < 8; ++qa) {
    const int pt = at8(qa, pb, pc);
    float gm[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const uint32_t word = qa < 2 ? g[m].x : qa < 4 ? g[m].y : qa < 6 ? g[m].z : g[m].w;
      gm[m] = (qa & 1) ? __builtin_bit_cast(float, word & 0xffff0000u) : __builtin_bit_cast(float, word << 16);
    }
    const float g0 = gm[0], g1 = gm[1], g2 = gm[2], g3 = gm[3], g4 = gm[4], g5 = gm[5];
    const float ur = G0[pt], us = G1[pt], ut = U[pt];
    G0[pt] = g0 * ur + g1 * us + g2 * ut;
    G1[pt] = g1 * ur + g3 * us + g4 * ut;
    U[pt] = g2 * ur + g4 * us + g5 * ut;
  }
  wave_lds_sync();
  // transposed gradient, summed into U
  contract8<2, false, SPLIT>(U, U, aDt, l);
  wave_lds_sync();
  contract8<0, true, SPLIT>(G0, U, aDt, l);
  wave_lds_sync();
  contract8<1, true, SPLIT>(G1, U, aDt, l);
  wave_lds_sync();
  // transposed interpolation back to the nodes: (a, b, c) -> (a, b, k) -> (a, j, k) -> (i, j, k)
  contract8<2, false, SPLIT>(U, G0, aIt, l);
  wave_lds_sync();
  contract8<1, false, SPLIT>(G0, G1, aIt, l);
  wave_lds_sync();
  contract8<0, false, SPLIT>(G1, U, aIt, l);
  wave_lds_sync();
  // colored scatter: owners store, the others add to the old value loaded above
  if (node_lane) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < P) y[nid[k]] = old[k] + U[at8(gi, gj, k)];
  }
}

// FP64 qdata [e][qc][m][qb][qa] (Q^3 points) -> bfloat16 [e][qc][m][qb][qa] padded to 8 x 8 x 8
// points, zero past Q (round to nearest even)
__global__ void k_qdata_bf16(int64_t nout, int Q, const double *__restrict__ a, uint16_t *__restrict__ b) {
  const int Q2 = Q * Q, Q3 = Q2 * Q;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nout; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / kQdBf16;
    const int r = (int)(t - e * kQdBf16);
    const int qc = r / 384, m = (r / 64) % 6, qb = (r / 8) % 8, qa = r % 8;
    float v = 0.f;
    if (qa < Q && qb < Q && qc < Q) v = (float)a[e * 6 * Q3 + (qc * 6 + m) * Q2 + qb * Q + qa];
    b[t] = f32_to_bf16_bits(v);
  }
}

}  // namespace

hx_status launch_apply_bf16(hx_op_s &op, bool split, const float *x, float *y, hipStream_t s) {
  if (op.kind != HX_DIFFUSION || op.ncomp != 1) return fail(HX_EUNSUPPORTED, "the bf16 operator supports scalar diffusion only");
  if (op.P > kBfMaxQ || op.Q > kBfMaxQ) return fail(HX_EUNSUPPORTED, "the bf16 operator supports p+1 <= 8 and q <= 8");
  if (!op.qdata_bf16.ptr) {
    const int64_t nout = op.mesh->nelem * (int64_t)kQdBf16;
    HX_HIP(op.qdata_bf16.alloc((size_t)nout));
    hipLaunchKernelGGL(k_qdata_bf16, dim3(1024), dim3(256), 0, s, nout, op.Q, op.qdata.ptr, op.qdata_bf16.ptr);
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
  const float *zero = reinterpret_cast<const float *>(m.zeros.ptr);
  for (int c = 0; c < m.ncolors; ++c) {
    const int64_t e0 = m.color_start[c], e1 = m.color_start[c + 1];
    if (e1 <= e0) continue;
    const dim3 grid((unsigned)((e1 - e0 + kBfWpb - 1) / kBfWpb)), block(kBfWpb * 64);
    if (m.idx_affine.ptr) {
      if (split)
        hipLaunchKernelGGL((k_diff_bf16<true, true>), grid, block, 0, s, op.P, op.Q, m.idx_affine.ptr, m.own.ptr,
                           op.qdata_bf16.ptr, op.tab_bf16.ptr, x, y, e0, e1, zero);
      else
        hipLaunchKernelGGL((k_diff_bf16<true, false>), grid, block, 0, s, op.P, op.Q, m.idx_affine.ptr, m.own.ptr,
                           op.qdata_bf16.ptr, op.tab_bf16.ptr, x, y, e0, e1, zero);
    } else {
      if (split)
        hipLaunchKernelGGL((k_diff_bf16<false, true>), grid, block, 0, s, op.P, op.Q, m.idx.ptr, m.own.ptr,
                           op.qdata_bf16.ptr, op.tab_bf16.ptr, x, y, e0, e1, zero);
      else
        hipLaunchKernelGGL((k_diff_bf16<false, false>), grid, block, 0, s, op.P, op.Q, m.idx.ptr, m.own.ptr,
                           op.qdata_bf16.ptr, op.tab_bf16.ptr, x, y, e0, e1, zero);
    }
  }
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace hx
