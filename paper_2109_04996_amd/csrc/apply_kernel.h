// Fused matrix-free operator apply on gfx950: y = G^T B^T D B G x in one pass.
//
// libCEED section (operator decomposition) and the Nek/MFEM section: the
// element restriction G, the basis evaluation B, the pointwise operator D at
// the quadrature points and the transposes are fused into one kernel, so the
// E-vectors and Q-vectors never leave the chip. Benchmarks section: B and its
// gradient are applied by tensor-product sum factorization -- three 1D
// contractions, one per reference direction -- never as dense element
// matrices.
//
// Work decomposition (one element per Q x Q thread tile):
//   thread (a, b) owns the column of points (a, b, 0..Q-1) along r3;
//   contractions along r3 run in registers over that column, contractions
//   along r1 and r2 read the element's plane of values from LDS.
// Per element, LDS holds three Q^3 buffers; several elements share a block
// (EPB) to fill 64-wide wavefronts.
//
// Kinds:
//   MODE_COLLOC  diffusion with q = p+1 GLL points on the nodes (BP5/BP6):
//                B is the identity, only the 1D derivative matrix D is used.
//   MODE_DIFF    diffusion with an interpolation step (BP3/BP4): interpolate
//                to the q^3 points with the 1D table, differentiate there with
//                the collocated derivative matrix of the q points.
//   MODE_MASS    mass (BP1/BP2): interpolate, scale by w detJ, project back.
// Pointwise data (qdata) per element: mass w*detJ; diffusion the 6 entries
// G11 G12 G13 G22 G23 G33 of w*kappa*detJ*J^-1 J^-T. Layout [e][qc][m][qb][qa]:
// plane by plane along r3, the components of a plane next to each other, so a
// wavefront reads each component of a plane as one contiguous run.
// HELM (the Helmholtz operator alpha A + beta B of the bake-off problems): the
// diffusion kinds also read qm [e][qc][qb][qa], beta * w * detJ, and add the
// mass term qm * u at each point to the field that the transposed basis sums.
//
// Scatter: no atomics. Elements of one launch never share a node (coloring);
// bit k of own[e][j][i] says element e is the first to write node (i,j,k),
// which it then stores; every later element read-modify-writes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hx {

enum { MODE_COLLOC = 0, MODE_DIFF = 1, MODE_MASS = 2 };

template <int Q>
struct EpbOf {
  // elements per block: fill whole wavefronts where Q^2 does not divide 64
  static constexpr int v = (Q == 2) ? 16 : (Q == 3) ? 7 : (Q == 4) ? 4 : (Q == 5) ? 5 : (Q == 6) ? 7
                         : (Q == 7) ? 5 : (Q == 8) ? 2 : (Q == 9) ? 3 : 2;
};

template <int P, int Q, int MODE>
struct TabLayout {
  // table offsets in units of T: collocated D [P][P]; otherwise interp [Q][P] then colloc [Q][Q]
  static constexpr int interp = 0;
  static constexpr int dq = (MODE == MODE_COLLOC) ? 0 : Q * P;
  static constexpr int size = (MODE == MODE_COLLOC) ? P * P : Q * P + Q * Q;
};

// Work item of block bid in a launch of G blocks. The hardware deals consecutive blocks
// round-robin to the 8 XCDs; item = the block's place in a contiguous run per XCD, so consecutive
// items -- the components of one element, then spatially neighbouring elements -- share an XCD
// and its L2.
__device__ __forceinline__ int xcd_item(int bid, int G) {
  const int xcd = bid & 7, loc = bid >> 3, base = G >> 3, rem = G & 7;
  return xcd * base + (xcd < rem ? xcd : rem) + loc;
}

// qdata loads: streaming (nontemporal) for one component; cached for several, whose workgroups
// (adjacent work items on one XCD) read the same qdata
template <int NC, typename TQ, typename T>
__device__ __forceinline__ T ld_q(const TQ *p) {
  if constexpr (NC > 1)
    return static_cast<T>(*p);
  else
    return static_cast<T>(__builtin_nontemporal_load(p));
}

// IDX: node ids, 0 one per element node, 2 the element's affine numbering {base, s_j, s_k} (16 bytes
// per element instead of 4 P^3)
template <int P, int Q, int MODE, int NC, typename T, typename TQ, bool EOUT, int IDX, bool HELM = false>
__global__ void __launch_bounds__(EpbOf<Q>::v * Q * Q) __attribute__((amdgpu_waves_per_eu(2)))
    k_apply(const int32_t *__restrict__ idx, const uint16_t *__restrict__ own, const TQ *__restrict__ qd,
            const T *__restrict__ tab, const T *__restrict__ x, T *__restrict__ y,
            const int32_t *__restrict__ order, int64_t e_begin, int64_t e_end, const TQ *__restrict__ qm = nullptr) {
  static_assert(!HELM || MODE != MODE_MASS, "the Helmholtz mass term rides on a diffusion kind");
  constexpr int EPB = EpbOf<Q>::v;
  constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
  constexpr int NCQ = (MODE == MODE_MASS) ? 1 : 6;
  using TL = TabLayout<P, Q, MODE>;
  __shared__ T s_tab[TL::size];
  __shared__ T s_buf[EPB][3][Q3];

  const int tid = threadIdx.x;
  for (int t = tid; t < TL::size; t += EPB * Q2) s_tab[t] = tab[t];

  // one component of EPB elements per block; XCD-aware order (components of a block adjacent)
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int eb = item / NC, c = item - eb * NC;
  const int slot = tid / Q2, lt = tid - slot * Q2;
  const int a = lt % Q, b = lt / Q;
  const int64_t e = e_begin + (int64_t)eb * EPB + slot;
  const bool live = e < e_end;
  const bool node_thread = live && a < P && b < P;  // owns node column (i=a, j=b)
  T *const A = s_buf[slot][0];
  T *const B = s_buf[slot][1];
  T *const C = s_buf[slot][2];
  const T *const tI = s_tab + TL::interp;
  const T *const tD = s_tab + TL::dq;

  int32_t nid[P];
  uint32_t ob = 0;
  if (node_thread) {
    if constexpr (IDX == 2) {
      const int32_t *af = idx + e * 4;
      const int32_t base = af[0] + a + b * af[1], sk = af[2];
#pragma unroll
      for (int k = 0; k < P; ++k) nid[k] = base + k * sk;
    } else {
      static_assert(IDX == 0, "full or affine node ids");
#pragma unroll
      for (int k = 0; k < P; ++k) nid[k] = idx[e * P3 + k * P2 + b * P + a];
    }
    ob = own[e * P2 + b * P + a];
  }
  const TQ *qe = qd + e * (int64_t)(NCQ * Q3) + b * Q + a;
  const TQ *qme = HELM ? qm + e * (int64_t)Q3 + b * Q + a : nullptr;
  __syncthreads();

  {
    T yv[P];
    if constexpr (MODE == MODE_COLLOC) {
      T u[P];
      if (node_thread) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          u[k] = x[(int64_t)nid[k] * NC + c];
          A[k * P2 + b * P + a] = u[k];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < P; ++k) yv[k] = T(0);
      if (node_thread) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T ur = 0, us = 0, ut = 0;
#pragma unroll
          for (int l = 0; l < P; ++l) {
            ur += tD[a * P + l] * A[k * P2 + b * P + l];
            us += tD[b * P + l] * A[k * P2 + l * P + a];
            ut += tD[k * P + l] * u[l];
          }
          const TQ *g = qe + k * 6 * Q2;
          const T g0 = ld_q<NC, TQ, T>(g), g1 = ld_q<NC, TQ, T>(g + Q2), g2 = ld_q<NC, TQ, T>(g + 2 * Q2);
          const T g3 = ld_q<NC, TQ, T>(g + 3 * Q2), g4 = ld_q<NC, TQ, T>(g + 4 * Q2), g5 = ld_q<NC, TQ, T>(g + 5 * Q2);
          B[k * P2 + b * P + a] = g0 * ur + g1 * us + g2 * ut;
          C[k * P2 + b * P + a] = g1 * ur + g3 * us + g4 * ut;
          const T vt = g2 * ur + g4 * us + g5 * ut;
#pragma unroll
          for (int m = 0; m < P; ++m) yv[m] += tD[k * P + m] * vt;
          if constexpr (HELM) yv[k] += ld_q<NC, TQ, T>(qme + k * Q2) * u[k];  // collocated mass: diagonal
        }
      }
      __syncthreads();
      if (node_thread) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < P; ++l) {
            s += tD[l * P + a] * B[k * P2 + b * P + l];
            s += tD[l * P + b] * C[k * P2 + l * P + a];
          }
          yv[k] += s;
        }
      }
    } else {
      // ---- gather into A[k][j][i]
      if (node_thread) {
#pragma unroll
        for (int k = 0; k < P; ++k) A[k * P2 + b * P + a] = x[(int64_t)nid[k] * NC + c];
      }
      __syncthreads();
      // ---- interpolate along r1: B[k][j][qa] = sum_i I[qa][i] A[k][j][i]
      if (live && b < P) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T s = 0;
#pragma unroll
          for (int i = 0; i < P; ++i) s += tI[a * P + i] * A[k * P2 + b * P + i];
          B[k * Q * P + b * Q + a] = s;
        }
      }
      __syncthreads();
      // ---- along r2 (to registers), then along r3 in registers
      T uq[Q];
      {
        T col[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T s = 0;
#pragma unroll
          for (int j = 0; j < P; ++j) s += tI[b * P + j] * B[k * Q * P + j * Q + a];
          col[k] = s;
        }
#pragma unroll
        for (int cq = 0; cq < Q; ++cq) {
          T s = 0;
#pragma unroll
          for (int k = 0; k < P; ++k) s += tI[cq * P + k] * col[k];
          uq[cq] = s;
        }
      }
      T w[Q];
      if constexpr (MODE == MODE_MASS) {
#pragma unroll
        for (int cq = 0; cq < Q; ++cq) w[cq] = live ? uq[cq] * ld_q<NC, TQ, T>(qe + cq * Q2) : T(0);
      } else {
#pragma unroll
        for (int cq = 0; cq < Q; ++cq) C[cq * Q2 + b * Q + a] = uq[cq];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < Q; ++m) w[m] = T(0);
        if (live) {
#pragma unroll
          for (int cq = 0; cq < Q; ++cq) {
            T ur = 0, us = 0, ut = 0;
#pragma unroll
            for (int l = 0; l < Q; ++l) {
              ur += tD[a * Q + l] * C[cq * Q2 + b * Q + l];
              us += tD[b * Q + l] * C[cq * Q2 + l * Q + a];
              ut += tD[cq * Q + l] * uq[l];
            }
            const TQ *g = qe + cq * 6 * Q2;
            const T g0 = ld_q<NC, TQ, T>(g), g1 = ld_q<NC, TQ, T>(g + Q2), g2 = ld_q<NC, TQ, T>(g + 2 * Q2);
            const T g3 = ld_q<NC, TQ, T>(g + 3 * Q2), g4 = ld_q<NC, TQ, T>(g + 4 * Q2), g5 = ld_q<NC, TQ, T>(g + 5 * Q2);
            A[cq * Q2 + b * Q + a] = g0 * ur + g1 * us + g2 * ut;
            B[cq * Q2 + b * Q + a] = g1 * ur + g3 * us + g4 * ut;
            const T vt = g2 * ur + g4 * us + g5 * ut;
#pragma unroll
            for (int m = 0; m < Q; ++m) w[m] += tD[cq * Q + m] * vt;
            if constexpr (HELM) w[cq] += ld_q<NC, TQ, T>(qme + cq * Q2) * uq[cq];  // mass term at the point
          }
        }
        __syncthreads();
        if (live) {
#pragma unroll
          for (int cq = 0; cq < Q; ++cq) {
            T s = 0;
#pragma unroll
            for (int l = 0; l < Q; ++l) {
              s += tD[l * Q + a] * A[cq * Q2 + b * Q + l];
              s += tD[l * Q + b] * B[cq * Q2 + l * Q + a];
            }
            w[cq] += s;
          }
        }
      }
      // ---- transpose along r3 (registers) into C[k][qb][qa]
#pragma unroll
      for (int k = 0; k < P; ++k) {
        T s = 0;
#pragma unroll
        for (int cq = 0; cq < Q; ++cq) s += tI[cq * P + k] * w[cq];
        C[k * Q2 + b * Q + a] = s;
      }
      __syncthreads();
      // ---- transpose along r2: A[k][j][qa] = sum_qb I[qb][j] C[k][qb][qa]
      if (live && b < P) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T s = 0;
#pragma unroll
          for (int bq = 0; bq < Q; ++bq) s += tI[bq * P + b] * C[k * Q2 + bq * Q + a];
          A[k * Q * P + b * Q + a] = s;
        }
      }
      __syncthreads();
      // ---- transpose along r1: y[k][j][i] = sum_qa I[qa][i] A[k][j][qa]
      if (node_thread) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T s = 0;
#pragma unroll
          for (int aq = 0; aq < Q; ++aq) s += tI[aq * P + a] * A[k * Q * P + b * Q + aq];
          yv[k] = s;
        }
      }
    }
    // ---- scatter (or E-vector store)
    if (node_thread) {
      if constexpr (EOUT) {
        T *ye = y + ((int64_t)order[e] * NC + c) * P3 + b * P + a;
#pragma unroll
        for (int k = 0; k < P; ++k) ye[k * P2] = yv[k];
      } else {
        T old[P];
#pragma unroll
        for (int k = 0; k < P; ++k) old[k] = (ob & (1u << k)) ? T(0) : y[(int64_t)nid[k] * NC + c];
#pragma unroll
        for (int k = 0; k < P; ++k) y[(int64_t)nid[k] * NC + c] = old[k] + yv[k];
      }
    }
  }
}

}  // namespace hx
