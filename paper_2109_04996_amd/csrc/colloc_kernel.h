// Fused collocated diffusion apply (GLL rule on the nodes, BP5/BP6) for p <= 7.
//
// Same operator as MODE_COLLOC of apply_kernel.h (Benchmarks section: integration
// on the (p+1)^3 GLL nodes, so the basis evaluation is the identity and only the
// 1D derivative matrix D acts; libCEED section: G^T B^T D B G fused into one
// pass), organised for gfx950:
//
// * every contraction runs on a whole line held in one thread's registers. The
//   P^2 threads of an element take the lines along r3 (thread = (i, j)), then
//   along r1 (thread = (j, k)), then along r2 (thread = (i, k)); values move
//   between these layouts through LDS, one write and one read per value,
//   instead of P reads per point when a thread owns a point and reads its
//   neighbours along r1 and r2.
// * the LDS layout [k][j][i] pads each r1-row to P+1 doubles: for P = 8 the row
//   stride is 18 dwords, so all three access patterns (rows along i, j, k) touch
//   32 distinct banks per 16 lanes, the unit in which a wave's 64-bit LDS access
//   is served.
// * D is applied in even-odd form (half-size products, 2h^2 + 2h coefficients), read with
//   wave-uniform addresses (scalar loads), never from LDS.
// * two LDS buffers per element; for P = 8 one element fills one wavefront and
//   a workgroup is one wavefront, so the workgroup barriers are cheap.
// * memory: the pointwise data streams with nontemporal loads, two planes ahead of
//   use (scheduling barriers keep the compiler from hoisting all 48 loads); every
//   load is branch-free -- a branch around a load makes the compiler wait for all
//   outstanding loads at the join -- so lanes past the last element read a valid
//   element, and the read-modify-write loads of nodes an element owns read a
//   zero buffer instead.
//
// Scatter as in apply_kernel.h: no atomics; element colors, and the ownership bit
// decides between a store (owner) and a read-modify-write.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hx {

template <int P>
struct CollocCfg {
  static constexpr int P2 = P * P;
  static constexpr int EPB = (P2 <= 64) ? (64 / P2) : 1;  // elements per workgroup (one wavefront)
  static constexpr int THREADS = EPB * P2;
  static constexpr int LS = P + 1;        // padded row stride (odd count of doubles)
  static constexpr int PL = P * LS;       // plane stride
  static constexpr int BUF = P * PL;      // one buffer
};

// Even-odd form of the GLL derivative matrix. The GLL nodes are symmetric about 0, so
// D[P-1-i][P-1-l] = -D[i][l] (centro-antisymmetric), and y = D u splits into two half-size
// products on u_e[l] = u[l] + u[P-1-l] and u_o[l] = u[l] - u[P-1-l] (l < h = P/2):
//   (y[i] - y[P-1-i]) / 2 = sum_l E[i][l] u_e[l],  (y[i] + y[P-1-i]) / 2 = sum_l O[i][l] u_o[l],
//   E[i][l] = (D[i][l] + D[i][P-1-l]) / 2,  O[i][l] = (D[i][l] - D[i][P-1-l]) / 2,
// and for odd P the middle node adds E[i][h] = D[i][h] (acting on u[h]) and y[h] = sum_l M[l] u_o[l],
// M[l] = D[h][l]. The transpose D^T has the same structure with E' = O^T, O' = E^T (first h
// columns), M'[l] = E[l][h], E'[i][h] = M[i], so one coefficient set serves both directions.
// Coefficient layout: E [h][h + odd], then O [h][h], then M [h] (odd P only).
template <int P>
struct EOLayout {
  static constexpr int h = P / 2, odd = P & 1, he = h + odd;
  static constexpr int E = 0, O = h * he, M = O + h * h, size = M + odd * h;
};

// Hide the table address from the optimizer so each product re-issues its (scalar-cache) loads
// instead of keeping every coefficient in scalar registers across the whole kernel.
// Constant address space: uniform loads from it are scalar (s_load), and the values land in SGPRs.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ const_ptr<T> launder_uniform(const T *p) {
  const_ptr<T> c = (const_ptr<T>)p;
  __asm__ volatile("" : "+s"(c));
  return c;
}

template <int P, typename T>
__device__ __forceinline__ void eo_apply(const T *__restrict__ C0, const T (&u)[P], T (&y)[P]) {
  const const_ptr<T> C = launder_uniform(C0);
  using L = EOLayout<P>;
  constexpr int h = L::h, he = L::he;
  T ue[he], uo[h > 0 ? h : 1];
#pragma unroll
  for (int l = 0; l < h; ++l) {
    ue[l] = u[l] + u[P - 1 - l];
    uo[l] = u[l] - u[P - 1 - l];
  }
  if constexpr (L::odd) ue[h] = u[h];
#pragma unroll
  for (int i = 0; i < h; ++i) {
    T d = 0, s = 0;
#pragma unroll
    for (int l = 0; l < he; ++l) d += C[L::E + i * he + l] * ue[l];
#pragma unroll
    for (int l = 0; l < h; ++l) s += C[L::O + i * h + l] * uo[l];
    y[i] = s + d;
    y[P - 1 - i] = s - d;
  }
  if constexpr (L::odd) {
    T s = 0;
#pragma unroll
    for (int l = 0; l < h; ++l) s += C[L::M + l] * uo[l];
    y[h] = s;
  }
}

template <int P, typename T>
__device__ __forceinline__ void eo_apply_t(const T *__restrict__ C0, const T (&v)[P], T (&y)[P]) {
  const const_ptr<T> C = launder_uniform(C0);
  using L = EOLayout<P>;
  constexpr int h = L::h, he = L::he;
  T ve[he], vo[h > 0 ? h : 1];
#pragma unroll
  for (int l = 0; l < h; ++l) {
    ve[l] = v[l] + v[P - 1 - l];
    vo[l] = v[l] - v[P - 1 - l];
  }
  if constexpr (L::odd) ve[h] = v[h];
#pragma unroll
  for (int i = 0; i < h; ++i) {
    T d = 0, s = 0;
#pragma unroll
    for (int l = 0; l < h; ++l) d += C[L::O + l * h + i] * ve[l];
    if constexpr (L::odd) d += C[L::M + i] * ve[h];
#pragma unroll
    for (int l = 0; l < h; ++l) s += C[L::E + l * he + i] * vo[l];
    y[i] = s + d;
    y[P - 1 - i] = s - d;
  }
  if constexpr (L::odd) {
    T s = 0;
#pragma unroll
    for (int l = 0; l < h; ++l) s += C[L::E + l * he + h] * vo[l];
    y[h] = s;
  }
}

// ROWS: idx holds one base id per r1-row ([e][k][j], node (i, j, k) = base + i) instead of
// one id per node. HELM: the Helmholtz operator alpha A + beta B; qm [e][k][j][i] holds
// beta * w * detJ at the nodes, where the collocated mass matrix is diagonal, so node (i, j, k)
// adds qm * u to its sum (u read again at the end: the element's x values are still in the L2).
template <int P, int NC, typename T, typename TQ, bool EOUT, bool ROWS, bool HELM = false>
__global__ void __launch_bounds__(CollocCfg<P>::THREADS)
    k_colloc(const int32_t *__restrict__ idx, const uint16_t *__restrict__ own, const TQ *__restrict__ qd,
             const T *__restrict__ Dg, const T *__restrict__ x, T *__restrict__ y, const int32_t *__restrict__ order,
             int64_t e_begin, int64_t e_end, const T *__restrict__ zero, const TQ *__restrict__ qm = nullptr) {
  using CF = CollocCfg<P>;
  constexpr int P2 = CF::P2, P3 = P2 * P, EPB = CF::EPB, LS = CF::LS, PL = CF::PL;
  __shared__ T s0[EPB][CF::BUF];
  __shared__ T s1[EPB][CF::BUF];

  const int tid = threadIdx.x;
  // one component of EPB elements per block, XCD-aware order (components of a block adjacent)
  const int G = gridDim.x, bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3, base = G >> 3, rem = G & 7;
  const int item = xcd * base + (xcd < rem ? xcd : rem) + loc;
  const int eb = item / NC, c = item - eb * NC;
  const int slot = tid / P2, lt = tid - slot * P2;
  const int a = lt % P, b = lt / P;
  const int64_t e_first = e_begin + (int64_t)eb * EPB;  // first element of this workgroup (always valid)
  const int64_t e = e_first + slot;
  const bool live = e < e_end;
  const int64_t ee = live ? e : e_first;  // every lane addresses a valid element
  T *const S0 = s0[slot];
  T *const S1 = s1[slot];
  const T *const C = Dg + P * P;  // even-odd coefficients
  // position of node (i, j, k) in a buffer
#define AT(i, j, k) ((k) * PL + (j) * LS + (i))

  int32_t nid[P];
  if constexpr (ROWS) {
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + ee * P2 + k * P + b) + a;
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + ee * P3 + k * P2 + b * P + a);
  }
  // a masked lane counts as owner of all its nodes: its read-modify-write loads read zeros
  const uint32_t ob = live ? (uint32_t)own[ee * P2 + b * P + a] : 0xffffu;

  // two planes of pointwise data in flight: plane k+2 is requested while plane k is used
  const TQ *const qe = qd + ee * (6 * P3) + b * P + a;
  T ga[6], gb[6];
  auto load_plane = [&](T(&g)[6], int k) {
#pragma unroll
    for (int m = 0; m < 6; ++m) g[m] = ld_q<NC, TQ, T>(qe + (k * 6 + m) * P2);
  };

  {
    // ---- lines along r3: thread (i=a, j=b). Gather, and the r3 derivative in registers.
    T ut[P];
    {
      T u[P];
#pragma unroll
      for (int k = 0; k < P; ++k) u[k] = x[(int64_t)nid[k] * NC + c];
      load_plane(ga, 0);
      if constexpr (P > 1) load_plane(gb, 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < P; ++k) S0[AT(a, b, k)] = u[k];
      eo_apply<P, T>(C, u, ut);
    }
    __syncthreads();
    // ---- read lines along r1 (thread (j=a, k=b)) and r2 (thread (i=a, k=b))
    T li[P], lj[P];
#pragma unroll
    for (int l = 0; l < P; ++l) {
      li[l] = S0[AT(l, a, b)];
      lj[l] = S0[AT(a, l, b)];
    }
    __syncthreads();
    // ---- derivatives along r1 -> S0, along r2 -> S1 (same layout [k][j][i])
    {
      T r[P];
      eo_apply<P, T>(C, li, r);
#pragma unroll
      for (int i = 0; i < P; ++i) S0[AT(i, a, b)] = r[i];
      eo_apply<P, T>(C, lj, r);
#pragma unroll
      for (int j = 0; j < P; ++j) S1[AT(a, j, b)] = r[j];
    }
    __syncthreads();
    // ---- pointwise: (vr, vs, vt) = G (ur, us, ut) on lines along r3 (thread (i=a, j=b))
    T vt[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      T(&g)[6] = (k & 1) ? gb : ga;
      const T ur = S0[AT(a, b, k)], us = S1[AT(a, b, k)];
      S0[AT(a, b, k)] = g[0] * ur + g[1] * us + g[2] * ut[k];
      S1[AT(a, b, k)] = g[1] * ur + g[3] * us + g[4] * ut[k];
      vt[k] = g[2] * ur + g[4] * us + g[5] * ut[k];
      if (k + 2 < P) load_plane(g, k + 2);
      __builtin_amdgcn_sched_barrier(0);
    }
    // the read-modify-write half of the scatter: request the old values of the nodes this element
    // does not own now, so they arrive during the transposed contractions (no other element of
    // this launch touches these nodes)
    T old[P];
#pragma unroll
    for (int k = 0; k < P; ++k) old[k] = *((EOUT || (ob & (1u << k))) ? zero : y + (int64_t)nid[k] * NC + c);
    T hm[HELM ? P : 1], xm[HELM ? P : 1];
    if constexpr (HELM) {
      const TQ *const qme = qm + ee * P3 + b * P + a;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        hm[k] = ld_q<NC, TQ, T>(qme + k * P2);
        xm[k] = x[(int64_t)nid[k] * NC + c];
      }
    }
    // transposed r3 derivative in registers: yt[m] = sum_k D[k][m] vt[k]
    T yt[P];
    eo_apply_t<P, T>(C, vt, yt);
    if constexpr (HELM) {
#pragma unroll
      for (int k = 0; k < P; ++k) yt[k] += hm[k] * xm[k];
    }
    __syncthreads();
    // ---- transposed r1 derivative on S0 (thread (j=a, k=b)), r2 on S1 (thread (i=a, k=b)), in place
#pragma unroll
    for (int l = 0; l < P; ++l) {
      li[l] = S0[AT(l, a, b)];
      lj[l] = S1[AT(a, l, b)];
    }
    {
      T r[P];
      eo_apply_t<P, T>(C, li, r);
#pragma unroll
      for (int i = 0; i < P; ++i) S0[AT(i, a, b)] = r[i];
      eo_apply_t<P, T>(C, lj, r);
#pragma unroll
      for (int j = 0; j < P; ++j) S1[AT(a, j, b)] = r[j];
    }
    __syncthreads();
    // ---- sum the three parts on lines along r3; store the E-vector or scatter
    if (live) {
      if constexpr (EOUT) {
        T *ye = y + ((int64_t)order[e] * NC + c) * P3 + b * P + a;
#pragma unroll
        for (int k = 0; k < P; ++k) ye[k * P2] = yt[k] + S0[AT(a, b, k)] + S1[AT(a, b, k)];
      } else {
#pragma unroll
        for (int k = 0; k < P; ++k)
          y[(int64_t)nid[k] * NC + c] = old[k] + (yt[k] + S0[AT(a, b, k)] + S1[AT(a, b, k)]);
      }
    }
  }
#undef AT
}

}  // namespace hx
