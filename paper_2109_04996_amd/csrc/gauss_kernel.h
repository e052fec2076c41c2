// Fused apply with an interpolation step (Gauss points, BP1-BP4) for q <= 9, line per thread.
//
// Same operator as MODE_DIFF / MODE_MASS of apply_kernel.h (Benchmarks section: tensor-product
// sum factorization; libCEED section: G^T B^T D B G in one pass), organised like the collocated
// kernel (colloc_kernel.h): one or two wavefronts per element (k_gauss, k_gauss_strip), or all
// components of an element in one workgroup (k_gauss_joint); every 1D contraction on a whole line
// held in one thread's registers, lines moving between the three directions through padded LDS
// buffers, the 1D tables read with wave-uniform (scalar) loads, branch-free global loads and the
// pointwise data streamed two planes ahead (or staged in LDS).
//
// Diffusion, thread (a, b) of the Q x Q tile:
//   interpolate x along r3 in registers (thread (i, j), P -> Q), then along r2 (thread (i, qk))
//   and r1 (thread (qj, qk)) through LDS; differentiate along r1 in registers, along r3 and r2
//   through LDS; pointwise on lines along r3 (thread (qi, qj)); the transposed derivatives; the
//   transposed interpolations along r1, r2 and last r3 in registers, which leaves thread (i, j)
//   with the line of node values (i, j, 0..P-1) that the colored scatter writes.
// Mass: interpolate, scale on lines along r1 (thread (qj, qk), where the pointwise data of a line
// is contiguous), then the transposed interpolations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "apply_kernel.h"
#include "colloc_kernel.h"
#include "hx_internal.h"

namespace hx {

// Even-odd form of the interpolation table B [Q][P] from P symmetric nodes to Q symmetric points:
// B[Q-1-q][P-1-i] = B[q][i] (centro-symmetric). With u_e[l] = u[l] + u[P-1-l], u_o[l] = u[l] -
// u[P-1-l] (l < hp = P/2; u_e[hp] = u[hp] for odd P), E[q][l] = (B[q][l] + B[q][P-1-l]) / 2
// (E[q][hp] = B[q][hp]) and O[q][l] = (B[q][l] - B[q][P-1-l]) / 2:
//   y[q] = E_q u_e + O_q u_o,  y[Q-1-q] = E_q u_e - O_q u_o  (q < hq = Q/2),  y[hq] = E_hq u_e (odd Q).
// The transpose uses the same E and O by columns. Half the products of the dense form.
// Coefficient layout: E [hq + oq][hp + op], then O [hq][hp].
template <int P, int Q>
struct EOInterp {
  static constexpr int hp = P / 2, op = P & 1, hq = Q / 2, oq = Q & 1;
  static constexpr int ew = hp + op;  // row length of E
  static constexpr int E = 0, O = (hq + oq) * ew, size = O + hq * hp;
};

// y[q] = sum_i B[q][i] u[i]
template <int P, int Q, typename T>
__device__ __forceinline__ void interp_fwd(const T *__restrict__ C0, const T (&u)[P], T (&y)[Q]) {
  const const_ptr<T> C = launder_uniform(C0);
  using L = EOInterp<P, Q>;
  T ue[L::ew], uo[L::hp > 0 ? L::hp : 1];
#pragma unroll
  for (int l = 0; l < L::hp; ++l) {
    ue[l] = u[l] + u[P - 1 - l];
    uo[l] = u[l] - u[P - 1 - l];
  }
  if constexpr (L::op) ue[L::hp] = u[L::hp];
#pragma unroll
  for (int q = 0; q < L::hq; ++q) {
    T d = 0, s = 0;
#pragma unroll
    for (int l = 0; l < L::ew; ++l) d += C[L::E + q * L::ew + l] * ue[l];
#pragma unroll
    for (int l = 0; l < L::hp; ++l) s += C[L::O + q * L::hp + l] * uo[l];
    y[q] = d + s;
    y[Q - 1 - q] = d - s;
  }
  if constexpr (L::oq) {
    T d = 0;
#pragma unroll
    for (int l = 0; l < L::ew; ++l) d += C[L::E + L::hq * L::ew + l] * ue[l];
    y[L::hq] = d;
  }
}

// y[i] = sum_q B[q][i] v[q]
template <int P, int Q, typename T>
__device__ __forceinline__ void interp_bwd(const T *__restrict__ C0, const T (&v)[Q], T (&y)[P]) {
  const const_ptr<T> C = launder_uniform(C0);
  using L = EOInterp<P, Q>;
  T ve[L::hq + L::oq], vo[L::hq > 0 ? L::hq : 1];
#pragma unroll
  for (int m = 0; m < L::hq; ++m) {
    ve[m] = v[m] + v[Q - 1 - m];
    vo[m] = v[m] - v[Q - 1 - m];
  }
  if constexpr (L::oq) ve[L::hq] = v[L::hq];
#pragma unroll
  for (int i = 0; i < L::hp; ++i) {
    T d = 0, s = 0;
#pragma unroll
    for (int m = 0; m < L::hq + L::oq; ++m) d += C[L::E + m * L::ew + i] * ve[m];
#pragma unroll
    for (int m = 0; m < L::hq; ++m) s += C[L::O + m * L::hp + i] * vo[m];
    y[i] = d + s;
    y[P - 1 - i] = d - s;
  }
  if constexpr (L::op) {
    T d = 0;
#pragma unroll
    for (int m = 0; m < L::hq + L::oq; ++m) d += C[L::E + m * L::ew + L::hp] * ve[m];
    y[L::hp] = d;
  }
}

// y = D u and y = D^T v for the Q x Q derivative on the q points: even-odd form (EOLayout of
// colloc_kernel.h; D is centro-antisymmetric on symmetric points)
template <int Q, typename T>
__device__ __forceinline__ void deriv_fwd(const T *__restrict__ C0, const T (&u)[Q], T (&y)[Q]) {
  eo_apply<Q, T>(C0, u, y);
}

template <int Q, typename T>
__device__ __forceinline__ void deriv_bwd(const T *__restrict__ C0, const T (&v)[Q], T (&y)[Q]) {
  eo_apply_t<Q, T>(C0, v, y);
}

// One element per workgroup: one wavefront for q <= 8, two for q = 9 (81 line tiles).
template <int Q>
struct GaussCfg {
  static constexpr int NT = (Q * Q <= 64) ? 64 : 128;
};

// LDS ordering between the steps of an element: within one wavefront LDS operations complete in
// order, so the fences only stop the compiler from moving accesses; two wavefronts need a barrier.
template <int NT>
__device__ __forceinline__ void elem_sync() {
  if constexpr (NT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// The element pipeline shared by the Gauss kernels: for one component c of element e, node lane
// (i, j) = (a, b) ends with z[k], its element's contribution at node (i, j, k), and old[k], the
// value its scatter adds it to (requested before the last contraction: zero where ob says the
// lane stores first). S0, S1: this element's two LDS buffers. NT: threads per element (64 syncs
// the wavefront, more a workgroup barrier).
// ONEBUF (mass only): S1 is S0, one LDS buffer per element; the two passes that read one layout and
// write another wait for every read before writing
// HELM (diffusion only): the Helmholtz operator alpha A + beta B; qm [e][qc][qb][qa] = beta * w * detJ, and
// the mass term qm * u joins the r3 line's sum before the transposed interpolations.
// QLDS: the caller has the element's pointwise data (qd's layout for one element) on its way to LDS at qs;
// stage() writes it there and is called once, right after the first pass's LDS writes, so that the
// loads overlap the node gather and the first interpolation; the pointwise step then reads qs, and
// the old values of the scatter are requested two passes early. EARLY_OLD: they are requested with
// the node gather instead, their latency hidden behind the whole pipeline (for kernels whose
// occupancy LDS bounds, which leaves the registers free).
struct NoStage {
  __device__ void operator()() const {}
};
// LS, PL: LDS strides (doubles) of the r2 rows and r3 planes of a buffer, AT(i, j, k) = k PL + j LS + i.
template <int P, int Q, int MODE, int NC, typename T, typename TQ, int NT, bool ONEBUF = false, bool HELM = false,
          bool QLDS = false, typename Stage = NoStage, int LS = Q + 1, int PL = Q *(Q + 1), bool EARLY_OLD = false>
__device__ __forceinline__ void gauss_element(T *S0, T *S1, int a, int b, bool lane_live,
                                              int64_t e, int c, const TQ *__restrict__ qd, const T *__restrict__ tab,
                                              const T *__restrict__ x, const int32_t (&nid)[P], uint32_t ob,
                                              const T *__restrict__ zero, const T *__restrict__ y, T (&old)[P],
                                              T (&z)[P], const TQ *__restrict__ qm = nullptr,
                                              const TQ *qs = nullptr, Stage stage = Stage()) {
  static_assert(!HELM || MODE == MODE_DIFF, "the Helmholtz mass term rides on the diffusion pipeline");
  constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
  static_assert(LS >= Q && PL >= (Q - 1) * LS + Q, "lines, rows and planes do not overlap");
#define AT(i, j, k) ((k) * PL + (j) * LS + (i))
  const T *const tI = tab + Q * P + Q * Q;       // even-odd interpolation
  const T *const tD = tI + EOInterp<P, Q>::size;  // even-odd derivative
  // node lanes: (i, j) = (a, b) for a, b < P; the others address node (min(a, P-1), min(b, P-1))
  const int an = a < P ? a : P - 1, bn = b < P ? b : P - 1;
  const bool node_lane = lane_live && a < P && b < P;
  // old values of the nodes this lane read-modify-writes (no other element of this launch touches them)
  auto load_old = [&]() {
#pragma unroll
    for (int k = 0; k < P; ++k) old[k] = *((ob & (1u << k)) ? zero : y + (int64_t)nid[k] * NC + c);
  };
    // ---- interpolate along r3 in registers: thread (i, j), S0[i][j][qk]
    {
      T u[P], uq[Q];
#pragma unroll
      for (int k = 0; k < P; ++k) u[k] = x[(int64_t)nid[k] * NC + c];
      if constexpr (QLDS && EARLY_OLD) load_old();
      interp_fwd<P, Q, T>(tI, u, uq);
      if (node_lane) {
#pragma unroll
        for (int q = 0; q < Q; ++q) S0[AT(a, b, q)] = uq[q];
      }
      if constexpr (QLDS) stage();
    }
    elem_sync<NT>();
    // ---- along r2: thread (i = a < P, qk = b), S1[i][qj][qk]
    {
      T u[P], uq[Q];
#pragma unroll
      for (int j = 0; j < P; ++j) u[j] = S0[AT(an, j, b)];
      interp_fwd<P, Q, T>(tI, u, uq);
      if constexpr (ONEBUF) elem_sync<NT>();
      if (lane_live && a < P) {
#pragma unroll
        for (int q = 0; q < Q; ++q) S1[AT(a, q, b)] = uq[q];
      }
    }
    elem_sync<NT>();
    // ---- along r1: thread (qj = a, qk = b) holds the line of u at (0..Q-1, a, b)
    T ul[Q];
    {
      T u[P];
#pragma unroll
      for (int i = 0; i < P; ++i) u[i] = S1[AT(i, a, b)];
      interp_fwd<P, Q, T>(tI, u, ul);
    }
    T w[Q];  // the field after the pointwise step and the transposed derivatives, on r3 lines of (a, b)
    if constexpr (MODE == MODE_MASS) {
      // pointwise on the r1 line: qdata (qi, qj=a, qk=b) is contiguous in qi
      T v[Q];
      if constexpr (QLDS) {
        const TQ *const ql = qs + b * Q2 + a * Q;
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = ul[q] * static_cast<T>(ql[q]);
        if constexpr (!EARLY_OLD) load_old();
      } else {
        const TQ *const ql = qd + e * Q3 + b * Q2 + a * Q;
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = ul[q] * ld_q<NC, TQ, T>(ql + q);
      }
      // transposed interpolation along r1 straight from registers: S0[i][qj][qk]
      T z[P];
      interp_bwd<P, Q, T>(tI, v, z);
      elem_sync<NT>();
      if (lane_live) {
#pragma unroll
        for (int i = 0; i < P; ++i) S0[AT(i, a, b)] = z[i];
      }
      (void)w;
    } else {
      // r1 derivative in registers; u to S0 (for the r3 and r2 lines) and ur to S1 (the r1
      // interpolation above was the last reader of S1)
      {
        T ur[Q];
        deriv_fwd<Q, T>(tD, ul, ur);
        elem_sync<NT>();
        if (lane_live) {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            S0[AT(q, a, b)] = ul[q];
            S1[AT(q, a, b)] = ur[q];
          }
        }
      }
      elem_sync<NT>();
      // r3 derivative on the r3 line of (qi = a, qj = b), kept in registers; r2 derivative on the
      // r2 line of (qi = a, qk = b), to S0 once every lane has read u
      T ut[Q];
      T um[HELM ? Q : 1];  // u on the r3 line, kept for the Helmholtz mass term
      {
        T lk[Q];
#pragma unroll
        for (int l = 0; l < Q; ++l) lk[l] = S0[AT(a, b, l)];
        deriv_fwd<Q, T>(tD, lk, ut);
        if constexpr (HELM) {
#pragma unroll
          for (int l = 0; l < Q; ++l) um[l] = lk[l];
        }
      }
      {
        T lj[Q], us[Q];
#pragma unroll
        for (int l = 0; l < Q; ++l) lj[l] = S0[AT(a, l, b)];
        deriv_fwd<Q, T>(tD, lj, us);
        elem_sync<NT>();
        if (lane_live) {
#pragma unroll
          for (int q = 0; q < Q; ++q) S0[AT(a, q, b)] = us[q];
        }
      }
      // pointwise on r3 lines: thread (qi = a, qj = b); S1 holds ur, S0 us; vr -> S1, vs -> S0
      T vt[Q];
      if constexpr (QLDS) {
        // the element's pointwise data is in LDS (planes along r3 of the (qi = a, qj = b) column)
        const TQ *const qp = qs + b * Q + a;
        elem_sync<NT>();
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          T g[6];
#pragma unroll
          for (int m = 0; m < 6; ++m) g[m] = static_cast<T>(qp[(k * 6 + m) * Q2]);
          const T r = S1[AT(a, b, k)], s = S0[AT(a, b, k)];
          const T t = ut[k];
          if (lane_live) {
            S1[AT(a, b, k)] = g[0] * r + g[1] * s + g[2] * t;
            S0[AT(a, b, k)] = g[1] * r + g[3] * s + g[4] * t;
          }
          vt[k] = g[2] * r + g[4] * s + g[5] * t;
        }
      } else {
        // plane-ahead pointwise data (planes along r3 of the (qi = a, qj = b) column)
        const TQ *const qe = qd + e * (6 * Q3) + b * Q + a;
        T ga[6], gb[6];
        auto load_plane = [&](T(&g)[6], int k) {
#pragma unroll
          for (int m = 0; m < 6; ++m) g[m] = ld_q<NC, TQ, T>(qe + (k * 6 + m) * Q2);
        };
        load_plane(ga, 0);
        load_plane(gb, 1);
        elem_sync<NT>();
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          T(&g)[6] = (k & 1) ? gb : ga;
          const T r = S1[AT(a, b, k)], s = S0[AT(a, b, k)];
          const T t = ut[k];
          if (lane_live) {
            S1[AT(a, b, k)] = g[0] * r + g[1] * s + g[2] * t;
            S0[AT(a, b, k)] = g[1] * r + g[3] * s + g[4] * t;
          }
          vt[k] = g[2] * r + g[4] * s + g[5] * t;
          if (k + 2 < Q) load_plane(g, k + 2);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      deriv_bwd<Q, T>(tD, vt, w);  // r3 part, on the r3 line of (a, b)
      if constexpr (HELM) {
        const TQ *const qme = qm + e * Q3 + b * Q + a;
#pragma unroll
        for (int k = 0; k < Q; ++k) w[k] += ld_q<NC, TQ, T>(qme + k * Q2) * um[k];
      }
      elem_sync<NT>();
      // transposed r1 (thread (qj = a, qk = b), from S1) and r2 (thread (qi = a, qk = b), from S0)
      {
        T ri[Q], rj[Q];
        {
          T li[Q];
#pragma unroll
          for (int l = 0; l < Q; ++l) li[l] = S1[AT(l, a, b)];
          deriv_bwd<Q, T>(tD, li, ri);
        }
        {
          T lj[Q];
#pragma unroll
          for (int l = 0; l < Q; ++l) lj[l] = S0[AT(a, l, b)];
          deriv_bwd<Q, T>(tD, lj, rj);
        }
        elem_sync<NT>();
        if (lane_live) {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            S1[AT(q, a, b)] = ri[q];
            S0[AT(a, q, b)] = rj[q];
          }
        }
      }
      elem_sync<NT>();
      // sum of the three parts on r3 lines, to S0 for the transposed interpolations
#pragma unroll
      for (int k = 0; k < Q; ++k) w[k] += S0[AT(a, b, k)] + S1[AT(a, b, k)];
      elem_sync<NT>();
      if (lane_live) {
#pragma unroll
        for (int k = 0; k < Q; ++k) S0[AT(a, b, k)] = w[k];
      }
      if constexpr (QLDS && !EARLY_OLD) load_old();
      elem_sync<NT>();
      // transposed interpolation along r1: thread (qj = a, qk = b), S0[i][qj][qk]
      {
        T v[Q], z[P];
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = S0[AT(q, a, b)];
        interp_bwd<P, Q, T>(tI, v, z);
        elem_sync<NT>();
        if (lane_live) {
#pragma unroll
          for (int i = 0; i < P; ++i) S0[AT(i, a, b)] = z[i];
        }
      }
    }
    elem_sync<NT>();
    // ---- transposed interpolation along r2: thread (i = a < P, qk = b), S1[i][j][qk]
    {
      T v[Q], z[P];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = S0[AT(an, q, b)];
      interp_bwd<P, Q, T>(tI, v, z);
      if constexpr (ONEBUF) elem_sync<NT>();
      if (lane_live && a < P) {
#pragma unroll
        for (int j = 0; j < P; ++j) S1[AT(a, j, b)] = z[j];
      }
    }
    if constexpr (!QLDS) load_old();  // requested before the last contraction
    elem_sync<NT>();
    // ---- transposed interpolation along r3 in registers: thread (i, j) -> node line (i, j, 0..P-1)
    {
      T v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = S1[AT(an, bn, q)];
      interp_bwd<P, Q, T>(tI, v, z);
    }
#undef AT
}

// One component of one element per workgroup (for several components k_gauss_joint is used up to
// q = 9; at q = 10 its FP64 form needs too much LDS). tab: interp [Q][P], D [Q][Q], then the even-odd
// coefficients of the interpolation (EOInterp) and of D (EOLayout).
// IDX: node ids as in k_gauss_joint (0 one per element node, 2 the element's affine numbering).
template <int P, int Q, int MODE, int NC, typename T, typename TQ, int IDX, bool HELM = false>
__global__ void __launch_bounds__(GaussCfg<Q>::NT)
    k_gauss(const int32_t *__restrict__ idx, const uint16_t *__restrict__ own, const TQ *__restrict__ qd,
            const T *__restrict__ tab, const T *__restrict__ x, T *__restrict__ y, int64_t e_begin, int64_t e_end,
            const T *__restrict__ zero, const TQ *__restrict__ qm = nullptr) {
  static_assert(Q * Q <= 128 && P <= Q, "at most two wavefronts per element, q >= p+1");
  static_assert(MODE == MODE_DIFF || MODE == MODE_MASS, "interpolating modes only");
  constexpr int NT = GaussCfg<Q>::NT;
  constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q;
  constexpr int BUF = Q * Q * (Q + 1);
  __shared__ T S0[BUF];
  __shared__ T S1[BUF];

  const int lt0 = threadIdx.x;
  const bool lane_live = lt0 < Q2;
  const int lt = lane_live ? lt0 : Q2 - 1;  // spare lanes shadow the last one (same values, no stores)
  const int a = lt % Q, b = lt / Q;
  // one component of one element per block (grid = (e_end - e_begin) NC); with several components an
  // XCD-aware order keeps an element's components on one XCD
  const int item = (NC > 1) ? xcd_item(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int64_t eo = item / NC;
  const int c = item - (int)eo * NC;
  const int64_t e = e_begin + eo;
  const int an = a < P ? a : P - 1, bn = b < P ? b : P - 1;
  const bool node_lane = lane_live && a < P && b < P;

  int32_t nid[P];
  if constexpr (IDX == 2) {
    const int32_t *af = idx + e * 4;
    const int32_t base = af[0] + an, sj = af[1], sk = af[2];
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = base + bn * sj + k * sk;
  } else {
    static_assert(IDX == 0, "full or affine node ids");
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + e * P3 + k * P2 + bn * P + an);
  }
  const uint32_t ob = node_lane ? (uint32_t)own[e * P2 + b * P + a] : 0xffffu;

  T old[P], z[P];
  gauss_element<P, Q, MODE, NC, T, TQ, NT, false, HELM>(S0, S1, a, b, lane_live, e, c, qd, tab, x, nid, ob, zero, y,
                                                       old, z, qm);
  if (node_lane) {
#pragma unroll
    for (int k = 0; k < P; ++k) y[(int64_t)nid[k] * NC + c] = old[k] + z[k];
  }
}

// Threads of the joint-component kernel: the NC Q x Q line tiles of an element, packed end to end
// and rounded up to whole wavefronts (Q = 9, NC = 3: 243 of 256 lanes live, against 81 of 128 with
// one workgroup per component; Q = 8: 192 of 192).
// LDS layout of its per-component buffers (strides in doubles): LS between r2 rows, PL between r3
// planes, CS between the components' buffers. Chosen, with the component-minor lane order, by
// counting LDS bank conflicts of the pipeline's access patterns (64 banks of 4 bytes, half a
// wavefront per pass; and 32 banks, a quarter per pass); the line tiles' own padding (LS = Q + 1)
// loses to these at every q.
template <int Q, int NC>
struct GaussJointCfg {
  static constexpr int NT = (NC * Q * Q + 63) / 64 * 64;
  // three wavefronts per SIMD where three workgroups' LDS fits a CU (q <= 8): the compiler then
  // keeps to 168 registers (the Helmholtz variant, with more live values, keeps its default); q = 9
  // fits two workgroups either way
  static constexpr bool WPE3 = Q <= 8;
  // LDS-bound occupancy (q = 9, and the Helmholtz variant): the scatter's old values load early
  static constexpr int LS = (Q == 6) ? 6 : (Q == 10) ? 10 : 9;
  static constexpr int PL = (Q == 10) ? 106 : (Q == 9) ? 83 : (Q == 8) ? 72 : (Q == 7) ? 71 : (Q == 6) ? 37 : Q * (Q + 1);
  static constexpr int CS = (Q == 10) ? 1067 : (Q == 9) ? 747 : (Q == 8) ? 587 : (Q == 7) ? 523 : (Q == 6) ? 235
                                                                                                : Q * Q * (Q + 1);
  static_assert(LS >= Q && PL >= (Q - 1) * LS + Q && CS >= (Q - 1) * PL + (Q - 1) * LS + Q, "disjoint buffers");
};

// Every component of one element per workgroup (vector problems, BP2 and BP4). Lane t works on
// component c = t mod NC at line tile t / NC, with its own pair of LDS buffers; the pipeline is
// gauss_element's, with workgroup barriers. Against a workgroup per component, this packs the
// lanes densely, fits one and a half times the element-components per CU at the same register
// budget, and reads the element's geometric factors once for all of its components: loaded whole
// and coalesced at the start, so that their latency overlaps the node gather and the first pass,
// and parked in LDS for the pointwise step (the NC lanes of a point read one address). The
// component-minor order also makes the lanes of a node gather and store NC adjacent values.
// IDX: node ids as in k_colloc_strip (0 one per element node; 2 {base, s_j, s_k} per element, read
// with scalar loads that the L2 serves, so the gather waits on no vector index load).
template <int P, int Q, int MODE, int NC, typename T, typename TQ, int IDX, bool HELM = false>
__global__ void __launch_bounds__((GaussJointCfg<Q, NC>::NT)) __attribute__((amdgpu_waves_per_eu((GaussJointCfg<Q, NC>::WPE3 && !HELM) ? 3 : 1)))
    k_gauss_joint(const int32_t *__restrict__ idx, const uint16_t *__restrict__ own, const TQ *__restrict__ qd,
                  const T *__restrict__ tab, const T *__restrict__ x, T *__restrict__ y, int64_t e_begin,
                  const T *__restrict__ zero, const TQ *__restrict__ qm = nullptr) {
  static_assert(P <= Q && NC > 1, "q >= p+1, several components");
  static_assert(MODE == MODE_DIFF || MODE == MODE_MASS, "interpolating modes only");
  using L = GaussJointCfg<Q, NC>;
  constexpr int NT = L::NT;
  static_assert(NT > 64, "workgroup barriers between the steps");
  constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q;
  __shared__ T S0[NC * L::CS];
  __shared__ T S1[NC * L::CS];

  const int t0 = threadIdx.x;
  const bool lane_live = t0 < NC * Q2;
  const int t = lane_live ? t0 : NC * Q2 - 1;  // spare lanes shadow the last one (same values, no stores)
  const int lt = t / NC;
  const int c = t - lt * NC;
  const int a = lt % Q, b = lt / Q;
  const int64_t e = e_begin + blockIdx.x;
  const int an = a < P ? a : P - 1, bn = b < P ? b : P - 1;
  const bool node_lane = lane_live && a < P && b < P;

  constexpr int QN = (MODE == MODE_MASS ? 1 : 6) * Q2 * Q;  // the element's pointwise data
  constexpr int QPL = (QN + NT - 1) / NT;
  __shared__ TQ QS[QN];
  TQ qv[QPL];
  {
    const TQ *const qsrc = qd + e * QN;
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
      const int o = i * NT + t0;
      qv[i] = (o < QN) ? __builtin_nontemporal_load(qsrc + o) : TQ(0);
    }
  }
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
      const int o = i * NT + t0;
      if (o < QN) QS[o] = qv[i];
    }
  };

  int32_t nid[P];
  if constexpr (IDX == 2) {
    const int32_t *af = idx + e * 4;
    const int32_t base = af[0] + an, sj = af[1], sk = af[2];
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = base + bn * sj + k * sk;
  } else {
    static_assert(IDX == 0, "full or affine node ids");
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + e * P3 + k * P2 + bn * P + an);
  }
  const uint32_t ob = node_lane ? (uint32_t)own[e * P2 + b * P + a] : 0xffffu;

  T old[P], z[P];
  gauss_element<P, Q, MODE, NC, T, TQ, NT, false, HELM, true, decltype(stage), L::LS, L::PL, !L::WPE3 || HELM>(
      S0 + c * L::CS, S1 + c * L::CS, a, b, lane_live, e, c, qd, tab, x, nid, ob, zero, y, old, z, qm, QS, stage);
  if (node_lane) {
#pragma unroll
    for (int k = 0; k < P; ++k) y[(int64_t)nid[k] * NC + c] = old[k] + z[k];
  }
}

// The Gauss kernel with the strip scatter of k_colloc_strip (degree 7 meshes with strips): a
// workgroup takes a strip of up to kStrip elements, one or two wavefronts per element, runs the
// element pipeline on each, and sums the shared r1 faces in LDS -- element w+1 leaves its r1 = -1
// face there, element w adds it to its own r1 = +1 face and writes it once. Other nodes follow the
// strip ownership (store by the first writer in strip order, read-modify-write by later ones).
// IDX: node ids as in k_colloc_strip (0 per node, 1 per r1-row, 2 affine per element).
// Mass keeps one LDS buffer per element (ONEBUF), and at q = 9 at most 64 registers: two 16-wavefront
// workgroups then fit on a CU, against one with two buffers.
template <int P, int Q, int MODE, int NC, typename T, typename TQ, int IDX, bool HELM = false>
__global__ void __launch_bounds__(kStrip * GaussCfg<Q>::NT)
    __attribute__((amdgpu_waves_per_eu((MODE == MODE_MASS && Q == 9) ? 8 : 1)))
    k_gauss_strip(const int32_t *__restrict__ idx, const uint16_t *__restrict__ sown, const TQ *__restrict__ qd,
                  const T *__restrict__ tab, const T *__restrict__ x, T *__restrict__ y,
                  const int32_t *__restrict__ selems, const uint8_t *__restrict__ slink, int64_t s_begin,
                  const T *__restrict__ zero, const TQ *__restrict__ qm = nullptr) {
  static_assert(Q * Q <= 128 && P <= Q, "at most two wavefronts per element, q >= p+1");
  constexpr int NTE = GaussCfg<Q>::NT;  // threads per element
  constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q;
  constexpr int BUF = Q * Q * (Q + 1);
  constexpr bool ONEBUF = MODE == MODE_MASS;
  __shared__ T s0[kStrip][BUF];
  __shared__ T s1[ONEBUF ? 1 : kStrip][ONEBUF ? 1 : BUF];
  __shared__ T face[kStrip][P2];  // element w's r1 = -1 face, [k][j]

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid / NTE);  // element slot (uniform in a wavefront)
  const int lt0 = tid - w * NTE;
  const bool lane_live = lt0 < Q2;
  const int lt = lane_live ? lt0 : Q2 - 1;
  const int a = lt % Q, b = lt / Q;
  // one component of one strip per block; several components: XCD-aware order
  const int item = (NC > 1) ? xcd_item(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int sl = item / NC, c = item - sl * NC;
  const int32_t *const se = selems + (s_begin + sl) * kStrip;
  const int32_t el = se[w];
  const bool live = el >= 0;
  const int64_t ee = live ? el : se[0];  // a slot past the strip's end works on a valid element
  // a group holds whole strips: bit w of its link byte says slot w + 1 continues slot w's strip
  const uint32_t link = slink[s_begin + sl];
  const bool has_prev = live && w > 0 && ((link >> (w > 0 ? w - 1 : 0)) & 1u);
  const bool has_next = live && (w + 1 < kStrip) && ((link >> w) & 1u);
  const int an = a < P ? a : P - 1, bn = b < P ? b : P - 1;
  const bool node_lane = lane_live && a < P && b < P;
  const bool skip = has_prev && node_lane && a == 0;  // written by the previous element

  int32_t nid[P];
  if constexpr (IDX == 2) {
    const int32_t *af = idx + ee * 4;
    const int32_t base = af[0] + an, sj = af[1], sk = af[2];
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = base + bn * sj + k * sk;
  } else if constexpr (IDX == 1) {
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + ee * P2 + k * P + bn) + an;
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + ee * P3 + k * P2 + bn * P + an);
  }
  const uint32_t ob = (live && node_lane && !skip) ? (uint32_t)sown[ee * P2 + b * P + a] : 0xffffu;

  T old[P], z[P];
  T *S1;
  if constexpr (ONEBUF) S1 = s0[w];
  else S1 = s1[w];
  gauss_element<P, Q, MODE, NC, T, TQ, NTE, ONEBUF, HELM>(s0[w], S1, a, b, lane_live, ee, c, qd, tab, x, nid, ob, zero,
                                                          y, old, z, qm);
  T out[P];
#pragma unroll
  for (int k = 0; k < P; ++k) out[k] = old[k] + z[k];
  if (skip) {
#pragma unroll
    for (int k = 0; k < P; ++k) face[w][k * P + b] = out[k];
  }
  __syncthreads();
  if (has_next && node_lane && a == P - 1) {
#pragma unroll
    for (int k = 0; k < P; ++k) out[k] += face[w + 1][k * P + b];
  }
  if (live && node_lane && !skip) {
#pragma unroll
    for (int k = 0; k < P; ++k) y[(int64_t)nid[k] * NC + c] = out[k];
  }
}

}  // namespace hx
