// Collocated diffusion apply with a strip scatter (P = p + 1 = 3, 4, 5 or 8 nodes per direction).
//
// The operator and the per-element work are those of k_colloc (colloc_kernel.h): a thread per
// line, LDS transposes, the even-odd derivative, and as many elements per wavefront as their
// P^2 lines fit (one for P = 8, two for P = 5, four for P = 4, seven for P = 3). What changes
// is the scatter G^T (libCEED section: G^T sums the element contributions
// into the L-vector). A workgroup takes a strip of up to StripCfg<P>::SL elements that follow
// each other along r1 (element w+1's r1 = -1 face is element w's r1 = +1 face, built by the
// mesh):
//
// * the shared faces are summed in LDS: element w+1 leaves its face values there, element w adds
//   them to its own and writes the node once -- no read-modify-write and no second store;
// * the r1-rows of a strip's elements join into rows of up to SL*p+1 consecutive nodes, written
//   by one workgroup within its lifetime, so the partially covered memory sectors of a row are
//   those at its two ends, not those at every element boundary;
// * strips have their own coloring (no two strips of a color share a node), one launch per
//   color, and their own ownership bits: the first writer of a node in strip order stores it,
//   later writers read-modify-write it.
//
// Each element's LDS buffers are its own, so the steps inside an element synchronise the
// wavefront only; the face exchange is the one workgroup barrier per component.

#pragma once

#include "colloc_kernel.h"
#include "hx_internal.h"

namespace hx {

// LDS ordering among the lanes of one wavefront: LDS operations of a wavefront complete in
// order, so the fences only stop the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Strip shape for P nodes per direction: EPW elements per wavefront, SL elements per strip
// (at most kStrip, the stride of the strip element lists), NW wavefronts per workgroup.
template <int P>
struct StripCfg {
  static constexpr int P2 = P * P;
  static constexpr int EPW = P2 <= 64 ? 64 / P2 : 1;
  static constexpr int SL = strip_len(P);
  static constexpr int NW = (SL + EPW - 1) / EPW;
  static_assert(SL <= kStrip, "strip longer than the element list stride");
  static_assert(P2 <= 64, "an element's lines must fit one wavefront");
};

// One workgroup per (group, component) of color [s_begin, s_begin + gridDim.x / NC); group s holds one or
// more whole strips of one color in selems[s][0..len) (internal positions), -1 past the end, and slink[s]
// marks which neighbouring slots belong to one strip. IDX: 0 one node id per element node,
// 1 one per r1-row (ROWS of k_colloc), 2 {base, s_j, s_k} per element, read with scalar loads
// (node (i, j, k) = base + i + j s_j + k s_k), so the gather does not wait on a vector load.
// sown: the strip-order ownership bits of each element.
// HELM: the Helmholtz operator alpha A + beta B, with qm [e][k][j][i] = beta * w * detJ at the
// nodes (the collocated mass matrix is diagonal), as in k_colloc.
template <int P, int NC, typename T, typename TQ, int IDX, bool HELM = false>
__global__ void __launch_bounds__(StripCfg<P>::NW * 64)
    k_colloc_strip(const int32_t *__restrict__ idx, const uint16_t *__restrict__ sown, const TQ *__restrict__ qd,
                   const T *__restrict__ Dg, const T *__restrict__ x, T *__restrict__ y,
                   const int32_t *__restrict__ selems, const uint8_t *__restrict__ slink, int64_t s_begin,
                   const T *__restrict__ zero, const TQ *__restrict__ qm = nullptr) {
  using SC = StripCfg<P>;
  constexpr int P2 = P * P, P3 = P2 * P, LS = P + 1, PL = P * LS, BUF = P * PL, SL = SC::SL, EPW = SC::EPW;
  __shared__ T s0[SL][BUF];
  __shared__ T s1[SL][BUF];
  __shared__ T face[SL][P2];  // element w's r1 = -1 face, [k][j]

  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), l64 = tid & 63;  // wv is wave-uniform
  const int sw = l64 / P2, lt = l64 - sw * P2;  // element slot in the wavefront, line in the element
  const int a = lt % P, b = lt / P;
  // w: the element's position in the strip; lanes past the last slot of a wavefront, or past the
  // strip length, work on slot 0 of the strip and store nothing
  const int wr = wv * EPW + sw;
  const bool lane_ok = (P2 == 64 && SC::NW == SL) ? true : (sw < EPW && wr < SL);  // P = 8: every lane
  const int w = lane_ok ? wr : 0;
  // one component of one strip per block: consecutive blocks take consecutive (spatially sorted)
  // strips; with several components, an XCD-aware order keeps a strip's components on one XCD
  const int item = (NC > 1) ? xcd_item(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int sl = item / NC, c = item - sl * NC;
  const int64_t s = s_begin + sl;
  const int32_t *const se = selems + s * kStrip;
  const int32_t el = se[w];
  const bool live = el >= 0 && lane_ok;
  const int64_t ee = el >= 0 ? el : se[0];  // a slot past the strip's end works on a valid element
  // a group holds whole strips: bit w of its link byte says slot w + 1 continues slot w's strip
  const uint32_t link = slink[s];
  const bool has_prev = live && w > 0 && ((link >> (w > 0 ? w - 1 : 0)) & 1u);
  const bool has_next = live && (w + 1 < SL) && ((link >> w) & 1u);
  // this lane's nodes are written by the previous element of the strip
  const bool skip = has_prev && a == 0;
  T *const S0 = s0[w];
  T *const S1 = s1[w];
  const T *const C = Dg + P * P;  // even-odd coefficients
#define AT(i, j, k) ((k) * PL + (j) * LS + (i))

  int32_t nid[P];
  if constexpr (IDX == 2) {
    const int32_t *af = idx + ee * 4;
    const int32_t base = af[0] + a, sj = af[1], sk = af[2];
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = base + b * sj + k * sk;
  } else if constexpr (IDX == 1) {
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + ee * P2 + k * P + b) + a;
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k) nid[k] = __builtin_nontemporal_load(idx + ee * P3 + k * P2 + b * P + a);
  }
  // skipped and dead lanes count as owners: their read-modify-write loads read zeros
  const uint32_t ob = (live && !skip) ? (uint32_t)sown[ee * P2 + b * P + a] : 0xffffu;

  const TQ *const qe = qd + ee * (6 * P3) + b * P + a;
  T ga[6], gb[6];
  auto load_plane = [&](T(&g)[6], int k) {
#pragma unroll
    for (int m = 0; m < 6; ++m) g[m] = ld_q<NC, TQ, T>(qe + (k * 6 + m) * P2);
  };
  // a lane that is not on a live element only reads (its slot-0 or padding element's data): it
  // never writes an LDS slot another lane uses
  const bool lds_ok = lane_ok;

  {
    // ---- lines along r3: thread (i=a, j=b). Gather, and the r3 derivative in registers.
    T ut[P];
    {
      T u[P];
#pragma unroll
      for (int k = 0; k < P; ++k) u[k] = x[(int64_t)nid[k] * NC + c];
      load_plane(ga, 0);
      load_plane(gb, 1);
      __builtin_amdgcn_sched_barrier(0);
      if (lds_ok) {
#pragma unroll
        for (int k = 0; k < P; ++k) S0[AT(a, b, k)] = u[k];
      }
      eo_apply<P, T>(C, u, ut);
    }
    wave_sync();
    // ---- read lines along r1 (thread (j=a, k=b)) and r2 (thread (i=a, k=b))
    T li[P], lj[P];
#pragma unroll
    for (int l = 0; l < P; ++l) {
      li[l] = S0[AT(l, a, b)];
      lj[l] = S0[AT(a, l, b)];
    }
    wave_sync();
    // ---- derivatives along r1 -> S0, along r2 -> S1 (same layout [k][j][i])
    {
      T r[P];
      eo_apply<P, T>(C, li, r);
      if (lds_ok) {
#pragma unroll
        for (int i = 0; i < P; ++i) S0[AT(i, a, b)] = r[i];
      }
      eo_apply<P, T>(C, lj, r);
      if (lds_ok) {
#pragma unroll
        for (int j = 0; j < P; ++j) S1[AT(a, j, b)] = r[j];
      }
    }
    wave_sync();
    // ---- pointwise: (vr, vs, vt) = G (ur, us, ut) on lines along r3 (thread (i=a, j=b))
    T vt[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      T(&g)[6] = (k & 1) ? gb : ga;
      const T ur = S0[AT(a, b, k)], us = S1[AT(a, b, k)];
      if (lds_ok) {
        S0[AT(a, b, k)] = g[0] * ur + g[1] * us + g[2] * ut[k];
        S1[AT(a, b, k)] = g[1] * ur + g[3] * us + g[4] * ut[k];
      }
      vt[k] = g[2] * ur + g[4] * us + g[5] * ut[k];
      if (k + 2 < P) load_plane(g, k + 2);
      __builtin_amdgcn_sched_barrier(0);
    }
    // old values of the nodes this lane read-modify-writes, requested early (no other strip of
    // this launch touches them)
    T old[P];
#pragma unroll
    for (int k = 0; k < P; ++k) old[k] = *((ob & (1u << k)) ? zero : y + (int64_t)nid[k] * NC + c);
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
    wave_sync();
    // ---- transposed r1 derivative on S0 (thread (j=a, k=b)), r2 on S1 (thread (i=a, k=b)), in place
#pragma unroll
    for (int l = 0; l < P; ++l) {
      li[l] = S0[AT(l, a, b)];
      lj[l] = S1[AT(a, l, b)];
    }
    {
      T r[P];
      eo_apply_t<P, T>(C, li, r);
      if (lds_ok) {
#pragma unroll
        for (int i = 0; i < P; ++i) S0[AT(i, a, b)] = r[i];
      }
      eo_apply_t<P, T>(C, lj, r);
      if (lds_ok) {
#pragma unroll
        for (int j = 0; j < P; ++j) S1[AT(a, j, b)] = r[j];
      }
    }
    wave_sync();
    // ---- element sums on lines along r3; shared faces through LDS; scatter
    T out[P];
#pragma unroll
    for (int k = 0; k < P; ++k) out[k] = old[k] + (yt[k] + S0[AT(a, b, k)] + S1[AT(a, b, k)]);
    if (skip) {
#pragma unroll
      for (int k = 0; k < P; ++k) face[w][k * P + b] = out[k];
    }
    if constexpr (SC::NW > 1)
      __syncthreads();
    else
      wave_sync();
    if (has_next && a == P - 1) {
#pragma unroll
      for (int k = 0; k < P; ++k) out[k] += face[w + 1][k * P + b];
    }
    if (live && !skip) {
#pragma unroll
      for (int k = 0; k < P; ++k) y[(int64_t)nid[k] * NC + c] = out[k];
    }
  }
#undef AT
}

}  // namespace hx
