// Host-side launch of the fused apply: one launch per element color, in color order.
#pragma once

#include <type_traits>

#include "apply_kernel.h"
#include "colloc_kernel.h"
#include "gauss_kernel.h"
#include "hx_internal.h"
#include "strip_kernel.h"

namespace hx {

// HELM: the Helmholtz operator alpha A + beta B (qd holds alpha times the diffusion factors, qm the
// mass factors beta w detJ at the points); the diffusion kernels add the mass term in the same pass.
template <int P, int Q, int MODE, int NC, typename T, typename TQ, bool EOUT, bool HELM = false>
hx_status launch_colors(const hx_op_s &op, const T *tab, const TQ *qd, const ApplyArgs &a, hipStream_t s,
                        const TQ *qm = nullptr) {
  // strips (one workgroup per group of whole strips and component)
  if constexpr (MODE == MODE_COLLOC && colloc_strips(P) && !EOUT) {
    const hx_mesh_s &m = *op.mesh;
    // below degree 7 a strip workgroup has 1-4 wavefronts: a launch needs two strips per CU on
    // average to fill the chip, else the element kernel (more, smaller workgroups) is faster
    if (m.nstrips > 0 && (P == kStripP || m.nstrip_groups >= (int64_t)kMinStripsPerColor * m.nstrip_colors)) {
      // strip scatter: one launch per strip color
      const T *zero = reinterpret_cast<const T *>(m.zeros.ptr);
      for (int c = 0; c < m.nstrip_colors; ++c) {
        const int64_t s0 = m.strip_color_start[c], s1 = m.strip_color_start[c + 1];
        if (s1 <= s0) continue;
        const dim3 grid((unsigned)((s1 - s0) * NC)), block(StripCfg<P>::NW * 64);
        if (m.idx_affine.ptr)
          hipLaunchKernelGGL((k_colloc_strip<P, NC, T, TQ, 2, HELM>), grid, block, 0, s, m.idx_affine.ptr, m.strip_own.ptr,
                             qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y), m.strip_elems.ptr, m.strip_link.ptr, s0, zero,
                             qm);
        else if (m.idx_rows.ptr)
          hipLaunchKernelGGL((k_colloc_strip<P, NC, T, TQ, 1, HELM>), grid, block, 0, s, m.idx_rows.ptr, m.strip_own.ptr,
                             qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y), m.strip_elems.ptr, m.strip_link.ptr, s0, zero,
                             qm);
        else
          hipLaunchKernelGGL((k_colloc_strip<P, NC, T, TQ, 0, HELM>), grid, block, 0, s, a.idx, m.strip_own.ptr, qd, tab,
                             static_cast<const T *>(a.x), static_cast<T *>(a.y), m.strip_elems.ptr, m.strip_link.ptr, s0, zero, qm);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "k_colloc_strip launch");
      return HX_OK;
    }
  }
  if constexpr (MODE == MODE_COLLOC && P <= 8) {
    // line-per-thread collocated kernel
    using CF = CollocCfg<P>;
    const hx_mesh_s &m = *op.mesh;
    const T *zero = reinterpret_cast<const T *>(m.zeros.ptr);
    // E-vector output writes no shared node: one launch over all elements
    const int ncol = EOUT ? 1 : m.ncolors;
    for (int c = 0; c < ncol; ++c) {
      const int64_t e0 = EOUT ? 0 : m.color_start[c], e1 = EOUT ? m.nelem : m.color_start[c + 1];
      if (e1 <= e0) continue;
      const int64_t nb = (e1 - e0 + CF::EPB - 1) / CF::EPB * NC;  // blocks: element groups x components
      if (m.idx_rows.ptr)
        hipLaunchKernelGGL((k_colloc<P, NC, T, TQ, EOUT, true, HELM>), dim3((unsigned)nb), dim3(CF::THREADS), 0, s,
                           m.idx_rows.ptr, a.own, qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y),
                           a.order, e0, e1, zero, qm);
      else
        hipLaunchKernelGGL((k_colloc<P, NC, T, TQ, EOUT, false, HELM>), dim3((unsigned)nb), dim3(CF::THREADS), 0, s,
                           a.idx, a.own, qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y), a.order, e0,
                           e1, zero, qm);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_colloc launch");
    return HX_OK;
  }
  // line-per-thread interpolating kernel, one element per workgroup: FP64 diffusion and FP64 mass
  // with q >= 7, where it beats the point-per-thread kernel; in FP32, and for mass at smaller q,
  // that kernel fills its wavefronts with several elements and wins
  constexpr bool kGaussQ = Q <= 10 && !EOUT && ((MODE == MODE_DIFF && Q >= 6) || (MODE == MODE_MASS && Q >= 7));
  constexpr bool kGauss = std::is_same<T, double>::value && kGaussQ;
  // several components in FP32: the joint-component kernel (all components of an element per
  // workgroup) beats the point-per-thread kernel too
  constexpr bool kJointF32 = std::is_same<T, float>::value && NC > 1 && kGaussQ;
  // several components in FP64: the joint kernel up to q = 9; at q = 10 its buffers and staged
  // factors (99 KB of LDS) leave one workgroup per CU, and a workgroup per component runs instead
  constexpr bool kJoint = NC > 1 && (kJointF32 || Q <= 9);
  if constexpr (kGauss && gauss_strips(P, Q, MODE == MODE_MASS, NC)) {
    // on a mesh with strips: the strip scatter
    const hx_mesh_s &m = *op.mesh;
    if (m.nstrips > 0) {
      const T *zero = reinterpret_cast<const T *>(m.zeros.ptr);
      const dim3 block(kStrip * GaussCfg<Q>::NT);
      for (int c = 0; c < m.nstrip_colors; ++c) {
        const int64_t s0 = m.strip_color_start[c], s1 = m.strip_color_start[c + 1];
        if (s1 <= s0) continue;
        const dim3 grid((unsigned)((s1 - s0) * NC));
        if (m.idx_affine.ptr)
          hipLaunchKernelGGL((k_gauss_strip<P, Q, MODE, NC, T, TQ, 2, HELM>), grid, block, 0, s, m.idx_affine.ptr,
                             m.strip_own.ptr, qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y),
                             m.strip_elems.ptr, m.strip_link.ptr, s0, zero, qm);
        else if (m.idx_rows.ptr)
          hipLaunchKernelGGL((k_gauss_strip<P, Q, MODE, NC, T, TQ, 1, HELM>), grid, block, 0, s, m.idx_rows.ptr,
                             m.strip_own.ptr, qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y),
                             m.strip_elems.ptr, m.strip_link.ptr, s0, zero, qm);
        else
          hipLaunchKernelGGL((k_gauss_strip<P, Q, MODE, NC, T, TQ, 0, HELM>), grid, block, 0, s, a.idx, m.strip_own.ptr,
                             qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y), m.strip_elems.ptr, m.strip_link.ptr, s0,
                             zero, qm);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "k_gauss_strip launch");
      return HX_OK;
    }
  }
  if constexpr (kGauss || kJointF32) {
    const hx_mesh_s &m = *op.mesh;
    const T *zero = reinterpret_cast<const T *>(m.zeros.ptr);
    for (int c = 0; c < m.ncolors; ++c) {
      const int64_t e0 = m.color_start[c], e1 = m.color_start[c + 1];
      if (e1 <= e0) continue;
      if constexpr (kJoint) {
        if (m.idx_affine.ptr)
          hipLaunchKernelGGL((k_gauss_joint<P, Q, MODE, NC, T, TQ, 2, HELM>), dim3((unsigned)(e1 - e0)),
                             dim3(GaussJointCfg<Q, NC>::NT), 0, s, m.idx_affine.ptr, a.own, qd, tab,
                             static_cast<const T *>(a.x), static_cast<T *>(a.y), e0, zero, qm);
        else
          hipLaunchKernelGGL((k_gauss_joint<P, Q, MODE, NC, T, TQ, 0, HELM>), dim3((unsigned)(e1 - e0)),
                             dim3(GaussJointCfg<Q, NC>::NT), 0, s, a.idx, a.own, qd, tab, static_cast<const T *>(a.x),
                             static_cast<T *>(a.y), e0, zero, qm);
      } else if (m.idx_affine.ptr) {
        hipLaunchKernelGGL((k_gauss<P, Q, MODE, NC, T, TQ, 2, HELM>), dim3((unsigned)((e1 - e0) * NC)),
                           dim3(GaussCfg<Q>::NT), 0, s, m.idx_affine.ptr, a.own, qd, tab, static_cast<const T *>(a.x),
                           static_cast<T *>(a.y), e0, e1, zero, qm);
      } else {
        hipLaunchKernelGGL((k_gauss<P, Q, MODE, NC, T, TQ, 0, HELM>), dim3((unsigned)((e1 - e0) * NC)),
                           dim3(GaussCfg<Q>::NT), 0, s, a.idx, a.own, qd, tab, static_cast<const T *>(a.x),
                           static_cast<T *>(a.y), e0, e1, zero, qm);
      }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_gauss launch");
    return HX_OK;
  }
  constexpr int EPB = EpbOf<Q>::v;
  const hx_mesh_s &m = *op.mesh;
  const int ncol = EOUT ? 1 : m.ncolors;  // E-vector output: one launch over all elements
  for (int c = 0; c < ncol; ++c) {
    const int64_t e0 = EOUT ? 0 : m.color_start[c], e1 = EOUT ? m.nelem : m.color_start[c + 1];
    if (e1 <= e0) continue;
    const int64_t nb = (e1 - e0 + EPB - 1) / EPB * NC;  // blocks: element groups x components
    if (m.idx_affine.ptr)
      hipLaunchKernelGGL((k_apply<P, Q, MODE, NC, T, TQ, EOUT, 2, HELM>), dim3((unsigned)nb), dim3(EPB * Q * Q), 0, s,
                         m.idx_affine.ptr, a.own, qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y), a.order,
                         e0, e1, qm);
    else
      hipLaunchKernelGGL((k_apply<P, Q, MODE, NC, T, TQ, EOUT, 0, HELM>), dim3((unsigned)nb), dim3(EPB * Q * Q), 0, s,
                         a.idx, a.own, qd, tab, static_cast<const T *>(a.x), static_cast<T *>(a.y), a.order, e0, e1,
                         qm);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_apply launch");
  return HX_OK;
}

template <int P, int Q, int MODE, int NC, bool HELM>
hx_status launch_prec_h(const hx_op_s &op, Prec prec, bool eout, const ApplyArgs &a, hipStream_t s) {
  if (eout) {
    if (prec != Prec::F64) return fail(HX_EUNSUPPORTED, "E-vector output is FP64 only");
    return launch_colors<P, Q, MODE, NC, double, double, true, HELM>(op, op.tab.ptr, op.qdata.ptr, a, s,
                                                                     op.qmass.ptr);
  }
  switch (prec) {
    case Prec::F64:
      return launch_colors<P, Q, MODE, NC, double, double, false, HELM>(op, op.tab.ptr, op.qdata.ptr, a, s,
                                                                        op.qmass.ptr);
    case Prec::F32_Q64:
      return launch_colors<P, Q, MODE, NC, float, double, false, HELM>(op, op.tab32.ptr, op.qdata.ptr, a, s,
                                                                       op.qmass.ptr);
    case Prec::F32_Q32:
      return launch_colors<P, Q, MODE, NC, float, float, false, HELM>(op, op.tab32.ptr, op.qdata32.ptr, a, s,
                                                                      op.qmass32.ptr);
  }
  return fail(HX_EINVAL, "bad precision");
}

template <int P, int Q, int MODE, int NC>
hx_status launch_prec(const hx_op_s &op, Prec prec, bool eout, const ApplyArgs &a, hipStream_t s) {
  if constexpr (MODE != MODE_MASS) {
    if (op.kind == HX_HELMHOLTZ) return launch_prec_h<P, Q, MODE, NC, true>(op, prec, eout, a, s);
  }
  return launch_prec_h<P, Q, MODE, NC, false>(op, prec, eout, a, s);
}

template <int P, int Q, int MODE>
hx_status launch_nc(const hx_op_s &op, Prec prec, bool eout, const ApplyArgs &a, hipStream_t s) {
  if (op.ncomp == 1) return launch_prec<P, Q, MODE, 1>(op, prec, eout, a, s);
  if (op.ncomp == 3) return launch_prec<P, Q, MODE, 3>(op, prec, eout, a, s);
  return fail(HX_EINVAL, "ncomp must be 1 or 3");
}

template <int P>
hx_status launch_apply_P(const hx_op_s &op, Prec prec, bool eout, const ApplyArgs &a, hipStream_t s) {
  if (op.colloc) return launch_nc<P, P, MODE_COLLOC>(op, prec, eout, a, s);
  const bool mass = op.kind == HX_MASS;
  if (op.Q == P) return mass ? launch_nc<P, P, MODE_MASS>(op, prec, eout, a, s)
                             : launch_nc<P, P, MODE_DIFF>(op, prec, eout, a, s);
  if (op.Q == P + 1) return mass ? launch_nc<P, P + 1, MODE_MASS>(op, prec, eout, a, s)
                                 : launch_nc<P, P + 1, MODE_DIFF>(op, prec, eout, a, s);
  return fail(HX_EUNSUPPORTED, "q must be p+1 or p+2");
}

}  // namespace hx
