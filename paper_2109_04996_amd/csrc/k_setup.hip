// Setup kernels, FP64: geometric factors at the quadrature points, the
// coefficient field, and the matrix-free diagonal.
//
// Benchmarks section: isoparametric Q_p bricks; the Jacobian of x^e(r) at a
// point is sum_n x_n (grad_r phi_n)(r) over the element's nodes. libCEED
// section: the pointwise operator D at the quadrature points is computed once
// and stored (partial assembly):
//   mass       w detJ
//   diffusion  w kappa detJ J^-1 J^-T = w kappa adj(J) adj(J)^T / detJ
// stored as 6 symmetric entries per point, layout [e][qc][m][qb][qa] (plane by plane);
// the Helmholtz operator alpha A + beta B stores alpha times the diffusion entries and,
// separately, beta w detJ.
// Miniapps section (Nekbone's diagonal preconditioner): the diagonal of the
// assembled operator is sum_e G_e^T diag(B^T D B), computed here point by
// point from the 1D tables without forming element matrices.
#include <cmath>

#include "hx_internal.h"

namespace hx {

namespace {

constexpr int kSetupThreads = 256;

struct KappaDev {
  int M;
  const double *omega;
  const double *phase;
  double scale, shift;
};

// One block per element: stage the element's node coordinates in LDS, then
// one thread per quadrature point.
// HX_HELMHOLTZ: qd gets alpha times the diffusion factors and qm [e][qc][qb][qa] beta * w * detJ.
__global__ void __launch_bounds__(kSetupThreads)
    k_qdata(int P, int Q, int kind, const int32_t *__restrict__ idx, const double *__restrict__ xyz,
            const double *__restrict__ interp, const double *__restrict__ grad, const double *__restrict__ qw,
            KappaDev kap, double *__restrict__ qd, int *__restrict__ bad, double alpha, double beta,
            double *__restrict__ qm) {
  __shared__ double sx[3][kMaxP * kMaxP * kMaxP];
  __shared__ double sI[kMaxQ * kMaxP], sG[kMaxQ * kMaxP], sw[kMaxQ];
  const int64_t e = blockIdx.x;
  const int P3 = P * P * P, Q3 = Q * Q * Q;
  for (int t = threadIdx.x; t < P3; t += blockDim.x) {
    const int64_t n = idx[e * P3 + t];
    sx[0][t] = xyz[n * 3 + 0];
    sx[1][t] = xyz[n * 3 + 1];
    sx[2][t] = xyz[n * 3 + 2];
  }
  for (int t = threadIdx.x; t < Q * P; t += blockDim.x) {
    sI[t] = interp[t];
    sG[t] = grad[t];
  }
  for (int t = threadIdx.x; t < Q; t += blockDim.x) sw[t] = qw[t];
  __syncthreads();
  const int ncq = (kind == HX_MASS) ? 1 : 6;
  for (int pt = threadIdx.x; pt < Q3; pt += blockDim.x) {
    const int qa = pt % Q, qb = (pt / Q) % Q, qc = pt / (Q * Q);
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double X[3] = {0, 0, 0};
    for (int k = 0; k < P; ++k) {
      const double Ik = sI[qc * P + k], Gk = sG[qc * P + k];
      for (int j = 0; j < P; ++j) {
        const double Ij = sI[qb * P + j], Gj = sG[qb * P + j];
        for (int i = 0; i < P; ++i) {
          const double Ii = sI[qa * P + i], Gi = sG[qa * P + i];
          const int l = i + P * (j + P * k);
          const double d0 = Gi * Ij * Ik, d1 = Ii * Gj * Ik, d2 = Ii * Ij * Gk, v = Ii * Ij * Ik;
          for (int r = 0; r < 3; ++r) {
            const double xr = sx[r][l];
            J[r][0] += xr * d0;
            J[r][1] += xr * d1;
            J[r][2] += xr * d2;
            X[r] += xr * v;
          }
        }
      }
    }
    // adjugate (transpose of the cofactor matrix): adj(J) J = det I
    double adj[3][3];
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    if (!(det > 0.0)) *bad = 1;
    const double w = sw[qa] * sw[qb] * sw[qc];
    // layout [e][qc][m][qb][qa]
    double *out = qd + e * (int64_t)(ncq * Q3) + (int64_t)qc * ncq * Q * Q + qb * Q + qa;
    const int Q2 = Q * Q;
    if (kind == HX_MASS) {
      out[0] = w * det;
    } else {
      if (kind == HX_HELMHOLTZ) qm[e * (int64_t)Q3 + pt] = beta * (w * det);
      double kappa = 1.0;
      if (kap.M > 0) {
        double g = 0.0;
        for (int m = 0; m < kap.M; ++m)
          g += cos(kap.omega[3 * m] * X[0] + kap.omega[3 * m + 1] * X[1] + kap.omega[3 * m + 2] * X[2] +
                   kap.phase[m]);
        g *= sqrt(2.0 / kap.M);
        kappa = exp(kap.scale * g + kap.shift);
      }
      const double s = (kind == HX_HELMHOLTZ ? alpha : 1.0) * (w * kappa / det);
      // J^-1 = adj / det, so w kappa det J^-1 J^-T = s * adj adj^T
      double G[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = r; c < 3; ++c)
          G[r][c] = s * (adj[r][0] * adj[c][0] + adj[r][1] * adj[c][1] + adj[r][2] * adj[c][2]);
      out[0 * Q2] = G[0][0];
      out[1 * Q2] = G[0][1];
      out[2 * Q2] = G[0][2];
      out[3 * Q2] = G[1][1];
      out[4 * Q2] = G[1][2];
      out[5 * Q2] = G[2][2];
    }
  }
}

// Diagonal: one block per element, one thread per element node; then the
// ownership scatter of the apply (store first, accumulate afterwards).
__global__ void __launch_bounds__(kSetupThreads)
    k_diag(int P, int Q, int kind, int ncomp, const int32_t *__restrict__ idx, const uint16_t *__restrict__ own,
           const double *__restrict__ interp, const double *__restrict__ grad, const double *__restrict__ qd,
           double *__restrict__ diag, int64_t e_begin, const double *__restrict__ qm) {
  __shared__ double sI[kMaxQ * kMaxP], sG[kMaxQ * kMaxP];
  const int64_t e = e_begin + blockIdx.x;
  const int P2 = P * P, P3 = P2 * P, Q3 = Q * Q * Q;
  for (int t = threadIdx.x; t < Q * P; t += blockDim.x) {
    sI[t] = interp[t];
    sG[t] = grad[t];
  }
  __syncthreads();
  const int ncq = (kind == HX_MASS) ? 1 : 6;
  const double *qe = qd + e * (int64_t)(ncq * Q3);
  for (int l = threadIdx.x; l < P3; l += blockDim.x) {
    const int i = l % P, j = (l / P) % P, k = l / P2;
    double s = 0.0;
    for (int qc = 0; qc < Q; ++qc) {
      const double Ik = sI[qc * P + k], Gk = sG[qc * P + k];
      for (int qb = 0; qb < Q; ++qb) {
        const double Ij = sI[qb * P + j], Gj = sG[qb * P + j];
        for (int qa = 0; qa < Q; ++qa) {
          const double Ii = sI[qa * P + i], Gi = sG[qa * P + i];
          // layout [qc][m][qb][qa]
          const double *g = qe + (qc * ncq) * Q * Q + qb * Q + qa;
          const int Q2 = Q * Q;
          if (kind == HX_MASS) {
            const double v = Ii * Ij * Ik;
            s += g[0] * v * v;
          } else {
            const double d0 = Gi * Ij * Ik, d1 = Ii * Gj * Ik, d2 = Ii * Ij * Gk;
            s += g[0] * d0 * d0 + g[3 * Q2] * d1 * d1 + g[5 * Q2] * d2 * d2 +
                 2.0 * (g[Q2] * d0 * d1 + g[2 * Q2] * d0 * d2 + g[4 * Q2] * d1 * d2);
            if (kind == HX_HELMHOLTZ) {
              const double v = Ii * Ij * Ik;
              s += qm[e * (int64_t)Q3 + (qc * Q + qb) * Q + qa] * v * v;
            }
          }
        }
      }
    }
    const int64_t n = idx[e * P3 + l];
    const bool first = (own[e * P2 + (l % P2)] >> k) & 1u;
    for (int c = 0; c < ncomp; ++c) {
      double *dst = diag + n * ncomp + c;
      if (first)
        *dst = s;
      else
        *dst += s;
    }
  }
}

__global__ void k_d2f(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = (float)a[t];
}

}  // namespace

hx_status launch_setup_qdata(hx_op_s &op, const hx_kappa_rff *kappa, hipStream_t s, int *bad_det) {
  const hx_mesh_s &m = *op.mesh;
  DevBuf<double> dI, dG, dW, dOm, dPh;
  DevBuf<int> dBad;
  HX_HIP(dI.upload(op.b.interp.data(), op.b.interp.size()));
  HX_HIP(dG.upload(op.b.grad.data(), op.b.grad.size()));
  HX_HIP(dW.upload(op.b.qw.data(), op.b.qw.size()));
  KappaDev kd{0, nullptr, nullptr, 0.0, 0.0};
  if (kappa && kappa->M > 0) {
    HX_HIP(dOm.upload(kappa->omega, (size_t)kappa->M * 3));
    HX_HIP(dPh.upload(kappa->phase, (size_t)kappa->M));
    kd = KappaDev{kappa->M, dOm.ptr, dPh.ptr, kappa->scale, kappa->shift};
  }
  HX_HIP(dBad.alloc(1));
  HX_HIP(hipMemsetAsync(dBad.ptr, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_qdata, dim3((unsigned)m.nelem), dim3(kSetupThreads), 0, s, op.P, op.Q, op.kind, m.idx.ptr,
                     m.xyz.ptr, dI.ptr, dG.ptr, dW.ptr, kd, op.qdata.ptr, dBad.ptr, op.alpha, op.beta, op.qmass.ptr);
  HX_HIP(hipGetLastError());
  HX_HIP(hipMemcpyAsync(bad_det, dBad.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  HX_HIP(hipStreamSynchronize(s));
  return HX_OK;
}

// the diagonal kernels on tables already in device memory (interp and grad, [Q][P] each); allocates nothing
hx_status launch_diagonal_tables(const hx_op_s &op, const double *interp, const double *grad, double *diag,
                                 hipStream_t s) {
  const hx_mesh_s &m = *op.mesh;
  if (m.nuntouched > 0) HX_HIP(hipMemsetAsync(diag, 0, sizeof(double) * m.nnodes * op.ncomp, s));
  for (int c = 0; c < m.ncolors; ++c) {
    const int64_t e0 = m.color_start[c], e1 = m.color_start[c + 1];
    if (e1 <= e0) continue;
    hipLaunchKernelGGL(k_diag, dim3((unsigned)(e1 - e0)), dim3(kSetupThreads), 0, s, op.P, op.Q, op.kind, op.ncomp,
                       m.idx.ptr, m.own.ptr, interp, grad, op.qdata.ptr, diag, e0, op.qmass.ptr);
  }
  HX_HIP(hipGetLastError());
  return HX_OK;
}

hx_status launch_diagonal(hx_op_s &op, double *diag, hipStream_t s) {
  if (op.kind == HX_LOR) return lor_diagonal(op, diag, s);
  DevBuf<double> dI, dG;
  HX_HIP(dI.upload(op.b.interp.data(), op.b.interp.size()));
  HX_HIP(dG.upload(op.b.grad.data(), op.b.grad.size()));
  if (hx_status st = launch_diagonal_tables(op, dI.ptr, dG.ptr, diag, s)) return st;
  // the temporary tables are freed when this returns: wait for the kernels that read them
  HX_HIP(hipStreamSynchronize(s));
  return HX_OK;
}

hx_status make_qdata32(hx_op_s &op, hipStream_t s) {
  if (op.qdata32.ptr) return HX_OK;
  if (op.qmass.count) {
    HX_HIP(op.qmass32.alloc(op.qmass.count));
    hipLaunchKernelGGL(k_d2f, dim3(1024), dim3(256), 0, s, (int64_t)op.qmass.count, op.qmass.ptr, op.qmass32.ptr);
  }
  HX_HIP(op.qdata32.alloc(op.qdata.count));
  hipLaunchKernelGGL(k_d2f, dim3(1024), dim3(256), 0, s, (int64_t)op.qdata.count, op.qdata.ptr, op.qdata32.ptr);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace hx
