// Low-order refined (LOR) operator.
//
// Preconditioning section: a high-order system can be preconditioned through a spectrally
// equivalent sparse matrix, the low-order discretization on a refined mesh (FEM-SEM equivalence
// for tensor-product elements). Here every degree-p element is split into p^3 trilinear
// sub-hexahedra whose corners are its GLL nodes; the sub-hex stiffness is the Q1 form integrated
// with the 2-point GLL (vertex) rule per direction, kappa at the vertices:
//   L_s[v][w] = sum_{q corner} kappa(x_q) (adj(J_q)^T grad phi_v(r_q)) . (adj(J_q)^T grad phi_w(r_q)) / det J_q.
// At a corner q only q and its three edge neighbours have a non-zero reference gradient, so two
// nodes couple only when they differ in at most two of the three local directions: 19 couplings
// per node of a lattice. The assembled matrix is stored in ELL layout, W entries per row (W the
// largest row length), column-major ([k][n]) so that consecutive rows read consecutive memory;
// rows shorter than W repeat their own index with value 0.
//
// Assembly on the device, deterministic and atomic-free: one thread per node walks the element
// slots that hold it (a node -> slot table in internal element order, ascending) and, for each,
// the sub-hexes of that element that have the node as a corner; it sums its own row only.
#include <algorithm>
#include <vector>

#include "hx_internal.h"

namespace hx {

namespace {

constexpr int kLorThreads = 128;
constexpr int kLorMaxW = 32;  // longest row the assembly supports

struct KappaLor {
  int M;
  const double *omega;
  const double *phase;
  double scale, shift;
};

__global__ void __launch_bounds__(256) k_lor_kappa(int64_t n, const double *__restrict__ xyz, KappaLor kap,
                                                   double *__restrict__ kn) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double k = 1.0;
    if (kap.M > 0) {
      const double x = xyz[3 * t], y = xyz[3 * t + 1], z = xyz[3 * t + 2];
      double g = 0.0;
      for (int m = 0; m < kap.M; ++m)
        g += cos(kap.omega[3 * m] * x + kap.omega[3 * m + 1] * y + kap.omega[3 * m + 2] * z + kap.phase[m]);
      g *= sqrt(2.0 / kap.M);
      k = exp(kap.scale * g + kap.shift);
    }
    kn[t] = k;
  }
}

// Row structure. Pass 0 counts each node's couplings into cnt; pass 1 writes them, ascending, to
// cols [W][n] (padded with the node's own index). sptr/sslot: the element slots of each node
// (internal element position e, local node l as e P^3 + l), ascending.
__global__ void __launch_bounds__(kLorThreads)
    k_lor_cols(int64_t n, int P, const int32_t *__restrict__ sptr, const int32_t *__restrict__ sslot,
               const int32_t *__restrict__ idx, int pass, int W, int32_t *__restrict__ cnt,
               int32_t *__restrict__ cols) {
  __shared__ int32_t nb[kLorThreads][kLorMaxW + 1];
  int32_t *const mine = nb[threadIdx.x];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int P2 = P * P, P3 = P2 * P;
  int m = 0;
  bool over = false;
  for (int64_t s = sptr[t]; s < sptr[t + 1]; ++s) {
    const int32_t sl = sslot[s];
    const int64_t e = sl / P3;
    const int l = sl - (int)e * P3;
    const int i = l % P, j = (l / P) % P, k = l / P2;
    for (int dk = -1; dk <= 1; ++dk)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          if (di != 0 && dj != 0 && dk != 0) continue;  // opposite corners of a sub-hex do not couple
          const int ii = i + di, jj = j + dj, kk = k + dk;
          if (ii < 0 || ii >= P || jj < 0 || jj >= P || kk < 0 || kk >= P) continue;
          const int32_t c = idx[e * P3 + ii + P * (jj + P * kk)];
          int pos = 0;
          while (pos < m && mine[pos] < c) ++pos;
          if (pos < m && mine[pos] == c) continue;
          if (m == kLorMaxW) {
            over = true;
            continue;
          }
          for (int q = m; q > pos; --q) mine[q] = mine[q - 1];
          mine[pos] = c;
          ++m;
        }
  }
  if (pass == 0) {
    cnt[t] = over ? kLorMaxW + 1 : m;
    return;
  }
  for (int q = 0; q < W; ++q) cols[(int64_t)q * n + t] = q < m ? mine[q] : (int32_t)t;
}

// Row values: for each slot of node t and each sub-hex of that element with t as a corner, the
// sub-hex matrix row of t, added at the columns of the sub-hex's corners. Rows are summed in
// LDS (this thread's own), slots and sub-hexes in a fixed order.
__global__ void __launch_bounds__(kLorThreads)
    k_lor_vals(int64_t n, int P, const int32_t *__restrict__ sptr, const int32_t *__restrict__ sslot,
               const int32_t *__restrict__ idx, const double *__restrict__ xyz, const double *__restrict__ kn, int W,
               const int32_t *__restrict__ cols, double *__restrict__ vals, int *__restrict__ bad) {
  __shared__ int32_t sc[kLorThreads][kLorMaxW + 1];
  __shared__ double sv[kLorThreads][kLorMaxW];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  int32_t *const mc = sc[threadIdx.x];
  double *const mv = sv[threadIdx.x];
  for (int q = 0; q < W; ++q) {
    mc[q] = cols[(int64_t)q * n + t];
    mv[q] = 0.0;
  }
  const int P2 = P * P, P3 = P2 * P;
  for (int64_t s = sptr[t]; s < sptr[t + 1]; ++s) {
    const int32_t sl = sslot[s];
    const int64_t e = sl / P3;
    const int l = sl - (int)e * P3;
    const int i = l % P, j = (l / P) % P, k = l / P2;
    // sub-hexes (i0, j0, k0) of this element with t as a corner (v = its corner index there)
    for (int c0 = 0; c0 < 2; ++c0)
      for (int b0 = 0; b0 < 2; ++b0)
        for (int a0 = 0; a0 < 2; ++a0) {
          const int i0 = i - a0, j0 = j - b0, k0 = k - c0;
          if (i0 < 0 || i0 > P - 2 || j0 < 0 || j0 > P - 2 || k0 < 0 || k0 > P - 2) continue;
          const int v = a0 + 2 * b0 + 4 * c0;
          int32_t nd[8];
          double X[8][3], kq[8];
          for (int w = 0; w < 8; ++w) {
            nd[w] = idx[e * P3 + (i0 + (w & 1)) + P * ((j0 + ((w >> 1) & 1)) + P * (k0 + (w >> 2)))];
            X[w][0] = xyz[3 * (int64_t)nd[w]];
            X[w][1] = xyz[3 * (int64_t)nd[w] + 1];
            X[w][2] = xyz[3 * (int64_t)nd[w] + 2];
            kq[w] = kn[nd[w]];
          }
          double row[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int q = 0; q < 8; ++q) {
            const double r[3] = {(q & 1) ? 1.0 : -1.0, ((q >> 1) & 1) ? 1.0 : -1.0, (q >> 2) ? 1.0 : -1.0};
            // reference gradients of the 8 corner functions at corner q
            double G[8][3];
            for (int w = 0; w < 8; ++w) {
              const double s0 = (w & 1) ? 1.0 : -1.0, s1 = ((w >> 1) & 1) ? 1.0 : -1.0, s2 = (w >> 2) ? 1.0 : -1.0;
              const double f0 = 0.5 * (1.0 + s0 * r[0]), f1 = 0.5 * (1.0 + s1 * r[1]), f2 = 0.5 * (1.0 + s2 * r[2]);
              G[w][0] = 0.5 * s0 * f1 * f2;
              G[w][1] = 0.5 * s1 * f0 * f2;
              G[w][2] = 0.5 * s2 * f0 * f1;
            }
            double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int w = 0; w < 8; ++w)
              for (int d = 0; d < 3; ++d)
                for (int c = 0; c < 3; ++c) J[d][c] += X[w][d] * G[w][c];
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
            if (!(det > 0.0)) {
              *bad = 1;
              continue;
            }
            // physical gradient times det: g_w[a] = sum_c adj[c][a] G[w][c] (J^-T = adj^T / det)
            double gv[3];
            for (int a = 0; a < 3; ++a) gv[a] = adj[0][a] * G[v][0] + adj[1][a] * G[v][1] + adj[2][a] * G[v][2];
            const double sq = kq[q] / det;
            for (int w = 0; w < 8; ++w) {
              double d = 0.0;
              for (int a = 0; a < 3; ++a) d += gv[a] * (adj[0][a] * G[w][0] + adj[1][a] * G[w][1] + adj[2][a] * G[w][2]);
              row[w] += sq * d;
            }
          }
          for (int w = 0; w < 8; ++w) {
            if ((w ^ v) == 7) continue;  // the opposite corner: no coupling (zero row entry)
            int pos = 0;
            while (pos < W - 1 && mc[pos] != nd[w]) ++pos;
            mv[pos] += row[w];
          }
        }
  }
  for (int q = 0; q < W; ++q) vals[(int64_t)q * n + t] = mv[q];
}

__global__ void __launch_bounds__(256) k_lor_spmv(int64_t n, int W, const int32_t *__restrict__ cols,
                                                  const double *__restrict__ vals, const double *__restrict__ x,
                                                  double *__restrict__ y) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < W; ++q) s += vals[(int64_t)q * n + t] * x[cols[(int64_t)q * n + t]];
    y[t] = s;
  }
}

__global__ void __launch_bounds__(256) k_lor_diag(int64_t n, int W, const int32_t *__restrict__ cols,
                                                  const double *__restrict__ vals, double *__restrict__ d) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < W; ++q)
      if (cols[(int64_t)q * n + t] == t) s += vals[(int64_t)q * n + t];
    d[t] = s;
  }
}

unsigned lor_grid(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 8192); }

}  // namespace

hx_status lor_assemble(hx_op_s &op, const hx_kappa_rff *kappa, hipStream_t s) {
  hx_mesh_s &m = *op.mesh;
  const int P = m.P;
  const int64_t n = m.nnodes;
  if (P < 2) return fail(HX_EUNSUPPORTED, "the low-order refined operator needs p >= 1");
  // node -> element slots, internal element order, ascending (kept by the mesh)
  if (hx_status st = mesh_slots(m)) return st;
  const int32_t *sptr = m.slot_ptr.ptr, *sslot = m.slot_idx.ptr;
  DevBuf<int32_t> dcnt;
  DevBuf<double> dk, dom, dph;
  HX_HIP(dcnt.alloc(n));
  HX_HIP(dk.alloc(n));
  KappaLor kap{0, nullptr, nullptr, 0.0, 0.0};
  if (kappa && kappa->M > 0) {
    HX_HIP(dom.upload(kappa->omega, (size_t)kappa->M * 3));
    HX_HIP(dph.upload(kappa->phase, (size_t)kappa->M));
    kap = KappaLor{kappa->M, dom.ptr, dph.ptr, kappa->scale, kappa->shift};
  }
  hipLaunchKernelGGL(k_lor_kappa, dim3(lor_grid(n)), dim3(256), 0, s, n, m.xyz.ptr, kap, dk.ptr);
  const unsigned nb = (unsigned)((n + kLorThreads - 1) / kLorThreads);
  hipLaunchKernelGGL(k_lor_cols, dim3(nb), dim3(kLorThreads), 0, s, n, P, sptr, sslot, m.idx.ptr, 0, 0,
                     dcnt.ptr, (int32_t *)nullptr);
  HX_HIP(hipGetLastError());
  std::vector<int32_t> cnt(n);
  HX_HIP(hipMemcpyAsync(cnt.data(), dcnt.ptr, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HX_HIP(hipStreamSynchronize(s));
  const int W = *std::max_element(cnt.begin(), cnt.end());
  if (W > kLorMaxW) return fail(HX_EUNSUPPORTED, "a node couples to more than 32 nodes in the refined mesh");
  op.lor_w = W;
  HX_HIP(op.lor_col.alloc((size_t)W * n));
  HX_HIP(op.lor_val.alloc((size_t)W * n));
  hipLaunchKernelGGL(k_lor_cols, dim3(nb), dim3(kLorThreads), 0, s, n, P, sptr, sslot, m.idx.ptr, 1, W,
                     dcnt.ptr, op.lor_col.ptr);
  DevBuf<int> dbad;
  HX_HIP(dbad.alloc(1));
  HX_HIP(hipMemsetAsync(dbad.ptr, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_lor_vals, dim3(nb), dim3(kLorThreads), 0, s, n, P, sptr, sslot, m.idx.ptr, m.xyz.ptr,
                     dk.ptr, W, op.lor_col.ptr, op.lor_val.ptr, dbad.ptr);
  HX_HIP(hipGetLastError());
  int bad = 0;
  HX_HIP(hipMemcpyAsync(&bad, dbad.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  HX_HIP(hipStreamSynchronize(s));  // the temporaries are freed on return
  if (bad) return fail(HX_EGEOM, "non-positive Jacobian determinant at a corner of a refined sub-hexahedron");
  return HX_OK;
}

hx_status lor_apply(const hx_op_s &op, const double *x, double *y, hipStream_t s) {
  const int64_t n = op.mesh->nnodes;
  hipLaunchKernelGGL(k_lor_spmv, dim3(lor_grid(n)), dim3(256), 0, s, n, op.lor_w, op.lor_col.ptr, op.lor_val.ptr, x,
                     y);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

hx_status lor_diagonal(const hx_op_s &op, double *diag, hipStream_t s) {
  const int64_t n = op.mesh->nnodes;
  hipLaunchKernelGGL(k_lor_diag, dim3(lor_grid(n)), dim3(256), 0, s, n, op.lor_w, op.lor_col.ptr, op.lor_val.ptr,
                     diag);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace hx

using namespace hx;

extern "C" hx_status hx_op_create_lor(hx_mesh mesh, const hx_kappa_rff *kappa, hx_stream stream, hx_op *out) {
  if (!out) return fail(HX_EINVAL, "out is null");
  *out = nullptr;
  if (!mesh) return fail(HX_EINVAL, "null mesh");
  if (mesh->host_only) return fail(HX_EINVAL, "the mesh is a host-only plan (hx_mesh_plan): create it with hx_mesh_create");
  if (kappa && (kappa->M < 0 || (kappa->M > 0 && (!kappa->omega || !kappa->phase))))
    return fail(HX_EINVAL, "kappa: M >= 0 and omega/phase non-null");
  int dev = 0;
  HX_HIP(hipGetDevice(&dev));
  if (dev != mesh->device) return fail(HX_EINVAL, "current device differs from the mesh's device");
  auto *op = new (std::nothrow) hx_op_s();
  if (!op) return fail(HX_ENOMEM, "host allocation failed");
  op->mesh = mesh;
  op->kind = HX_LOR;
  op->ncomp = 1;
  op->P = mesh->P;
  op->Q = 2;
  op->b.p = mesh->p;
  op->b.P = mesh->P;
  op->b.q = 2;
  op->b.rule = HX_GLL;
  op->ncq = 0;
  if (hx_status st = lor_assemble(*op, kappa, static_cast<hipStream_t>(stream))) {
    delete op;
    return st;
  }
  *out = op;
  return HX_OK;
}

extern "C" hx_status hx_op_lor_matrix(hx_op op, int *width, int32_t *cols, double *vals) {
  if (!op || !width) return fail(HX_EINVAL, "null argument");
  if (op->kind != HX_LOR) return fail(HX_EINVAL, "not a low-order refined operator");
  *width = op->lor_w;
  const size_t cnt = (size_t)op->lor_w * op->mesh->nnodes;
  if (cols) HX_HIP(hipMemcpy(cols, op->lor_col.ptr, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
  if (vals) HX_HIP(hipMemcpy(vals, op->lor_val.ptr, sizeof(double) * cnt, hipMemcpyDeviceToHost));
  return HX_OK;
}
