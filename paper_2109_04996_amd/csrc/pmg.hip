// p-multigrid transfers between polynomial degrees on one mesh (preconditioning section: multigrid
// over a hierarchy of degrees with matrix-free smoothers), and the hierarchy's host-side setup.
//
// Prolongation y_f = P x_c: each element interpolates the coarse values at its coarse GLL nodes to
// its fine GLL nodes by three 1D contractions (the coarse Lagrange basis evaluated at the fine
// nodes, Pf x Pc), and writes only the fine nodes it owns (the fine mesh's ownership bits: the
// first element in internal order that holds the node), so each node is written exactly once
// (no scatter). Restriction y_c = P^T r_f: each element applies the transposed contractions to the
// fine values it owns (zero elsewhere) and stores a coarse E-vector; a second kernel sums every
// coarse node's E-vector slots in ascending slot order (deterministic, no atomics).
//
// One wavefront per element, four per workgroup; the element's intermediate tensors (at most
// 9^3 values) stay in LDS. The transfers run a few times per V-cycle against the smoothers'
// operator applies, and move 8 B per fine node plus the coarse vector.

#include <algorithm>
#include <cmath>
#include <numeric>

#include "hx_internal.h"
#include "mlp_internal.h"

namespace hx {
namespace {

constexpr int kTW = 4;  // wavefronts (elements) per workgroup

// LDS doubles per element: the two intermediate tensors of each transfer (A, then B)
__host__ __device__ constexpr int prolong_lds_a(int Pf, int Pc) { return Pc * Pf * Pf > Pc * Pc * Pc ? Pc * Pf * Pf : Pc * Pc * Pc; }
__host__ __device__ constexpr int prolong_lds_b(int Pf, int Pc) { return Pc * Pc * Pf; }
__host__ __device__ constexpr int restrict_lds_a(int Pf, int Pc) { return Pf * Pf * Pf; }
__host__ __device__ constexpr int restrict_lds_b(int Pf, int Pc) { return Pc * Pf * Pf; }

// fine node of local (line ji = i + Pf j, layer k): from the affine numbering {base, s_j, s_k}, or the index
template <bool AFF>
__device__ __forceinline__ int32_t fine_node(const int32_t *__restrict__ idx_f, const int32_t *__restrict__ aff,
                                             int64_t e, int Pf, int ji, int k) {
  if constexpr (AFF) {
    const int i = ji % Pf, j = ji / Pf;
    return aff[e * 4] + i + j * aff[e * 4 + 1] + k * aff[e * 4 + 2];
  } else {
    return idx_f[e * Pf * Pf * Pf + k * Pf * Pf + ji];
  }
}

// T: the vectors' type (the contractions run in FP64 either way)
template <bool AFF, typename T>
__global__ void __launch_bounds__(kTW * 64)
k_prolong(int64_t E, int Pf, int Pc, const int32_t *__restrict__ cmap, const int32_t *__restrict__ idx_f,
          const int32_t *__restrict__ aff, const int32_t *__restrict__ idx_c, const uint16_t *__restrict__ own,
          const double *__restrict__ I, const uint8_t *__restrict__ fm, int nc, const T *__restrict__ xc,
          T *__restrict__ yf) {
  const int comp = blockIdx.y;  // component of an interleaved vector (node * nc + comp)
  extern __shared__ double smem[];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * kTW + w;
  const bool live = e < E;
  double *A = smem + w * (prolong_lds_a(Pf, Pc) + prolong_lds_b(Pf, Pc)), *B = A + prolong_lds_a(Pf, Pc);
  const int Pc3 = Pc * Pc * Pc, Pf2 = Pf * Pf, Pf3 = Pf2 * Pf;
  if (live) {
    const int64_t ec = cmap[e];
    for (int t = l; t < Pc3; t += 64) A[t] = (double)xc[(int64_t)idx_c[ec * Pc3 + t] * nc + comp];
  }
  __syncthreads();
  if (live)  // r1: B[k][j][i] = sum_a I[i][a] A[k][j][a]   (k, j < Pc; i < Pf)
    for (int t = l; t < Pc * Pc * Pf; t += 64) {
      const int i = t % Pf, kj = t / Pf;
      double v = 0.0;
      for (int a = 0; a < Pc; ++a) v += I[i * Pc + a] * A[kj * Pc + a];
      B[t] = v;
    }
  __syncthreads();
  if (live)  // r2: A[k][j][i] = sum_b I[j][b] B[k][b][i]   (k < Pc; j, i < Pf)
    for (int t = l; t < Pc * Pf2; t += 64) {
      const int i = t % Pf, j = (t / Pf) % Pf, k = t / Pf2;
      double v = 0.0;
      for (int b = 0; b < Pc; ++b) v += I[j * Pc + b] * B[(k * Pc + b) * Pf + i];
      A[t] = v;
    }
  __syncthreads();
  if (live)  // r3: y[k][j][i] = sum_c I[k][c] A[c][j][i], stored at the nodes this element owns
    for (int t = l; t < Pf3; t += 64) {
      const int ji = t % Pf2, k = t / Pf2;
      double v = 0.0;
      for (int c = 0; c < Pc; ++c) v += I[k * Pc + c] * A[c * Pf2 + ji];
      if ((own[e * Pf2 + ji] >> k) & 1) {
        const int32_t node = fine_node<AFF>(idx_f, aff, e, Pf, ji, k);
        yf[(int64_t)node * nc + comp] = (fm && !fm[node]) ? T(0) : (T)v;
      }
    }
}

template <bool AFF, typename T>
__global__ void __launch_bounds__(kTW * 64)
k_restrict_elem(int64_t E, int Pf, int Pc, const int32_t *__restrict__ cmap, const int32_t *__restrict__ idx_f,
                const int32_t *__restrict__ aff, const uint16_t *__restrict__ own, const double *__restrict__ I,
                int nc, const T *__restrict__ rf, const T *__restrict__ rb, const uint8_t *__restrict__ fmf,
                T *__restrict__ ec_out) {
  const int comp = blockIdx.y;
  extern __shared__ double smem[];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * kTW + w;
  const bool live = e < E;
  double *A = smem + w * (restrict_lds_a(Pf, Pc) + restrict_lds_b(Pf, Pc)), *B = A + restrict_lds_a(Pf, Pc);
  const int Pc2 = Pc * Pc, Pc3 = Pc2 * Pc, Pf2 = Pf * Pf, Pf3 = Pf2 * Pf;
  if (live)
    for (int t = l; t < Pf3; t += 64) {
      const int ji = t % Pf2, k = t / Pf2;
      double v = 0.0;
      if ((own[e * Pf2 + ji] >> k) & 1) {
        const int32_t node = fine_node<AFF>(idx_f, aff, e, Pf, ji, k);
        const int64_t g = (int64_t)node * nc + comp;
        // rb: restrict the masked residual rb - rf instead of rf
        v = rb ? (fmf[node] ? (double)rb[g] - (double)rf[g] : 0.0) : (double)rf[g];
      }
      A[t] = v;
    }
  __syncthreads();
  if (live)  // r3: B[c][j][i] = sum_k I[k][c] A[k][j][i]   (c < Pc; j, i < Pf)
    for (int t = l; t < Pc * Pf2; t += 64) {
      const int ji = t % Pf2, c = t / Pf2;
      double v = 0.0;
      for (int k = 0; k < Pf; ++k) v += I[k * Pc + c] * A[k * Pf2 + ji];
      B[t] = v;
    }
  __syncthreads();
  if (live)  // r2: A[c][b][i] = sum_j I[j][b] B[c][j][i]   (c, b < Pc; i < Pf)
    for (int t = l; t < Pc2 * Pf; t += 64) {
      const int i = t % Pf, b = (t / Pf) % Pc, c = t / (Pf * Pc);
      double v = 0.0;
      for (int j = 0; j < Pf; ++j) v += I[j * Pc + b] * B[(c * Pf + j) * Pf + i];
      A[t] = v;
    }
  __syncthreads();
  if (live) {  // r1: z[c][b][a] = sum_i I[i][a] A[c][b][i]
    const int64_t ec = cmap[e];
    for (int t = l; t < Pc3; t += 64) {
      const int a = t % Pc, cb = t / Pc;
      double v = 0.0;
      for (int i = 0; i < Pf; ++i) v += I[i * Pc + a] * A[cb * Pf + i];
      ec_out[(comp * E + ec) * Pc3 + t] = (T)v;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_restrict_sum(int64_t n, int nc, int64_t ev_stride, const int64_t *__restrict__ ptr, const int32_t *__restrict__ slot,
               const T *__restrict__ ev, const uint8_t *__restrict__ fm, T *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int c = 0; c < nc; ++c) {
      double v = 0.0;
      for (int64_t s = ptr[i]; s < ptr[i + 1]; ++s) v += (double)ev[c * ev_stride + slot[s]];
      y[i * nc + c] = (fm && !fm[i]) ? T(0) : (T)v;
    }
}

int64_t blocks_for(int64_t E) { return (E + kTW - 1) / kTW; }

}  // namespace

template <typename T>
hx_status launch_prolong(const hx_pmg_s &mg, int l, const T *xc, T *yf, const uint8_t *fm, hipStream_t s) {
  const auto &F = *mg.lv[l];
  const hx_mesh mf = F.op->mesh, mc = mg.lv[l + 1]->op->mesh;
  if (mf->nelem == 0) return HX_OK;
  const int nc = F.op->ncomp;
  const dim3 g((unsigned)blocks_for(mf->nelem), (unsigned)nc), b(kTW * 64);
  const size_t lds = sizeof(double) * kTW * (prolong_lds_a(mf->P, F.Pc) + prolong_lds_b(mf->P, F.Pc));
  if (mf->idx_affine.count)
    hipLaunchKernelGGL((k_prolong<true, T>), g, b, lds, s, mf->nelem, mf->P, F.Pc, F.cmap.ptr, mf->idx.ptr,
                       mf->idx_affine.ptr, mc->idx.ptr, mf->own.ptr, F.interp.ptr, fm, nc, xc, yf);
  else
    hipLaunchKernelGGL((k_prolong<false, T>), g, b, lds, s, mf->nelem, mf->P, F.Pc, F.cmap.ptr, mf->idx.ptr,
                       mf->idx_affine.ptr, mc->idx.ptr, mf->own.ptr, F.interp.ptr, fm, nc, xc, yf);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

template <typename T>
hx_status launch_restrict(const hx_pmg_s &mg, int l, const T *rf, T *yc, const uint8_t *fm, hipStream_t s,
                          const T *rb) {
  T *ev = reinterpret_cast<T *>(mg.lv[l]->ecoarse.ptr);  // FP64 storage, large enough for either type
  const int nc = mg.lv[l]->op->ncomp;
  const auto &F = *mg.lv[l];
  const hx_mesh mf = F.op->mesh, mc = mg.lv[l + 1]->op->mesh;
  if (mf->nelem > 0) {
    const dim3 g((unsigned)blocks_for(mf->nelem), (unsigned)nc), b(kTW * 64);
    const size_t lds = sizeof(double) * kTW * (restrict_lds_a(mf->P, F.Pc) + restrict_lds_b(mf->P, F.Pc));
    if (mf->idx_affine.count)
      hipLaunchKernelGGL((k_restrict_elem<true, T>), g, b, lds, s, mf->nelem, mf->P, F.Pc, F.cmap.ptr, mf->idx.ptr,
                         mf->idx_affine.ptr, mf->own.ptr, F.interp.ptr, nc, rf, rb, mf->freemask.ptr, ev);
    else
      hipLaunchKernelGGL((k_restrict_elem<false, T>), g, b, lds, s, mf->nelem, mf->P, F.Pc, F.cmap.ptr, mf->idx.ptr,
                         mf->idx_affine.ptr, mf->own.ptr, F.interp.ptr, nc, rf, rb, mf->freemask.ptr, ev);
  }
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((mc->nnodes + 255) / 256, 4096));
  hipLaunchKernelGGL((k_restrict_sum<T>), dim3(nb), dim3(256), 0, s, mc->nnodes, nc, mf->nelem * (int64_t)F.Pc * F.Pc * F.Pc,
                     F.csr_ptr.ptr, F.csr_slot.ptr, ev, fm, yc);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

template hx_status launch_prolong<double>(const hx_pmg_s &, int, const double *, double *, const uint8_t *, hipStream_t);
template hx_status launch_prolong<float>(const hx_pmg_s &, int, const float *, float *, const uint8_t *, hipStream_t);
template hx_status launch_restrict<double>(const hx_pmg_s &, int, const double *, double *, const uint8_t *, hipStream_t,
                                           const double *);
template hx_status launch_restrict<float>(const hx_pmg_s &, int, const float *, float *, const uint8_t *, hipStream_t,
                                          const float *);

}  // namespace hx

using namespace hx;

namespace {

// The transfer between fine level l and coarse level l + 1: element map, the coarse
// node -> E-vector slot lists and the 1D interpolation table.
hx_status build_transfer(hx_pmg_s::Level &F, const hx_pmg_s::Level &C) {
  const hx_mesh mf = F.op->mesh, mc = C.op->mesh;
  const int Pf = mf->P, Pc = mc->P;
  const int64_t E = mf->nelem;
  const int Pf3 = Pf * Pf * Pf, Pc3 = Pc * Pc * Pc;
  std::vector<int32_t> idf((size_t)E * Pf3), idc((size_t)E * Pc3);
  if (E > 0) {
    HX_HIP(hipMemcpy(idf.data(), mf->idx.ptr, sizeof(int32_t) * idf.size(), hipMemcpyDeviceToHost));
    HX_HIP(hipMemcpy(idc.data(), mc->idx.ptr, sizeof(int32_t) * idc.size(), hipMemcpyDeviceToHost));
  }
  // element correspondence through the caller's element ids
  std::vector<int32_t> inv_c(E), cmap(E);
  for (int64_t t = 0; t < E; ++t) inv_c[mc->order[t]] = (int32_t)t;
  for (int64_t t = 0; t < E; ++t) cmap[t] = inv_c[mf->order[t]];
  // same hexahedra in the same local orientation: the eight corners coincide
  double scale = 0.0;
  for (double v : mc->h_xyz) scale = std::max(scale, std::fabs(v));
  const double tol = 1e-10 * std::max(1.0, scale);
  for (int64_t t = 0; t < E; ++t)
    for (int c = 0; c < 8; ++c) {
      const int a = c & 1, b = (c >> 1) & 1, k = c >> 2;
      const int lf = (a + Pf * (b + Pf * k)) * (Pf - 1), lc = (a + Pc * (b + Pc * k)) * (Pc - 1);
      const int64_t nf = idf[(size_t)t * Pf3 + lf], nc = idc[(size_t)cmap[t] * Pc3 + lc];
      for (int d = 0; d < 3; ++d)
        if (std::fabs(mf->h_xyz[nf * 3 + d] - mc->h_xyz[nc * 3 + d]) > tol)
          return fail(HX_EINVAL, "p-multigrid levels do not share the element geometry (element " +
                                     std::to_string(mf->order[t]) + ", corner " + std::to_string(c) + ")");
    }
  // coarse node -> E-vector slots (coarse internal order), ascending
  std::vector<int64_t> ptr(mc->nnodes + 1, 0);
  for (int32_t g : idc) ++ptr[g + 1];
  for (int64_t i = 0; i < mc->nnodes; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> slot(idc.size());
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (size_t s = 0; s < idc.size(); ++s) slot[fill[idc[s]]++] = (int32_t)s;
  // I[i][a]: coarse Lagrange basis (GLL nodes of degree Pc - 1) at the fine GLL nodes
  std::vector<double> xf, wf, xc, wc, I, dI;
  gll_nodes_weights(Pf - 1, xf, wf);
  gll_nodes_weights(Pc - 1, xc, wc);
  lagrange_tables(xc, xf, I, dI);
  F.Pc = Pc;
  HX_HIP(F.interp.upload(I.data(), I.size()));
  HX_HIP(F.cmap.upload(cmap.data(), cmap.size()));
  HX_HIP(F.csr_ptr.upload(ptr.data(), ptr.size()));
  HX_HIP(F.csr_slot.upload(slot.data(), slot.size()));
  HX_HIP(F.ecoarse.alloc((size_t)E * Pc3 * F.op->ncomp));
  return HX_OK;
}

}  // namespace

extern "C" void hx_pmg_opts_default(hx_pmg_opts *o) {
  if (!o) return;
  o->smooth_degree = 3;
  o->smooth_ratio = 15.0;
  o->lanczos_steps = 20;
  o->coarse_maxit = 30;
  o->coarse_rtol = 0.1;
  o->prec = HX_FP64;
  o->smoother_mlp = nullptr;
  o->cycles = 1;
}

extern "C" hx_status hx_pmg_create(const hx_op *ops, int nlevels, const hx_pmg_opts *opts, hx_stream stream,
                                   hx_pmg *out) {
  if (!ops || !opts || !out) return fail(HX_EINVAL, "null argument");
  *out = nullptr;
  if (nlevels < 2 || nlevels > 8) return fail(HX_EINVAL, "nlevels must be in 2..8");
  const hx_pmg_opts &o = *opts;
  if (o.cycles < 1 || (o.cycles > 1 && o.prec != HX_FP64))
    return fail(HX_EINVAL, "cycles must be >= 1 (more than one cycle per application in FP64 hierarchies only)");
  if (o.smooth_degree < 1 || !(o.smooth_ratio > 1.0) || o.lanczos_steps < 2 || o.coarse_maxit < 1 ||
      !(o.coarse_rtol >= 0.0 && o.coarse_rtol < 1.0))
    return fail(HX_EINVAL, "need smooth_degree >= 1, smooth_ratio > 1, lanczos_steps >= 2, coarse_maxit >= 1, "
                           "0 <= coarse_rtol < 1");
  if (o.prec != HX_FP64 && o.prec != HX_FP32 && o.prec != HX_BF16 && o.prec != HX_BF16_SPLIT)
    return fail(HX_EINVAL, "prec must be HX_FP64, HX_FP32, HX_BF16 or HX_BF16_SPLIT");
  if ((o.prec == HX_BF16 || o.prec == HX_BF16_SPLIT) &&
      (ops[0]->kind != HX_DIFFUSION || ops[0]->ncomp != 1 || ops[0]->P > 8 || ops[0]->Q > 8))
    return fail(HX_EUNSUPPORTED, "bf16 p-multigrid needs a scalar diffusion finest level with p+1 <= 8 and q <= 8");
  for (int l = 0; l < nlevels; ++l) {
    if (!ops[l]) return fail(HX_EINVAL, "null operator in ops");
    if (ops[l]->ncomp != ops[0]->ncomp) return fail(HX_EINVAL, "the levels' operators differ in components");
    if (ops[l]->mesh->nuntouched > 0) return fail(HX_EINVAL, "p-multigrid needs every node in some element");
    if (l == 0) continue;
    // a low-order refined finest level sits on diffusion levels of the same coefficient
    const int kind0 = ops[0]->kind == HX_LOR ? HX_DIFFUSION : ops[0]->kind;
    if (ops[l]->kind != kind0) return fail(HX_EINVAL, "the levels' operators differ in kind");
    if (ops[l]->P >= ops[l - 1]->P) return fail(HX_EINVAL, "degrees must decrease strictly from level 0");
    if (ops[l]->mesh->nelem != ops[0]->mesh->nelem) return fail(HX_EINVAL, "the levels' meshes differ in elements");
    if (ops[l]->mesh->device != ops[0]->mesh->device) return fail(HX_EINVAL, "the levels are on different devices");
  }
  auto mg = std::make_unique<hx_pmg_s>();
  if (ops[0] && ops[0]->kind == HX_LOR && (o.prec != HX_FP64 || o.smoother_mlp))
    return fail(HX_EUNSUPPORTED, "a low-order refined finest level needs an FP64 hierarchy without a learned smoother");
  if (o.smoother_mlp) {
    if (o.prec != HX_FP64) return fail(HX_EUNSUPPORTED, "a learned smoother needs an FP64 hierarchy");
    if (ops[0]->kind != HX_DIFFUSION || ops[0]->ncomp != 1)
      return fail(HX_EUNSUPPORTED, "a learned smoother needs a scalar diffusion finest level");
    const int P3 = ops[0]->P * ops[0]->P * ops[0]->P;
    if (o.smoother_mlp->n_in != 2 * P3 || o.smoother_mlp->n_out != P3)
      return fail(HX_EINVAL, "the smoother network's shape does not match the finest level");
  }
  mg->opts = o;
  for (int l = 0; l < nlevels; ++l) {
    mg->lv.push_back(std::make_unique<hx_pmg_s::Level>());
    mg->lv[l]->op = ops[l];
    mg->lv[l]->n = ops[l]->mesh->nnodes * ops[l]->ncomp;
  }
  for (int l = 0; l + 1 < nlevels; ++l)
    if (hx_status st = build_transfer(*mg->lv[l], *mg->lv[l + 1])) return st;
  if (hx_status st = pmg_setup_levels(*mg, static_cast<hipStream_t>(stream))) return st;
  *out = mg.release();
  return HX_OK;
}

extern "C" int hx_pmg_levels(hx_pmg mg) { return mg ? (int)mg->lv.size() : 0; }

extern "C" hx_status hx_pmg_lambda_max(hx_pmg mg, int level, double *lam_max) {
  if (!mg || !lam_max) return fail(HX_EINVAL, "null argument");
  if (level < 0 || level >= (int)mg->lv.size()) return fail(HX_EINVAL, "level out of range");
  *lam_max = mg->lv[level]->lam_max;
  return HX_OK;
}

extern "C" hx_status hx_pmg_prolong(hx_pmg mg, int level, const double *x_coarse, double *y_fine, hx_stream s) {
  if (!mg || !x_coarse || !y_fine) return fail(HX_EINVAL, "null argument");
  if (level < 0 || level + 1 >= (int)mg->lv.size()) return fail(HX_EINVAL, "level out of range");
  return launch_prolong(*mg, level, x_coarse, y_fine, nullptr, static_cast<hipStream_t>(s));
}

extern "C" hx_status hx_pmg_restrict(hx_pmg mg, int level, const double *r_fine, double *y_coarse, hx_stream s) {
  if (!mg || !r_fine || !y_coarse) return fail(HX_EINVAL, "null argument");
  if (level < 0 || level + 1 >= (int)mg->lv.size()) return fail(HX_EINVAL, "level out of range");
  return launch_restrict<double>(*mg, level, r_fine, y_coarse, nullptr, static_cast<hipStream_t>(s), nullptr);
}

extern "C" void hx_pmg_destroy(hx_pmg mg) { delete mg; }
