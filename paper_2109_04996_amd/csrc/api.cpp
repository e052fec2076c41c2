// C ABI: error reporting, bases, operators and applies.
#include <cmath>
#include <cstring>
#include <string>

#include "hx_internal.h"

namespace hx {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }

hx_status fail(hx_status code, const std::string &msg) {
  g_err = msg;
  return code;
}

hx_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return e == hipErrorOutOfMemory ? HX_ENOMEM : HX_EHIP;
}

template <int P>
hx_status launch_apply_P(const hx_op_s &op, Prec prec, bool eout, const ApplyArgs &a, hipStream_t s);

hx_status launch_apply(const hx_op_s &op, Prec prec, bool out_elem, const ApplyArgs &a, hipStream_t s) {
  if (op.kind == HX_LOR) {
    if (prec != Prec::F64 || out_elem)
      return fail(HX_EUNSUPPORTED, "the low-order refined operator applies in FP64 to L-vectors only");
    return lor_apply(op, static_cast<const double *>(a.x), static_cast<double *>(a.y), s);
  }
  switch (op.P) {
    case 2: return launch_apply_P<2>(op, prec, out_elem, a, s);
    case 3: return launch_apply_P<3>(op, prec, out_elem, a, s);
    case 4: return launch_apply_P<4>(op, prec, out_elem, a, s);
    case 5: return launch_apply_P<5>(op, prec, out_elem, a, s);
    case 6: return launch_apply_P<6>(op, prec, out_elem, a, s);
    case 7: return launch_apply_P<7>(op, prec, out_elem, a, s);
    case 8: return launch_apply_P<8>(op, prec, out_elem, a, s);
    case 9: return launch_apply_P<9>(op, prec, out_elem, a, s);
  }
  return fail(HX_EUNSUPPORTED, "p out of range");
}

hx_status make_qdata32(hx_op_s &op, hipStream_t s);

}  // namespace hx

using namespace hx;

extern "C" const char *hx_last_error(void) { return g_err.c_str(); }

extern "C" const char *hx_version(void) { return "hexpa 0.1 (gfx950)"; }

// ------------------------------------------------------------------ bases
extern "C" hx_status hx_basis_create(int p, int q, int qrule, hx_basis *out) {
  if (!out) return fail(HX_EINVAL, "out is null");
  *out = nullptr;
  auto *b = new (std::nothrow) hx_basis_s();
  if (!b) return fail(HX_ENOMEM, "host allocation failed");
  std::string err;
  if (!make_basis(p, q, qrule, b->b, err)) {
    delete b;
    return fail(HX_EINVAL, err);
  }
  *out = b;
  return HX_OK;
}

extern "C" hx_status hx_basis_get_tables(hx_basis basis, double *nodes, double *qpts, double *qweights,
                                         double *interp, double *grad) {
  if (!basis) return fail(HX_EINVAL, "null basis");
  const Basis1D &b = basis->b;
  if (nodes) std::memcpy(nodes, b.nodes.data(), sizeof(double) * b.nodes.size());
  if (qpts) std::memcpy(qpts, b.qpts.data(), sizeof(double) * b.qpts.size());
  if (qweights) std::memcpy(qweights, b.qw.data(), sizeof(double) * b.qw.size());
  if (interp) std::memcpy(interp, b.interp.data(), sizeof(double) * b.interp.size());
  if (grad) std::memcpy(grad, b.grad.data(), sizeof(double) * b.grad.size());
  return HX_OK;
}

extern "C" void hx_basis_destroy(hx_basis basis) { delete basis; }

// ------------------------------------------------------------------ operators
namespace {

hx_status op_create(hx_mesh mesh, hx_basis basis, int kind, int ncomp, double alpha, double beta,
                    const hx_kappa_rff *kappa, hx_stream stream, hx_op *out) {
  if (!out) return fail(HX_EINVAL, "out is null");
  *out = nullptr;
  if (!mesh || !basis) return fail(HX_EINVAL, "null mesh or basis");
  if (mesh->host_only) return fail(HX_EINVAL, "the mesh is a host-only plan (hx_mesh_plan): create it with hx_mesh_create");
  if (ncomp != 1 && ncomp != 3) return fail(HX_EINVAL, "ncomp must be 1 or 3");
  if (basis->b.p != mesh->p) return fail(HX_EUNSUPPORTED, "basis degree differs from the mesh degree");
  if (kappa && kind == HX_MASS) return fail(HX_EINVAL, "a coefficient applies to HX_DIFFUSION only");
  if (kappa && (kappa->M < 0 || (kappa->M > 0 && (!kappa->omega || !kappa->phase))))
    return fail(HX_EINVAL, "kappa: M >= 0 and omega/phase non-null");
  if (kind == HX_MASS && basis->b.rule == HX_GLL && basis->b.q == basis->b.P) {
    // collocated mass is diagonal: handled by the interpolation kernel with an identity table
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  HX_HIP(hipGetDevice(&dev));
  if (dev != mesh->device) return fail(HX_EINVAL, "current device differs from the mesh's device");

  auto *op = new (std::nothrow) hx_op_s();
  if (!op) return fail(HX_ENOMEM, "host allocation failed");
  op->mesh = mesh;
  op->b = basis->b;
  op->kind = kind;
  op->ncomp = ncomp;
  op->P = op->b.P;
  op->Q = op->b.q;
  op->colloc = (kind != HX_MASS && op->b.rule == HX_GLL && op->Q == op->P);
  op->ncq = kind == HX_MASS ? 1 : 6;
  op->alpha = alpha;
  op->beta = beta;
  const int64_t Q3 = (int64_t)op->Q * op->Q * op->Q;

  // device tables: collocated D [P][P]; otherwise interp [Q][P] then the q-point derivative [Q][Q]
  std::vector<double> tab;
  if (op->colloc) {
    // D [P][P], then its even-odd coefficients E [h][h+odd], O [h][h], M [h] (odd P)
    tab = op->b.grad;
    const int P = op->P, h = P / 2, odd = P & 1, he = h + odd;
    const std::vector<double> &D = op->b.grad;
    std::vector<double> E(h * he), O(h * h), M(odd * h);
    for (int i = 0; i < h; ++i) {
      for (int l = 0; l < h; ++l) {
        E[i * he + l] = 0.5 * (D[i * P + l] + D[i * P + P - 1 - l]);
        O[i * h + l] = 0.5 * (D[i * P + l] - D[i * P + P - 1 - l]);
      }
      if (odd) E[i * he + h] = D[i * P + h];
    }
    for (int l = 0; l < odd * h; ++l) M[l] = D[h * P + l];
    tab.insert(tab.end(), E.begin(), E.end());
    tab.insert(tab.end(), O.begin(), O.end());
    tab.insert(tab.end(), M.begin(), M.end());
  } else {
    // interp [Q][P], the q-point derivative [Q][Q], then the even-odd coefficients of both: the
    // interpolation table is centro-symmetric (symmetric nodes and points), E [hq+oq][hp+op] and
    // O [hq][hp] (hp = P/2, op = P odd, likewise q); the derivative is centro-antisymmetric,
    // E [h][h+odd], O [h][h], M [h] (odd Q), h = Q/2, as for the collocated D above
    tab = op->b.interp;
    tab.insert(tab.end(), op->b.colloc.begin(), op->b.colloc.end());
    const int P = op->P, Q = op->Q, hp = P / 2, opd = P & 1, hq = Q / 2, oq = Q & 1;
    const std::vector<double> &B = op->b.interp;
    std::vector<double> EI((hq + oq) * (hp + opd)), OI(hq * hp);
    for (int q = 0; q < hq + oq; ++q) {
      for (int l = 0; l < hp; ++l) EI[q * (hp + opd) + l] = 0.5 * (B[q * P + l] + B[q * P + P - 1 - l]);
      if (opd) EI[q * (hp + opd) + hp] = B[q * P + hp];
    }
    for (int q = 0; q < hq; ++q)
      for (int l = 0; l < hp; ++l) OI[q * hp + l] = 0.5 * (B[q * P + l] - B[q * P + P - 1 - l]);
    tab.insert(tab.end(), EI.begin(), EI.end());
    tab.insert(tab.end(), OI.begin(), OI.end());
    const std::vector<double> &D = op->b.colloc;
    const int h = hq, odd = oq, he = h + odd;
    std::vector<double> E(h * he), O(h * h), M(odd * h);
    for (int i = 0; i < h; ++i) {
      for (int l = 0; l < h; ++l) {
        E[i * he + l] = 0.5 * (D[i * Q + l] + D[i * Q + Q - 1 - l]);
        O[i * h + l] = 0.5 * (D[i * Q + l] - D[i * Q + Q - 1 - l]);
      }
      if (odd) E[i * he + h] = D[i * Q + h];
    }
    for (int l = 0; l < odd * h; ++l) M[l] = D[h * Q + l];
    tab.insert(tab.end(), E.begin(), E.end());
    tab.insert(tab.end(), O.begin(), O.end());
    tab.insert(tab.end(), M.begin(), M.end());
  }
  std::vector<float> tab32(tab.begin(), tab.end());
  hipError_t e;
  if ((e = op->tab.upload(tab.data(), tab.size())) != hipSuccess ||
      (e = op->tab32.upload(tab32.data(), tab32.size())) != hipSuccess ||
      (e = op->qdata.alloc((size_t)mesh->nelem * op->ncq * Q3)) != hipSuccess ||
      (kind == HX_HELMHOLTZ && (e = op->qmass.alloc((size_t)mesh->nelem * Q3)) != hipSuccess)) {
    delete op;
    return hip_fail(e, "operator allocation");
  }
  if (kappa && kappa->M > 0) {
    op->kappa_M = kappa->M;
    op->kappa_omega.assign(kappa->omega, kappa->omega + 3 * kappa->M);
    op->kappa_phase.assign(kappa->phase, kappa->phase + kappa->M);
    op->kappa_scale = kappa->scale;
    op->kappa_shift = kappa->shift;
  }
  int bad = 0;
  if (hx_status st = launch_setup_qdata(*op, kappa, s, &bad)) {
    delete op;
    return st;
  }
  if (bad) {
    delete op;
    return fail(HX_EGEOM, "non-positive Jacobian determinant at a quadrature point");
  }
  *out = op;
  return HX_OK;
}

}  // namespace

extern "C" hx_status hx_op_create(hx_mesh mesh, hx_basis basis, int kind, int ncomp, const hx_kappa_rff *kappa,
                                  hx_stream stream, hx_op *out) {
  if (kind != HX_MASS && kind != HX_DIFFUSION) {
    if (out) *out = nullptr;
    return fail(HX_EINVAL, "kind must be HX_MASS or HX_DIFFUSION (hx_op_create_helmholtz makes HX_HELMHOLTZ)");
  }
  return op_create(mesh, basis, kind, ncomp, 1.0, 0.0, kappa, stream, out);
}

extern "C" hx_status hx_op_create_helmholtz(hx_mesh mesh, hx_basis basis, int ncomp, double alpha, double beta,
                                            const hx_kappa_rff *kappa, hx_stream stream, hx_op *out) {
  if (!(std::isfinite(alpha) && std::isfinite(beta) && alpha >= 0.0 && beta >= 0.0 && alpha + beta > 0.0)) {
    if (out) *out = nullptr;
    return fail(HX_EINVAL, "alpha and beta must be finite, >= 0 and not both 0");
  }
  return op_create(mesh, basis, HX_HELMHOLTZ, ncomp, alpha, beta, kappa, stream, out);
}

extern "C" hx_status hx_op_apply(hx_op op, const double *x, double *y, hx_stream s) {
  if (!op || !x || !y) return fail(HX_EINVAL, "null argument");
  hipStream_t st = static_cast<hipStream_t>(s);
  if (op->mesh->nuntouched > 0) HX_HIP(hipMemsetAsync(y, 0, sizeof(double) * op->mesh->nnodes * op->ncomp, st));
  ApplyArgs a{op->mesh->idx.ptr, op->mesh->own.ptr, nullptr, nullptr, nullptr, x, y, nullptr, 0, 0, op->mesh->nnodes};
  return launch_apply(*op, Prec::F64, false, a, st);
}

extern "C" hx_status hx_op_apply_f32(hx_op op, int qdata_prec, const float *x, float *y, hx_stream s) {
  if (!op || !x || !y) return fail(HX_EINVAL, "null argument");
  if (qdata_prec != HX_FP64 && qdata_prec != HX_FP32) return fail(HX_EINVAL, "qdata_prec must be HX_FP64 or HX_FP32");
  if (op->kind == HX_LOR) return fail(HX_EUNSUPPORTED, "the low-order refined operator applies in FP64 only");
  hipStream_t st = static_cast<hipStream_t>(s);
  if (qdata_prec == HX_FP32)
    if (hx_status e = make_qdata32(*op, st)) return e;
  if (op->mesh->nuntouched > 0) HX_HIP(hipMemsetAsync(y, 0, sizeof(float) * op->mesh->nnodes * op->ncomp, st));
  ApplyArgs a{op->mesh->idx.ptr, op->mesh->own.ptr, nullptr, nullptr, nullptr, x, y, nullptr, 0, 0, op->mesh->nnodes};
  return launch_apply(*op, qdata_prec == HX_FP32 ? Prec::F32_Q32 : Prec::F32_Q64, false, a, st);
}

extern "C" hx_status hx_op_apply_bf16(hx_op op, int prec, const float *x, float *y, hx_stream s) {
  if (!op || !x || !y) return fail(HX_EINVAL, "null argument");
  if (prec != HX_BF16 && prec != HX_BF16_SPLIT) return fail(HX_EINVAL, "prec must be HX_BF16 or HX_BF16_SPLIT");
  if (op->kind != HX_DIFFUSION || op->ncomp != 1) return fail(HX_EUNSUPPORTED, "the bf16 operator supports scalar diffusion only");
  return launch_apply_bf16(*op, prec == HX_BF16_SPLIT, x, y, static_cast<hipStream_t>(s));
}

extern "C" hx_status hx_op_apply_elem(hx_op op, const double *x, double *y_e, hx_stream s) {
  if (!op || !x || !y_e) return fail(HX_EINVAL, "null argument");
  ApplyArgs a{op->mesh->idx.ptr, op->mesh->own.ptr, nullptr, nullptr, nullptr, x, y_e, op->mesh->order_d.ptr, 0, 0,
              op->mesh->nnodes};
  return launch_apply(*op, Prec::F64, true, a, static_cast<hipStream_t>(s));
}

extern "C" hx_status hx_op_diagonal(hx_op op, double *diag, hx_stream s) {
  if (!op || !diag) return fail(HX_EINVAL, "null argument");
  return launch_diagonal(*op, diag, static_cast<hipStream_t>(s));
}

extern "C" hx_status hx_op_get_stats(hx_op op, hx_op_stats *st) {
  if (!op || !st) return fail(HX_EINVAL, "null argument");
  st->p = op->b.p;
  st->q = op->Q;
  st->qrule = op->b.rule;
  st->kind = op->kind;
  st->ncomp = op->ncomp;
  st->nnodes = op->mesh->nnodes;
  st->nelem = op->mesh->nelem;
  st->qdata_bytes = (int64_t)op->qdata.count * 8;
  st->index_bytes = (int64_t)op->mesh->idx.count * 4;
  return HX_OK;
}

extern "C" void hx_op_destroy(hx_op op) { delete op; }
