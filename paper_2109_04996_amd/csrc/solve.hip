// Preconditioned conjugate gradients on the GPU.
//
// Benchmarks section: the bake-off problems are CG solves of the Dirichlet
// problem; CG mixes the local operator work with global reductions (two dot
// products per iteration). Miniapps section (Nekbone): CG with a diagonal
// preconditioner. Here the scalars alpha, beta, r'z, p'Ap stay in device
// memory: every iteration is a fixed sequence of kernels on the caller's
// stream, and the host reads a few bytes every check_every iterations.
//
// Reductions are deterministic: each block sums a fixed contiguous slice in a
// fixed order (wavefront shuffles, then LDS), then one block adds the block
// sums in index order. Products of FP32 vectors are accumulated in FP64.
//
// Not in the paper: the Chebyshev polynomial preconditioner (textbook
// Chebyshev acceleration of D^-1 A, degree k, k-1 operator applies), the
// Lanczos estimate of lambda_max(D^-1 A) from CG coefficients, and mixed
// precision iterative refinement (FP64 residual and update, FP32 inner PCG).
#include <chrono>
#include <cmath>
#include <functional>
#include <mutex>
#include <random>
#include <type_traits>

#include "mlp_internal.h"

extern "C" hx_status hx_op_diagonal(hx_op op, double *diag, hx_stream s);

namespace hx {

hx_status make_qdata32(hx_op_s &op, hipStream_t s);

namespace {

constexpr int kVecThreads = 256;
constexpr int kVecBlocks = 1024;

enum { S_RZ = 0, S_PAP, S_ALPHA, S_RZNEW, S_BETA, S_RR, S_FLAG, S_BB, S_TMP, S_RZPREV, S_NSCAL = 16 };
enum { FIN_SUM = 0, FIN_PAP, FIN_RZ_RR, FIN_RZ, FIN_FLEX };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum in a fixed order, result on every thread
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[kVecThreads / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kVecThreads / 64; ++w) s += sh[w];
  return s;
}

// contiguous slice of [0, n) for this block: a deterministic partition
__device__ __forceinline__ void slice(int64_t n, int64_t &lo, int64_t &hi) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  lo = min(n, (int64_t)blockIdx.x * per);
  hi = min(n, lo + per);
}

template <int NC>
__device__ __forceinline__ bool is_free(const uint8_t *fm, int64_t t) {
  return fm[NC == 1 ? t : t / NC] != 0;
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_dot(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
                                                       double *__restrict__ part) {
  int64_t lo, hi;
  slice(n, lo, hi);
  double s = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) s += (double)a[t] * (double)b[t];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sum_t r_t z_t and sum_t (r_t - rp_t) z_t (flexible CG)
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_dot_flex(int64_t n, const T *__restrict__ r, const T *__restrict__ rp,
                                                            const T *__restrict__ z, double *__restrict__ part0,
                                                            double *__restrict__ part2) {
  int64_t lo, hi;
  slice(n, lo, hi);
  double s0 = 0.0, s2 = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const double zz = (double)z[t];
    s0 += (double)r[t] * zz;
    s2 += ((double)r[t] - (double)rp[t]) * zz;
  }
  s0 = block_sum(s0);
  s2 = block_sum(s2);
  if (threadIdx.x == 0) {
    part0[blockIdx.x] = s0;
    part2[blockIdx.x] = s2;
  }
}

// one block: reduce the partials (p1 optional) and derive the CG scalars
__global__ void __launch_bounds__(kVecThreads) k_final(const double *__restrict__ p0, const double *__restrict__ p1,
                                                         int nb, double *__restrict__ S, int what, int slot) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    a += p0[i];
    if (p1) b += p1[i];
  }
  a = block_sum(a);
  if (p1) b = block_sum(b);
  if (threadIdx.x != 0) return;
  switch (what) {
    case FIN_SUM:
      S[slot] = a;
      break;
    case FIN_PAP: {
      S[S_PAP] = a;
      const bool ok = a > 0.0 && isfinite(a);
      S[S_ALPHA] = ok ? S[S_RZ] / a : 0.0;
      if (!ok) S[S_FLAG] = 1.0;
      break;
    }
    case FIN_RZ_RR: {  // a = r'z of the new residual, b = r'r
      const double rz_old = S[S_RZ];
      S[S_RZNEW] = a;
      S[S_RR] = b;
      S[S_BETA] = (rz_old != 0.0) ? a / rz_old : 0.0;
      S[S_RZ] = a;
      if (!(a > 0.0) && b > 0.0) S[S_FLAG] = 2.0;
      if (!isfinite(a) || !isfinite(b)) S[S_FLAG] = 3.0;
      break;
    }
    case FIN_FLEX: {  // flexible CG: a = r'z, b = (r - r_prev)'z; beta = b / r'z of the previous step
      const double rz_old = S[S_RZ];
      S[S_RZNEW] = a;
      S[S_BETA] = (rz_old != 0.0) ? b / rz_old : 0.0;
      S[S_RZ] = a;
      if (!(a > 0.0) && S[S_RR] > 0.0) S[S_FLAG] = 2.0;
      if (!isfinite(a) || !isfinite(b)) S[S_FLAG] = 3.0;
      break;
    }
    case FIN_RZ:
      S[S_RZ] = a;
      if (!(a > 0.0) && S[S_RR] > 0.0) S[S_FLAG] = 2.0;
      if (!isfinite(a)) S[S_FLAG] = 3.0;
      break;
  }
}

// r = m (scale * b - w), partial r'r; w may be null
template <typename T, typename TB, int NC>
__global__ void __launch_bounds__(kVecThreads)
    k_resid(int64_t n, double scale, const TB *__restrict__ b, const double *__restrict__ w,
            const uint8_t *__restrict__ fm, T *__restrict__ r, double *__restrict__ part_rr) {
  int64_t lo, hi;
  slice(n, lo, hi);
  double s = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const double v = is_free<NC>(fm, t) ? scale * (double)b[t] - (w ? w[t] : 0.0) : 0.0;
    const T rv = (T)v;
    r[t] = rv;
    s += (double)rv * (double)rv;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// z = dinv r, partial r'z (dinv is 0 on constrained nodes)
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_jacobi(int64_t n, const T *__restrict__ dinv, const T *__restrict__ r,
                                                          T *__restrict__ z, double *__restrict__ part_rz) {
  int64_t lo, hi;
  slice(n, lo, hi);
  double s = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const T zv = dinv[t] * r[t];
    z[t] = zv;
    s += (double)r[t] * (double)zv;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = s;
}

// x += alpha p; r -= alpha m w; with JAC also z = dinv r; partials r'z (JAC) and r'r; rp (if given) = old r
template <typename T, int NC, bool JAC>
__global__ void __launch_bounds__(kVecThreads)
    k_update(int64_t n, const double *__restrict__ S, T *__restrict__ x, const T *__restrict__ p, T *__restrict__ r,
             const T *__restrict__ w, const uint8_t *__restrict__ fm, const T *__restrict__ dinv, T *__restrict__ z,
             double *__restrict__ part_rz, double *__restrict__ part_rr, T *__restrict__ rp) {
  const T alpha = (T)S[S_ALPHA];
  int64_t lo, hi;
  slice(n, lo, hi);
  double srz = 0.0, srr = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    x[t] += alpha * p[t];
    if (rp) rp[t] = r[t];
    const T rv = is_free<NC>(fm, t) ? r[t] - alpha * w[t] : T(0);
    r[t] = rv;
    srr += (double)rv * (double)rv;
    if constexpr (JAC) {
      const T zv = dinv[t] * rv;
      z[t] = zv;
      srz += (double)rv * (double)zv;
    }
  }
  srr = block_sum(srr);
  if constexpr (JAC) srz = block_sum(srz);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = srr;
    if constexpr (JAC) part_rz[blockIdx.x] = srz;
  }
}

// Sum of nb block partials in a fixed order, on every thread: the order of k_final, so every block of a
// kernel that reduces the partials itself gets the bits k_final would have written.
__device__ __forceinline__ double reduce_partials(const double *__restrict__ p, int nb) {
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) a += p[i];
  return block_sum(a);
}

// The update of a PCG iteration with the step length reduced in place: every block sums the p'Ap
// partials (part_pap, written by the dot kernel before it) itself, alpha = r'z / p'Ap, and block 0
// keeps the scalars for the host's checks (p'Ap, alpha, and r'z of this step for the next kernel's beta).
// Then as k_update: x += alpha p; r -= alpha m w; with JAC z = dinv r; partials r'z (JAC) and r'r;
// rp (if given) = old r.
template <typename T, int NC, bool JAC>
__global__ void __launch_bounds__(kVecThreads)
    k_update_red(int64_t n, double *__restrict__ S, const double *__restrict__ part_pap, int nb, T *__restrict__ x,
                 const T *__restrict__ p, T *__restrict__ r, const T *__restrict__ w, const uint8_t *__restrict__ fm,
                 const T *__restrict__ dinv, T *__restrict__ z, double *__restrict__ part_rz,
                 double *__restrict__ part_rr, T *__restrict__ rp) {
  const double pap = reduce_partials(part_pap, nb);
  const bool ok = pap > 0.0 && isfinite(pap);
  const double rz = S[S_RZ];
  const double alpha_d = ok ? rz / pap : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S[S_PAP] = pap;
    S[S_ALPHA] = alpha_d;
    S[S_RZPREV] = rz;
    if (!ok) S[S_FLAG] = 1.0;
  }
  const T alpha = (T)alpha_d;
  int64_t lo, hi;
  slice(n, lo, hi);
  double srz = 0.0, srr = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    x[t] += alpha * p[t];
    if (rp) rp[t] = r[t];
    const T rv = is_free<NC>(fm, t) ? r[t] - alpha * w[t] : T(0);
    r[t] = rv;
    srr += (double)rv * (double)rv;
    if constexpr (JAC) {
      const T zv = dinv[t] * rv;
      z[t] = zv;
      srz += (double)rv * (double)zv;
    }
  }
  srr = block_sum(srr);
  if constexpr (JAC) srz = block_sum(srz);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = srr;
    if constexpr (JAC) part_rz[blockIdx.x] = srz;
  }
}

// p = z + beta p with beta reduced in place: every block sums the r'z partials (part_rz) and, for flexible
// CG, the (r - r_prev)'z partials (part_flex); beta = r'z / r'z_prev (or (r - r_prev)'z / r'z_prev). Block 0
// keeps r'z, r'r (part_rr) and beta for the host's checks and raises the breakdown flags as k_final does.
template <typename T, bool FLEX>
__global__ void __launch_bounds__(kVecThreads)
    k_pupd_red(int64_t n, double *__restrict__ S, const double *__restrict__ part_rz,
               const double *__restrict__ part_rr, const double *__restrict__ part_flex, int nb,
               const T *__restrict__ z, T *__restrict__ p) {
  const double rz = reduce_partials(part_rz, nb);
  const double rr = reduce_partials(part_rr, nb);
  const double num = FLEX ? reduce_partials(part_flex, nb) : rz;
  const double rz_old = S[S_RZPREV];
  const double beta_d = (rz_old != 0.0) ? num / rz_old : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S[S_RR] = rr;
    S[S_RZNEW] = rz;
    S[S_BETA] = beta_d;
    S[S_RZ] = rz;
    if (!(rz > 0.0) && rr > 0.0) S[S_FLAG] = 2.0;
    if (FLEX ? (!isfinite(rz) || !isfinite(num)) : (!isfinite(rz) || !isfinite(rr))) S[S_FLAG] = 3.0;
  }
  const T beta = (T)beta_d;
  int64_t lo, hi;
  slice(n, lo, hi);
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) p[t] = z[t] + beta * p[t];
}

// Node gather of an E-vector (the transpose of the element restriction): w[t] = sum of the node's slots in
// ascending order (component c of slot e*P3 + l sits at (e*NC + c)*P3 + l), fused with the partial sums of
// p'w over the same deterministic slices as k_dot.
template <int NC>
__global__ void __launch_bounds__(kVecThreads)
    k_gather_dot(int64_t n, int P3, const int32_t *__restrict__ gptr, const int32_t *__restrict__ gslot,
                 const double *__restrict__ ye, const double *__restrict__ p, double *__restrict__ w,
                 double *__restrict__ part) {
  int64_t lo, hi;
  slice(n, lo, hi);
  double s = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const int64_t nd = NC == 1 ? t : t / NC;
    const int c = NC == 1 ? 0 : (int)(t - nd * NC);
    double v = 0.0;
    for (int32_t k = gptr[nd]; k < gptr[nd + 1]; ++k) {
      const int32_t sl = gslot[k];
      v += NC == 1 ? ye[sl] : ye[((int64_t)(sl / P3) * NC + c) * P3 + sl % P3];
    }
    w[t] = v;
    s += p[t] * v;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_pupd(int64_t n, const double *__restrict__ S, const T *__restrict__ z,
                                                        T *__restrict__ p) {
  const T beta = (T)S[S_BETA];
  int64_t lo, hi;
  slice(n, lo, hi);
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) p[t] = z[t] + beta * p[t];
}

// Chebyshev first step: d = dinv r / theta, z = d
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_cheb0(int64_t n, T inv_theta, const T *__restrict__ dinv,
                                                         const T *__restrict__ r, T *__restrict__ d,
                                                         T *__restrict__ z) {
  int64_t lo, hi;
  slice(n, lo, hi);
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const T v = inv_theta * dinv[t] * r[t];
    d[t] = v;
    z[t] = v;
  }
}

// Chebyshev step: d = c1 d + c2 dinv (r - A z), z += d
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_cheb(int64_t n, T c1, T c2, const T *__restrict__ dinv,
                                                        const T *__restrict__ r, const T *__restrict__ az,
                                                        T *__restrict__ d, T *__restrict__ z) {
  int64_t lo, hi;
  slice(n, lo, hi);
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const T v = c1 * d[t] + c2 * dinv[t] * (r[t] - az[t]);
    d[t] = v;
    z[t] += v;
  }
}

// first Chebyshev step from a nonzero iterate: d = c2 dinv (r - A z), z += d
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_cheb_first(int64_t n, T c2, const T *__restrict__ dinv,
                                                              const T *__restrict__ r, const T *__restrict__ az,
                                                              T *__restrict__ d, T *__restrict__ z) {
  int64_t lo, hi;
  slice(n, lo, hi);
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const T v = c2 * dinv[t] * (r[t] - az[t]);
    d[t] = v;
    z[t] += v;
  }
}

// dinv = m / diag, or m alone when diag is null (no preconditioner)
template <typename T, int NC>
__global__ void __launch_bounds__(kVecThreads) k_dinv(int64_t n, const double *__restrict__ diag,
                                                        const uint8_t *__restrict__ fm, T *__restrict__ dinv) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dinv[t] = is_free<NC>(fm, t) ? (diag ? (T)(1.0 / diag[t]) : T(1)) : T(0);
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(kVecThreads) k_convert(int64_t n, double scale, const TA *__restrict__ a,
                                                           TB *__restrict__ b) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = (TB)(scale * (double)a[t]);
}

// w = m (r - w): masked residual, in place over w = A z (nc interleaved components share a node's mask)
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_mresid(int64_t n, int nc, const T *__restrict__ r,
                                                          const uint8_t *__restrict__ fm, T *__restrict__ w) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = fm[nc == 1 ? i : i / nc] ? r[i] - w[i] : T(0);
}

// Chebyshev step with a general base map: d = a d + b m, z += d (k == 0: d = b m, z = d)
__global__ void __launch_bounds__(kVecThreads) k_cheb_m(int64_t n, double a, double b, const double *__restrict__ m,
                                                          double *__restrict__ d, double *__restrict__ z, int first) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (first) {
      const double v = b * m[i];
      d[i] = v;
      z[i] = v;
    } else {
      const double v = a * d[i] + b * m[i];
      d[i] = v;
      z[i] += v;
    }
  }
}

// x += scale * d (FP64 x)
template <typename TD>
__global__ void __launch_bounds__(kVecThreads) k_axpy(int64_t n, double scale, const TD *__restrict__ d,
                                                        double *__restrict__ x) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    x[t] += scale * (double)d[t];
}

template <int NC>
__global__ void __launch_bounds__(kVecThreads) k_maskset(int64_t n, const uint8_t *__restrict__ fm, double *__restrict__ x) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    if (!is_free<NC>(fm, t)) x[t] = 0.0;
}

// largest eigenvalue of a symmetric tridiagonal matrix (diagonal d, off-diagonal e) by Sturm bisection
double tridiag_max_eig(const std::vector<double> &d, const std::vector<double> &e) {
  const int n = (int)d.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
      q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-14 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= n) hi = mid;
    else lo = mid;
  }
  return hi;
}

template <typename T>
struct Vecs {
  T *r, *z, *p, *w, *dinv, *cd, *ct, *x, *rp, *m;
};

struct Ctx {
  hx_op_s &op;
  hipStream_t s;
  int64_t n;
  int nc;
  double *part0, *part1, *S, *part2;
  double *hS;  // pinned host copy of S
  int applies = 0;
  bool graph = false;   // replay PCG iterations as a captured graph
  bool gather = false;  // FP64 CG operator as an E-vector apply plus a node gather (HX_SCATTER_GATHER)
};

// Synchronises a stream when the scope ends (the solve is synchronous on every return path).
struct StreamSync {
  hipStream_t s = nullptr;
  ~StreamSync() {
    if (s) (void)hipStreamSynchronize(s);
  }
};

#define LAUNCH_V(kern, ...) hipLaunchKernelGGL(kern, dim3(kVecBlocks), dim3(kVecThreads), 0, c.s, __VA_ARGS__)
#define FINAL(p0, p1, what, slot) \
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kVecThreads), 0, c.s, p0, p1, kVecBlocks, c.S, (int)(what), (int)(slot))

hx_status apply_T(Ctx &c, const double *x, double *y, int) {
  ApplyArgs a{c.op.mesh->idx.ptr, c.op.mesh->own.ptr, nullptr, nullptr, nullptr, x, y, nullptr, 0, 0,
              c.op.mesh->nnodes};
  if (c.op.mesh->nuntouched > 0) HX_HIP(hipMemsetAsync(y, 0, sizeof(double) * c.n, c.s));
  ++c.applies;
  return launch_apply(c.op, Prec::F64, false, a, c.s);
}

// prec: HX_FP64 (FP64 qdata), HX_FP32 (FP32 qdata), HX_BF16 / HX_BF16_SPLIT (matrix-core operator)
hx_status apply_T(Ctx &c, const float *x, float *y, int prec) {
  ++c.applies;
  if (prec == HX_BF16 || prec == HX_BF16_SPLIT) return launch_apply_bf16(c.op, prec == HX_BF16_SPLIT, x, y, c.s);
  ApplyArgs a{c.op.mesh->idx.ptr, c.op.mesh->own.ptr, nullptr, nullptr, nullptr, x, y, nullptr, 0, 0,
              c.op.mesh->nnodes};
  if (c.op.mesh->nuntouched > 0) HX_HIP(hipMemsetAsync(y, 0, sizeof(float) * c.n, c.s));
  return launch_apply(c.op, prec == HX_FP32 ? Prec::F32_Q32 : Prec::F32_Q64, false, a, c.s);
}

hx_status read_scalars(Ctx &c) {
  HX_HIP(hipMemcpyAsync(c.hS, c.S, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, c.s));
  HX_HIP(hipStreamSynchronize(c.s));
  return HX_OK;
}

struct Cheb {
  int degree = 4;
  double lam_lo = 0, lam_hi = 0;
};

// z = s(D^-1 A) D^-1 r: degree steps from z = 0, degree-1 operator applies
template <typename T>
hx_status cheb_apply(Ctx &c, const Cheb &ch, const Vecs<T> &v, const T *r, T *z, int op_prec) {
  const double theta = 0.5 * (ch.lam_hi + ch.lam_lo), delta = 0.5 * (ch.lam_hi - ch.lam_lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  LAUNCH_V((k_cheb0<T>), c.n, (T)(1.0 / theta), v.dinv, r, v.cd, z);
  for (int k = 1; k < ch.degree; ++k) {
    if (hx_status st = apply_T(c, z, v.ct, op_prec)) return st;
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    LAUNCH_V((k_cheb<T>), c.n, (T)(rho_new * rho), (T)(2.0 * rho_new / delta), v.dinv, r, v.ct, v.cd, z);
    rho = rho_new;
  }
  HX_HIP(hipGetLastError());
  return HX_OK;
}

// The same polynomial on the error equation from the iterate already in z: z += s(D^-1 A) D^-1 (r - A z),
// degree steps and degree operator applies (the first one forms the residual). Uses v.cd and v.ct.
template <typename T>
hx_status cheb_apply_from(Ctx &c, const Cheb &ch, const Vecs<T> &v, const T *r, T *z, int op_prec) {
  const double theta = 0.5 * (ch.lam_hi + ch.lam_lo), delta = 0.5 * (ch.lam_hi - ch.lam_lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  for (int k = 0; k < ch.degree; ++k) {
    if (hx_status st = apply_T(c, z, v.ct, op_prec)) return st;
    if (k == 0) {
      LAUNCH_V((k_cheb_first<T>), c.n, (T)(1.0 / theta), v.dinv, r, v.ct, v.cd, z);
    } else {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      LAUNCH_V((k_cheb<T>), c.n, (T)(rho_new * rho), (T)(2.0 * rho_new / delta), v.dinv, r, v.ct, v.cd, z);
      rho = rho_new;
    }
  }
  HX_HIP(hipGetLastError());
  return HX_OK;
}

// Preconditioner that is not fused into the update: computes z from r, then the partial r'z into part0.
template <typename T>
using PrecFn = std::function<hx_status(const T *r, T *z)>;

// Chebyshev steps on M A e = M r from e = 0 with a general base map M in place of D^-1 (the same
// recurrence as cheb_apply): z = s(M A) M r. Uses v.cd (d), v.ct (A z, then the masked residual)
// and v.m (M of it); the FP64 operator.
hx_status cheb_apply_base(Ctx &c, const Cheb &ch, const Vecs<double> &v, const PrecFn<double> &base, const double *r,
                          double *z) {
  const double theta = 0.5 * (ch.lam_hi + ch.lam_lo), delta = 0.5 * (ch.lam_hi - ch.lam_lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (hx_status st = base(r, v.m)) return st;
  LAUNCH_V(k_cheb_m, c.n, 0.0, 1.0 / theta, v.m, v.cd, z, 1);
  for (int k = 1; k < ch.degree; ++k) {
    if (hx_status st = apply_T(c, z, v.ct, HX_FP64)) return st;
    LAUNCH_V((k_mresid<double>), c.n, 1, r, c.op.mesh->freemask.ptr, v.ct);
    if (hx_status st = base(v.ct, v.m)) return st;
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    LAUNCH_V(k_cheb_m, c.n, rho_new * rho, 2.0 * rho_new / delta, v.m, v.cd, z, 0);
    rho = rho_new;
  }
  HX_HIP(hipGetLastError());
  return HX_OK;
}

// PCG on vectors of type T. On entry v.r holds the masked right-hand side with r'r = rr0; solves for v.x
// from 0. Jacobi (and none, with dinv = mask) is fused into the update kernel; other preconditioners
// go through pc. Stops when r'r <= stop2, at maxit, or on breakdown.
constexpr hx_status kStalled = -100;  // internal: the residual stopped falling (learned preconditioner)

// Called at every host check with the recurrence r'r; may replace the residual (and r'z on the device)
// and returns the r'r the loop goes on with.
using CheckFn = std::function<hx_status(double rr, double *rr_next)>;

template <typename T>
hx_status pcg_core(Ctx &c, const Vecs<T> &v, const PrecFn<T> *pc, int op_prec, double rr0, double stop2, int maxit,
                   int check_every, bool flexible, int *iters, double *rr_out, int stall_window = 0,
                   double stall_factor = 0.0, const CheckFn *on_check = nullptr) {
  std::vector<std::pair<int, double>> hist;  // (iteration, r'r) at the host checks (stall check only)
  if (stall_window > 0) hist.emplace_back(0, rr0);
  HX_HIP(hipMemsetAsync(v.x, 0, sizeof(T) * c.n, c.s));
  HX_HIP(hipMemsetAsync(c.S, 0, sizeof(double) * S_NSCAL, c.s));
  flexible = flexible && pc;  // Jacobi is linear and symmetric: plain CG
  if (!pc) {
    LAUNCH_V((k_jacobi<T>), c.n, v.dinv, v.r, v.z, c.part0);
  } else {
    if (hx_status st = (*pc)(v.r, v.z)) return st;
    LAUNCH_V((k_dot<T>), c.n, v.r, v.z, c.part0);
  }
  FINAL(c.part0, (const double *)nullptr, FIN_RZ, 0);
  HX_HIP(hipMemcpyAsync(v.p, v.z, sizeof(T) * c.n, hipMemcpyDeviceToDevice, c.s));
  int it = 0;
  double rr = rr0;
  T *rp = flexible ? v.rp : nullptr;
  // one iteration: kernels only, every scalar device-resident (no host work between them)
  // The scalars are reduced where they are used: the update kernel sums the p'Ap partials itself and
  // the direction update the r'z (and r'r) partials, each block in the fixed order of k_final, so there
  // is no single-block finishing kernel between them and the results are those of that sequence, bit
  // for bit. Partials: p'Ap in part2; r'z in part0, r'r in part1, (r - r_prev)'z in part2 (flexible CG,
  // after the update has read the p'Ap partials).
  auto iteration = [&]() -> hx_status {
    bool dot_done = false;
    if constexpr (std::is_same<T, double>::value) {
      if (c.gather && op_prec == HX_FP64) {
        // w = G^T (A_e p_e): one E-vector launch over all elements, then the node gather with p'w fused
        ApplyArgs a{c.op.mesh->idx.ptr, c.op.mesh->own.ptr, nullptr, nullptr, nullptr, v.p, c.op.evec.ptr,
                    c.op.mesh->order_d.ptr, 0, 0, c.op.mesh->nnodes};
        ++c.applies;
        if (hx_status st = launch_apply(c.op, Prec::F64, true, a, c.s)) return st;
        const int P3 = c.op.P * c.op.P * c.op.P;
        const int32_t *gp = c.op.mesh->gather_ptr.ptr, *gs = c.op.mesh->gather_slot.ptr;
        if (c.nc == 1) LAUNCH_V((k_gather_dot<1>), c.n, P3, gp, gs, c.op.evec.ptr, v.p, v.w, c.part2);
        else LAUNCH_V((k_gather_dot<3>), c.n, P3, gp, gs, c.op.evec.ptr, v.p, v.w, c.part2);
        dot_done = true;
      }
    }
    if (!dot_done) {
      if (hx_status st = apply_T(c, v.p, v.w, op_prec)) return st;
      LAUNCH_V((k_dot<T>), c.n, v.p, v.w, c.part2);
    }
    const uint8_t *fm = c.op.mesh->freemask.ptr;
    if (!pc) {
      if (c.nc == 1)
        LAUNCH_V((k_update_red<T, 1, true>), c.n, c.S, c.part2, kVecBlocks, v.x, v.p, v.r, v.w, fm, v.dinv, v.z,
                 c.part0, c.part1, rp);
      else
        LAUNCH_V((k_update_red<T, 3, true>), c.n, c.S, c.part2, kVecBlocks, v.x, v.p, v.r, v.w, fm, v.dinv, v.z,
                 c.part0, c.part1, rp);
      LAUNCH_V((k_pupd_red<T, false>), c.n, c.S, c.part0, c.part1, (const double *)nullptr, kVecBlocks, v.z, v.p);
    } else {
      if (c.nc == 1)
        LAUNCH_V((k_update_red<T, 1, false>), c.n, c.S, c.part2, kVecBlocks, v.x, v.p, v.r, v.w, fm, v.dinv, v.z,
                 c.part0, c.part1, rp);
      else
        LAUNCH_V((k_update_red<T, 3, false>), c.n, c.S, c.part2, kVecBlocks, v.x, v.p, v.r, v.w, fm, v.dinv, v.z,
                 c.part0, c.part1, rp);
      if (hx_status st = (*pc)(v.r, v.z)) return st;
      if (flexible) {
        // Polak-Ribiere beta = (r - r_prev)'z / r_prev'z_prev keeps CG robust with a preconditioner
        // that is not exactly linear or symmetric (rounded operator)
        LAUNCH_V((k_dot_flex<T>), c.n, v.r, v.rp, v.z, c.part0, c.part2);
        LAUNCH_V((k_pupd_red<T, true>), c.n, c.S, c.part0, c.part1, c.part2, kVecBlocks, v.z, v.p);
      } else {
        LAUNCH_V((k_dot<T>), c.n, v.r, v.z, c.part0);
        LAUNCH_V((k_pupd_red<T, false>), c.n, c.S, c.part0, c.part1, (const double *)nullptr, kVecBlocks, v.z, v.p);
      }
    }
    HX_HIP(hipGetLastError());
    return HX_OK;
  };
  // graph replay: captured at the second iteration (the first one, launched eagerly, makes the
  // buffers the kernels allocate on first use) and replayed for the rest
  hipGraphExec_t gx = nullptr;
  struct GraphExec {
    hipGraphExec_t &g;
    ~GraphExec() {
      if (g) (void)hipGraphExecDestroy(g);
    }
  } gx_guard{gx};
  int graph_applies = 0;
  while (it < maxit && rr > stop2) {
    if (c.graph && it >= 1) {
      if (!gx) {
        const int applies0 = c.applies;
        HX_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
        const hx_status st = iteration();
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c.s, &g);
        if (st != HX_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return hip_fail(e, "PCG iteration capture");
        const hipError_t ei = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return hip_fail(ei, "PCG iteration graph");
        graph_applies = c.applies - applies0;
        c.applies = applies0;
      }
      HX_HIP(hipGraphLaunch(gx, c.s));
      c.applies += graph_applies;
    } else {
      if (hx_status st = iteration()) return st;
    }
    ++it;
    if (it % check_every == 0 || it == maxit) {
      if (hx_status e = read_scalars(c)) return e;
      rr = c.hS[S_RR];
      if (c.hS[S_FLAG] != 0.0) {
        *iters = it;
        *rr_out = rr;
        return fail(HX_EBREAKDOWN, "CG breakdown: p'Ap <= 0, r'z <= 0 or a non-finite scalar (flag " +
                                       std::to_string((int)c.hS[S_FLAG]) + ")");
      }
      if (on_check) {
        if (hx_status st = (*on_check)(rr, &rr)) {
          *iters = it;
          *rr_out = rr;
          return st;
        }
      }
      if (stall_window > 0) {
        hist.emplace_back(it, rr);
        for (const auto &h : hist)
          if (h.first <= it - stall_window && h.first > it - stall_window - check_every && rr > stall_factor * stall_factor * h.second) {
            *iters = it;
            *rr_out = rr;
            return kStalled;
          }
      }
    }
  }
  *iters = it;
  *rr_out = rr;
  return HX_OK;
}

// Lanczos estimate of the largest eigenvalue of D^-1 A: `steps` Jacobi-PCG iterations from a seeded random right-hand
// side; the CG coefficients give the Lanczos tridiagonal T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
// T_{j,j+1} = sqrt(beta_j)/alpha_j, whose largest eigenvalue approaches lambda_max from below.
hx_status lanczos_lambda_max(Ctx &c, const Vecs<double> &v, int steps, double *lmax) {
  std::vector<double> h(c.n);
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (auto &t : h) t = U(rng);
  HX_HIP(hipMemcpyAsync(v.r, h.data(), sizeof(double) * c.n, hipMemcpyHostToDevice, c.s));
  if (c.nc == 1) LAUNCH_V((k_maskset<1>), c.n, c.op.mesh->freemask.ptr, v.r);
  else LAUNCH_V((k_maskset<3>), c.n, c.op.mesh->freemask.ptr, v.r);
  HX_HIP(hipMemsetAsync(c.S, 0, sizeof(double) * S_NSCAL, c.s));
  LAUNCH_V((k_jacobi<double>), c.n, v.dinv, v.r, v.z, c.part0);
  FINAL(c.part0, (const double *)nullptr, FIN_RZ, 0);
  HX_HIP(hipMemcpyAsync(v.p, v.z, sizeof(double) * c.n, hipMemcpyDeviceToDevice, c.s));
  HX_HIP(hipMemsetAsync(v.x, 0, sizeof(double) * c.n, c.s));
  std::vector<double> al, be;
  for (int it = 0; it < steps; ++it) {
    if (hx_status st = apply_T(c, v.p, v.w, HX_FP64)) return st;
    LAUNCH_V((k_dot<double>), c.n, v.p, v.w, c.part0);
    FINAL(c.part0, (const double *)nullptr, FIN_PAP, 0);
    if (c.nc == 1) LAUNCH_V((k_update<double, 1, true>), c.n, c.S, v.x, v.p, v.r, v.w, c.op.mesh->freemask.ptr, v.dinv, v.z, c.part0, c.part1, (double *)nullptr);
    else LAUNCH_V((k_update<double, 3, true>), c.n, c.S, v.x, v.p, v.r, v.w, c.op.mesh->freemask.ptr, v.dinv, v.z, c.part0, c.part1, (double *)nullptr);
    FINAL(c.part0, c.part1, FIN_RZ_RR, 0);
    LAUNCH_V((k_pupd<double>), c.n, c.S, v.z, v.p);
    if (hx_status e = read_scalars(c)) return e;
    if (c.hS[S_FLAG] != 0.0 || !(c.hS[S_ALPHA] > 0)) break;
    al.push_back(c.hS[S_ALPHA]);
    be.push_back(c.hS[S_BETA]);
    if (c.hS[S_RR] == 0.0) break;
  }
  if (al.empty()) return fail(HX_EBREAKDOWN, "Lanczos estimate failed (zero right-hand side or breakdown)");
  const int m = (int)al.size();
  std::vector<double> d(m), e(m > 1 ? m - 1 : 0);
  for (int j = 0; j < m; ++j) {
    d[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < m) e[j] = std::sqrt(be[j]) / al[j];
  }
  *lmax = tridiag_max_eig(d, e);
  return HX_OK;
}

// Largest eigenvalue of M A for a general base map M (scalar operator), by power iteration from a
// seeded random vector: `steps` products v <- M A v / |M A v|; the last norm ratio approaches
// |lambda_max| from below. Uses v.p, v.w, v.z.
hx_status power_lambda_max(Ctx &c, const Vecs<double> &v, const PrecFn<double> &base, int steps, double *lmax) {
  std::vector<double> h(c.n);
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (auto &t : h) t = U(rng);
  HX_HIP(hipMemcpyAsync(v.p, h.data(), sizeof(double) * c.n, hipMemcpyHostToDevice, c.s));
  LAUNCH_V((k_maskset<1>), c.n, c.op.mesh->freemask.ptr, v.p);
  auto norm = [&](const double *a, double *out) -> hx_status {
    LAUNCH_V((k_dot<double>), c.n, a, a, c.part0);
    FINAL(c.part0, (const double *)nullptr, FIN_SUM, S_TMP);
    if (hx_status st = read_scalars(c)) return st;
    *out = std::sqrt(c.hS[S_TMP]);
    return HX_OK;
  };
  double nv = 0.0, lam = 0.0;
  if (hx_status st = norm(v.p, &nv)) return st;
  for (int it = 0; it < steps; ++it) {
    if (hx_status st = apply_T(c, v.p, v.w, HX_FP64)) return st;
    LAUNCH_V((k_maskset<1>), c.n, c.op.mesh->freemask.ptr, v.w);
    if (hx_status st = base(v.w, v.z)) return st;
    double nz = 0.0;
    if (hx_status st = norm(v.z, &nz)) return st;
    if (!(nz > 0.0) || !std::isfinite(nz) || !(nv > 0.0))
      return fail(HX_EBREAKDOWN, "power iteration for lambda_max(M A): zero or non-finite product");
    lam = nz / nv;
    LAUNCH_V((k_convert<double, double>), c.n, 1.0 / nz, v.z, v.p);
    nv = 1.0;
  }
  *lmax = lam;
  return HX_OK;
}

template <typename T>
hx_status carve(DevBuf<T> &buf, int64_t n, Vecs<T> &v) {
  if (buf.count < (size_t)(10 * n)) HX_HIP(buf.alloc((size_t)10 * n));
  T *b = buf.ptr;
  v = Vecs<T>{b, b + n, b + 2 * n, b + 3 * n, b + 4 * n, b + 5 * n, b + 6 * n, b + 7 * n, b + 8 * n, b + 9 * n};
  return HX_OK;
}

struct PinnedHost {
  double *p = nullptr;
  ~PinnedHost() {
    if (p) (void)hipHostFree(p);
  }
};

// ---------------------------------------------------------------- p-multigrid V-cycle

Ctx level_ctx(hx_pmg_s &mg, hx_pmg_s::Level &L, hipStream_t s) {
  double *red = L.red.ptr;
  return Ctx{*L.op, s, L.n, L.op->ncomp, red, red + kVecBlocks, red + 3 * kVecBlocks, red + 2 * kVecBlocks, mg.hS, 0};
}

// the level's work vectors of type T (carved at setup)
hx_status level_vecs(hx_pmg_s::Level &L, Vecs<double> &v) { return carve(L.work, L.n, v); }
hx_status level_vecs(hx_pmg_s::Level &L, Vecs<float> &v) { return carve(L.work32, L.n, v); }

// x += d
template <typename T>
__global__ void __launch_bounds__(kVecThreads) k_add(int64_t n, const T *__restrict__ d, T *__restrict__ x) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    x[t] += d[t];
}

// z = V_l r on vectors of type T (operators in the matching precision: FP32 ones read FP32 geometric
// factors). Level l's vectors: r and z are the caller's at level 0 and v.r, v.x below it; the level
// itself uses v.w, v.cd, v.ct and v.dinv. The coarsest level runs Jacobi-PCG from 0.
template <typename T>
hx_status pmg_level(hx_pmg_s &mg, size_t l, const T *r, T *z, hipStream_t s) {
  // FP32 hierarchies with a bf16 precision run the finest level's operator on matrix cores
  const bool mfma = l == 0 && (mg.opts.prec == HX_BF16 || mg.opts.prec == HX_BF16_SPLIT);
  const int op_prec = std::is_same<T, float>::value ? (mfma ? mg.opts.prec : HX_FP32) : HX_FP64;
  auto &L = *mg.lv[l];
  Ctx c = level_ctx(mg, L, s);
  Vecs<T> v;
  if (hx_status st = level_vecs(L, v)) return st;
  const int64_t n = L.n;
  if (l + 1 == mg.lv.size()) {
    if (r != v.r) HX_HIP(hipMemcpyAsync(v.r, r, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    double rr0 = 1.0, stop2 = 0.0;
    int check = mg.opts.coarse_maxit;
    if (mg.opts.coarse_rtol > 0.0) {
      HX_HIP(hipMemsetAsync(c.S, 0, sizeof(double) * S_NSCAL, s));
      LAUNCH_V((k_dot<T>), n, v.r, v.r, c.part0);
      FINAL(c.part0, (const double *)nullptr, FIN_SUM, S_TMP);
      if (hx_status st = read_scalars(c)) return st;
      rr0 = c.hS[S_TMP];
      stop2 = mg.opts.coarse_rtol * mg.opts.coarse_rtol * rr0;
      check = std::min(10, mg.opts.coarse_maxit);
    }
    int it = 0;
    double rr = 0.0;
    hx_status st = rr0 > 0.0 ? pcg_core<T>(c, v, nullptr, op_prec, rr0, stop2, mg.opts.coarse_maxit, check, false,
                                           &it, &rr)
                             : (hipMemsetAsync(v.x, 0, sizeof(T) * n, s) == hipSuccess ? HX_OK : HX_EHIP);
    if (st == HX_EBREAKDOWN) st = HX_OK;  // keep the iterate reached (a residual that vanished exactly)
    L.applies += c.applies;
    if (st) return st;
    if (z != v.x) HX_HIP(hipMemcpyAsync(z, v.x, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    return HX_OK;
  }
  const uint8_t *fm = L.op->mesh->freemask.ptr;
  Cheb ch;
  ch.degree = mg.opts.smooth_degree;
  ch.lam_hi = 1.1 * L.lam_max;
  ch.lam_lo = ch.lam_hi / mg.opts.smooth_ratio;
  auto &C = *mg.lv[l + 1];
  Vecs<T> vc;
  if (hx_status st = level_vecs(C, vc)) return st;
  // a learned smoother on the finest level of an FP64 hierarchy: the same polynomial on the mode-1
  // learned map M in place of D^-1 (v.cd, v.ct and v.m carry its recurrence; v.p and v.z the
  // post-smoothing residual and correction)
  const PrecFn<double> *learned = nullptr;
  PrecFn<double> mlp_base;
  if constexpr (std::is_same<T, double>::value) {
    if (l == 0 && mg.opts.smoother_mlp) {
      mlp_base = [&](const double *rr, double *zz) -> hx_status {
        return mlp_precond_apply(*L.op, *mg.opts.smoother_mlp, 1, rr, zz, s);
      };
      learned = &mlp_base;
    }
  }
  // pre-smoothing from 0; the restriction reads the masked residual r - A z
  if constexpr (std::is_same<T, double>::value) {
    if (learned) {
      if (hx_status st = cheb_apply_base(c, ch, v, *learned, r, z)) return st;
    } else {
      if (hx_status st = cheb_apply<T>(c, ch, v, r, z, op_prec)) return st;
    }
  } else {
    if (hx_status st = cheb_apply<T>(c, ch, v, r, z, op_prec)) return st;
  }
  if (hx_status st = apply_T(c, z, v.w, op_prec)) return st;
  // coarse correction
  if (hx_status st = launch_restrict<T>(mg, (int)l, v.w, vc.r, C.op->mesh->freemask.ptr, s, r)) return st;
  if (hx_status st = pmg_level<T>(mg, l + 1, vc.r, vc.x, s)) return st;
  if (hx_status st = launch_prolong<T>(mg, (int)l, vc.x, v.w, fm, s)) return st;
  LAUNCH_V((k_add<T>), n, v.w, z);
  // post-smoothing: the same polynomial on the error equation, from the corrected iterate
  if constexpr (std::is_same<T, double>::value) {
    if (learned) {
      if (hx_status st = apply_T(c, z, v.w, op_prec)) return st;
      LAUNCH_V((k_resid<double, double, 1>), n, 1.0, r, v.w, fm, v.p, c.part1);
      if (hx_status st = cheb_apply_base(c, ch, v, *learned, v.p, v.z)) return st;
      LAUNCH_V((k_add<T>), n, v.z, z);
    } else {
      if (hx_status st = cheb_apply_from<T>(c, ch, v, r, z, op_prec)) return st;
    }
  } else {
    if (hx_status st = cheb_apply_from<T>(c, ch, v, r, z, op_prec)) return st;
  }
  L.applies += c.applies;
  HX_HIP(hipGetLastError());
  return HX_OK;
}

// z = V_0 r on FP64 vectors; an FP32 hierarchy converts at the finest level (its v.m and v.rp carry
// the FP32 input and output: the level itself does not use them)
hx_status pmg_vcycle(hx_pmg_s &mg, const double *r, double *z, hipStream_t s) {
  if (mg.opts.prec == HX_FP64) {
    if (hx_status st = pmg_level<double>(mg, 0, r, z, s)) return st;
    if (mg.opts.cycles > 1) {
      // further cycles on the residual: z += V(r - A z), level 0's v.r and v.x (free at level 0) carry it
      auto &L = *mg.lv[0];
      Ctx c = level_ctx(mg, L, s);
      Vecs<double> v;
      if (hx_status st = level_vecs(L, v)) return st;
      const uint8_t *fm = L.op->mesh->freemask.ptr;
      for (int k = 1; k < mg.opts.cycles; ++k) {
        if (hx_status st = apply_T(c, z, v.w, HX_FP64)) return st;
        if (L.op->ncomp == 1) LAUNCH_V((k_resid<double, double, 1>), L.n, 1.0, r, v.w, fm, v.r, c.part1);
        else LAUNCH_V((k_resid<double, double, 3>), L.n, 1.0, r, v.w, fm, v.r, c.part1);
        if (hx_status st = pmg_level<double>(mg, 0, v.r, v.x, s)) return st;
        LAUNCH_V((k_add<double>), L.n, v.x, z);
      }
      L.applies += c.applies;
      HX_HIP(hipGetLastError());
    }
    return HX_OK;
  }
  auto &L = *mg.lv[0];
  Ctx c = level_ctx(mg, L, s);
  Vecs<float> v;
  if (hx_status st = level_vecs(L, v)) return st;
  LAUNCH_V((k_convert<double, float>), L.n, 1.0, r, v.m);
  if (hx_status st = pmg_level<float>(mg, 0, v.m, v.rp, s)) return st;
  LAUNCH_V((k_convert<float, double>), L.n, 1.0, v.rp, z);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace

// each level's work vectors, D^-1 and (above the coarsest) lam_max of D^-1 A by Lanczos; an FP32
// hierarchy also gets FP32 vectors, D^-1 and geometric factors
hx_status pmg_setup_levels(hx_pmg_s &mg, hipStream_t s) {
  if (!mg.hS) HX_HIP(hipHostMalloc(reinterpret_cast<void **>(&mg.hS), sizeof(double) * S_NSCAL));
  for (size_t l = 0; l < mg.lv.size(); ++l) {
    auto &L = *mg.lv[l];
    hx_op_s &op = *L.op;
    HX_HIP(L.red.alloc(3 * kVecBlocks + S_NSCAL));
    Vecs<double> v;
    if (hx_status st = carve(L.work, L.n, v)) return st;
    if (!op.diag_valid) {
      if (op.diag.count < (size_t)L.n) HX_HIP(op.diag.alloc(L.n));
      if (hx_status st = hx_op_diagonal(&op, op.diag.ptr, s)) return st;
      op.diag_valid = true;
    }
    Ctx c = level_ctx(mg, L, s);
    if (op.ncomp == 1) LAUNCH_V((k_dinv<double, 1>), L.n, op.diag.ptr, op.mesh->freemask.ptr, v.dinv);
    else LAUNCH_V((k_dinv<double, 3>), L.n, op.diag.ptr, op.mesh->freemask.ptr, v.dinv);
    HX_HIP(hipGetLastError());
    if (mg.opts.prec != HX_FP64) {
      Vecs<float> v32;
      if (hx_status st = carve(L.work32, L.n, v32)) return st;
      LAUNCH_V((k_convert<double, float>), L.n, 1.0, v.dinv, v32.dinv);
      // FP32 geometric factors, except where the finest level runs on matrix cores (bf16 copy, made on first use)
      if (mg.opts.prec == HX_FP32 || l > 0)
        if (hx_status st = make_qdata32(op, s)) return st;
    }
    if (l == 0 && mg.opts.smoother_mlp) {
      // the learned smoother's interval: lam_max of M A by power iteration
      if (hx_status st = mlp_prepare(op, s)) return st;
      PrecFn<double> base = [&](const double *rr, double *zz) -> hx_status {
        return mlp_precond_apply(op, *mg.opts.smoother_mlp, 1, rr, zz, s);
      };
      if (hx_status st = power_lambda_max(c, v, base, mg.opts.lanczos_steps, &L.lam_max)) return st;
    } else if (l + 1 < mg.lv.size()) {
      if (hx_status st = lanczos_lambda_max(c, v, mg.opts.lanczos_steps, &L.lam_max)) return st;
    }
  }
  HX_HIP(hipStreamSynchronize(s));
  return HX_OK;
}

}  // namespace hx

extern "C" hx_status hx_pmg_vcycle(hx_pmg mg, const double *r, double *z, hx_stream s) {
  if (!mg || !r || !z) return hx::fail(HX_EINVAL, "null argument");
  if (r == z) return hx::fail(HX_EINVAL, "z must not alias r");
  return hx::pmg_vcycle(*mg, r, z, static_cast<hipStream_t>(s));
}

using namespace hx;

extern "C" void hx_solve_opts_default(hx_solve_opts *o) {
  if (!o) return;
  o->mode = HX_SOLVE_FP64;
  o->precond = HX_PC_JACOBI;
  o->rtol = 1e-8;
  o->maxit = 10000;
  o->check_every = 10;
  o->use_x0 = 0;
  o->cheb_degree = 4;
  o->cheb_ratio = 30.0;
  o->cheb_prec = HX_FP32;
  o->lanczos_steps = 20;
  o->inner_rtol = 1e-4;
  o->inner_maxit = 10000;
  o->inner_qdata = HX_FP64;
  o->flexible = 0;
  o->mlp = nullptr;
  o->fallback = HX_PC_JACOBI;
  o->stall_window = 20;
  o->stall_factor = 0.1;
  o->mlp_mode = 1;
  o->graph = 0;
  o->pmg = nullptr;
  o->scatter = HX_SCATTER_COLORS;
  o->reliable_delta = 0.25;
}

extern "C" hx_status hx_pcg_solve(hx_op op, const double *b, double *x, const hx_solve_opts *opts,
                                  hx_solve_info *info, hx_stream stream) {
  if (!op || !b || !x || !opts || !info) return fail(HX_EINVAL, "null argument");
  const hx_solve_opts &o = *opts;
  if (o.mode != HX_SOLVE_FP64 && o.mode != HX_SOLVE_IR && o.mode != HX_SOLVE_MIXED)
    return fail(HX_EINVAL, "mode must be HX_SOLVE_FP64, HX_SOLVE_IR or HX_SOLVE_MIXED");
  const bool mixed = o.mode == HX_SOLVE_MIXED;
  if (mixed && !(o.reliable_delta > 0.0 && o.reliable_delta < 1.0))
    return fail(HX_EINVAL, "HX_SOLVE_MIXED needs 0 < reliable_delta < 1");
  if (o.precond < HX_PC_NONE || o.precond > HX_PC_PMG) return fail(HX_EINVAL, "precond out of range");
  const bool pmg = o.precond == HX_PC_PMG;
  if (pmg && !o.pmg) return fail(HX_EINVAL, "HX_PC_PMG needs opts.pmg");
  // the hierarchy's finest operator is the solved one, or the low-order refined operator of its nodes
  // (same node count, and the same coordinates at 1024 sampled nodes)
  if (pmg && o.pmg->lv[0]->op != op) {
    const hx_op_s &f = *o.pmg->lv[0]->op;
    bool same = f.kind == HX_LOR && o.pmg->lv[0]->n == op->mesh->nnodes * op->ncomp &&
                f.mesh->nnodes == op->mesh->nnodes;
    const int64_t nn = op->mesh->nnodes;
    for (int64_t t = 0; same && t < nn; t += std::max<int64_t>(1, nn / 1024))
      for (int d = 0; d < 3; ++d) same = same && f.mesh->h_xyz[3 * t + d] == op->mesh->h_xyz[3 * t + d];
    if (!same) return fail(HX_EINVAL, "the hierarchy's finest operator is not the solved one");
  }
  if (pmg && o.mode != HX_SOLVE_FP64) return fail(HX_EUNSUPPORTED, "HX_PC_PMG runs in HX_SOLVE_FP64 mode");
  if (!(o.rtol > 0) || o.maxit < 1 || o.check_every < 1) return fail(HX_EINVAL, "need rtol > 0, maxit >= 1, check_every >= 1");
  const bool mlp = o.precond == HX_PC_MLP;
  if (mlp && !o.mlp) return fail(HX_EINVAL, "HX_PC_MLP needs opts.mlp");
  if (mlp && o.mode != HX_SOLVE_FP64) return fail(HX_EUNSUPPORTED, "HX_PC_MLP runs in HX_SOLVE_FP64 mode");
  if (mlp && (op->kind != HX_DIFFUSION || op->ncomp != 1))
    return fail(HX_EUNSUPPORTED, "the learned preconditioner supports scalar diffusion only");
  if (mlp && o.fallback != HX_PC_JACOBI && o.fallback != HX_PC_CHEBYSHEV)
    return fail(HX_EINVAL, "fallback must be HX_PC_JACOBI or HX_PC_CHEBYSHEV");
  if (mlp && (o.mlp_mode < 0 || o.mlp_mode > 2)) return fail(HX_EINVAL, "mlp_mode must be 0, 1 or 2");
  if (mlp && o.mlp_mode == 2 && (o.cheb_degree < 1 || !(o.cheb_ratio > 1.0) || o.lanczos_steps < 2))
    return fail(HX_EINVAL, "mlp_mode 2 needs cheb_degree >= 1, cheb_ratio > 1, lanczos_steps >= 2");
  if (mlp && (o.stall_window < 0 || !(o.stall_factor > 0 && o.stall_factor < 1)))
    return fail(HX_EINVAL, "stall_window >= 0 and 0 < stall_factor < 1");
  // Chebyshev runs as the preconditioner, or as the fallback of the learned one
  const bool cheb = o.precond == HX_PC_CHEBYSHEV || (mlp && o.fallback == HX_PC_CHEBYSHEV);
  if (cheb && (o.cheb_degree < 1 || !(o.cheb_ratio > 1.0) || o.lanczos_steps < 2))
    return fail(HX_EINVAL, "Chebyshev needs cheb_degree >= 1, cheb_ratio > 1, lanczos_steps >= 2");
  const bool cheb_bf16 = o.cheb_prec == HX_BF16 || o.cheb_prec == HX_BF16_SPLIT;
  if (cheb && o.cheb_prec != HX_FP64 && o.cheb_prec != HX_FP32 && !cheb_bf16)
    return fail(HX_EINVAL, "cheb_prec must be HX_FP64, HX_FP32, HX_BF16 or HX_BF16_SPLIT");
  if (o.mode == HX_SOLVE_IR && (!(o.inner_rtol > 0 && o.inner_rtol < 1) || o.inner_maxit < 1))
    return fail(HX_EINVAL, "IR needs 0 < inner_rtol < 1 and inner_maxit >= 1");
  if ((o.mode == HX_SOLVE_IR || mixed) && o.inner_qdata != HX_FP64 && o.inner_qdata != HX_FP32)
    return fail(HX_EINVAL, "inner_qdata must be HX_FP64 or HX_FP32");
  if ((o.mode == HX_SOLVE_IR || mixed) && cheb && o.cheb_prec == HX_FP64)
    return fail(HX_EINVAL, "the FP32 solve needs cheb_prec HX_FP32, HX_BF16 or HX_BF16_SPLIT");
  if (cheb && cheb_bf16 && (op->kind != HX_DIFFUSION || op->ncomp != 1))
    return fail(HX_EUNSUPPORTED, "the bf16 operator supports scalar diffusion only");
  if (o.scatter != HX_SCATTER_COLORS && o.scatter != HX_SCATTER_GATHER)
    return fail(HX_EINVAL, "scatter must be HX_SCATTER_COLORS or HX_SCATTER_GATHER");
  if (op->kind == HX_LOR && (o.mode != HX_SOLVE_FP64 || (cheb && o.cheb_prec != HX_FP64) || mlp ||
                             o.scatter != HX_SCATTER_COLORS))
    return fail(HX_EUNSUPPORTED, "the low-order refined operator solves in FP64 with Jacobi, FP64 Chebyshev or p-multigrid");
  *info = hx_solve_info{};
  hipStream_t s = static_cast<hipStream_t>(stream);
  // graph replay needs a stream that can be captured: the solve then runs on the operator's own
  // stream, after the caller's queued work; it is synchronous, so it has finished on return
  const bool use_graph = o.graph != 0 && !mlp && !pmg && op->mesh->nuntouched == 0;
  StreamSync solve_done;
  if (use_graph) {
    if (!op->solve_stream) HX_HIP(hipStreamCreateWithFlags(&op->solve_stream, hipStreamNonBlocking));
    HX_HIP(hipStreamSynchronize(s));
    s = op->solve_stream;
    stream = s;
    solve_done.s = s;
  }
  const int64_t n = op->mesh->nnodes * op->ncomp;
  const int NC = op->ncomp;
  const auto t_setup0 = std::chrono::steady_clock::now();

  if (op->red.count < (size_t)(3 * kVecBlocks + S_NSCAL)) HX_HIP(op->red.alloc(3 * kVecBlocks + S_NSCAL));
  PinnedHost hs;
  HX_HIP(hipHostMalloc(reinterpret_cast<void **>(&hs.p), sizeof(double) * S_NSCAL));
  Ctx c{*op, s, n, NC, op->red.ptr, op->red.ptr + kVecBlocks, op->red.ptr + 3 * kVecBlocks,
        op->red.ptr + 2 * kVecBlocks, hs.p, 0};
  c.graph = use_graph;
  if (o.scatter == HX_SCATTER_GATHER) {
    const size_t ne = (size_t)op->mesh->nelem * NC * op->P * op->P * op->P;
    if (op->evec.count < ne) HX_HIP(op->evec.alloc(ne));
    if (hx_status st = mesh_gather_csr(*op->mesh)) return st;
    c.gather = true;
  }

  Vecs<double> v;
  if (hx_status st = carve(op->work, n, v)) return st;
  const bool need_diag = o.precond != HX_PC_NONE;
  if (need_diag && !op->diag_valid) {
    if (op->diag.count < (size_t)n) HX_HIP(op->diag.alloc(n));
    if (hx_status st = hx_op_diagonal(op, op->diag.ptr, stream)) return st;
    op->diag_valid = true;
  }
  const double *dg = need_diag ? op->diag.ptr : nullptr;
  if (NC == 1) LAUNCH_V((k_dinv<double, 1>), n, dg, op->mesh->freemask.ptr, v.dinv);
  else LAUNCH_V((k_dinv<double, 3>), n, dg, op->mesh->freemask.ptr, v.dinv);
  HX_HIP(hipGetLastError());

  const bool use32 = o.mode == HX_SOLVE_IR || mixed || (cheb && o.cheb_prec != HX_FP64);
  Vecs<float> v32{};
  if (use32) {
    if (hx_status st = carve(op->work32, n, v32)) return st;
    LAUNCH_V((k_convert<double, float>), n, 1.0, v.dinv, v32.dinv);
    const bool q32 = ((o.mode == HX_SOLVE_IR || mixed) && o.inner_qdata == HX_FP32) || (cheb && o.cheb_prec == HX_FP32);
    if (q32)
      if (hx_status st = make_qdata32(*op, s)) return st;
    HX_HIP(hipGetLastError());
  }

  Cheb ch;
  ch.degree = o.cheb_degree;
  if (cheb) {
    double lmax = 0;
    if (hx_status st = lanczos_lambda_max(c, v, o.lanczos_steps, &lmax)) return st;
    ch.lam_hi = 1.1 * lmax;
    ch.lam_lo = ch.lam_hi / o.cheb_ratio;
    info->lam_max = lmax;
  }
  // learned maps: mode 1 base M r = D^-1 r + network correction; mode 2 runs Chebyshev steps over it
  PrecFn<double> mlp_base = [&](const double *r, double *z) -> hx_status {
    return mlp_precond_apply(*op, *o.mlp, 1, r, z, s);
  };
  Cheb chm;
  chm.degree = o.cheb_degree;
  if (mlp) {
    if (hx_status st = mlp_prepare(*op, s)) return st;
    if (o.mlp_mode == 2) {
      double lmax = 0;
      if (hx_status st = power_lambda_max(c, v, mlp_base, o.lanczos_steps, &lmax)) return st;
      chm.lam_hi = 1.1 * lmax;
      chm.lam_lo = chm.lam_hi / o.cheb_ratio;
      info->lam_max = lmax;
    }
  }
  HX_HIP(hipStreamSynchronize(s));
  const auto t0 = std::chrono::steady_clock::now();
  info->setup_seconds = std::chrono::duration<double>(t0 - t_setup0).count();
  c.applies = 0;
  const int64_t pmg_applies0 = pmg ? o.pmg->lv[0]->applies : 0;

  if (o.use_x0) {
    if (NC == 1) LAUNCH_V((k_maskset<1>), n, op->mesh->freemask.ptr, x);
    else LAUNCH_V((k_maskset<3>), n, op->mesh->freemask.ptr, x);
  } else {
    HX_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  }
  // ||b|| over the free nodes
  if (NC == 1) LAUNCH_V((k_resid<double, double, 1>), n, 1.0, b, (const double *)nullptr, op->mesh->freemask.ptr, v.r, c.part1);
  else LAUNCH_V((k_resid<double, double, 3>), n, 1.0, b, (const double *)nullptr, op->mesh->freemask.ptr, v.r, c.part1);
  FINAL(c.part1, (const double *)nullptr, FIN_SUM, S_BB);
  if (hx_status st = read_scalars(c)) return st;
  const double bb = c.hS[S_BB];
  if (!std::isfinite(bb)) return fail(HX_EBREAKDOWN, "right-hand side is not finite");
  if (bb == 0.0) {
    HX_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    HX_HIP(hipStreamSynchronize(s));
    info->solve_seconds = 0.0;
    return HX_OK;
  }
  const double bn = std::sqrt(bb);

  // v.r = m (b - A x) in FP64; returns r'r
  auto residual = [&](double *rr_out) -> hx_status {
    if (hx_status st = apply_T(c, x, v.w, HX_FP64)) return st;
    if (NC == 1) LAUNCH_V((k_resid<double, double, 1>), n, 1.0, b, v.w, op->mesh->freemask.ptr, v.r, c.part1);
    else LAUNCH_V((k_resid<double, double, 3>), n, 1.0, b, v.w, op->mesh->freemask.ptr, v.r, c.part1);
    HX_HIP(hipMemsetAsync(c.S, 0, sizeof(double) * S_NSCAL, s));
    FINAL(c.part1, (const double *)nullptr, FIN_SUM, S_RR);
    if (hx_status st = read_scalars(c)) return st;
    *rr_out = c.hS[S_RR];
    return HX_OK;
  };

  hx_status result = HX_OK;
  double rr = 0.0;
  if (hx_status st = residual(&rr)) return st;
  if (o.mode == HX_SOLVE_FP64) {
    // solve A d = r0 in FP64 for the correction d (v.x), then x += d
    PrecFn<double> pc64 = [&](const double *r, double *z) -> hx_status {
      return cheb_apply<double>(c, ch, v, r, z, HX_FP64);
    };
    PrecFn<double> pc32 = [&](const double *r, double *z) -> hx_status {
      LAUNCH_V((k_convert<double, float>), n, 1.0, r, v32.r);
      if (hx_status st = cheb_apply<float>(c, ch, v32, v32.r, v32.z, o.cheb_prec)) return st;
      LAUNCH_V((k_convert<float, double>), n, 1.0, v32.z, z);
      return HX_OK;
    };
    PrecFn<double> pcm = [&](const double *r, double *z) -> hx_status {
      if (o.mlp_mode == 0) return mlp_precond_apply(*op, *o.mlp, 0, r, z, s);
      if (o.mlp_mode == 1) return mlp_base(r, z);
      return cheb_apply_base(c, chm, v, mlp_base, r, z);
    };
    PrecFn<double> pcp = [&](const double *r, double *z) -> hx_status { return pmg_vcycle(*o.pmg, r, z, s); };
    const PrecFn<double> *pc_cheb = cheb ? ((o.cheb_prec == HX_FP64) ? &pc64 : &pc32) : nullptr;
    const PrecFn<double> *pc = mlp ? &pcm : pmg ? &pcp : pc_cheb;
    const double stop2 = o.rtol * o.rtol * bb;
    int it = 0;
    double rre = 0;
    // the learned preconditioner and the V-cycle (its coarse PCG) are nonlinear in r: flexible CG,
    // with a stall check for the learned one's fallback
    result = pcg_core<double>(c, v, pc, HX_FP64, rr, stop2, o.maxit, o.check_every, o.flexible != 0 || mlp || pmg, &it,
                              &rre, mlp ? o.stall_window : 0, o.stall_factor);
    if (mlp) HX_HIP(hipMemcpyAsync(v.cd, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));  // x before the learned phase
    LAUNCH_V((k_axpy<double>), n, 1.0, v.x, x);
    info->iterations = it;
    if (mlp && (result == HX_EBREAKDOWN || result == kStalled || (result == HX_OK && rre > stop2))) {
      // check and fallback: Jacobi or Chebyshev PCG from the current iterate, or from the iterate
      // before the learned phase when its correction is not finite or did not lower the true residual
      info->fallback_used = 1;
      info->fallback_reason = result == HX_EBREAKDOWN ? 1 : result == kStalled ? 2 : 3;
      double rr2 = 0;
      if (hx_status st = residual(&rr2)) return st;
      if (!std::isfinite(rr2) || rr2 >= rr) {
        HX_HIP(hipMemcpyAsync(x, v.cd, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (hx_status st = residual(&rr2)) return st;
      }
      int it2 = 0;
      result = pcg_core<double>(c, v, o.fallback == HX_PC_CHEBYSHEV ? pc_cheb : nullptr, HX_FP64, rr2, stop2,
                                std::max(1, o.maxit - it), o.check_every, o.flexible != 0, &it2, &rre);
      LAUNCH_V((k_axpy<double>), n, 1.0, v.x, x);
      info->fallback_iterations = it2;
      info->iterations += it2;
    }
    info->rel_residual = std::sqrt(rre) / bn;
  } else if (mixed) {
    // One FP32 PCG on A d = r0 with reliable updates: whenever the recurrence residual has fallen by
    // reliable_delta since the last replacement (or below the target), the FP32 correction d is added
    // to x in FP64, r = m (b - A x) is formed with the FP64 operator and replaces the FP32 residual,
    // z and r'z are recomputed from it, and the search direction is kept, so the Krylov space built so
    // far is not discarded as an iterative-refinement restart would. Convergence is decided on the
    // FP64 residual.
    // as in refinement: the Chebyshev polynomial's operator in cheb_prec, the CG operator on FP32
    // vectors with the geometric factors inner_qdata names
    const int inner_prec = cheb ? o.cheb_prec : o.inner_qdata;
    const int op32 = (o.inner_qdata == HX_FP32) ? HX_FP32 : HX_FP64;
    PrecFn<float> pcc = [&](const float *r, float *z) -> hx_status {
      return cheb_apply<float>(c, ch, v32, r, z, inner_prec);
    };
    const double stop2 = o.rtol * o.rtol * bb;
    const double d2 = o.reliable_delta * o.reliable_delta;
    double rr_ref = rr;
    int updates = 0;
    LAUNCH_V((k_convert<double, float>), n, 1.0, v.r, v32.r);
    CheckFn reliable = [&](double rr_s, double *rr_next) -> hx_status {
      *rr_next = rr_s;
      if (rr_s > std::max(stop2, d2 * rr_ref)) return HX_OK;
      LAUNCH_V((k_axpy<float>), n, 1.0, v32.x, x);
      HX_HIP(hipMemsetAsync(v32.x, 0, sizeof(float) * n, s));
      if (hx_status st = apply_T(c, x, v.w, HX_FP64)) return st;
      const uint8_t *fm = op->mesh->freemask.ptr;
      if (NC == 1) LAUNCH_V((k_resid<float, double, 1>), n, 1.0, b, v.w, fm, v32.r, c.part1);
      else LAUNCH_V((k_resid<float, double, 3>), n, 1.0, b, v.w, fm, v32.r, c.part1);
      if (cheb) {
        if (hx_status st = pcc(v32.r, v32.z)) return st;
        LAUNCH_V((k_dot<float>), n, v32.r, v32.z, c.part0);
      } else {
        LAUNCH_V((k_jacobi<float>), n, v32.dinv, v32.r, v32.z, c.part0);
      }
      FINAL(c.part1, (const double *)nullptr, FIN_SUM, S_RR);
      FINAL(c.part0, (const double *)nullptr, FIN_RZ, 0);
      if (hx_status st = read_scalars(c)) return st;
      ++updates;
      rr_ref = c.hS[S_RR];
      *rr_next = rr_ref;
      if (c.hS[S_FLAG] != 0.0) return fail(HX_EBREAKDOWN, "r'z <= 0 or a non-finite scalar after a residual replacement");
      return HX_OK;
    };
    int it = 0;
    double rre = 0;
    result = pcg_core<float>(c, v32, cheb ? &pcc : nullptr, op32, rr, stop2, o.maxit,
                             o.check_every, o.flexible != 0, &it, &rre, 0, 0.0, &reliable);
    LAUNCH_V((k_axpy<float>), n, 1.0, v32.x, x);  // the part since the last replacement
    HX_HIP(hipGetLastError());
    info->iterations = it;
    info->outer_iterations = updates;
    info->rel_residual = std::sqrt(rre) / bn;
  } else {
    // iterative refinement: FP64 residual, FP32 inner PCG on r / ||r||, FP64 update x += ||r|| d
    int outer = 0, inner_total = 0;
    const int inner_prec = cheb ? o.cheb_prec : o.inner_qdata;
    const int cg_prec = (o.inner_qdata == HX_FP32) ? HX_FP32 : HX_FP64;  // FP32 vectors, qdata precision
    PrecFn<float> pcc = [&](const float *r, float *z) -> hx_status {
      return cheb_apply<float>(c, ch, v32, r, z, inner_prec);
    };
    while (rr > o.rtol * o.rtol * bb) {
      if (!std::isfinite(rr)) {
        result = fail(HX_EBREAKDOWN, "non-finite residual in refinement");
        break;
      }
      if (outer >= o.maxit) {
        result = fail(HX_ENOCONV, "iterative refinement reached maxit outer steps");
        break;
      }
      const double rn = std::sqrt(rr);
      LAUNCH_V((k_convert<double, float>), n, 1.0 / rn, v.r, v32.r);
      int it = 0;
      double rri = 0;
      // inner r'r starts at ~1 (the residual is normalised)
      // inner target: inner_rtol, loosened on the last steps to what the outer tolerance still needs
      // (half of rtol ||b|| / ||r||), and at least a halving
      const double inner_rel = std::min(0.5, std::max(o.inner_rtol, 0.5 * o.rtol * bn / rn));
      hx_status st = pcg_core<float>(c, v32, cheb ? &pcc : nullptr, cg_prec, 1.0, inner_rel * inner_rel,
                                     o.inner_maxit, std::min(o.check_every, o.inner_maxit), o.flexible != 0, &it, &rri);
      if (st == HX_EBREAKDOWN && it > 1) st = HX_OK;  // keep the partial correction; the FP64 residual decides
      if (st) return st;
      inner_total += it;
      LAUNCH_V((k_axpy<float>), n, rn, v32.x, x);
      HX_HIP(hipGetLastError());
      ++outer;
      if (hx_status st2 = residual(&rr)) return st2;
    }
    info->iterations = inner_total;
    info->outer_iterations = outer;
    info->rel_residual = std::sqrt(rr) / bn;
  }
  HX_HIP(hipStreamSynchronize(s));
  const auto t1 = std::chrono::steady_clock::now();
  info->solve_seconds = std::chrono::duration<double>(t1 - t0).count();
  info->operator_applies = c.applies + ((pmg && o.pmg->lv[0]->op == op) ? (int)(o.pmg->lv[0]->applies - pmg_applies0) : 0);
  double rr_true = 0;
  if (hx_status st = residual(&rr_true)) return st;
  info->true_rel_residual = std::sqrt(rr_true) / bn;
  if (result == HX_OK && (o.mode == HX_SOLVE_FP64 || mixed) && info->rel_residual > o.rtol)
    result = fail(HX_ENOCONV, "PCG reached maxit without meeting rtol");
  return result;
}

// ---------------------------------------------------------------- the solve that allocates nothing

namespace {

// Layout of the no-allocation solve's device memory, in doubles: the two 1D tables of the diagonal
// kernel (interpolation and gradient, [q][p+1] each), the reduction partials and device scalars, and
// seven vectors of up to HX_NOALLOC_MAX_DOFS entries (r, z, p, A p, D^-1, the correction, the diagonal).
constexpr size_t kNaTab = 2 * kMaxQ * kMaxP;
constexpr size_t kNaRedOff = 256;
constexpr size_t kNaVecOff = kNaRedOff + ((3 * kVecBlocks + S_NSCAL + 31) / 32) * 32;
constexpr size_t kNaDoubles = kNaVecOff + 7 * (size_t)HX_NOALLOC_MAX_DOFS;
static_assert(kNaTab <= kNaRedOff, "tables overlap the reduction buffers");

}  // namespace

// Each device holds its own copy from the time the library's code is loaded on it until the process ends
// (about 56 MiB). Host code must not pass this name to a kernel or a copy: in host code it is a stand-in,
// not a device address. Host code uses the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kNaDoubles];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on device dev (the current device), looked up once per device
hx_status scratch_address(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HX_EUNSUPPORTED, "device ordinal beyond the supported range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HX_EHIP, "hipGetSymbolAddress returned a null address for the solver's scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return HX_OK;
}

}  // namespace

extern "C" hx_status hx_pcg_solve_noalloc(hx_op op, const double *b, double *x, const hx_solve_opts *opts,
                                          hx_solve_info *info, hx_stream stream) {
  if (!op || !b || !x || !opts || !info) return fail(HX_EINVAL, "null argument");
  const hx_solve_opts &o = *opts;
  if (o.mode != HX_SOLVE_FP64) return fail(HX_EUNSUPPORTED, "the no-allocation solve runs in HX_SOLVE_FP64 mode");
  if (o.precond != HX_PC_NONE && o.precond != HX_PC_JACOBI)
    return fail(HX_EUNSUPPORTED, "the no-allocation solve supports HX_PC_NONE and HX_PC_JACOBI");
  if (o.scatter != HX_SCATTER_COLORS) return fail(HX_EUNSUPPORTED, "the no-allocation solve needs HX_SCATTER_COLORS");
  if (o.graph != 0) return fail(HX_EUNSUPPORTED, "the no-allocation solve does not replay graphs");
  if (!(o.rtol > 0) || o.maxit < 1 || o.check_every < 1) return fail(HX_EINVAL, "need rtol > 0, maxit >= 1, check_every >= 1");
  const int64_t n = op->mesh->nnodes * op->ncomp;
  if (n > (int64_t)HX_NOALLOC_MAX_DOFS)
    return fail(HX_EINVAL, "nnodes*ncomp = " + std::to_string(n) + " exceeds HX_NOALLOC_MAX_DOFS = " +
                               std::to_string((long long)HX_NOALLOC_MAX_DOFS));
  if (op->b.interp.size() + op->b.grad.size() > kNaTab) return fail(HX_EUNSUPPORTED, "1D tables exceed the scratch slot");
  int dev = -1;
  HX_HIP(hipGetDevice(&dev));
  if (dev != op->mesh->device) return fail(HX_EINVAL, "current device differs from the operator's device");
  double *sc = nullptr;
  if (hx_status st = scratch_address(dev, &sc)) return st;

  *info = hx_solve_info{};
  hipStream_t s = static_cast<hipStream_t>(stream);
  StreamSync solve_done;
  solve_done.s = s;  // synchronous on every return path, like hx_pcg_solve
  const int NC = op->ncomp;
  const auto t_setup0 = std::chrono::steady_clock::now();
  double hS[S_NSCAL] = {};  // host copy of the device scalars (pageable: nothing is allocated)
  double *red = sc + kNaRedOff;
  Ctx c{*op, s, n, NC, red, red + kVecBlocks, red + 3 * kVecBlocks, red + 2 * kVecBlocks, hS, 0};
  double *vb = sc + kNaVecOff;
  // r, z, p, w, dinv, (cd, ct unused), x, (rp, m unused): Jacobi PCG reads none of the unused ones
  Vecs<double> v{vb, vb + n, vb + 2 * n, vb + 3 * n, vb + 4 * n, nullptr, nullptr, vb + 5 * n, nullptr, nullptr};
  const double *dg = nullptr;
  if (o.precond == HX_PC_JACOBI) {
    if (op->diag_valid) {
      dg = op->diag.ptr;  // the diagonal an earlier solve cached: already in memory the operator owns
    } else {
      // the diagonal into the seventh vector, its kernel reading the 1D tables staged in the scratch array
      double *d = vb + 6 * n, *ti = sc, *tg = sc + op->b.interp.size();
      if (op->kind == HX_LOR) {
        if (hx_status st = lor_diagonal(*op, d, s)) return st;
      } else {
        HX_HIP(hipMemcpyAsync(ti, op->b.interp.data(), sizeof(double) * op->b.interp.size(), hipMemcpyHostToDevice, s));
        HX_HIP(hipMemcpyAsync(tg, op->b.grad.data(), sizeof(double) * op->b.grad.size(), hipMemcpyHostToDevice, s));
        if (hx_status st = launch_diagonal_tables(*op, ti, tg, d, s)) return st;
      }
      dg = d;
    }
  }
  if (NC == 1) LAUNCH_V((k_dinv<double, 1>), n, dg, op->mesh->freemask.ptr, v.dinv);
  else LAUNCH_V((k_dinv<double, 3>), n, dg, op->mesh->freemask.ptr, v.dinv);
  HX_HIP(hipGetLastError());
  HX_HIP(hipStreamSynchronize(s));
  const auto t0 = std::chrono::steady_clock::now();
  info->setup_seconds = std::chrono::duration<double>(t0 - t_setup0).count();

  // the device scalars start at zero: an earlier call on this device left its own there
  HX_HIP(hipMemsetAsync(c.S, 0, sizeof(double) * S_NSCAL, s));
  if (o.use_x0) {
    if (NC == 1) LAUNCH_V((k_maskset<1>), n, op->mesh->freemask.ptr, x);
    else LAUNCH_V((k_maskset<3>), n, op->mesh->freemask.ptr, x);
  } else {
    HX_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  }
  if (NC == 1) LAUNCH_V((k_resid<double, double, 1>), n, 1.0, b, (const double *)nullptr, op->mesh->freemask.ptr, v.r, c.part1);
  else LAUNCH_V((k_resid<double, double, 3>), n, 1.0, b, (const double *)nullptr, op->mesh->freemask.ptr, v.r, c.part1);
  FINAL(c.part1, (const double *)nullptr, FIN_SUM, S_BB);
  if (hx_status st = read_scalars(c)) return st;
  const double bb = c.hS[S_BB];
  if (!std::isfinite(bb)) return fail(HX_EBREAKDOWN, "right-hand side is not finite");
  if (bb == 0.0) {
    HX_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    return HX_OK;
  }
  const double bn = std::sqrt(bb);
  // v.r = m (b - A x); r'r
  auto residual = [&](double *rr_out) -> hx_status {
    if (hx_status st = apply_T(c, x, v.w, HX_FP64)) return st;
    if (NC == 1) LAUNCH_V((k_resid<double, double, 1>), n, 1.0, b, v.w, op->mesh->freemask.ptr, v.r, c.part1);
    else LAUNCH_V((k_resid<double, double, 3>), n, 1.0, b, v.w, op->mesh->freemask.ptr, v.r, c.part1);
    HX_HIP(hipMemsetAsync(c.S, 0, sizeof(double) * S_NSCAL, s));
    FINAL(c.part1, (const double *)nullptr, FIN_SUM, S_RR);
    if (hx_status st = read_scalars(c)) return st;
    *rr_out = c.hS[S_RR];
    return HX_OK;
  };
  double rr = 0.0;
  if (hx_status st = residual(&rr)) return st;
  int it = 0;
  double rre = 0.0;
  hx_status result = pcg_core<double>(c, v, nullptr, HX_FP64, rr, o.rtol * o.rtol * bb, o.maxit, o.check_every,
                                      false, &it, &rre);
  LAUNCH_V((k_axpy<double>), n, 1.0, v.x, x);
  HX_HIP(hipGetLastError());
  info->iterations = it;
  info->rel_residual = std::sqrt(rre) / bn;
  HX_HIP(hipStreamSynchronize(s));
  info->solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  info->operator_applies = c.applies;
  double rr_true = 0.0;
  if (hx_status st = residual(&rr_true)) return st;
  info->true_rel_residual = std::sqrt(rr_true) / bn;
  if (result == HX_OK && info->rel_residual > o.rtol) result = fail(HX_ENOCONV, "PCG reached maxit without meeting rtol");
  return result;
}
