// Two-layer tanh network y = W2 tanh(W1 x + b1) + b2: FP32 training (forward, loss, backward,
// Adam) and bf16 matrix-core inference, all in kernels of this file.
//
// Not in the paper: the network is the element-local learned preconditioner added on top of
// the method. Loss: mean squared error over every output entry of a batch. Adam: Kingma and
// Ba (2015), with bias correction. Reductions (bias gradients, loss) are deterministic.
#include <type_traits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "mlp_internal.h"

namespace hx {

namespace {

constexpr int TS = 64;   // FP32 GEMM tile (M and N)
constexpr int TK = 16;   // FP32 GEMM tile (K)

enum { EPI_STORE = 0, EPI_BIAS_TANH = 1, EPI_BIAS = 2, EPI_DTANH = 3 };

// C[M x N] = op(A)[M x K] * op(B)[K x N], then the epilogue:
//   EPI_BIAS_TANH: tanh(acc + bias[n]); EPI_BIAS: acc + bias[n];
//   EPI_DTANH: acc * (1 - aux[m, n]^2) (aux: the tanh activations, ldc layout).
// op(A)(m, k) = TA ? A[k * lda + m] : A[m * lda + k]; op(B)(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n].
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256)
    k_sgemm(int M, int N, int K, const float *__restrict__ A, int lda, const float *__restrict__ B, int ldb,
            float *__restrict__ C, int ldc, const float *__restrict__ bias, const float *__restrict__ aux) {
  __shared__ float As[TK][TS + 1], Bs[TK][TS + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * TS, n0 = blockIdx.x * TS;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int t = tid; t < TK * TS; t += 256) {
      const int kk = t / TS, mm = t % TS;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? (TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k]) : 0.f;
      const int n = n0 + mm;
      Bs[kk][mm] = (n < N && k < K) ? (TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[kk][ty * 4 + i];
        b[i] = Bs[kk][tx * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= N) continue;
      float v = acc[i][j];
      if (EPI == EPI_BIAS_TANH) v = tanhf(v + bias[n]);
      if (EPI == EPI_BIAS) v = v + bias[n];
      if (EPI == EPI_DTANH) {
        const float h = aux[(int64_t)m * ldc + n];
        v = v * (1.f - h * h);
      }
      C[(int64_t)m * ldc + n] = v;
    }
  }
}

template <bool TA, bool TB, int EPI>
void sgemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
           const float *bias, const float *aux, hipStream_t s) {
  dim3 grid((N + TS - 1) / TS, (M + TS - 1) / TS);
  hipLaunchKernelGGL((k_sgemm<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, aux);
}

// out[n] = sum_m A[m * N + n] (fixed order per column)
__global__ void k_colsum(int M, int N, const float *__restrict__ A, float *__restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += A[(int64_t)m * N + n];
  out[n] = s;
}

// dY = 2 (Y - T) / count; per-block partial sums of (Y - T)^2
__global__ void __launch_bounds__(256) k_mse(int64_t n, const float *__restrict__ Y, const float *__restrict__ T,
                                               float *__restrict__ dY, float inv_count, double *__restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[t] - T[t];
    dY[t] = 2.f * d * inv_count;
    s += (double)d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(int nb, const double *__restrict__ part, double scale, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[i];
    *out = s * scale;
  }
}

// Adam with bias correction: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr mhat / (sqrt(vhat) + eps)
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
  }
}

// rows of src (width w) picked by rows[] into dst
__global__ void k_gather_rows(int64_t nrows, int w, const int32_t *__restrict__ rows, const float *__restrict__ src,
                              float *__restrict__ dst) {
  const int64_t total = nrows * w;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / w, c = t - r * w;
    dst[t] = src[(int64_t)rows[r] * w + c];
  }
}

__global__ void k_f2bf(int64_t n, const float *__restrict__ a, uint16_t *__restrict__ b) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = f32_to_bf16_bits(a[t]);
}

// bf16 matrix-core forward of one layer: Out[M x N] = act(In[M x K] W^T + bias), W (N x K) bf16, both
// row-major. gfx950's 16x16x32 bf16 product: lane l holds A[l%16][8(l/16) + t] and B[8(l/16) + t][l%16]
// (t < 8) and receives D[4(l/16) + t][l%16] (t < 4) (layout checked on the device). One wavefront owns
// 16 rows and NT tiles of 16 output columns, so a layer runs ceil(M/16) ceil(N/16 NT) wavefronts; per
// 32-wide step of K a lane loads its 8 input values and, per tile, the 8 weights of its column, each as
// one 16-byte load when K is a multiple of 8 (the rows are then 16-byte aligned). The input is FP32
// (converted in registers) or bf16.
template <typename TIN>
__device__ __forceinline__ bf16x8 load8_bf16(const TIN *__restrict__ p, bool full, int valid) {
  bf16x8 v;
  if constexpr (std::is_same<TIN, uint16_t>::value) {
    if (full) {
      const uint4 q = *reinterpret_cast<const uint4 *>(p);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        v[2 * t] = (short)(w[t] & 0xffffu);
        v[2 * t + 1] = (short)(w[t] >> 16);
      }
      return v;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = t < valid ? (short)p[t] : (short)0;
  } else {
    if (full) {
      const float4 q0 = *reinterpret_cast<const float4 *>(p), q1 = *reinterpret_cast<const float4 *>(p + 4);
      const float f[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = (short)f32_to_bf16_bits(f[t]);
      return v;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = t < valid ? (short)f32_to_bf16_bits(p[t]) : (short)0;
  }
  return v;
}

template <typename TIN, bool TANH, typename TOUT, int NT, int RT, int U>
__global__ void __launch_bounds__(256)
    k_layer_bf16(int64_t M, int N, int K, const TIN *__restrict__ In, const uint16_t *__restrict__ W,
                 const float *__restrict__ bias, const float *__restrict__ row_scale, TOUT *__restrict__ Out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // RT tiles of 16 rows share every weight load; consecutive blocks take the column groups of one row block
  const int64_t m0 = ((int64_t)blockIdx.y * 4 + wave) * 16 * RT;
  const int n0 = blockIdx.x * (16 * NT);
  if (m0 >= M) return;  // whole wavefront exits together
  const int r = lane & 15, kq = 8 * (lane >> 4);
  const bool vec = (K & 7) == 0;
  f32x4 acc[RT][NT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  // U steps of 32 along K per iteration: every load of the U steps is issued before their products
  for (int kb0 = 0; kb0 < K; kb0 += 32 * U) {
    bf16x8 a[U][RT], b[U][NT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb0 + 32 * u + kq, valid = K - k;  // this lane's 8 values along K: k .. k + 7
      const bool full = vec && valid >= 8;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int64_t row = m0 + 16 * i + r;
        a[u][i] = (row < M && valid > 0) ? load8_bf16<TIN>(In + row * K + k, full, valid) : zero8;
      }
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int n = n0 + j * 16 + r;  // lane's column in this tile
        b[u][j] = (n < N && valid > 0) ? load8_bf16<uint16_t>(W + (int64_t)n * K + k, full, valid) : zero8;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int i = 0; i < RT; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a[u][i]),
                                                              __builtin_bit_cast(bf16x8_t, b[u][j]), acc[i][j], 0, 0, 0);
  }
  // accumulator: lane holds rows m0 + 16 i + 4 (lane / 16) + t of column n0 + 16 j + r
  const int rb = 4 * (lane >> 4);
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int n = n0 + j * 16 + r;
      if (n >= N) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t m = m0 + 16 * i + rb + t;
        if (m >= M) continue;
        float v = acc[i][j][t] + bias[n];
        if (TANH) v = tanhf(v);
        if (row_scale) v *= row_scale[m];
        store_as(Out + m * N + n, v);
      }
    }
}

// A layer with at most 16 NT outputs (the hidden layer): a workgroup takes 64 rows, 16 per
// wavefront, and every output column, so each input row is read once; per chunk of KC = 32 U values
// along K the weights of all columns are staged in LDS once for the four wavefronts (rows padded to
// KC + 8 values: the 16 lanes of one row group read 16 distinct banks quadruples). Lane layout of
// the products and the epilogue as in k_layer_bf16.
template <typename TIN, bool TANH, typename TOUT, int NT, int U>
__global__ void __launch_bounds__(256)
    k_layer_wide(int64_t M, int N, int K, const TIN *__restrict__ In, const uint16_t *__restrict__ W,
                 const float *__restrict__ bias, const float *__restrict__ row_scale, TOUT *__restrict__ Out) {
  constexpr int KC = 32 * U, KP = KC + 8, SEGS = KC / 8;
  __shared__ __align__(16) uint16_t Bs[NT * 16][KP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const int r = lane & 15, kq = 8 * (lane >> 4);
  const bool vec = (K & 7) == 0;
  const int64_t row = m0 + r;
  const bf16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  f32x4 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kb0 = 0; kb0 < K; kb0 += KC) {
    // this wavefront's input values of the chunk, requested before the weights are staged
    bf16x8 a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb0 + 32 * u + kq, valid = K - k;
      a[u] = (row < M && valid > 0) ? load8_bf16<TIN>(In + row * K + k, vec && valid >= 8, valid) : zero8;
    }
    __syncthreads();  // every wavefront is done with the previous chunk's weights
    for (int t = threadIdx.x; t < NT * 16 * SEGS; t += 256) {
      const int n = t / SEGS, k8 = (t - n * SEGS) * 8, k = kb0 + k8, valid = K - k;
      const bf16x8 v = (n < N && valid > 0) ? load8_bf16<uint16_t>(W + (int64_t)n * K + k, vec && valid >= 8, valid)
                                            : zero8;
      *reinterpret_cast<bf16x8 *>(&Bs[n][k8]) = v;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[j * 16 + r][32 * u + kq]);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a[u]),
                                                         __builtin_bit_cast(bf16x8_t, b), acc[j], 0, 0, 0);
      }
  }
  const int rb = 4 * (lane >> 4);
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int n = j * 16 + r;
    if (n >= N) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t m = m0 + rb + t;
      if (m >= M) continue;
      float v = acc[j][t] + bias[n];
      if (TANH) v = tanhf(v);
      if (row_scale) v *= row_scale[m];
      store_as(Out + m * N + n, v);
    }
  }
}

// launch one layer: NT = 2 column tiles and RT = 4 row tiles per wavefront up to 128 columns, else 4 and 2;
// loads of U = 4 K steps in flight for K > 256, else 1; row_scale (optional) multiplies output row m
template <typename TIN, bool TANH, typename TOUT>
void launch_layer(int64_t M, int N, int K, const TIN *In, const uint16_t *W, const float *bias, TOUT *Out,
                  hipStream_t s, const float *row_scale = nullptr) {
  if (N <= 128) {
    const dim3 g((unsigned)((N + 31) / 32), (unsigned)((M + 255) / 256));
    if (K > 256)
      hipLaunchKernelGGL((k_layer_bf16<TIN, TANH, TOUT, 2, 4, 4>), g, dim3(256), 0, s, M, N, K, In, W, bias, row_scale,
                         Out);
    else
      hipLaunchKernelGGL((k_layer_bf16<TIN, TANH, TOUT, 2, 4, 1>), g, dim3(256), 0, s, M, N, K, In, W, bias, row_scale,
                         Out);
  } else {
    const dim3 g((unsigned)((N + 63) / 64), (unsigned)((M + 127) / 128));
    if (K > 256)
      hipLaunchKernelGGL((k_layer_bf16<TIN, TANH, TOUT, 4, 2, 4>), g, dim3(256), 0, s, M, N, K, In, W, bias, row_scale,
                         Out);
    else
      hipLaunchKernelGGL((k_layer_bf16<TIN, TANH, TOUT, 4, 2, 1>), g, dim3(256), 0, s, M, N, K, In, W, bias, row_scale,
                         Out);
  }
}

}  // namespace

hx_status mlp_layers_bf16(hx_mlp_s &net, const uint16_t *X16, int64_t batch, uint16_t *H16, float *Y, hipStream_t s,
                          const float *row_scale) {
  if (hx_status st = mlp_refresh_bf16(net, s)) return st;
  // the hidden layer: every column per workgroup, weights shared through LDS, where there are rows
  // for more than about 1.25 workgroups per CU (below that, fewer rows per wavefront group win:
  // 15.6k rows, p = 7, 0.167 against 0.176 ms per map; 24.4k, p = 6, 0.309 against 0.220)
  if (net.n_hid <= 128 && batch >= 20000)
    hipLaunchKernelGGL((k_layer_wide<uint16_t, true, uint16_t, 8, 4>), dim3((unsigned)((batch + 63) / 64)), dim3(256),
                       0, s, batch, net.n_hid, net.n_in, X16, net.W1b.ptr, net.p.ptr + net.off_b1, nullptr, H16);
  else
    launch_layer<uint16_t, true, uint16_t>(batch, net.n_hid, net.n_in, X16, net.W1b.ptr, net.p.ptr + net.off_b1, H16,
                                           s);
  launch_layer<uint16_t, false, float>(batch, net.n_out, net.n_hid, H16, net.W2b.ptr, net.p.ptr + net.off_b2, Y, s,
                                       row_scale);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

hx_status mlp_forward_bf16(hx_mlp_s &net, const float *X, int64_t batch, float *Y, hipStream_t s) {
  if (hx_status st = mlp_refresh_bf16(net, s)) return st;
  if (net.act16.count < (size_t)(batch * net.n_hid)) HX_HIP(net.act16.alloc((size_t)batch * net.n_hid));
  launch_layer<float, true, uint16_t>(batch, net.n_hid, net.n_in, X, net.W1b.ptr, net.p.ptr + net.off_b1,
                                     net.act16.ptr, s);
  launch_layer<uint16_t, false, float>(batch, net.n_out, net.n_hid, net.act16.ptr, net.W2b.ptr, net.p.ptr + net.off_b2,
                                       Y, s);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

hx_status mlp_refresh_bf16(hx_mlp_s &net, hipStream_t s) {
  if (net.bf16_valid) return HX_OK;
  if (!net.W1b.ptr) {
    HX_HIP(net.W1b.alloc((size_t)net.n_hid * net.n_in));
    HX_HIP(net.W2b.alloc((size_t)net.n_out * net.n_hid));
  }
  hipLaunchKernelGGL(k_f2bf, dim3(256), dim3(256), 0, s, (int64_t)net.n_hid * net.n_in, net.p.ptr + net.off_W1,
                     net.W1b.ptr);
  hipLaunchKernelGGL(k_f2bf, dim3(256), dim3(256), 0, s, (int64_t)net.n_out * net.n_hid, net.p.ptr + net.off_W2,
                     net.W2b.ptr);
  HX_HIP(hipGetLastError());
  net.bf16_valid = true;
  return HX_OK;
}

// FP32 forward into net.Z/Hact/Y work buffers (batch rows of X)
static hx_status forward_f32(hx_mlp_s &net, const float *X, int64_t B, float *Y, hipStream_t s) {
  if (net.hact.count < (size_t)(B * net.n_hid)) HX_HIP(net.hact.alloc((size_t)B * net.n_hid));
  const float *W1 = net.p.ptr + net.off_W1, *b1 = net.p.ptr + net.off_b1;
  const float *W2 = net.p.ptr + net.off_W2, *b2 = net.p.ptr + net.off_b2;
  // H = tanh(X W1^T + b1)
  sgemm<false, true, EPI_BIAS_TANH>((int)B, net.n_hid, net.n_in, X, net.n_in, W1, net.n_in, net.hact.ptr, net.n_hid,
                                    b1, nullptr, s);
  // Y = H W2^T + b2
  sgemm<false, true, EPI_BIAS>((int)B, net.n_out, net.n_hid, net.hact.ptr, net.n_hid, W2, net.n_hid, Y, net.n_out, b2,
                               nullptr, s);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

// loss and gradients of one batch into net.g (same layout as net.p); loss (device double) if non-null
static hx_status loss_grad(hx_mlp_s &net, const float *X, const float *T, int64_t B, double *loss_dev, hipStream_t s) {
  if (net.yout.count < (size_t)(B * net.n_out)) HX_HIP(net.yout.alloc((size_t)B * net.n_out));
  if (net.dy.count < (size_t)(B * net.n_out)) HX_HIP(net.dy.alloc((size_t)B * net.n_out));
  if (net.dz.count < (size_t)(B * net.n_hid)) HX_HIP(net.dz.alloc((size_t)B * net.n_hid));
  if (hx_status st = forward_f32(net, X, B, net.yout.ptr, s)) return st;
  const int64_t cnt = B * net.n_out;
  const int nb = 256;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, cnt, net.yout.ptr, T, net.dy.ptr, 1.f / (float)cnt,
                     net.part.ptr);
  if (loss_dev) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, s, nb, net.part.ptr, 1.0 / (double)cnt, loss_dev);
  float *g = net.g.ptr;
  const float *W2 = net.p.ptr + net.off_W2;
  // gW2 = dY^T H (O x H), gb2 = colsum(dY)
  sgemm<true, false, EPI_STORE>(net.n_out, net.n_hid, (int)B, net.dy.ptr, net.n_out, net.hact.ptr, net.n_hid,
                                g + net.off_W2, net.n_hid, nullptr, nullptr, s);
  hipLaunchKernelGGL(k_colsum, dim3((net.n_out + 255) / 256), dim3(256), 0, s, (int)B, net.n_out, net.dy.ptr,
                     g + net.off_b2);
  // dZ = (dY W2) * (1 - H^2)   (B x H)
  sgemm<false, false, EPI_DTANH>((int)B, net.n_hid, net.n_out, net.dy.ptr, net.n_out, W2, net.n_hid, net.dz.ptr,
                                 net.n_hid, nullptr, net.hact.ptr, s);
  // gW1 = dZ^T X (H x I), gb1 = colsum(dZ)
  sgemm<true, false, EPI_STORE>(net.n_hid, net.n_in, (int)B, net.dz.ptr, net.n_hid, X, net.n_in, g + net.off_W1,
                                net.n_in, nullptr, nullptr, s);
  hipLaunchKernelGGL(k_colsum, dim3((net.n_hid + 255) / 256), dim3(256), 0, s, (int)B, net.n_hid, net.dz.ptr,
                     g + net.off_b1);
  HX_HIP(hipGetLastError());
  return HX_OK;
}

}  // namespace hx

using namespace hx;

// ------------------------------------------------------------------ ABI
extern "C" hx_status hx_mlp_create(int n_in, int n_hidden, int n_out, uint64_t seed, hx_mlp *out) {
  if (!out) return fail(HX_EINVAL, "out is null");
  *out = nullptr;
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || n_in > (1 << 16) || n_hidden > (1 << 12) || n_out > (1 << 16))
    return fail(HX_EINVAL, "network sizes out of range");
  auto *net = new (std::nothrow) hx_mlp_s();
  if (!net) return fail(HX_ENOMEM, "host allocation failed");
  net->n_in = n_in;
  net->n_hid = n_hidden;
  net->n_out = n_out;
  net->off_W1 = 0;
  net->off_b1 = (int64_t)n_hidden * n_in;
  net->off_W2 = net->off_b1 + n_hidden;
  net->off_b2 = net->off_W2 + (int64_t)n_out * n_hidden;
  net->nparam = net->off_b2 + n_out;
  // uniform(-1, 1) / sqrt(fan_in) weights, zero biases
  std::vector<float> h(net->nparam, 0.f);
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (int64_t t = 0; t < net->off_b1; ++t) h[t] = (float)(U(rng) / std::sqrt((double)n_in));
  for (int64_t t = net->off_W2; t < net->off_b2; ++t) h[t] = (float)(U(rng) / std::sqrt((double)n_hidden));
  hipError_t e;
  if ((e = net->p.upload(h.data(), h.size())) != hipSuccess || (e = net->g.alloc(net->nparam)) != hipSuccess ||
      (e = net->part.alloc(256)) != hipSuccess) {
    delete net;
    return hip_fail(e, "network allocation");
  }
  *out = net;
  return HX_OK;
}

extern "C" void hx_mlp_destroy(hx_mlp net) { delete net; }

extern "C" hx_status hx_mlp_get_shape(hx_mlp net, int *n_in, int *n_hidden, int *n_out) {
  if (!net) return fail(HX_EINVAL, "null network");
  if (n_in) *n_in = net->n_in;
  if (n_hidden) *n_hidden = net->n_hid;
  if (n_out) *n_out = net->n_out;
  return HX_OK;
}

extern "C" hx_status hx_mlp_set_params(hx_mlp net, const float *params) {
  if (!net || !params) return fail(HX_EINVAL, "null argument");
  HX_HIP(hipMemcpy(net->p.ptr, params, sizeof(float) * net->nparam, hipMemcpyHostToDevice));
  net->bf16_valid = false;
  net->adam_t = 0;
  return HX_OK;
}

extern "C" hx_status hx_mlp_get_params(hx_mlp net, float *params) {
  if (!net || !params) return fail(HX_EINVAL, "null argument");
  HX_HIP(hipMemcpy(params, net->p.ptr, sizeof(float) * net->nparam, hipMemcpyDeviceToHost));
  return HX_OK;
}

extern "C" hx_status hx_mlp_forward(hx_mlp net, int prec, const float *X, int64_t batch, float *Y, hx_stream stream) {
  if (!net || !X || !Y) return fail(HX_EINVAL, "null argument");
  if (batch < 1 || batch > INT32_MAX) return fail(HX_EINVAL, "batch out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (prec == HX_FP32) return forward_f32(*net, X, batch, Y, s);
  if (prec == HX_BF16) return mlp_forward_bf16(*net, X, batch, Y, s);
  return fail(HX_EINVAL, "prec must be HX_FP32 or HX_BF16");
}

extern "C" hx_status hx_mlp_loss_grad(hx_mlp net, const float *X, const float *T, int64_t batch, double *loss,
                                      float *grads, hx_stream stream) {
  if (!net || !X || !T) return fail(HX_EINVAL, "null argument");
  if (batch < 1 || batch > INT32_MAX) return fail(HX_EINVAL, "batch out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf<double> dl;
  HX_HIP(dl.alloc(1));
  if (hx_status st = loss_grad(*net, X, T, batch, dl.ptr, s)) return st;
  if (loss) HX_HIP(hipMemcpyAsync(loss, dl.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grads) HX_HIP(hipMemcpyAsync(grads, net->g.ptr, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, s));
  HX_HIP(hipStreamSynchronize(s));
  return HX_OK;
}

extern "C" void hx_train_opts_default(hx_train_opts *o) {
  if (!o) return;
  o->epochs = 200;
  o->batch = 256;
  o->lr = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
  o->seed = 7;
}

extern "C" hx_status hx_mlp_train(hx_mlp net, const float *X, const float *T, int64_t nsamples,
                                  const hx_train_opts *opts, hx_train_info *info, hx_stream stream) {
  if (!net || !X || !T || !opts || !info) return fail(HX_EINVAL, "null argument");
  if (nsamples < 1 || nsamples > INT32_MAX) return fail(HX_EINVAL, "nsamples out of range");
  const hx_train_opts &o = *opts;
  if (o.epochs < 1 || o.batch < 1 || !(o.lr > 0)) return fail(HX_EINVAL, "epochs, batch >= 1 and lr > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  *info = hx_train_info{};
  const int64_t B = std::min<int64_t>(o.batch, nsamples);
  DevBuf<float> xb, tb, m, v;
  DevBuf<int32_t> rows;
  DevBuf<double> loss_dev;
  HX_HIP(xb.alloc((size_t)B * net->n_in));
  HX_HIP(tb.alloc((size_t)B * net->n_out));
  HX_HIP(m.alloc(net->nparam));
  HX_HIP(v.alloc(net->nparam));
  HX_HIP(hipMemsetAsync(m.ptr, 0, sizeof(float) * net->nparam, s));
  HX_HIP(hipMemsetAsync(v.ptr, 0, sizeof(float) * net->nparam, s));
  HX_HIP(rows.alloc((size_t)nsamples));
  HX_HIP(loss_dev.alloc((size_t)o.epochs));
  std::vector<int32_t> perm(nsamples);
  for (int64_t t = 0; t < nsamples; ++t) perm[t] = (int32_t)t;
  std::mt19937_64 rng(o.seed);
  const auto t0 = std::chrono::steady_clock::now();
  int64_t step = 0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    HX_HIP(hipMemcpyAsync(rows.ptr, perm.data(), sizeof(int32_t) * nsamples, hipMemcpyHostToDevice, s));
    // the copy reads perm from the host: finish it before the next shuffle
    HX_HIP(hipStreamSynchronize(s));
    for (int64_t b0 = 0; b0 + B <= nsamples; b0 += B) {
      hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, s, B, net->n_in, rows.ptr + b0, X, xb.ptr);
      hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, s, B, net->n_out, rows.ptr + b0, T, tb.ptr);
      // the last batch of an epoch records the epoch's loss
      const bool last = b0 + 2 * B > nsamples;
      if (hx_status st = loss_grad(*net, xb.ptr, tb.ptr, B, last ? loss_dev.ptr + ep : nullptr, s)) return st;
      ++step;
      const float c1 = (float)(1.0 - std::pow(o.beta1, (double)step));
      const float c2 = (float)(1.0 - std::pow(o.beta2, (double)step));
      hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, s, net->nparam, net->p.ptr, net->g.ptr, m.ptr, v.ptr,
                         (float)o.lr, (float)o.beta1, (float)o.beta2, (float)o.eps, c1, c2);
    }
    HX_HIP(hipGetLastError());
  }
  std::vector<double> losses(o.epochs);
  HX_HIP(hipMemcpyAsync(losses.data(), loss_dev.ptr, sizeof(double) * o.epochs, hipMemcpyDeviceToHost, s));
  HX_HIP(hipStreamSynchronize(s));
  net->bf16_valid = false;
  info->steps = step;
  info->first_loss = losses.front();
  info->final_loss = losses.back();
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return HX_OK;
}

// file: "HXMLP1\0\0", int32 n_in, n_hidden, n_out, reserved; then the FP32 parameters (W1, b1, W2, b2)
extern "C" hx_status hx_mlp_save(hx_mlp net, const char *path) {
  if (!net || !path) return fail(HX_EINVAL, "null argument");
  std::vector<float> h(net->nparam);
  HX_HIP(hipMemcpy(h.data(), net->p.ptr, sizeof(float) * net->nparam, hipMemcpyDeviceToHost));
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(HX_EINVAL, std::string("cannot open ") + path);
  const char magic[8] = {'H', 'X', 'M', 'L', 'P', '1', 0, 0};
  const int32_t hdr[4] = {net->n_in, net->n_hid, net->n_out, 0};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
            std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HX_OK : fail(HX_EINVAL, std::string("write failed: ") + path);
}

extern "C" hx_status hx_mlp_load(const char *path, hx_mlp *out) {
  if (!path || !out) return fail(HX_EINVAL, "null argument");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(HX_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[4];
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "HXMLP1", 6) != 0 || std::fread(hdr, 4, 4, f) != 4) {
    std::fclose(f);
    return fail(HX_EINVAL, "not a network file");
  }
  hx_mlp net = nullptr;
  if (hx_status st = hx_mlp_create(hdr[0], hdr[1], hdr[2], 0, &net)) {
    std::fclose(f);
    return st;
  }
  std::vector<float> h(net->nparam);
  const bool ok = std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
  std::fclose(f);
  if (!ok) {
    hx_mlp_destroy(net);
    return fail(HX_EINVAL, "truncated network file");
  }
  if (hx_status st = hx_mlp_set_params(net, h.data())) {
    hx_mlp_destroy(net);
    return st;
  }
  *out = net;
  return HX_OK;
}
