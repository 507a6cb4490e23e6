// Residual MLP of the learned warm start: forward, backward and Adam.
//
//   y = x[:, :n_out] + W3 relu(W2 relu(W1 x + b1) + b2) + b3     (row-wise)
//
// Parameters live in one FP32 buffer (the master copy), in the order
// W1 [H][In], b1 [H], W2 [H][H], b2 [H], W3 [Out][H], b3 [Out]; gradients
// and the Adam moments use the same layout.  Every product runs on
// v_mfma_f32_32x32x16_bf16: operands are rounded to BF16 (nearest even) as
// they are loaded, accumulation is FP32.  Each workgroup computes a 64 x 64
// block of C = A B with four wavefronts of 32 x 32; A and B are addressed
// through strides, so the transposed products of the backward pass need no
// copies.  Epilogues fuse the bias, the rectifier, the residual and the
// rectifier mask of the backward pass.
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

typedef __bf16 bf16x8m __attribute__((ext_vector_type(8)));
typedef float f32x16m __attribute__((ext_vector_type(16)));

namespace {

constexpr int NT = 256;

struct GemmArgs {
  int M, N, K;
  const float* A; int64_t sam, sak;   // A(m, k) = A[m * sam + k * sak]
  const float* B; int64_t sbk, sbn;   // B(k, n) = B[k * sbk + n * sbn]
  float* C; int64_t ldc;              // C(m, n) = C[m * ldc + n]
  const float* bias;                  // [N]
  const float* aux; int64_t ldaux;    // residual input or rectified activation
};

// epilogues
enum { EPI_STORE = 0, EPI_BIAS_RELU = 1, EPI_BIAS_RESID = 2, EPI_MASK = 3 };

// lane l supplies A rows l % 32 with k = 8 (l / 32) .. + 7, the same for the
// columns of B; element i of the result belongs to row 8 (i / 4) +
// 4 (l / 32) + i % 4 and column l % 32 of the 32 x 32 tile.
template <int EPI>
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(GemmArgs g) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int tm = blockIdx.x * 64 + (wave / 2) * 32;
  const int tn = blockIdx.y * 64 + (wave % 2) * 32;
  const int row = tm + lane % 32, col = tn + lane % 32;
  const int kh = 8 * (lane / 32);
  const bool rok = row < g.M, cok = col < g.N;
  const float* Ar = g.A + (int64_t)(rok ? row : 0) * g.sam;
  const float* Bc = g.B + (int64_t)(cok ? col : 0) * g.sbn;
  f32x16m acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x8m a, b;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + kh + q;
      const bool kok = k < g.K;
      a[q] = (__bf16)((rok && kok) ? Ar[(int64_t)k * g.sak] : 0.f);
      b[q] = (__bf16)((cok && kok) ? Bc[(int64_t)k * g.sbk] : 0.f);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = tm + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
    if (r < g.M && cok) {
      float v = acc[i];
      if constexpr (EPI == EPI_BIAS_RELU) {
        v += g.bias[col];
        v = v > 0.f ? v : 0.f;
      } else if constexpr (EPI == EPI_BIAS_RESID) {
        v += g.bias[col] + g.aux[(int64_t)r * g.ldaux + col];
      } else if constexpr (EPI == EPI_MASK) {
        v = g.aux[(int64_t)r * g.ldaux + col] > 0.f ? v : 0.f;
      }
      g.C[(int64_t)r * g.ldc + col] = v;
    }
  }
}

// out[c] = sum over rows of X[r][c], rows in order (deterministic)
__global__ void colsum_kernel(const float* __restrict__ X, int64_t n, int m,
                              float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  float s = 0.f;
  for (int64_t r = 0; r < n; ++r) s += X[r * m + c];
  out[c] = s;
}

// dY = 2 (Y - T) / (n m); block partial sums of (Y - T)^2 in FP64
__global__ __launch_bounds__(NT) void mse_kernel(const float* __restrict__ Y,
                                                 const float* __restrict__ T, int64_t cnt,
                                                 float* __restrict__ dY,
                                                 double* __restrict__ partials) {
  __shared__ double red[NT];
  const float scale = 2.f / (float)cnt;
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * NT) {
    const float d = Y[e] - T[e];
    dY[e] = scale * d;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void sum_kernel(const double* __restrict__ partials, int n,
                                                 double scale, double* __restrict__ out) {
  __shared__ double red[NT];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += NT) s += partials[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// Adam (Kingma and Ba, Algorithm 1) on the FP32 master parameters;
// c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float beta1, float beta2, float eps, float c1, float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = beta1 * m[e] + (1.f - beta1) * ge;
    const float ve = beta2 * v[e] + (1.f - beta2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

template <int EPI>
hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, int64_t sam, int64_t sak,
                const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                const float* bias = nullptr, const float* aux = nullptr, int64_t ldaux = 0) {
  if (M <= 0 || N <= 0) return hipSuccess;
  GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, aux, ldaux};
  const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL(gemm_bf16_kernel<EPI>, grid, dim3(NT), 0, s, g);
  return hipGetLastError();
}

}  // namespace

int64_t mlp_param_count(int nin, int nh, int nout) {
  return (int64_t)nh * nin + nh + (int64_t)nh * nh + nh + (int64_t)nout * nh + nout;
}

MlpLayout mlp_layout(int nin, int nh, int nout) {
  MlpLayout L;
  L.nin = nin; L.nh = nh; L.nout = nout;
  L.W1 = 0;
  L.b1 = L.W1 + (int64_t)nh * nin;
  L.W2 = L.b1 + nh;
  L.b2 = L.W2 + (int64_t)nh * nh;
  L.W3 = L.b2 + nh;
  L.b3 = L.W3 + (int64_t)nout * nh;
  L.total = L.b3 + nout;
  return L;
}

hipError_t mlp_forward(hipStream_t s, const MlpLayout& L, const float* w, const float* X, int64_t n,
                       float* H1, float* H2, float* Y) {
  const int nin = L.nin, nh = L.nh, nout = L.nout;
  hipError_t e = gemm<EPI_BIAS_RELU>(s, (int)n, nh, nin, X, nin, 1, w + L.W1, 1, nin, H1, nh,
                                     w + L.b1);
  if (e == hipSuccess)
    e = gemm<EPI_BIAS_RELU>(s, (int)n, nh, nh, H1, nh, 1, w + L.W2, 1, nh, H2, nh, w + L.b2);
  if (e == hipSuccess)
    e = gemm<EPI_BIAS_RESID>(s, (int)n, nout, nh, H2, nh, 1, w + L.W3, 1, nh, Y, nout, w + L.b3,
                             X, nin);
  return e;
}

hipError_t mlp_backward(hipStream_t s, const MlpLayout& L, const float* w, const float* X,
                        int64_t n, const float* H1, const float* H2, const float* dY, float* dZ2,
                        float* dZ1, float* grad) {
  const int nin = L.nin, nh = L.nh, nout = L.nout;
  const int N = (int)n;
  // gW3 = dY^T H2, gb3 = column sums of dY
  hipError_t e = gemm<EPI_STORE>(s, nout, nh, N, dY, 1, nout, H2, nh, 1, grad + L.W3, nh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((nout + 255) / 256), dim3(256), 0, s, dY, n, nout,
                     grad + L.b3);
  // dZ2 = (dY W3) masked by H2 > 0
  e = gemm<EPI_MASK>(s, N, nh, nout, dY, nout, 1, w + L.W3, nh, 1, dZ2, nh, nullptr, H2, nh);
  if (e != hipSuccess) return e;
  e = gemm<EPI_STORE>(s, nh, nh, N, dZ2, 1, nh, H1, nh, 1, grad + L.W2, nh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((nh + 255) / 256), dim3(256), 0, s, dZ2, n, nh,
                     grad + L.b2);
  // dZ1 = (dZ2 W2) masked by H1 > 0
  e = gemm<EPI_MASK>(s, N, nh, nh, dZ2, nh, 1, w + L.W2, nh, 1, dZ1, nh, nullptr, H1, nh);
  if (e != hipSuccess) return e;
  e = gemm<EPI_STORE>(s, nh, nin, N, dZ1, 1, nh, X, nin, 1, grad + L.W1, nin);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((nh + 255) / 256), dim3(256), 0, s, dZ1, n, nh,
                     grad + L.b1);
  return hipGetLastError();
}

hipError_t mlp_mse(hipStream_t s, const float* Y, const float* T, int64_t cnt, float* dY,
                   double* partials, int nparts, double* loss) {
  int g = (int)((cnt + NT - 1) / NT);
  if (g > nparts) g = nparts;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(mse_kernel, dim3(g), dim3(NT), 0, s, Y, T, cnt, dY, partials);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(NT), 0, s, partials, g, 1.0 / (double)cnt, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t s, float* w, const float* g, float* m, float* v, int64_t n,
                    float lr, float beta1, float beta2, float eps, int64_t step) {
  const float c1 = 1.f - powf(beta1, (float)step);
  const float c2 = 1.f - powf(beta2, (float)step);
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, s, w, g, m, v, n, lr, beta1, beta2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace octen
