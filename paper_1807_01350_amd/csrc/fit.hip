// Fitness terms of Sec. 5.1 over dense slices: sum (X - [[A,B,C]])^2 and
// sum X^2, accumulated in FP64 with a fixed reduction order (deterministic).
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int MAXR = 32;

// Block b handles rows (k, i) = b, b + nparts, ... of the t*I slice rows.
template <typename T>
__global__ __launch_bounds__(256) void fit_kernel(const T* __restrict__ X, int64_t t, int64_t I,
                                                  int64_t J, int R, int64_t k0,
                                                  const double* __restrict__ A,
                                                  const double* __restrict__ B,
                                                  const double* __restrict__ C,
                                                  double* __restrict__ partials) {
  __shared__ double ac[MAXR];
  __shared__ double r1[256], r2[256];
  const int tid = threadIdx.x;
  double sse = 0.0, nx = 0.0;
  const int64_t rows = t * I;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int64_t k = row / I, i = row % I;
    __syncthreads();
    if (tid < R) ac[tid] = A[i * R + tid] * C[(k0 + k) * R + tid];
    __syncthreads();
    const T* x = X + row * J;
    for (int64_t j = tid; j < J; j += 256) {
      double xh = 0.0;
      for (int r = 0; r < R; ++r) xh = fma(ac[r], B[j * R + r], xh);
      const double xv = (double)x[j];
      const double d = xv - xh;
      sse = fma(d, d, sse);
      nx = fma(xv, xv, nx);
    }
  }
  r1[tid] = sse;
  r2[tid] = nx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) { r1[tid] += r1[tid + w]; r2[tid] += r2[tid + w]; }
    __syncthreads();
  }
  if (tid == 0) { partials[2 * blockIdx.x] = r1[0]; partials[2 * blockIdx.x + 1] = r2[0]; }
}

__global__ __launch_bounds__(256) void fit_reduce(const double* __restrict__ partials, int n,
                                                  double* __restrict__ out) {
  __shared__ double r1[256], r2[256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int e = tid; e < n; e += 256) { a += partials[2 * e]; b += partials[2 * e + 1]; }
  r1[tid] = a;
  r2[tid] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) { r1[tid] += r1[tid + w]; r2[tid] += r2[tid + w]; }
    __syncthreads();
  }
  if (tid == 0) { out[0] = r1[0]; out[1] = r2[0]; }
}

}  // namespace

hipError_t fit_dense(hipStream_t s, const void* X, bool x_f64, int64_t t, int64_t I, int64_t J,
                     int R, int64_t k0, const double* A, const double* B, const double* C,
                     double* partials, int nparts, double* out2) {
  if (R > MAXR) return hipErrorInvalidValue;
  if (x_f64)
    hipLaunchKernelGGL(fit_kernel<double>, dim3(nparts), dim3(256), 0, s, (const double*)X, t, I,
                       J, R, k0, A, B, C, partials);
  else
    hipLaunchKernelGGL(fit_kernel<float>, dim3(nparts), dim3(256), 0, s, (const float*)X, t, I, J,
                       R, k0, A, B, C, partials);
  hipLaunchKernelGGL(fit_reduce, dim3(1), dim3(256), 0, s, partials, nparts, out2);
  return hipGetLastError();
}

}  // namespace octen
