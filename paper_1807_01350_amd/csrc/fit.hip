// Fitness terms of Sec. 5.1 over dense slices: sum (X - [[A,B,C]])^2 and
// sum X^2, accumulated in FP64 with a fixed reduction order (deterministic).
#include <hip/hip_runtime.h>

#include <mutex>

#include "octen.h"
#include "octen_internal.h"

// Partial sums of octen_fit_noalloc: 2 doubles per block of fit_kernel, then
// the 2 reduced terms.  The library holds this array on every device it runs
// on until the process ends; host code reaches it only through the address
// taken by hipGetSymbolAddress (the array's name is not a device address in
// host code).
constexpr int NOALLOC_PARTS = 2048;
static __device__ __align__(256) double scratch[2 * NOALLOC_PARTS + 2];

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

namespace octen {
namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, taken once per device.
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace octen

extern "C" octen_status octen_fit_noalloc(const void* X, int32_t x_dtype, int64_t t, int64_t I,
                                          int64_t J, int32_t R, int64_t k0, const double* A,
                                          const double* B, const double* C, void* stream,
                                          double* out_host) {
  if (!X || !A || !B || !C || !out_host) return OCTEN_ERR_ARG;
  if (t < 1 || I < 1 || J < 1 || k0 < 0 || R < 1 || R > 32) return OCTEN_ERR_ARG;
  if (x_dtype != OCTEN_F64 && x_dtype != OCTEN_F32) return OCTEN_ERR_ARG;
  if (I > ((int64_t)1 << 40) / t) return OCTEN_ERR_ARG;   // t * I rows must stay addressable
  double* sp = nullptr;
  if (octen::scratch_address(&sp) != hipSuccess) return OCTEN_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  const int64_t rows = t * I;
  // the grid never exceeds the array: at most NOALLOC_PARTS partial pairs;
  // every pair is written before fit_reduce reads it, so nothing is cleared
  const int parts = rows < NOALLOC_PARTS ? (int)rows : NOALLOC_PARTS;
  double* partials = sp;
  double* terms = sp + 2 * NOALLOC_PARTS;
  if (octen::fit_dense(s, X, x_dtype == OCTEN_F64, t, I, J, R, k0, A, B, C, partials, parts,
                       terms) != hipSuccess)
    return OCTEN_ERR_HIP;
  double o[2];
  if (hipMemcpyAsync(o, terms, sizeof(o), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return OCTEN_ERR_HIP;
  out_host[0] += o[0];
  out_host[1] += o[1];
  return OCTEN_OK;
}
