// Per-replica rank-R CP-ALS (Sec. 4.1: every replica summary is decomposed on
// its own; the CP model and its unfoldings are those of Sec. 2).
//
// Reference kernel: one workgroup owns one replica for the whole iteration
// loop, so no grid-wide synchronisation is needed.  MTTKRP, Gram matrices,
// the R x R Cholesky solve and the column normalisation all run in FP64.
#include <hip/hip_runtime.h>
#include <math.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int MAXR = 32;
constexpr int NT = 256;

template <typename T>
__global__ __launch_bounds__(NT) void als_ref_kernel(const T* __restrict__ Y, int Q, int R, int nch,
                                                     const double* init,
                                                     double* Fout,
                                                     double* __restrict__ lamout,
                                                     int* __restrict__ iters_out,
                                                     int* __restrict__ flags, int max_iters,
                                                     double tol) {
  extern __shared__ double sm[];
  const int QR = Q * R;
  double* F = sm;                    // [3][Q][R]
  double* part = F + 3 * QR;         // [nch][Q][R]; part[0] holds M after reduction
  double* G = part + nch * QR;       // [R][R]
  double* L = G + R * R;             // [R][R]
  double* lam = L + R * R;           // [R]
  double* red = lam + MAXR;          // [NT] reduction scratch
  __shared__ int bad;
  __shared__ double sh_nx2, sh_fit_old;
  __shared__ int have_old;

  const int p = blockIdx.x, tid = threadIdx.x;
  const int64_t Q3 = (int64_t)Q * Q * Q;
  const T* X = Y + (int64_t)p * Q3;

  for (int e = tid; e < 3 * QR; e += NT) F[e] = init[(int64_t)p * 3 * QR + e];
  if (tid < R) lam[tid] = 1.0;
  if (tid == 0) { bad = 0; sh_fit_old = 0.0; have_old = 0; }
  // ||X||^2 for the tolerance test
  double s2 = 0.0;
  if (tol > 0.0)
    for (int64_t e = tid; e < Q3; e += NT) { double v = (double)X[e]; s2 = fma(v, v, s2); }
  red[tid] = s2;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) sh_nx2 = red[0];
  __syncthreads();

  int done = 0;
  for (int it = 0; it < max_iters; ++it) {
    for (int n = 0; n < 3; ++n) {
      // ---- MTTKRP: M(q, r) = sum_{x,y} X(idx(q,x,y)) Fa(x, r) Fb(y, r)
      const double* Fa = F + (n == 0 ? 1 : 0) * QR;
      const double* Fb = F + (n == 2 ? 1 : 2) * QR;
      if (tid < Q * nch) {
        const int q = tid % Q, ch = tid / Q;
        double acc[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) acc[r] = 0.0;
        for (int pr = ch; pr < Q * Q; pr += nch) {
          const int x = pr / Q, y = pr % Q;
          int64_t idx;
          if (n == 0) idx = ((int64_t)q * Q + x) * Q + y;
          else if (n == 1) idx = ((int64_t)x * Q + q) * Q + y;
          else idx = ((int64_t)x * Q + y) * Q + q;
          const double xv = (double)X[idx];
#pragma unroll
          for (int r = 0; r < MAXR; ++r)
            if (r < R) acc[r] = fma(xv * Fa[x * R + r], Fb[y * R + r], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < MAXR; ++r)
          if (r < R) part[(ch * Q + q) * R + r] = acc[r];
      }
      __syncthreads();
      for (int e = tid; e < QR; e += NT) {
        double s = part[e];
        for (int c = 1; c < nch; ++c) s += part[c * QR + e];
        part[e] = s;
      }
      // ---- Hadamard product of the other two Gram matrices
      for (int e = tid; e < R * R; e += NT) {
        const int r1 = e / R, r2 = e % R;
        double g = 1.0;
        for (int m = 0; m < 3; ++m) {
          if (m == n) continue;
          const double* Fm = F + m * QR;
          double d = 0.0;
          for (int q = 0; q < Q; ++q) d = fma(Fm[q * R + r1], Fm[q * R + r2], d);
          g *= d;
        }
        G[e] = g;
      }
      __syncthreads();
      // ---- Cholesky G = L L^T (row-oriented)
      for (int j = 0; j < R; ++j) {
        if (tid == 0) {
          double d = G[j * R + j];
          for (int k = 0; k < j; ++k) d -= L[j * R + k] * L[j * R + k];
          if (!(d > 0.0)) { bad = 1; d = 1e-300; }
          L[j * R + j] = sqrt(d);
        }
        __syncthreads();
        if (tid > j && tid < R) {
          double v = G[tid * R + j];
          for (int k = 0; k < j; ++k) v -= L[tid * R + k] * L[j * R + k];
          L[tid * R + j] = v / L[j * R + j];
        }
        __syncthreads();
      }
      // ---- F_n(q, :) = M(q, :) G^{-1}
      double* Fn = F + n * QR;
      if (tid < Q) {
        double y[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) y[r] = r < R ? part[tid * R + r] : 0.0;
        for (int r = 0; r < R; ++r) {
          double v = y[r];
          for (int k = 0; k < r; ++k) v -= L[r * R + k] * y[k];
          y[r] = v / L[r * R + r];
        }
        for (int r = R - 1; r >= 0; --r) {
          double v = y[r];
          for (int k = r + 1; k < R; ++k) v -= L[k * R + r] * y[k];
          y[r] = v / L[r * R + r];
        }
        for (int r = 0; r < R; ++r) Fn[tid * R + r] = y[r];
      }
      __syncthreads();
      // ---- unit 2-norm columns; lambda = norms
      if (tid < R) {
        double s = 0.0;
        for (int q = 0; q < Q; ++q) s = fma(Fn[q * R + tid], Fn[q * R + tid], s);
        s = sqrt(s);
        lam[tid] = s > 0.0 ? s : 1.0;
      }
      __syncthreads();
      for (int e = tid; e < QR; e += NT) Fn[e] /= lam[e % R];
      __syncthreads();
    }
    ++done;
    if (tol > 0.0) {
      // replica fit from the Gram identity; part holds M for mode 3
      if (tid == 0) {
        double inner = 0.0;
        for (int r = 0; r < R; ++r) {
          double d = 0.0;
          for (int q = 0; q < Q; ++q) d = fma(part[q * R + r], F[2 * QR + q * R + r], d);
          inner += lam[r] * d;
        }
        double nh = 0.0;
        for (int r1 = 0; r1 < R; ++r1)
          for (int r2 = 0; r2 < R; ++r2) {
            double g = 1.0;
            for (int m = 0; m < 3; ++m) {
              double d = 0.0;
              for (int q = 0; q < Q; ++q) d = fma(F[m * QR + q * R + r1], F[m * QR + q * R + r2], d);
              g *= d;
            }
            nh += lam[r1] * g * lam[r2];
          }
        double res = sh_nx2 - 2.0 * inner + nh;
        if (res < 0.0) res = 0.0;
        double fit = sh_nx2 > 0.0 ? 1.0 - sqrt(res) / sqrt(sh_nx2) : 0.0;
        red[0] = (have_old && fabs(fit - sh_fit_old) < tol) ? 1.0 : 0.0;
        sh_fit_old = fit;
        have_old = 1;
      }
      __syncthreads();
      const bool stop = red[0] > 0.5;
      __syncthreads();
      if (stop) break;
    }
  }
  for (int e = tid; e < 3 * QR; e += NT) Fout[(int64_t)p * 3 * QR + e] = F[e];
  if (tid < R) lamout[(int64_t)p * R + tid] = lam[tid];
  if (tid == 0) {
    iters_out[p] = done;
    if (bad) flags[p] |= 1;
  }
}

}  // namespace

hipError_t als_reference(hipStream_t s, const void* Y, bool y_f64, int P, int Q, int R,
                         const double* init, double* F, double* lam, int* iters, int* flags,
                         int max_iters, double tol) {
  if (R > MAXR || Q > 128) return hipErrorInvalidValue;
  const int QR = Q * R;
  const size_t fixed = (size_t)(3 * QR + 2 * R * R + MAXR + NT) * sizeof(double);
  int nch = NT / Q;
  while (nch > 1 && fixed + (size_t)nch * QR * sizeof(double) > 150 * 1024) --nch;
  const size_t lds = fixed + (size_t)nch * QR * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (y_f64) {
    hipFuncSetAttribute((const void*)als_ref_kernel<double>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(als_ref_kernel<double>, dim3(P), dim3(NT), lds, s, (const double*)Y, Q, R,
                       nch, init, F, lam, iters, flags, max_iters, tol);
  } else {
    hipFuncSetAttribute((const void*)als_ref_kernel<float>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(als_ref_kernel<float>, dim3(P), dim3(NT), lds, s, (const float*)Y, Q, R,
                       nch, init, F, lam, iters, flags, max_iters, tol);
  }
  return hipGetLastError();
}

}  // namespace octen
