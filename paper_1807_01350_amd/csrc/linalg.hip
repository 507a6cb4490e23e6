// FP64 building blocks: a strided batched GEMM, SPD inversion and small SPD
// solves.  They carry the least-squares steps of the method (Sec. 4.3, Eq. 7)
// and the set-up of its operators; all arithmetic is double precision.
#include <hip/hip_runtime.h>
#include <math.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int GT = 64;   // output tile (GT x GT)
constexpr int GK = 16;   // k step

template <typename TA>
__global__ __launch_bounds__(256) void gemm_kernel(
    int M, int N, int K, const TA* __restrict__ A, int64_t sam, int64_t sak, int64_t sab,
    const double* __restrict__ B, int64_t sbk, int64_t sbn, int64_t sbb, double* __restrict__ C,
    int64_t scm, int64_t scn, int64_t scb, const double* __restrict__ d, double alpha,
    double beta) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  A += (int64_t)b * sab;
  B += (int64_t)b * sbb;
  C += (int64_t)b * scb;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GK * GT; e += 256) {
      // A tile: m fastest when A is k-major, else k fastest
      int kk, mm;
      if (sam == 1) { mm = e % GT; kk = e / GT; } else { kk = e % GK; mm = e / GK; }
      int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < M && gk < K) {
        v = (double)A[(int64_t)gm * sam + (int64_t)gk * sak];
        if (d) v *= d[gk];
      }
      As[kk][mm] = v;
      int nn, kb;
      if (sbn == 1) { nn = e % GT; kb = e / GT; } else { kb = e % GK; nn = e / GK; }
      int gn = n0 + nn, gk2 = k0 + kb;
      Bs[kb][nn] = (gn < N && gk2 < K) ? B[(int64_t)gk2 * sbk + (int64_t)gn * sbn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      double* c = C + (int64_t)gm * scm + (int64_t)gn * scn;
      double v = alpha * acc[i][j];
      if (beta != 0.0) v += beta * (*c);
      *c = v;
    }
  }
}

template <typename TA>
hipError_t gemm_launch(hipStream_t s, int M, int N, int K, int batch, const TA* A, int64_t sam,
                       int64_t sak, int64_t sab, const double* B, int64_t sbk, int64_t sbn,
                       int64_t sbb, double* C, int64_t scm, int64_t scn, int64_t scb,
                       const double* d, double alpha, double beta) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch);
  hipLaunchKernelGGL(gemm_kernel<TA>, grid, dim3(256), 0, s, M, N, K, A, sam, sak, sab, B, sbk, sbn,
                     sbb, C, scm, scn, scb, d, alpha, beta);
  return hipGetLastError();
}

// Gauss-Jordan step k: save row k and column k before the in-place update.
__global__ void gj_save(const double* __restrict__ A, int n, int k, double* __restrict__ row,
                        double* __restrict__ col) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    row[i] = A[(int64_t)k * n + i];
    col[i] = A[(int64_t)i * n + k];
  }
}

__global__ void gj_update(double* __restrict__ A, int n, int k, const double* __restrict__ row,
                          const double* __restrict__ col, int* info) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (j >= n) return;
  double piv = row[k];
  if (!(piv > 0.0)) {
    if (i == 0 && j == 0 && *info == 0) *info = k + 1;
    return;
  }
  double inv = 1.0 / piv;
  double v;
  if (i == k && j == k) v = inv;
  else if (i == k) v = row[j] * inv;
  else if (j == k) v = -col[i] * inv;
  else v = A[(int64_t)i * n + j] - col[i] * row[j] * inv;
  A[(int64_t)i * n + j] = v;
}

// One workgroup: in-place Cholesky of N (lower factor), then two triangular
// solves for nrhs right-hand sides.  One barrier per column: step j updates
// the trailing lower triangle from the still unscaled column j divided by the
// pivot, and scales column j - 1 (nobody reads it any more) in the same pass.
// The substitutions write each solved row into Z and update the remaining
// rows from the unsolved value, again one barrier per step.
__global__ __launch_bounds__(1024) void spd_solve_kernel(double* __restrict__ Nm, int n,
                                                         double* __restrict__ Bm, int nrhs,
                                                         double* __restrict__ Z, int* info) {
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double djj = Nm[(int64_t)j * n + j];
    if (tid == 0 && !(djj > 0.0) && !bad) bad = j + 1;
    const double inv = djj > 0.0 ? 1.0 / djj : 0.0;
    // scale column j - 1 by its pivot (kept on the diagonal until now)
    if (j > 0) {
      const double lp = sqrt(fmax(Nm[(int64_t)(j - 1) * n + (j - 1)], 1e-300));
      for (int i = j + tid; i < n; i += nt) Nm[(int64_t)i * n + (j - 1)] /= lp;
    }
    const int m = n - j - 1;
    const int64_t tri = (int64_t)m * (m + 1) / 2;
    for (int64_t e = tid; e < tri; e += nt) {
      int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((int64_t)ii * (ii + 1) / 2 > e) --ii;
      while ((int64_t)(ii + 1) * (ii + 2) / 2 <= e) ++ii;
      const int kk = (int)(e - (int64_t)ii * (ii + 1) / 2);
      const int gi = j + 1 + ii, gk = j + 1 + kk;
      Nm[(int64_t)gi * n + gk] -= Nm[(int64_t)gi * n + j] * Nm[(int64_t)gk * n + j] * inv;
    }
    __syncthreads();
  }
  // the diagonal becomes the factor's diagonal (the last column has nothing below it)
  for (int j = tid; j < n; j += nt) Z[j] = sqrt(fmax(Nm[(int64_t)j * n + j], 1e-300));
  __syncthreads();
  for (int j = tid; j < n; j += nt) Nm[(int64_t)j * n + j] = Z[j];
  __syncthreads();
  // forward: L y = b; row j solved into Bm (scaled) while the rest is updated
  for (int j = 0; j < n; ++j) {
    const double ljj = Nm[(int64_t)j * n + j];
    const int64_t tot = (int64_t)(n - j - 1) * nrhs;
    for (int64_t e = tid; e < tot; e += nt) {
      const int i = j + 1 + (int)(e / nrhs), c = (int)(e % nrhs);
      Bm[(int64_t)i * nrhs + c] -= Nm[(int64_t)i * n + j] * (Bm[(int64_t)j * nrhs + c] / ljj);
    }
    __syncthreads();
    for (int c = tid; c < nrhs; c += nt) Bm[(int64_t)j * nrhs + c] /= ljj;
  }
  __syncthreads();
  // backward: L^T x = y
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = Nm[(int64_t)j * n + j];
    const int64_t tot = (int64_t)j * nrhs;
    for (int64_t e = tid; e < tot; e += nt) {
      const int i = (int)(e / nrhs), c = (int)(e % nrhs);
      Bm[(int64_t)i * nrhs + c] -= Nm[(int64_t)j * n + i] * (Bm[(int64_t)j * nrhs + c] / ljj);
    }
    __syncthreads();
    for (int c = tid; c < nrhs; c += nt) Bm[(int64_t)j * nrhs + c] /= ljj;
  }
  if (tid == 0 && bad && *info == 0) *info = bad;
}

// Small systems (n <= 112, nrhs <= 32): Gauss-Jordan elimination without
// pivoting on [N | B] held in LDS, one workgroup; for symmetric positive
// definite N every pivot is positive (an SPD Schur complement stays SPD).
// Per pivot j: every row i != j loses N(i,j)/N(j,j) times row j, columns right
// of j only (the ones left of j are already eliminated, column j is not read
// again).  Rows are not divided by their pivots during the elimination: a step
// writes only columns right of j of rows other than j and reads only column j
// and row j, so one barrier per pivot suffices; N ends diagonal with its
// pivots unchanged, and the right-hand columns of row i are divided by N(i,i)
// at the end, giving N^{-1} B.  Thread t owns rows t/16 + 16k and columns
// t%16 + 16m, so no element index is divided at run time.  Per pivot a
// thread first loads every operand of its KR x KC elements (they are
// independent), then updates and stores them: one LDS latency per pivot
// instead of one per element.  info = j + 1 for a pivot that is not positive
// (the elimination continues with it skipped and its row is returned
// undivided).
constexpr int GJ_NMAX = 112, GJ_RMAX = 32;
template <int KR, int KC>
__global__ __launch_bounds__(256) void spd_solve_gj_kernel(const double* __restrict__ Nm, int n,
                                                           double* __restrict__ Bm, int nrhs,
                                                           int* info) {
  extern __shared__ double gj_lds[];
  __shared__ int bad;
  const int tid = threadIdx.x, w = n + nrhs, ld = w + 1;
  const int rg = tid >> 4, cg = tid & 15;
  auto M = [&](int i, int c) -> double& { return gj_lds[i * ld + c]; };
  if (tid == 0) bad = 0;
  for (int i = rg; i < n; i += 16)
    for (int c = cg; c < w; c += 16)
      M(i, c) = c < n ? Nm[(int64_t)i * n + c] : Bm[(int64_t)i * nrhs + (c - n)];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double p = M(j, j);
    if (p > 0.0) {
      const double ip = 1.0 / p;
      double f[KR], rj[KC], x[KR][KC];
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = rg + 16 * k;
        f[k] = (i < n && i != j) ? M(i, j) : 0.0;
      }
#pragma unroll
      for (int m = 0; m < KC; ++m) {
        const int c = cg + 16 * m;
        rj[m] = (c > j && c < w) ? M(j, c) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < KR; ++k)
#pragma unroll
        for (int m = 0; m < KC; ++m) {
          const int i = rg + 16 * k, c = cg + 16 * m;
          x[k][m] = (i < n && i != j && c > j && c < w) ? M(i, c) : 0.0;
        }
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = rg + 16 * k;
        const double fk = f[k] * ip;
#pragma unroll
        for (int m = 0; m < KC; ++m) {
          const int c = cg + 16 * m;
          if (i < n && i != j && c > j && c < w) M(i, c) = fma(-fk, rj[m], x[k][m]);
        }
      }
    } else if (tid == 0 && !bad) {
      bad = j + 1;
    }
    __syncthreads();
  }
  for (int i = rg; i < n; i += 16) {
    const double p = M(i, i);
    const double ip = p > 0.0 ? 1.0 / p : 1.0;
    for (int c = cg; c < nrhs; c += 16) Bm[(int64_t)i * nrhs + c] = M(i, n + c) * ip;
  }
  if (tid == 0 && bad && *info == 0) *info = bad;
}

// Set-up of one ALS call in one launch: F0 = src (the starting factors, given
// back to a replica whose fit fails), lam0 = lam_src or ones, the replica
// flags cleared, and (for a cooperative launch) its barrier words cleared.
__global__ void als_prep_kernel(int64_t nf, double* __restrict__ F0, const double* __restrict__ src,
                                int64_t nl, double* __restrict__ lam0,
                                const double* __restrict__ lam_src, int P, int* __restrict__ flags,
                                unsigned* __restrict__ ctr, int nctr, int* __restrict__ err) {
  int64_t n = nf > nl ? nf : nl;
  if (P > n) n = P;
  if (nctr > n) n = nctr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nf) F0[i] = src[i];
    if (i < nl) lam0[i] = lam_src ? lam_src[i] : 1.0;
    if (i < P) flags[i] = 0;
    if (ctr && i < nctr) ctr[i] = 0u;
    if (err && i == 0) *err = 0;
  }
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_i32_kernel(int* p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void cvt_kernel(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
// Y_p += Z_p where replica p's compressed batch is finite (n values each).
template <typename T>
__global__ void update_masked_kernel(T* __restrict__ y, const T* __restrict__ x, int P, int64_t n,
                                     const int* __restrict__ zbad, int* __restrict__ health) {
  const int64_t tot = (int64_t)P * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(i / n);
    if (zbad[p] == 0) y[i] += x[i];
    else if (i == (int64_t)p * n) atomicOr(health, 1);
  }
}

// One workgroup per replica: keep or roll back the replica's new factors.
__global__ void als_commit_kernel(int QR3, int R, double* __restrict__ F, double* __restrict__ lam,
                                  const double* __restrict__ F0, const double* __restrict__ lam0,
                                  int* __restrict__ flags, int* __restrict__ health) {
  const int p = blockIdx.x;
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  double* f = F + (int64_t)p * QR3;
  int bad = 0;
  for (int e = threadIdx.x; e < QR3; e += blockDim.x) bad |= isfinite(f[e]) ? 0 : 1;
  for (int e = threadIdx.x; e < R; e += blockDim.x) bad |= isfinite(lam[(int64_t)p * R + e]) ? 0 : 1;
  if (bad) atomicOr(&s_bad, 1);
  __syncthreads();
  const int fl = flags[p] | (s_bad ? 4 : 0);
  const bool back = (fl & 7) != 0;
  if (back) {
    for (int e = threadIdx.x; e < QR3; e += blockDim.x) f[e] = F0[(int64_t)p * QR3 + e];
    for (int e = threadIdx.x; e < R; e += blockDim.x) lam[(int64_t)p * R + e] = lam0[(int64_t)p * R + e];
  }
  if (threadIdx.x == 0) {
    flags[p] = fl | (back ? 8 : 0);
    if (back) atomicOr(health, 2);
  }
}

__global__ void scale_kernel(double* X, int64_t rows, int64_t cols, const double* vr,
                             const double* vc) {
  const int64_t tot = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    double f = 1.0;
    if (vr) f *= vr[e / cols];
    if (vc) f *= vc[e % cols];
    X[e] *= f;
  }
}

inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t scale_cols(hipStream_t s, double* X, int64_t rows, int64_t cols, const double* v) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, X, rows, cols,
                     (const double*)nullptr, v);
  return hipGetLastError();
}
hipError_t scale_rows(hipStream_t s, double* X, int64_t rows, int64_t cols, const double* v) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, X, rows, cols, v,
                     (const double*)nullptr);
  return hipGetLastError();
}
hipError_t scale_rows_cols(hipStream_t s, double* X, int64_t n, const double* v) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n * n)), dim3(256), 0, s, X, n, n, v, v);
  return hipGetLastError();
}

hipError_t gemm_f64(hipStream_t s, int M, int N, int K, int batch, const double* A, int64_t sam,
                    int64_t sak, int64_t sab, const double* B, int64_t sbk, int64_t sbn,
                    int64_t sbb, double* C, int64_t scm, int64_t scn, int64_t scb,
                    const double* d, double alpha, double beta) {
  return gemm_launch<double>(s, M, N, K, batch, A, sam, sak, sab, B, sbk, sbn, sbb, C, scm, scn,
                             scb, d, alpha, beta);
}

hipError_t gemm_f32in_f64(hipStream_t s, int M, int N, int K, int batch, const float* A,
                          int64_t sam, int64_t sak, int64_t sab, const double* B, int64_t sbk,
                          int64_t sbn, int64_t sbb, double* C, int64_t scm, int64_t scn,
                          int64_t scb, const double* d, double alpha, double beta) {
  return gemm_launch<float>(s, M, N, K, batch, A, sam, sak, sab, B, sbk, sbn, sbb, C, scm, scn,
                            scb, d, alpha, beta);
}

hipError_t spd_invert(hipStream_t s, double* A, int n, double* work, int* info) {
  double* row = work;
  double* col = work + n;
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(gj_save, dim3((n + 255) / 256), dim3(256), 0, s, A, n, k, row, col);
    hipLaunchKernelGGL(gj_update, dim3((n + 255) / 256, n), dim3(256), 0, s, A, n, k, row, col,
                       info);
  }
  return hipGetLastError();
}

hipError_t spd_solve_small(hipStream_t s, double* N, int n, double* Bm, int nrhs, double* work,
                           int* info) {
  if (n <= 0) return hipSuccess;
  if (n <= GJ_NMAX && nrhs <= GJ_RMAX) {
    const size_t lds = (size_t)n * (n + nrhs + 1) * sizeof(double);
    // row and column slots per thread (rows t/16 + 16k, columns t%16 + 16m)
    const int kr = (n + 15) / 16, kc = (n + nrhs + 15) / 16;
    const void* fn = (kr <= 4 && kc <= 4)   ? (const void*)spd_solve_gj_kernel<4, 4>
                     : (kr <= 4 && kc <= 6) ? (const void*)spd_solve_gj_kernel<4, 6>
                                            : (const void*)spd_solve_gj_kernel<7, 9>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    void* args[] = {&N, &n, &Bm, &nrhs, &info};
    return hipLaunchKernel(fn, dim3(1), dim3(256), args, lds, s);
  }
  hipLaunchKernelGGL(spd_solve_kernel, dim3(1), dim3(1024), 0, s, N, n, Bm, nrhs, work, info);
  return hipGetLastError();
}

hipError_t als_prep(hipStream_t s, int64_t nf, double* F0, const double* src, int64_t nl,
                    double* lam0, const double* lam_src, int P, int* flags, unsigned* ctr,
                    int nctr, int* err) {
  int64_t n = nf > nl ? nf : nl;
  if (P > n) n = P;
  if (nctr > n) n = nctr;
  hipLaunchKernelGGL(als_prep_kernel, dim3(grid_for(n)), dim3(256), 0, s, nf, F0, src, nl, lam0,
                     lam_src, P, flags, ctr, nctr, err);
  return hipGetLastError();
}

hipError_t fill_f64(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t fill_i32(hipStream_t s, int* p, int64_t n, int v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t convert_f64_to_f32(hipStream_t s, const double* in, float* out, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cvt_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t update_masked(hipStream_t s, void* Y, const void* Z, int P, int64_t n, bool f64,
                         const int* zbad, int* health) {
  if (f64)
    hipLaunchKernelGGL(update_masked_kernel<double>, dim3(grid_for(P * n)), dim3(256), 0, s,
                       (double*)Y, (const double*)Z, P, n, zbad, health);
  else
    hipLaunchKernelGGL(update_masked_kernel<float>, dim3(grid_for(P * n)), dim3(256), 0, s,
                       (float*)Y, (const float*)Z, P, n, zbad, health);
  return hipGetLastError();
}

hipError_t als_commit(hipStream_t s, int P, int QR3, int R, double* F, double* lam,
                      const double* F0, const double* lam0, int* flags, int* health) {
  hipLaunchKernelGGL(als_commit_kernel, dim3(P), dim3(256), 0, s, QR3, R, F, lam, F0, lam0, flags,
                     health);
  return hipGetLastError();
}

}  // namespace octen

// ---------------------------------------------------------------------------
// Products with a small output width: out(i, r) = alpha * sum_k A(i,k) d(k) B(k,r)
// + beta * out(i, r) for r < ncols (<= any), one wavefront per (row i, block of
// 32 columns, range of k); lanes split k, partial sums meet in a butterfly.
// Operands are strided: A(i,k) = A[i*sai + k*sak], B(k,r) = B[k*sbk + r*sbr].
namespace octen {
namespace {
// One product of the kernels below; nsplit, kchunk and part from rowdot_plan.
struct RowdotJob {
  int64_t nrows;
  int ncols;
  int64_t K;
  const double* A;
  int64_t sai, sak;
  const double* B;
  int64_t sbk, sbr;
  const double* d;
  double alpha, beta;
  double* out;
  int64_t ldo;
  int nsplit;
  int64_t kchunk;
  double* part;
};

// Up to two independent products in one launch: blocks [0, blocks0) work on
// j0, the rest on j1.
__global__ __launch_bounds__(256) void rowdot_kernel(RowdotJob j0, RowdotJob j1, int64_t blocks0) {
  const bool second = (int64_t)blockIdx.x >= blocks0;
  const RowdotJob& j = second ? j1 : j0;
  const int64_t nrows = j.nrows, K = j.K, sai = j.sai, sak = j.sak, sbk = j.sbk, sbr = j.sbr;
  const int ncols = j.ncols, nsplit = j.nsplit;
  const double* __restrict__ A = j.A;
  const double* __restrict__ B = j.B;
  const double* __restrict__ d = j.d;
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x - (second ? blocks0 : 0)) * 4 + threadIdx.x / 64;
  const int nblk = (ncols + 31) / 32;
  if (wid >= nrows * nblk * nsplit) return;
  const int sp = (int)(wid % nsplit);
  const int64_t rest = wid / nsplit;
  const int64_t i = rest / nblk;
  const int r0 = (int)(rest % nblk) * 32;
  const int nr = ncols - r0 < 32 ? ncols - r0 : 32;
  const int64_t k0 = sp * j.kchunk, k1 = k0 + j.kchunk < K ? k0 + j.kchunk : K;
  double acc[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) acc[r] = 0.0;
  const double* a = A + i * sai;
  for (int64_t k = k0 + lane; k < k1; k += 64) {
    double av = a[k * sak];
    if (d) av *= d[k];
    const double* b = B + k * sbk + (int64_t)r0 * sbr;
#pragma unroll
    for (int r = 0; r < 32; ++r)
      if (r < nr) acc[r] = fma(av, b[r * sbr], acc[r]);
  }
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    if (r < nr) {
      double v = acc[r];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[r] = v;
    }
  }
  if (lane == 0) {
    if (nsplit == 1) {
      double* o = j.out + i * j.ldo + r0;
#pragma unroll
      for (int r = 0; r < 32; ++r)
        if (r < nr) o[r] = j.beta != 0.0 ? j.alpha * acc[r] + j.beta * o[r] : j.alpha * acc[r];
    } else {
      double* o = j.part + ((int64_t)sp * nrows + i) * ncols + r0;
#pragma unroll
      for (int r = 0; r < 32; ++r)
        if (r < nr) o[r] = acc[r];
    }
  }
}

// out(i, r) = alpha * sum over the splits (in order) + beta * out(i, r), for
// up to two products as in rowdot_kernel (256 threads per block).
__global__ void rowdot_reduce_kernel(RowdotJob j0, RowdotJob j1, int64_t blocks0) {
  const bool second = (int64_t)blockIdx.x >= blocks0;
  const RowdotJob& j = second ? j1 : j0;
  const int64_t e = ((int64_t)blockIdx.x - (second ? blocks0 : 0)) * blockDim.x + threadIdx.x;
  if (e >= j.nrows * j.ncols) return;
  const int64_t i = e / j.ncols;
  const int r = (int)(e % j.ncols);
  const double* __restrict__ part = j.part;
  const int64_t stride = j.nrows * j.ncols;
  // split order kept; eight partials loaded ahead of their adds
  double sum = 0.0;
#pragma unroll 8
  for (int sp = 0; sp < j.nsplit; ++sp) sum += part[(int64_t)sp * stride + e];
  double* o = j.out + i * j.ldo + r;
  *o = j.beta != 0.0 ? j.alpha * sum + j.beta * *o : j.alpha * sum;
}

// Small Gram-type products over a long index: part[g][i][r] = sum over the
// k range of block g of A[k*sak + i] * B[k*sbk + r], i < n <= 32, r < ncols
// <= 32.  Each block stages 64 rows of A and B in LDS at a time (every row
// of both read once from HBM); thread t owns the pairs t + 256 j.  The
// partials are summed in block order by rowdot_reduce_kernel.
constexpr int GR_KB = 64;
__global__ __launch_bounds__(256) void gram_part_kernel(int n, int ncols, int64_t K,
                                                        const double* __restrict__ A, int64_t sak,
                                                        const double* __restrict__ B, int64_t sbk,
                                                        int64_t kchunk, double* __restrict__ part) {
  __shared__ double As[GR_KB][33], Bs[GR_KB][33];
  const int tid = threadIdx.x, np = n * ncols;
  const int64_t k0 = (int64_t)blockIdx.x * kchunk;
  const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
  double acc[4];
  int pi[4], pr[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = tid + 256 * j;
    acc[j] = 0.0;
    pi[j] = p < np ? p / ncols : 0;
    pr[j] = p < np ? p % ncols : 0;
  }
  for (int64_t kb = k0; kb < k1; kb += GR_KB) {
    for (int e = tid; e < GR_KB * 32; e += 256) {
      const int kk = e >> 5, c = e & 31;
      const int64_t k = kb + kk;
      As[kk][c] = (k < k1 && c < n) ? A[k * sak + c] : 0.0;
      Bs[kk][c] = (k < k1 && c < ncols) ? B[k * sbk + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (tid + 256 * j < np) {
        double a = acc[j];
        for (int kk = 0; kk < GR_KB; ++kk) a = fma(As[kk][pi[j]], Bs[kk][pr[j]], a);
        acc[j] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = tid + 256 * j;
    if (p < np) part[(int64_t)blockIdx.x * np + p] = acc[j];
  }
}

typedef double tg_f64x4 __attribute__((ext_vector_type(4)));
constexpr int TG_KC = 128;   // k rows of B per LDS chunk

// out[i][r] = alpha sum_k A[i][k] B[k][r] (+ beta out[i][r]) for a tall A
// (n x K, row stride lda, unit column stride) and B (K x R, row stride ldb),
// R <= 32, on v_mfma_f64_16x16x4f64: each wavefront owns 16 rows of A and
// both 16-column halves of the output; the four wavefronts of a workgroup
// share a chunk of TG_KC rows of B in LDS (zero past K and past R, row
// padded to 33 against bank conflicts).  A is read once, in the MFMA
// operand layout (16 rows x 4 consecutive k per load, clamped into range:
// the zero rows of the B chunk cancel the clamped terms).  Per group of 8
// steps, all operand loads are issued before the MFMAs.
__global__ __launch_bounds__(256) void tall_gemm_kernel(int64_t n, int R, int64_t K,
                                                        const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ B, int64_t ldb,
                                                        double alpha, double beta,
                                                        double* __restrict__ out, int64_t ldo) {
  __shared__ double Bs[TG_KC][33];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid & 63;
  const int kq = lane / 16, nl = lane % 16;
  const int64_t i0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t row = i0 + nl;
  const double* a = A + (row < n ? row : n - 1) * lda;
  const bool two = R > 16;
  tg_f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int64_t kc = 0; kc < K; kc += TG_KC) {
    __syncthreads();
    for (int e = tid; e < TG_KC * 32; e += 256) {
      const int kk = e >> 5, rr = e & 31;
      const int64_t k = kc + kk;
      Bs[kk][rr] = (k < K && rr < R) ? B[k * ldb + rr] : 0.0;
    }
    __syncthreads();
    const int steps = K - kc < TG_KC ? (int)(K - kc) : TG_KC;
    for (int s0 = 0; s0 < steps; s0 += 32) {
      double av[8], b0[8], b1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t k = kc + s0 + 4 * u + kq;
        av[u] = a[k < K ? k : K - 1];
        b0[u] = Bs[s0 + 4 * u + kq][nl];
        b1[u] = Bs[s0 + 4 * u + kq][16 + nl];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b0[u], acc0, 0, 0, 0);
        if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b1[u], acc1, 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // element i of lane l holds D[l/16 + 4 i][l%16]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t orow = i0 + kq + 4 * i;
    if (orow >= n) continue;
    double* o = out + orow * ldo;
    if (nl < R) o[nl] = beta != 0.0 ? alpha * acc0[i] + beta * o[nl] : alpha * acc0[i];
    if (two && 16 + nl < R)
      o[16 + nl] = beta != 0.0 ? alpha * acc1[i] + beta * o[16 + nl] : alpha * acc1[i];
  }
}

}  // namespace

namespace {

RowdotJob make_job(int64_t nrows, int ncols, int64_t K, const double* A, int64_t sai, int64_t sak,
                   const double* B, int64_t sbk, int64_t sbr, const double* d, double alpha,
                   double beta, double* out, int64_t ldo) {
  RowdotJob j;
  j.nrows = nrows; j.ncols = ncols; j.K = K; j.A = A; j.sai = sai; j.sak = sak; j.B = B;
  j.sbk = sbk; j.sbr = sbr; j.d = d; j.alpha = alpha; j.beta = beta; j.out = out; j.ldo = ldo;
  j.nsplit = 1; j.kchunk = K; j.part = nullptr;
  return j;
}

// The tall and Gram-type products have kernels of their own (rowdot_special).
bool rowdot_is_tall(const RowdotJob& j) {
  return j.sak == 1 && j.sbr == 1 && !j.d && j.ncols <= 32 && j.nrows >= 16384 && j.K >= 32;
}
bool rowdot_is_gram(const RowdotJob& j, const double* work) {
  return j.sai == 1 && j.sbr == 1 && !j.d && j.nrows <= 32 && j.ncols <= 32 && j.K >= 8192 && work;
}

// Splits of the long index for rowdot_kernel: when there are too few rows to
// fill the GPU, partial sums go to work (added in split order by
// rowdot_reduce_kernel).  Returns the kernel's blocks.
int64_t rowdot_plan(RowdotJob& j, double* work, int64_t work_len) {
  const int nblk = (j.ncols + 31) / 32;
  int64_t nsplit = 1;
  const int64_t waves = j.nrows * nblk;
  if (work && waves < 2048 && j.K >= 256) {
    nsplit = (2048 + waves - 1) / waves;
    const int64_t maxs = j.K / 128;   // at least two 64-wide steps per wavefront
    if (nsplit > maxs) nsplit = maxs;
    if (nsplit > 64) nsplit = 64;
    while (nsplit > 1 && nsplit * j.nrows * j.ncols > work_len) --nsplit;
    if (nsplit < 1) nsplit = 1;
  }
  int64_t kchunk = (j.K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 63) / 64 * 64;
  j.nsplit = (int)nsplit;
  j.kchunk = kchunk;
  j.part = nsplit > 1 ? work : nullptr;
  return (waves * nsplit + 3) / 4;
}

int64_t reduce_blocks(const RowdotJob& j) {
  return j.nsplit > 1 ? (j.nrows * j.ncols + 255) / 256 : 0;
}

hipError_t rowdot_special(hipStream_t s, const RowdotJob& j, double* work, int64_t work_len,
                          bool* done) {
  *done = false;
  if (rowdot_is_tall(j)) {
    // tall product with unit inner strides and enough 64-row blocks to fill
    // the GPU: FP64 MFMA, A streamed once
    hipLaunchKernelGGL(tall_gemm_kernel, dim3((unsigned)((j.nrows + 63) / 64)), dim3(256), 0, s,
                       j.nrows, j.ncols, j.K, j.A, j.sai, j.B, j.sbk, j.alpha, j.beta, j.out,
                       j.ldo);
    *done = true;
    return hipGetLastError();
  }
  if (rowdot_is_gram(j, work)) {
    // R x R Gram-type product over a long index: blocks over k, partials
    // summed in block order
    const int64_t np = j.nrows * j.ncols;
    int64_t g = j.K / 256;
    if (g > 256) g = 256;
    if (g * np > work_len) g = work_len / np;
    if (g >= 2) {
      int64_t kchunk = (j.K + g - 1) / g;
      kchunk = (kchunk + GR_KB - 1) / GR_KB * GR_KB;
      g = (j.K + kchunk - 1) / kchunk;
      hipLaunchKernelGGL(gram_part_kernel, dim3((unsigned)g), dim3(256), 0, s, (int)j.nrows,
                         j.ncols, j.K, j.A, j.sak, j.B, j.sbk, kchunk, work);
      RowdotJob r = j;
      r.nsplit = (int)g;
      r.part = work;
      const int64_t rb = reduce_blocks(r);
      hipLaunchKernelGGL(rowdot_reduce_kernel, dim3((unsigned)rb), dim3(256), 0, s, r, r, rb);
      *done = true;
      return hipGetLastError();
    }
  }
  return hipSuccess;
}

hipError_t rowdot_job(hipStream_t s, RowdotJob j, double* work, int64_t work_len) {
  if (j.nrows <= 0 || j.ncols <= 0) return hipSuccess;
  bool done = false;
  hipError_t e = rowdot_special(s, j, work, work_len, &done);
  if (e != hipSuccess || done) return e;
  const int64_t blocks = rowdot_plan(j, work, work_len);
  hipLaunchKernelGGL(rowdot_kernel, dim3((unsigned)blocks), dim3(256), 0, s, j, j, blocks);
  const int64_t rb = reduce_blocks(j);
  if (rb > 0)
    hipLaunchKernelGGL(rowdot_reduce_kernel, dim3((unsigned)rb), dim3(256), 0, s, j, j, rb);
  return hipGetLastError();
}

}  // namespace

hipError_t rowdot(hipStream_t s, int64_t nrows, int ncols, int64_t K, const double* A, int64_t sai,
                  int64_t sak, const double* B, int64_t sbk, int64_t sbr, const double* d,
                  double alpha, double beta, double* out, int64_t ldo, double* work,
                  int64_t work_len) {
  return rowdot_job(s, make_job(nrows, ncols, K, A, sai, sak, B, sbk, sbr, d, alpha, beta, out, ldo),
                    work, work_len);
}

hipError_t rowdot_pair(hipStream_t s, const RowdotArgs& x, const RowdotArgs& y, double* work,
                       int64_t work_len) {
  RowdotJob j0 = make_job(x.nrows, x.ncols, x.K, x.A, x.sai, x.sak, x.B, x.sbk, x.sbr, x.d,
                          x.alpha, x.beta, x.out, x.ldo);
  RowdotJob j1 = make_job(y.nrows, y.ncols, y.K, y.A, y.sai, y.sak, y.B, y.sbk, y.sbr, y.d,
                          y.alpha, y.beta, y.out, y.ldo);
  const int64_t half = work ? work_len / 2 : 0;
  double* work1 = work ? work + half : nullptr;
  if (j0.nrows <= 0 || j0.ncols <= 0 || j1.nrows <= 0 || j1.ncols <= 0 || rowdot_is_tall(j0) ||
      rowdot_is_tall(j1) || rowdot_is_gram(j0, work) || rowdot_is_gram(j1, work)) {
    hipError_t e = rowdot_job(s, j0, work, half);
    return e != hipSuccess ? e : rowdot_job(s, j1, work1, half);
  }
  const int64_t b0 = rowdot_plan(j0, work, half);
  const int64_t b1 = rowdot_plan(j1, work1, half);
  hipLaunchKernelGGL(rowdot_kernel, dim3((unsigned)(b0 + b1)), dim3(256), 0, s, j0, j1, b0);
  const int64_t r0 = reduce_blocks(j0), r1 = reduce_blocks(j1);
  if (r0 > 0 && r1 > 0)
    hipLaunchKernelGGL(rowdot_reduce_kernel, dim3((unsigned)(r0 + r1)), dim3(256), 0, s, j0, j1, r0);
  else if (r0 > 0)
    hipLaunchKernelGGL(rowdot_reduce_kernel, dim3((unsigned)r0), dim3(256), 0, s, j0, j0, r0);
  else if (r1 > 0)
    hipLaunchKernelGGL(rowdot_reduce_kernel, dim3((unsigned)r1), dim3(256), 0, s, j1, j1, r1);
  return hipGetLastError();
}
}  // namespace octen
