// Reference compression path (Sec. 4.1, Eq. 1): plain FP64-accumulating
// kernels for any slice type, used for the FP64 form and as the baseline the
// MFMA path is measured against.
//
// The multi-mode product is evaluated as
//   T2[k] = X_k V            (contract j; one strided GEMM over all slices)
//   M[k][p] = U_p^T T2[k]_p  (contract i per replica; Q x Q per slice)
//   Z_p = sum_k M[k][p] (x) W_p(k, :)   (contract k)
// which is the same trilinear form as the paper's mode-1, mode-2, mode-3
// order; only the order of the two non-temporal contractions differs.
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

namespace {

__device__ __forceinline__ int rep_col(int p, int q, int Q, int S) {
  return q < S ? q : S + p * (Q - S) + (q - S);
}

constexpr int S2_ROWS = 16;   // output rows a per block
constexpr int S2_KT = 32;     // i per LDS tile

// M[k][p][a][b] = sum_i U[i][col_p(a)] * T2[k][i][col_p(b)], a in a block of 16.
__global__ __launch_bounds__(256) void stage2_kernel(const double* __restrict__ U,
                                                     const double* __restrict__ T2, int64_t I,
                                                     int M1, int P, int Q, int S,
                                                     double* __restrict__ Mout) {
  extern __shared__ double sm[];
  double* Us = sm;                      // [S2_KT][S2_ROWS]
  double* Ts = sm + S2_KT * S2_ROWS;    // [S2_KT][Q]
  const int k = blockIdx.x, p = blockIdx.y, a0 = blockIdx.z * S2_ROWS;
  const int tid = threadIdx.x;
  const int nout = S2_ROWS * Q;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  const double* T2k = T2 + (int64_t)k * I * M1;
  for (int64_t i0 = 0; i0 < I; i0 += S2_KT) {
    for (int e = tid; e < S2_KT * S2_ROWS; e += 256) {
      int ii = e / S2_ROWS, aa = e % S2_ROWS;
      int64_t gi = i0 + ii;
      int a = a0 + aa;
      Us[e] = (gi < I && a < Q) ? U[gi * M1 + rep_col(p, a, Q, S)] : 0.0;
    }
    for (int e = tid; e < S2_KT * Q; e += 256) {
      int ii = e / Q, b = e % Q;
      int64_t gi = i0 + ii;
      Ts[e] = gi < I ? T2k[gi * M1 + rep_col(p, b, Q, S)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int o = tid + u * 256;
      if (o < nout) {
        int aa = o / Q, b = o % Q;
        double s = acc[u];
        for (int ii = 0; ii < S2_KT; ++ii) s = fma(Us[ii * S2_ROWS + aa], Ts[ii * Q + b], s);
        acc[u] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    int o = tid + u * 256;
    if (o < nout) {
      int aa = o / Q, b = o % Q;
      int a = a0 + aa;
      if (a < Q) Mout[(((int64_t)k * P + p) * Q + a) * Q + b] = acc[u];
    }
  }
}

constexpr int S3_KT = 32;  // k per LDS tile

// Z[p][a][b][c] = sum_k M[k][p][a][b] * W[k][col_p(c)] (k ascending, FP64
// sums of the row-block partials first), for Q <= 64.  One workgroup per
// (p, a) covers all (b, c): thread (ty, tx) owns 4 x 4 outputs of the 64 x 64
// block, so that a k step reads 4 + 4 values from LDS for 16 products and W
// is staged once per workgroup.
template <typename TM, typename TZ>
__global__ __launch_bounds__(256) void mode3_kernel(const TM* __restrict__ Mk,
                                                    const double* __restrict__ W, int64_t t,
                                                    int nrb, int M1, int P, int Q, int S,
                                                    TZ* __restrict__ Z, int* __restrict__ zbad) {
  extern __shared__ double sm[];
  constexpr int QP = 64;
  double* Ms = sm;                     // [S3_KT][QP]
  double* Ws = sm + S3_KT * QP;        // [S3_KT][QP]
  const int p = blockIdx.x, a = blockIdx.y;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t k0 = 0; k0 < t; k0 += S3_KT) {
    for (int e = tid; e < S3_KT * QP; e += 256) {
      const int kk = e / QP, b = e - kk * QP;
      const int64_t gk = k0 + kk;
      double v = 0.0, wv = 0.0;
      if (gk < t && b < Q) {
        for (int rb = 0; rb < nrb; ++rb) v += (double)Mk[(((gk * nrb + rb) * P + p) * Q + a) * Q + b];
        wv = W[gk * M1 + rep_col(p, b, Q, S)];
      }
      Ms[e] = v;
      Ws[e] = wv;
    }
    __syncthreads();
    for (int kk = 0; kk < S3_KT; ++kk) {
      double mb[4], wc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) mb[i] = Ms[kk * QP + ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) wc[j] = Ws[kk * QP + tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(mb[i], wc[j], acc[i][j]);
    }
    __syncthreads();
  }
  int bad = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = ty * 4 + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = tx * 4 + j;
      if (b < Q && c < Q) {
        const TZ z = (TZ)acc[i][j];
        bad |= isfinite((double)z) ? 0 : 1;
        Z[(((int64_t)p * Q + a) * Q + b) * Q + c] = z;
      }
    }
  }
  // a non-finite slice value reaches every replica's Z: flag the replica
  if (bad) atomicOr(zbad + p, 1);
}

constexpr int S3_B = 16;   // b per block

// The same for Q > 64, one workgroup per (p, a, block of 16 b): the 4 x 4
// tiles of mode3_kernel would leave most of a 128 x 128 block idle there.
template <typename TM, typename TZ>
__global__ __launch_bounds__(256) void mode3_bblock_kernel(const TM* __restrict__ Mk,
                                                    const double* __restrict__ W, int64_t t,
                                                    int nrb, int M1, int P, int Q, int S,
                                                    TZ* __restrict__ Z, int* __restrict__ zbad) {
  extern __shared__ double sm[];
  double* Ms = sm;                     // [S3_KT][S3_B]
  double* Ws = sm + S3_KT * S3_B;      // [S3_KT][Q]
  const int p = blockIdx.x, a = blockIdx.y, b0 = blockIdx.z * S3_B;
  const int tid = threadIdx.x;
  const int nout = S3_B * Q;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  for (int64_t k0 = 0; k0 < t; k0 += S3_KT) {
    for (int e = tid; e < S3_KT * S3_B; e += 256) {
      int kk = e / S3_B, bb = e % S3_B;
      int64_t gk = k0 + kk;
      int b = b0 + bb;
      double v = 0.0;
      if (gk < t && b < Q)
        for (int rb = 0; rb < nrb; ++rb) v += (double)Mk[(((gk * nrb + rb) * P + p) * Q + a) * Q + b];
      Ms[e] = v;
    }
    for (int e = tid; e < S3_KT * Q; e += 256) {
      int kk = e / Q, c = e % Q;
      int64_t gk = k0 + kk;
      Ws[e] = gk < t ? W[gk * M1 + rep_col(p, c, Q, S)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int o = tid + u * 256;
      if (o < nout) {
        int bb = o / Q, c = o % Q;
        double s = acc[u];
        for (int kk = 0; kk < S3_KT; ++kk) s = fma(Ms[kk * S3_B + bb], Ws[kk * Q + c], s);
        acc[u] = s;
      }
    }
    __syncthreads();
  }
  int bad = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    int o = tid + u * 256;
    if (o < nout) {
      int bb = o / Q, c = o % Q;
      int b = b0 + bb;
      if (b < Q) {
        const TZ z = (TZ)acc[u];
        bad |= isfinite((double)z) ? 0 : 1;
        Z[(((int64_t)p * Q + a) * Q + b) * Q + c] = z;
      }
    }
  }
  // a non-finite slice value reaches every replica's Z: flag the replica
  if (bad) atomicOr(zbad + p, 1);
}

}  // namespace

hipError_t compress_mode3_partials(hipStream_t s, const CompressShape& sh, int64_t t, int nrb,
                                  const float* Mpart, const double* W, float* Z, int* zbad) {
  if (sh.Q > 128) return hipErrorInvalidValue;
  dim3 grid(sh.P, sh.Q);
  if (sh.Q <= 64) {
    const size_t lds = (size_t)2 * S3_KT * 64 * sizeof(double);
    hipLaunchKernelGGL((mode3_kernel<float, float>), grid, dim3(256), lds, s, Mpart, W, t, nrb,
                       sh.M1, sh.P, sh.Q, sh.S, Z, zbad);
  } else {
    dim3 g3(sh.P, sh.Q, (sh.Q + S3_B - 1) / S3_B);
    const size_t lds = (size_t)(S3_KT * S3_B + S3_KT * sh.Q) * sizeof(double);
    hipLaunchKernelGGL((mode3_bblock_kernel<float, float>), g3, dim3(256), lds, s, Mpart, W, t,
                       nrb, sh.M1, sh.P, sh.Q, sh.S, Z, zbad);
  }
  return hipGetLastError();
}

namespace {
template <typename TM, typename TZ>
hipError_t launch_mode3(hipStream_t s, const CompressShape& sh, int64_t t, const TM* M,
                        const double* W, TZ* Z, int* zbad) {
  dim3 grid(sh.P, sh.Q);
  if (sh.Q <= 64) {
    hipLaunchKernelGGL((mode3_kernel<TM, TZ>), grid, dim3(256),
                       (size_t)2 * S3_KT * 64 * sizeof(double), s, M, W, t, 1, sh.M1, sh.P, sh.Q,
                       sh.S, Z, zbad);
  } else {
    dim3 g3(sh.P, sh.Q, (sh.Q + S3_B - 1) / S3_B);
    const size_t lds = (size_t)(S3_KT * S3_B + S3_KT * sh.Q) * sizeof(double);
    hipLaunchKernelGGL((mode3_bblock_kernel<TM, TZ>), g3, dim3(256), lds, s, M, W, t, 1, sh.M1,
                       sh.P, sh.Q, sh.S, Z, zbad);
  }
  return hipGetLastError();
}
}  // namespace

hipError_t compress_mode3(hipStream_t s, const CompressShape& sh, int64_t t, const void* M,
                          bool m_f64, const double* W, void* Z, bool z_f64, int* zbad) {
  if (sh.Q > 128) return hipErrorInvalidValue;
  if (m_f64 && z_f64) return launch_mode3(s, sh, t, (const double*)M, W, (double*)Z, zbad);
  if (m_f64 && !z_f64) return launch_mode3(s, sh, t, (const double*)M, W, (float*)Z, zbad);
  if (!m_f64 && z_f64) return launch_mode3(s, sh, t, (const float*)M, W, (double*)Z, zbad);
  return launch_mode3(s, sh, t, (const float*)M, W, (float*)Z, zbad);
}

hipError_t compress_reference(hipStream_t s, const CompressShape& sh, const void* X, bool x_f64,
                              int64_t t, const double* U, const double* V, const double* W,
                              double* T2work, int64_t t2_rows_cap, double* Mwork, void* Z,
                              bool z_f64, int* zbad) {
  const int64_t I = sh.I, J = sh.J;
  const int M1 = sh.M1;
  int64_t chunk = t2_rows_cap / I;
  if (chunk < 1) return hipErrorInvalidValue;
  for (int64_t k0 = 0; k0 < t; k0 += chunk) {
    int64_t tc = t - k0 < chunk ? t - k0 : chunk;
    // T2 (tc*I x M1) = X[k0:k0+tc] (tc*I x J) * V (J x M1)
    hipError_t e;
    if (x_f64)
      e = gemm_f64(s, (int)(tc * I), M1, (int)J, 1, (const double*)X + k0 * I * J, J, 1, 0, V, M1,
                   1, 0, T2work, M1, 1, 0, nullptr, 1.0, 0.0);
    else
      e = gemm_f32in_f64(s, (int)(tc * I), M1, (int)J, 1, (const float*)X + k0 * I * J, J, 1, 0,
                         V, M1, 1, 0, T2work, M1, 1, 0, nullptr, 1.0, 0.0);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)tc, sh.P, (sh.Q + S2_ROWS - 1) / S2_ROWS);
    size_t lds = (size_t)(S2_KT * S2_ROWS + S2_KT * sh.Q) * sizeof(double);
    hipLaunchKernelGGL(stage2_kernel, grid, dim3(256), lds, s, U, T2work, I, M1, sh.P, sh.Q, sh.S,
                       Mwork + k0 * sh.P * sh.Q * sh.Q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return compress_mode3(s, sh, t, Mwork, true, W, Z, z_f64, zbad);
}

}  // namespace octen
