// Learned warm start of the replica ALS: batch sketch, column features and
// targets, candidate factors and the judge that keeps a candidate only when
// its replica fit (Sec. 5.1 on the summary) is at least that of the plain
// warm start of Algorithm 1 (the previous factors).
//
// Column r of replica p (previous unit columns a, b, c, weight lambda):
//   a~ = lambda^(1/3) a etc. (the lambda distribution of Sec. 4.2);
//   s_a, s_b = sign of the entry of largest magnitude of a~, b~ (first on ties)
//   u = (Z_p x1 a~ x2 b~) / (||a~||^2 ||b~||^2): the change of the mode-3
//       least-squares column caused by the new batch with a~, b~ held
//   features = [s_a a~ ; s_b b~ ; s_a s_b (c~ + u) ; s_a s_b u ; sketch_p]
//              (FP32, 4Q + D)
//   sketch_p = G vec(Z_p) / ||Z_p||                         (G: D x Q^3)
// Candidate = network output with the signs undone (FP64 factors).
#include <hip/hip_runtime.h>
#include <math.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int NT = 256;
constexpr int DMAX = 32;   // sketch length
constexpr int MAXR = 32;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sketch as one contraction S[p][d] = sum_e Z_p[e] G[d][e] on
// v_mfma_f32_32x32x2f32: rows are the replicas (up to 32), columns the
// sketch rows.  Each wavefront walks a range of e eight entries at a time:
// lane (r, h) loads four consecutive entries 4h .. 4h + 3 of row r of Z and
// of G, and four MFMAs take entry i of both halves (the pairing over k is
// the same on both operands, so the sum is unchanged).  The squared norms of
// the rows of Z come along in the same pass.
// part[ch][32][33]: dots (32 x 32, replica-major) then the squared norms.
typedef float f32x16w __attribute__((ext_vector_type(16)));
typedef float f32x4w __attribute__((ext_vector_type(4)));
constexpr int SK_CHUNK = 4096;   // entries per workgroup (1024 per wavefront)

template <typename TZ>
__global__ __launch_bounds__(NT) void sketch_mfma_kernel(const TZ* __restrict__ Z,
                                                         const float* __restrict__ G, int P,
                                                         int64_t Q3, int D, int nch,
                                                         float* __restrict__ part) {
  __shared__ float red[4][32 * 33];
  const int ch = blockIdx.x;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = lane % 32, h = lane / 32;
  const int64_t w0 = (int64_t)ch * SK_CHUNK + (int64_t)wave * (SK_CHUNK / 4);
  const int64_t w1 = w0 + SK_CHUNK / 4 < Q3 ? w0 + SK_CHUNK / 4 : Q3;
  const bool zrow = r < P, grow = r < D;
  const TZ* zr = Z + (int64_t)(zrow ? r : 0) * Q3;
  const float* gr = G + (int64_t)(grow ? r : 0) * Q3;
  f32x16w acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  float zz = 0.f;
  for (int64_t e0 = w0; e0 < w1; e0 += 8) {
    float zv[4], gv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t e = e0 + 4 * h + i;
      const bool ok = e < w1;
      zv[i] = (zrow && ok) ? (float)zr[e] : 0.f;
      gv[i] = (grow && ok) ? gr[e] : 0.f;
      zz = fmaf(zv[i], zv[i], zz);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(zv[i], gv[i], acc, 0, 0, 0);
  }
  // D[i] of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4 (replica), column l % 32
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = 8 * (i / 4) + 4 * h + (i % 4);
    red[wave][row * 33 + r] = acc[i];
  }
  zz += __shfl_xor(zz, 32, 64);
  if (h == 0) red[wave][r * 33 + 32] = zz;
  __syncthreads();
  float* out = part + (int64_t)ch * 32 * 33;
  for (int e = threadIdx.x; e < 32 * 33; e += NT)
    out[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
}

// sk[p][d] = sum_ch dots / sqrt(sum_ch norms), chunks in order (FP64 sums)
__global__ void sketch_final_kernel(const float* __restrict__ part, int nch, int D,
                                    float* __restrict__ sk) {
  const int p = blockIdx.x, d = threadIdx.x;
  if (d >= D) return;
  double s = 0.0, zz = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    s += part[(int64_t)ch * 32 * 33 + p * 33 + d];
    zz += part[(int64_t)ch * 32 * 33 + p * 33 + 32];
  }
  sk[p * D + d] = zz > 0.0 ? (float)(s / sqrt(zz)) : 0.f;
}

// index of the entry of largest magnitude of x[0..Q) (first on ties), over
// one wavefront; x read with stride
__device__ int wave_argmax_abs(const double* __restrict__ x, int64_t stride, int Q, int lane) {
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int q = lane; q < Q; q += 64) {
    const double v = fabs(x[q * stride]);
    if (v > best) { best = v; bi = q; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  return bi;
}

// u[(p R + r) Q + c] for c in one range of at most UC values: one workgroup
// per (range, r, p), threads over the (a, b) pairs, FP64 sums.
constexpr int UC = 8;
template <typename TZ>
__global__ __launch_bounds__(NT) void mode3_change_kernel(const TZ* __restrict__ Z,
                                                          const double* __restrict__ F,
                                                          const double* __restrict__ lam, int Q,
                                                          int R, double* __restrict__ u) {
  __shared__ double av[128], bv[128];
  __shared__ double red[4][UC + 2];
  const int split = blockIdx.x, r = blockIdx.y, p = blockIdx.z;
  const int c0 = split * UC, nc = Q - c0 < UC ? Q - c0 : UC;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const double* Fp = F + (int64_t)p * 3 * Q * R;
  const double c3 = cbrt(lam[p * R + r]);
  for (int q = threadIdx.x; q < Q; q += NT) {
    av[q] = c3 * Fp[(int64_t)q * R + r];
    bv[q] = c3 * Fp[(int64_t)(Q + q) * R + r];
  }
  __syncthreads();
  const TZ* Zp = Z + (int64_t)p * Q * Q * Q;
  double acc[UC], na = 0.0, nb = 0.0;
#pragma unroll
  for (int j = 0; j < UC; ++j) acc[j] = 0.0;
  for (int ab = threadIdx.x; ab < Q * Q; ab += NT) {
    const double w = av[ab / Q] * bv[ab % Q];
    const TZ* z = Zp + (int64_t)ab * Q + c0;
#pragma unroll
    for (int j = 0; j < UC; ++j)
      if (j < nc) acc[j] = fma((double)z[j], w, acc[j]);
  }
  for (int q = threadIdx.x; q < Q; q += NT) {
    na = fma(av[q], av[q], na);
    nb = fma(bv[q], bv[q], nb);
  }
#pragma unroll
  for (int j = 0; j < UC; ++j) {
    const double sj = wave_sum(acc[j]);
    if (lane == 0) red[wave][j] = sj;
  }
  {
    const double sa = wave_sum(na), sb = wave_sum(nb);
    if (lane == 0) { red[wave][UC] = sa; red[wave][UC + 1] = sb; }
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    const int j = threadIdx.x;
    const double num = red[0][j] + red[1][j] + red[2][j] + red[3][j];
    const double den = (red[0][UC] + red[1][UC] + red[2][UC] + red[3][UC]) *
                       (red[0][UC + 1] + red[1][UC + 1] + red[2][UC + 1] + red[3][UC + 1]);
    u[((int64_t)p * R + r) * Q + c0 + j] = den > 0.0 ? num / den : 0.0;
  }
}

// One wavefront per column (p, r).  mode 0: features (and signs, and the
// plain scaled start); mode 1: targets with the stored signs.
__global__ __launch_bounds__(64) void columns_kernel(const double* __restrict__ F,
                                                     const double* __restrict__ lam, int P,
                                                     int Q, int R, const float* __restrict__ sk,
                                                     const double* __restrict__ u, int D,
                                                     int mode, float* __restrict__ out,
                                                     double* __restrict__ signs,
                                                     double* __restrict__ plain) {
  const int pr = blockIdx.x, p = pr / R, r = pr % R, lane = threadIdx.x;
  const double* Fp = F + (int64_t)p * 3 * Q * R;
  const double c3 = cbrt(lam[p * R + r]);
  double sa, sb;
  if (mode == 0) {
    const int ia = wave_argmax_abs(Fp + r, R, Q, lane);
    const int ib = wave_argmax_abs(Fp + (int64_t)Q * R + r, R, Q, lane);
    const double va = Fp[(int64_t)ia * R + r], vb = Fp[(int64_t)Q * R + (int64_t)ib * R + r];
    sa = va < 0.0 ? -1.0 : 1.0;
    sb = vb < 0.0 ? -1.0 : 1.0;
    if (lane == 0) { signs[2 * pr] = sa; signs[2 * pr + 1] = sb; }
  } else {
    sa = signs[2 * pr];
    sb = signs[2 * pr + 1];
  }
  const int width = mode == 0 ? 4 * Q + D : 3 * Q;
  float* row = out + (int64_t)pr * width;
  const double* ur = u + (int64_t)pr * Q;
  for (int e = lane; e < 3 * Q; e += 64) {
    const int n = e / Q, q = e % Q;
    const double v = c3 * Fp[((int64_t)n * Q + q) * R + r];
    const double sg = n == 0 ? sa : (n == 1 ? sb : sa * sb);
    const double add = (mode == 0 && n == 2) ? ur[q] : 0.0;
    row[e] = (float)(sg * (v + add));
    if (mode == 0) plain[((int64_t)p * 3 * Q + (int64_t)n * Q + q) * R + r] = v;
  }
  if (mode == 0) {
    for (int q = lane; q < Q; q += 64) row[3 * Q + q] = (float)(sa * sb * ur[q]);
    for (int d = lane; d < D; d += 64) row[4 * Q + d] = sk[p * D + d];
  }
}

// network outputs [P*R][3Q] -> candidate factors [P][3][Q][R] (signs undone)
__global__ void candidate_kernel(const float* __restrict__ Y, const double* __restrict__ signs,
                                 int P, int Q, int R, double* __restrict__ cand) {
  const int64_t total = (int64_t)P * 3 * Q * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % R);
    const int64_t t = e / R;
    const int q = (int)(t % Q), n = (int)((t / Q) % 3), p = (int)(t / (3 * Q));
    const int pr = p * R + r;
    const double sa = signs[2 * pr], sb = signs[2 * pr + 1];
    const double s = n == 0 ? sa : (n == 1 ? sb : sa * sb);
    cand[e] = s * (double)Y[(int64_t)pr * 3 * Q + (int64_t)n * Q + q];
  }
}

// Partial fitness terms of two starting points per replica over a range of
// the third index: <Y_p, [[A, B, C]]> and ||Y_p||^2.  One thread per (a, b)
// pair at a time, products A(a,:) * B(b,:) held in registers, C(c0:c1, :)
// in LDS.  part[p][which][split][2].
template <typename TY>
__global__ __launch_bounds__(NT) void judge_partial_kernel(const TY* __restrict__ Y, int P, int Q,
                                                           int R, const double* __restrict__ plain,
                                                           const double* __restrict__ cand,
                                                           int nsplit, double* __restrict__ part) {
  extern __shared__ double Cs[];   // [c1 - c0][R]
  __shared__ double red[2][4];
  const int split = blockIdx.x, which = blockIdx.y, p = blockIdx.z;
  const int c0 = (int)((int64_t)split * Q / nsplit), c1 = (int)((int64_t)(split + 1) * Q / nsplit);
  const double* Fp = (which == 0 ? plain : cand) + (int64_t)p * 3 * Q * R;
  const double *A = Fp, *B = Fp + (int64_t)Q * R, *C = Fp + 2 * (int64_t)Q * R;
  for (int e = threadIdx.x; e < (c1 - c0) * R; e += NT) Cs[e] = C[(int64_t)c0 * R + e];
  __syncthreads();
  const TY* Yp = Y + (int64_t)p * Q * Q * Q;
  double inner = 0.0, yy = 0.0;
  for (int ab = threadIdx.x; ab < Q * Q; ab += NT) {
    const int a = ab / Q, b = ab % Q;
    double w[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) w[r] = r < R ? A[(int64_t)a * R + r] * B[(int64_t)b * R + r] : 0.0;
    const TY* y = Yp + (int64_t)ab * Q;
    for (int c = c0; c < c1; ++c) {
      const double* cr = Cs + (int64_t)(c - c0) * R;
      double xh = 0.0;
#pragma unroll
      for (int r = 0; r < MAXR; ++r)
        if (r < R) xh = fma(w[r], cr[r], xh);
      const double v = (double)y[c];
      inner = fma(v, xh, inner);
      yy = fma(v, v, yy);
    }
  }
  inner = wave_sum(inner);
  yy = wave_sum(yy);
  const int wave = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) { red[0][wave] = inner; red[1][wave] = yy; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + (((int64_t)p * 2 + which) * nsplit + split) * 2;
    o[0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    o[1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Per replica: fit of both starting points, the choice, and the chosen init.
// fits[p][2] (plain, candidate); keep[p] = 1 when the candidate is kept.
__global__ __launch_bounds__(NT) void judge_final_kernel(const double* __restrict__ part,
                                                         int nsplit, int P, int Q, int R,
                                                         const double* __restrict__ plain,
                                                         const double* __restrict__ cand,
                                                         double* __restrict__ fits,
                                                         int* __restrict__ keep,
                                                         double* __restrict__ init) {
  __shared__ double gsum[2][NT];
  __shared__ int s_keep;
  const int p = blockIdx.x;
  const int64_t QR = (int64_t)Q * R;
  // ||[[A,B,C]]||^2 = sum_{r,s} (A^T A)(B^T B)(C^T C) for both starting points
  for (int which = 0; which < 2; ++which) {
    const double* Fp = (which == 0 ? plain : cand) + (int64_t)p * 3 * QR;
    double s = 0.0;
    for (int rs = threadIdx.x; rs < R * R; rs += NT) {
      const int r = rs / R, t = rs % R;
      double g = 1.0;
      for (int n = 0; n < 3; ++n) {
        double d = 0.0;
        for (int q = 0; q < Q; ++q) d = fma(Fp[n * QR + (int64_t)q * R + r], Fp[n * QR + (int64_t)q * R + t], d);
        g *= d;
      }
      s += g;
    }
    gsum[which][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      gsum[0][threadIdx.x] += gsum[0][threadIdx.x + w];
      gsum[1][threadIdx.x] += gsum[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double f[2];
    for (int which = 0; which < 2; ++which) {
      double inner = 0.0, yy = 0.0;
      for (int sp = 0; sp < nsplit; ++sp) {
        const double* o = part + (((int64_t)p * 2 + which) * nsplit + sp) * 2;
        inner += o[0];
        yy += o[1];
      }
      const double sse = yy - 2.0 * inner + gsum[which][0];
      f[which] = yy > 0.0 ? 1.0 - sqrt(sse > 0.0 ? sse : 0.0) / sqrt(yy) : 0.0;
      fits[2 * p + which] = f[which];
    }
    s_keep = f[1] >= f[0] ? 1 : 0;
    keep[p] = s_keep;
  }
  __syncthreads();
  const double* src = (s_keep ? cand : plain) + (int64_t)p * 3 * QR;
  for (int64_t e = threadIdx.x; e < 3 * QR; e += NT) init[(int64_t)p * 3 * QR + e] = src[e];
}

}  // namespace

hipError_t ws_sketch(hipStream_t s, const void* Z, bool z_f64, int P, int Q, const float* G, int D,
                     double* part, int64_t part_cap, float* sk) {
  if (D < 1 || D > DMAX || P > 32) return hipErrorInvalidValue;
  const int64_t Q3 = (int64_t)Q * Q * Q;
  const int nch = (int)((Q3 + SK_CHUNK - 1) / SK_CHUNK);
  // the partials are FP32: part_cap counts doubles
  if ((int64_t)nch * 32 * 33 > 2 * part_cap) return hipErrorInvalidValue;
  float* pf = (float*)part;
  if (z_f64)
    hipLaunchKernelGGL(sketch_mfma_kernel<double>, dim3(nch), dim3(NT), 0, s, (const double*)Z, G,
                       P, Q3, D, nch, pf);
  else
    hipLaunchKernelGGL(sketch_mfma_kernel<float>, dim3(nch), dim3(NT), 0, s, (const float*)Z, G, P,
                       Q3, D, nch, pf);
  hipLaunchKernelGGL(sketch_final_kernel, dim3(P), dim3(64), 0, s, pf, nch, D, sk);
  return hipGetLastError();
}

int64_t ws_sketch_part_len(int P, int Q, int D) {
  (void)P;
  (void)D;
  const int64_t Q3 = (int64_t)Q * Q * Q;
  return ((Q3 + SK_CHUNK - 1) / SK_CHUNK) * 32 * 33 / 2 + 1;
}

hipError_t ws_mode3_change(hipStream_t s, const void* Z, bool z_f64, const double* F,
                           const double* lam, int P, int Q, int R, double* u) {
  if (Q > 128) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((Q + UC - 1) / UC), (unsigned)R, (unsigned)P);
  if (z_f64)
    hipLaunchKernelGGL(mode3_change_kernel<double>, grid, dim3(NT), 0, s, (const double*)Z, F, lam,
                       Q, R, u);
  else
    hipLaunchKernelGGL(mode3_change_kernel<float>, grid, dim3(NT), 0, s, (const float*)Z, F, lam,
                       Q, R, u);
  return hipGetLastError();
}

hipError_t ws_columns(hipStream_t s, const double* F, const double* lam, int P, int Q, int R,
                      const float* sk, const double* u, int D, bool targets, float* out,
                      double* signs, double* plain) {
  hipLaunchKernelGGL(columns_kernel, dim3(P * R), dim3(64), 0, s, F, lam, P, Q, R, sk, u, D,
                     targets ? 1 : 0, out, signs, plain);
  return hipGetLastError();
}

hipError_t ws_candidate(hipStream_t s, const float* Y, const double* signs, int P, int Q, int R,
                        double* cand) {
  const int64_t total = (int64_t)P * 3 * Q * R;
  int grid = (int)((total + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(candidate_kernel, dim3(grid), dim3(256), 0, s, Y, signs, P, Q, R, cand);
  return hipGetLastError();
}

int ws_judge_splits(int Q) { return Q >= 8 ? Q / 8 : 1; }

hipError_t ws_judge(hipStream_t s, const void* Y, bool y_f64, int P, int Q, int R,
                    const double* plain, const double* cand, double* part, double* fits,
                    int* keep, double* init) {
  if (R > MAXR) return hipErrorInvalidValue;
  const int nsplit = ws_judge_splits(Q);
  const int cmax = (Q + nsplit - 1) / nsplit + 1;
  const size_t lds = (size_t)cmax * R * sizeof(double);
  const dim3 grid((unsigned)nsplit, 2, (unsigned)P);
  if (y_f64)
    hipLaunchKernelGGL(judge_partial_kernel<double>, grid, dim3(NT), lds, s, (const double*)Y, P,
                       Q, R, plain, cand, nsplit, part);
  else
    hipLaunchKernelGGL(judge_partial_kernel<float>, grid, dim3(NT), lds, s, (const float*)Y, P, Q,
                       R, plain, cand, nsplit, part);
  hipLaunchKernelGGL(judge_final_kernel, dim3(P), dim3(NT), 0, s, part, nsplit, P, Q, R, plain,
                     cand, fits, keep, init);
  return hipGetLastError();
}

}  // namespace octen
