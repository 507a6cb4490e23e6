// Factor matching and recovery (Sec. 4.2, Eq. 5; Sec. 4.3, Eq. 6-7;
// Algorithm 1 matching loop and final solve).  All FP64.
//
// Matching reads only the anchor rows (the first S rows of every replica
// factor, produced by the shared compression columns of Eq. 1).  Pairing is
// an exclusive greedy assignment done by one wavefront: each round every lane
// scans a strided share of the free entries and a butterfly reduction picks
// the maximum, ties going to the smallest reference column, then the
// smallest replica column.
#include <hip/hip_runtime.h>
#include <math.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int MAXR = 32;

// A candidate entry: its value and key = (reference column << 6) | replica
// row, so that the smaller key is the tie-break order (column first, then
// row); KEY_NONE marks no candidate.
struct Cand {
  double v;
  int key;
};
constexpr int KEY_NONE = 0x7fffffff;

__device__ __forceinline__ bool better(const Cand& a, const Cand& b) {
  return a.v > b.v || (a.v == b.v && a.key < b.key);
}

__device__ __forceinline__ Cand wave_best(Cand x) {
  for (int off = 32; off > 0; off >>= 1) {
    Cand y;
    y.v = __shfl_xor(x.v, off, 64);
    y.key = __shfl_xor(x.key, off, 64);
    if (better(y, x)) x = y;
  }
  return x;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Exclusive greedy assignment on sim[r][c] (R x R in LDS, R <= 32) by one
// wavefront of 64 lanes.  perm[r] = c.  Returns the smallest gap between a
// chosen entry and its best free competitor in the same row or column (+inf
// if none).  Each lane keeps its entries (e = lane + 64 k) in registers and
// every lane tracks the free rows and columns as the same bit masks, so a
// round is two butterfly reductions with no barrier.
// EPL entries per lane: R * R <= 64 * EPL.
template <int EPL>
__device__ double greedy_wave(const double* sim, int R, int* perm) {
  const int lane = threadIdx.x;
  const int n = R * R, kmax = (n + 63) / 64;
  double sv[EPL];
  int sk[EPL];   // (c << 6) | r; 63 in both fields (bits never free) past n
#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    const int e = lane + 64 * k;
    const bool in = e < n;
    sv[k] = in ? sim[e] : -INFINITY;
    sk[k] = in ? ((e % R) << 6) | (e / R) : (63 << 6) | 63;
  }
  unsigned long long rowm = (1ull << R) - 1ull, colm = rowm;
  auto is_free = [&](int key) {
    return ((rowm >> (key & 63)) & 1ull) && ((colm >> (key >> 6)) & 1ull);
  };
  double margin = INFINITY;
  for (int round = 0; round < R; ++round) {
    Cand best{-INFINITY, KEY_NONE};
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      if (k < kmax && is_free(sk[k])) {
        const Cand x{sv[k], sk[k]};
        if (better(x, best)) best = x;
      }
    }
    best = wave_best(best);
    int br, bc;
    if (best.key == KEY_NONE) {   // every free entry is NaN: take the first free pair
      br = __builtin_ctzll(rowm);
      bc = __builtin_ctzll(colm);
    } else {
      br = best.key & 63;
      bc = best.key >> 6;
    }
    double rival = -INFINITY;
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      if (k < kmax && is_free(sk[k])) {
        const int r = sk[k] & 63, c = sk[k] >> 6;
        if ((r == br) != (c == bc)) rival = sv[k] > rival ? sv[k] : rival;
      }
    }
    rival = wave_max(rival);
    if (rival > -INFINITY) {
      const double g = best.v - rival;
      margin = g < margin ? g : margin;
    }
    if (lane == 0) perm[br] = bc;
    rowm &= ~(1ull << br);
    colm &= ~(1ull << bc);
  }
  __syncthreads();
  return margin;
}

// One block (64 lanes) per replica p.
template <int EPL>
__global__ __launch_bounds__(64) void align_kernel(int P, int Q, int R, int S,
                                                   const double* __restrict__ F,
                                                   const double* __restrict__ lam,
                                                   double* __restrict__ aligned,
                                                   int* __restrict__ perm_out,
                                                   double* __restrict__ margin_out) {
  extern __shared__ double sm[];
  const int SR = S * R;
  double* a0 = sm;                 // [3][S][R] reference anchors (lambda distributed)
  double* ap = a0 + 3 * SR;        // [3][S][R] this replica's anchors
  double* sim = ap + 3 * SR;       // [R][R]
  __shared__ double c0[MAXR], cp[MAXR];
  __shared__ int perm[MAXR];
  const int p = blockIdx.x, lane = threadIdx.x;
  const int64_t QR = (int64_t)Q * R;
  const double* F0 = F;
  const double* Fp = F + (int64_t)p * 3 * QR;
  if (lane < R) {
    c0[lane] = cbrt(lam[lane]);
    cp[lane] = cbrt(lam[(int64_t)p * R + lane]);
  }
  __syncthreads();
  double* Ap = aligned + (int64_t)p * 3 * QR;
  // element loops over [3][Q][R]: lane = (row offset lq, column lr), rows
  // stepped by rpl = 64 / R; no division inside the loops
  const int rpl = 64 / R, lq = lane / R, lr = lane - (lane / R) * R;
  if (p == 0) {
    if (lq < rpl)
      for (int n = 0; n < 3; ++n)
#pragma unroll 8
        for (int q = lq; q < Q; q += rpl) {
          const int64_t e = n * QR + (int64_t)q * R + lr;
          Ap[e] = F0[e] * c0[lr];
        }
    if (lane < R) perm_out[lane] = lane;
    if (lane == 0) margin_out[0] = INFINITY;
    return;
  }
  for (int e = lane; e < 3 * SR; e += 64) {
    const int n = e / SR, rem = e % SR;       // rem = s * R + r
    const int r = rem % R;
    a0[e] = F0[n * QR + rem] * c0[r];
    ap[e] = Fp[n * QR + rem] * cp[r];
  }
  __syncthreads();
  // sim[r][c] = prod_n |cos(ap[n][:, r], a0[n][:, c])|
  for (int e = lane; e < R * R; e += 64) {
    const int r = e / R, c = e % R;
    double s = 1.0;
    for (int n = 0; n < 3; ++n) {
      double num = 0.0, na = 0.0, nb = 0.0;
      for (int q = 0; q < S; ++q) {
        const double x = ap[n * SR + q * R + r], y = a0[n * SR + q * R + c];
        num = fma(x, y, num);
        na = fma(x, x, na);
        nb = fma(y, y, nb);
      }
      const double den = sqrt(na) * sqrt(nb);
      s *= den > 0.0 ? fabs(num) / den : 0.0;
    }
    sim[e] = s;
  }
  __syncthreads();
  const double margin = greedy_wave<EPL>(sim, R, perm);
  if (lane == 0) margin_out[p] = margin;
  if (lane < R) perm_out[(int64_t)p * R + lane] = perm[lane];
  // least-squares scale of each anchor column onto the reference's
  for (int e = lane; e < 3 * R; e += 64) {
    const int n = e / R, r = e % R, rr = perm[r];
    double num = 0.0, den = 0.0;
    for (int q = 0; q < S; ++q) {
      const double x = ap[n * SR + q * R + r];
      num = fma(a0[n * SR + q * R + rr], x, num);
      den = fma(x, x, den);
    }
    sim[e] = den > 0.0 ? num / den : 0.0;   // sim reused as d[n][r]
  }
  __syncthreads();
  if (lq < rpl) {
    const int pr = perm[lr];
    for (int n = 0; n < 3; ++n) {
      const double d = sim[n * R + lr];
      // eight rows' loads in flight before their stores
#pragma unroll 8
      for (int q = lq; q < Q; q += rpl) {
        const int64_t e = n * QR + (int64_t)q * R + lr;
        Ap[n * QR + (int64_t)q * R + pr] = d * (Fp[e] * cp[lr]);
      }
    }
  }
}

__global__ void stack_kernel(int P, int Q, int R, int S, const double* __restrict__ aligned,
                             double* __restrict__ rhs) {
  const int M1 = S + P * (Q - S);
  const int64_t tot = (int64_t)3 * M1 * R;
  const int64_t QR = (int64_t)Q * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / ((int64_t)M1 * R));
    const int64_t rem = e % ((int64_t)M1 * R);
    const int row = (int)(rem / R), r = (int)(rem % R);
    double v;
    if (row < S) {
      v = 0.0;
      for (int p = 0; p < P; ++p) v += aligned[((int64_t)p * 3 + n) * QR + (int64_t)row * R + r];
      v /= (double)P;
    } else {
      const int p = (row - S) / (Q - S), q = S + (row - S) % (Q - S);
      v = aligned[((int64_t)p * 3 + n) * QR + (int64_t)q * R + r];
    }
    rhs[e] = v;
  }
}

// Column r of X [n][R]: 2-norm and first index of the largest |x|; one block
// per column (short columns: one launch).
__device__ void column_stats(int64_t n, int R, const double* X, int r, double* s_sum, double* s_val,
                             int64_t* s_idx, double* nrm, double* signv) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double s = 0.0, best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = tid; i < n; i += nt) {
    const double v = X[i * R + r];
    s = fma(v, v, s);
    const double a = fabs(v);
    if (a > best) { best = a; bi = i; }
  }
  s_sum[tid] = s;
  s_val[tid] = best;
  s_idx[tid] = bi;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s_sum[tid] += s_sum[tid + w];
      const double ov = s_val[tid + w];
      const int64_t oi = s_idx[tid + w];
      if (ov > s_val[tid] || (ov == s_val[tid] && oi < s_idx[tid])) { s_val[tid] = ov; s_idx[tid] = oi; }
    }
    __syncthreads();
  }
  *nrm = sqrt(s_sum[0]);
  const int64_t idx = s_idx[0];
  *signv = idx < n ? X[idx * R + r] : 0.0;
}

__global__ __launch_bounds__(256) void canon_kernel(int64_t n, int R, const double* __restrict__ X,
                                                    double* __restrict__ out,
                                                    double* __restrict__ kfac) {
  __shared__ double s_sum[256], s_val[256];
  __shared__ int64_t s_idx[256];
  const int r = blockIdx.x;
  double nrm, sv;
  column_stats(n, R, X, r, s_sum, s_val, s_idx, &nrm, &sv);
  const double sg = sv > 0.0 ? 1.0 : (sv < 0.0 ? -1.0 : 1.0);
  const double k = (nrm > 0.0 ? nrm : 1.0) * sg;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) out[i * R + r] = X[i * R + r] / k;
  if (threadIdx.x == 0) kfac[r] = k;
}

__global__ __launch_bounds__(256) void colnorm_kernel(int64_t n, int R, const double* __restrict__ X,
                                                      double* __restrict__ norms) {
  __shared__ double s_sum[256], s_val[256];
  __shared__ int64_t s_idx[256];
  const int r = blockIdx.x;
  double nrm, sv;
  column_stats(n, R, X, r, s_sum, s_val, s_idx, &nrm, &sv);
  if (threadIdx.x == 0) norms[r] = nrm;
}

// colnorm_kernel over four matrices at once: block b takes matrix b / R
// (Ac, Ap with nA rows, Bc, Bp with nB rows), column b % R.
__global__ __launch_bounds__(256) void colnorm4_kernel(int64_t nA, int64_t nB, int R,
                                                       const double* __restrict__ X0,
                                                       const double* __restrict__ X1,
                                                       const double* __restrict__ X2,
                                                       const double* __restrict__ X3,
                                                       double* __restrict__ norms) {
  __shared__ double s_sum[256], s_val[256];
  __shared__ int64_t s_idx[256];
  const int m = blockIdx.x / R, r = blockIdx.x % R;
  const double* X = m == 0 ? X0 : m == 1 ? X1 : m == 2 ? X2 : X3;
  const int64_t n = m < 2 ? nA : nB;
  double nrm, sv;
  column_stats(n, R, X, r, s_sum, s_val, s_idx, &nrm, &sv);
  if (threadIdx.x == 0) norms[m * R + r] = nrm;
}

// canon_kernel over two matrices at once: block b takes matrix b / R, column
// b % R.
__global__ __launch_bounds__(256) void canon2_kernel(int64_t nA, int64_t nB, int R,
                                                     const double* __restrict__ XA,
                                                     double* __restrict__ outA,
                                                     double* __restrict__ kA,
                                                     const double* __restrict__ XB,
                                                     double* __restrict__ outB,
                                                     double* __restrict__ kB) {
  __shared__ double s_sum[256], s_val[256];
  __shared__ int64_t s_idx[256];
  const int m = blockIdx.x / R, r = blockIdx.x % R;
  const double* X = m == 0 ? XA : XB;
  double* out = m == 0 ? outA : outB;
  const int64_t n = m == 0 ? nA : nB;
  double nrm, sv;
  column_stats(n, R, X, r, s_sum, s_val, s_idx, &nrm, &sv);
  const double sg = sv > 0.0 ? 1.0 : (sv < 0.0 ? -1.0 : 1.0);
  const double k = (nrm > 0.0 ? nrm : 1.0) * sg;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) out[i * R + r] = X[i * R + r] / k;
  if (threadIdx.x == 0) (m == 0 ? kA : kB)[r] = k;
}

__global__ __launch_bounds__(256) void copy3_kernel(double* __restrict__ d1,
                                                    const double* __restrict__ s1, int64_t n1,
                                                    double* __restrict__ d2,
                                                    const double* __restrict__ s2, int64_t n2,
                                                    double* __restrict__ d3,
                                                    const double* __restrict__ s3, int64_t n3) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n1; e += stride) d1[e] = s1[e];
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n2; e += stride) d2[e] = s2[e];
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n3; e += stride) d3[e] = s3[e];
}

// Column statistics of X [n][R] (R <= 32) in two passes.  Pass 1: block b
// takes rows [b rows_per, (b + 1) rows_per); its threads form groups of R,
// thread (g, r) reads column r of rows g, g + ngrp, ... (a group reads whole
// rows: coalesced); per block and column it keeps the sum of squares and the
// largest |x| with its first row, combining the groups in order.
// part: [2][G][R] f64 (sums, largest |x|), pidx: [G][R] rows.
__global__ __launch_bounds__(256) void colstat_part_kernel(int64_t n, int R, int64_t rows_per,
                                                           const double* __restrict__ X,
                                                           double* __restrict__ part,
                                                           int64_t* __restrict__ pidx, int G) {
  __shared__ double s_sum[256], s_val[256];
  __shared__ int64_t s_idx[256];
  const int tid = threadIdx.x, ngrp = 256 / R;
  const int grp = tid / R, r = tid - grp * R;
  const int64_t i0 = (int64_t)blockIdx.x * rows_per;
  const int64_t i1 = i0 + rows_per < n ? i0 + rows_per : n;
  double sum = 0.0, best = -1.0;
  int64_t bi = INT64_MAX;
  if (grp < ngrp) {
    for (int64_t i = i0 + grp; i < i1; i += ngrp) {
      const double v = X[i * R + r];
      sum = fma(v, v, sum);
      const double av = fabs(v);
      if (av > best) { best = av; bi = i; }
    }
  }
  s_sum[tid] = sum;
  s_val[tid] = best;
  s_idx[tid] = bi;
  __syncthreads();
  if (tid < R) {
    double ss = 0.0, bv = -1.0;
    int64_t bx = INT64_MAX;
    for (int g = 0; g < ngrp; ++g) {
      const int t = g * R + tid;
      ss += s_sum[t];
      if (s_val[t] > bv || (s_val[t] == bv && s_idx[t] < bx)) { bv = s_val[t]; bx = s_idx[t]; }
    }
    part[(int64_t)blockIdx.x * R + tid] = ss;
    part[((int64_t)G + blockIdx.x) * R + tid] = bv;
    pidx[(int64_t)blockIdx.x * R + tid] = bx;
  }
}

// Pass 2 (one block): for column r, eight threads take the blocks b = g,
// g + 8, ... (g = 0..7, in order, loads unrolled four deep), then thread g = 0
// combines the eight in order: 2-norm; with kfac, also kfac[r] = norm (1 when
// zero) times the sign of the first largest-magnitude entry.
__global__ __launch_bounds__(256) void colstat_final_kernel(int64_t n, int R, int G,
                                                            const double* __restrict__ part,
                                                            const int64_t* __restrict__ pidx,
                                                            const double* __restrict__ X,
                                                            double* __restrict__ norms,
                                                            double* __restrict__ kfac) {
  __shared__ double s_sum[256], s_val[256];
  __shared__ int64_t s_idx[256];
  const int tid = threadIdx.x, r = tid & 31, g = tid >> 5;
  double ss = 0.0, bv = -1.0;
  int64_t bx = INT64_MAX;
  if (r < R) {
    for (int b0 = g; b0 < G; b0 += 32) {
      double sv[4], vv[4];
      int64_t xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + 8 * u;
        const bool ok = b < G;
        sv[u] = ok ? part[(int64_t)b * R + r] : 0.0;
        vv[u] = ok ? part[((int64_t)G + b) * R + r] : -1.0;
        xv[u] = ok ? pidx[(int64_t)b * R + r] : INT64_MAX;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ss += sv[u];
        if (vv[u] > bv || (vv[u] == bv && xv[u] < bx)) { bv = vv[u]; bx = xv[u]; }
      }
    }
  }
  s_sum[tid] = ss;
  s_val[tid] = bv;
  s_idx[tid] = bx;
  __syncthreads();
  if (g != 0 || r >= R) return;
  for (int h = 1; h < 8; ++h) {
    const int t = h * 32 + r;
    ss += s_sum[t];
    if (s_val[t] > bv || (s_val[t] == bv && s_idx[t] < bx)) { bv = s_val[t]; bx = s_idx[t]; }
  }
  const double nrm = sqrt(ss);
  if (norms) norms[r] = nrm;
  if (kfac) {
    const double sv = bx < n ? X[bx * R + r] : 0.0;
    const double sg = sv > 0.0 ? 1.0 : (sv < 0.0 ? -1.0 : 1.0);
    kfac[r] = (nrm > 0.0 ? nrm : 1.0) * sg;
  }
}

// out[i][r] = X[i][r] / kfac[r].
__global__ __launch_bounds__(256) void colscale_kernel(int64_t n, int R, const double* __restrict__ X,
                                                       const double* __restrict__ kfac,
                                                       double* __restrict__ out) {
  const int64_t total = n * R;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256)
    out[e] = X[e] / kfac[e % R];
}

// cross: [2][R][R] = Ac^T Ap and Bc^T Bp; norms: [4][R] = |Ac|, |Ap|, |Bc|, |Bp|.
template <int EPL>
__global__ __launch_bounds__(64) void tmatch_kernel(int R, const double* __restrict__ cross,
                                                    const double* __restrict__ norms,
                                                    int* __restrict__ tperm,
                                                    double* __restrict__ tsign,
                                                    double* __restrict__ tmargin) {
  __shared__ double sim[MAXR * MAXR];
  __shared__ int perm[MAXR];
  const int lane = threadIdx.x;
  const double* ca = cross;
  const double* cb = cross + R * R;
  const double *nac = norms, *nap = norms + R, *nbc = norms + 2 * R, *nbp = norms + 3 * R;
  for (int e = lane; e < R * R; e += 64) {
    const int r = e / R, c = e % R;
    const double da = nac[r] * nap[c], db = nbc[r] * nbp[c];
    sim[e] = fabs(ca[e]) / (da > 0.0 ? da : 1.0) * fabs(cb[e]) / (db > 0.0 ? db : 1.0);
  }
  __syncthreads();
  const double margin = greedy_wave<EPL>(sim, R, perm);
  if (lane < R) {
    const int c = perm[lane];
    const double a = ca[lane * R + c], b = cb[lane * R + c];
    double s = (a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0)) * (b > 0.0 ? 1.0 : (b < 0.0 ? -1.0 : 0.0));
    tperm[lane] = c;
    tsign[lane] = s == 0.0 ? 1.0 : s;
  }
  if (lane == 0) *tmargin = margin;
}

__global__ void temporal_prep_kernel(int M1, int R, const double* __restrict__ H,
                                     const int* __restrict__ tperm,
                                     const double* __restrict__ tsign,
                                     const double* __restrict__ ka, const double* __restrict__ kb,
                                     double* __restrict__ kappa, double* __restrict__ Hcur,
                                     const double* __restrict__ rhs2, double* __restrict__ rhs_c,
                                     int have_prev) {
  const int64_t tot = (int64_t)M1 * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / R;
    const int r = (int)(e % R);
    const double kap = ka[r] * kb[r];
    if (e < R) kappa[e] = ka[e] * kb[e];
    double h = 0.0;
    if (have_prev) h = H[m * R + tperm[r]] * tsign[r];
    Hcur[e] = h;
    rhs_c[e] = rhs2[e] - h / kap;
  }
}

__global__ void temporal_finish_kernel(int R, int64_t Kold, int64_t t,
                                       const double* __restrict__ kappa,
                                       const int* __restrict__ tperm,
                                       const double* __restrict__ tsign,
                                       double* __restrict__ Cnew, double* __restrict__ Chist,
                                       double* __restrict__ tmp, int have_prev, int phase) {
  if (phase == 0) {
    // tmp = old rows permuted and sign-fixed; Cnew scaled by kappa
    const int64_t tot = Kold * R;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t k = e / R;
      const int r = (int)(e % R);
      tmp[e] = have_prev ? Chist[k * R + tperm[r]] * tsign[r] : Chist[e];
    }
    const int64_t tn = t * R;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tn;
         e += (int64_t)gridDim.x * blockDim.x)
      Cnew[e] *= kappa[e % R];
  } else {
    const int64_t tot = (Kold + t) * R;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x)
      Chist[e] = e < Kold * R ? tmp[e] : Cnew[e - Kold * R];
  }
}

__global__ void weights_kernel(int M1, int S, int P, double* w, double* w2) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < M1; m += gridDim.x * blockDim.x) {
    w[m] = m < S ? sqrt((double)P) : 1.0;
    w2[m] = m < S ? (double)P : 1.0;
  }
}

inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t rec_align(hipStream_t s, int P, int Q, int R, int S, const double* F,
                     const double* lam, double* aligned, int* perm, double* margin) {
  if (R > MAXR) return hipErrorInvalidValue;
  const int simn = R * R > 3 * R ? R * R : 3 * R;
  size_t lds = (size_t)(6 * S * R + simn) * sizeof(double);
  if (R * R <= 256)
    hipLaunchKernelGGL(align_kernel<4>, dim3(P), dim3(64), lds, s, P, Q, R, S, F, lam, aligned,
                       perm, margin);
  else if (R * R <= 512)
    hipLaunchKernelGGL(align_kernel<8>, dim3(P), dim3(64), lds, s, P, Q, R, S, F, lam, aligned,
                       perm, margin);
  else
    hipLaunchKernelGGL(align_kernel<16>, dim3(P), dim3(64), lds, s, P, Q, R, S, F, lam, aligned,
                       perm, margin);
  return hipGetLastError();
}

hipError_t rec_stack(hipStream_t s, int P, int Q, int R, int S, const double* aligned, double* rhs) {
  const int M1 = S + P * (Q - S);
  hipLaunchKernelGGL(stack_kernel, dim3(grid_for((int64_t)3 * M1 * R)), dim3(256), 0, s, P, Q, R,
                     S, aligned, rhs);
  return hipGetLastError();
}

// Blocks of pass 1: at least 64 rows each, at most 256 blocks (and within
// the work buffer: 3 G R values).
static int colstat_blocks(int64_t n, int R, int64_t work_len, int64_t* rows_per) {
  int64_t rp = (n + 255) / 256;
  if (rp < 64) rp = 64;
  int64_t G = (n + rp - 1) / rp;
  while (G > 1 && 3 * G * R > work_len) {
    rp *= 2;
    G = (n + rp - 1) / rp;
  }
  *rows_per = rp;
  return (int)(G < 1 ? 1 : G);
}

static hipError_t colstat(hipStream_t s, int64_t n, int R, const double* X, double* norms,
                          double* kfac, double* work, int64_t work_len) {
  if (R > 32 || 3 * (int64_t)R > work_len) return hipErrorInvalidValue;
  int64_t rows_per;
  const int G = colstat_blocks(n, R, work_len, &rows_per);
  double* part = work;
  int64_t* pidx = (int64_t*)(work + 2 * (int64_t)G * R);
  hipLaunchKernelGGL(colstat_part_kernel, dim3(G), dim3(256), 0, s, n, R, rows_per, X, part, pidx, G);
  hipLaunchKernelGGL(colstat_final_kernel, dim3(1), dim3(256), 0, s, n, R, G, part, pidx, X, norms,
                     kfac);
  return hipGetLastError();
}

// Columns shorter than this take the one-launch kernels (one block per column).
constexpr int64_t COLSTAT_SHORT = 16384;

hipError_t rec_canon(hipStream_t s, int64_t n, int R, const double* X, double* out, double* kfac,
                     double* work, int64_t work_len) {
  if (n < COLSTAT_SHORT) {
    hipLaunchKernelGGL(canon_kernel, dim3(R), dim3(256), 0, s, n, R, X, out, kfac);
    return hipGetLastError();
  }
  hipError_t e = colstat(s, n, R, X, nullptr, kfac, work, work_len);
  if (e != hipSuccess) return e;
  const int64_t total = n * R;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(colscale_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, R, X, kfac, out);
  return hipGetLastError();
}

hipError_t rec_col_norms(hipStream_t s, int64_t n, int R, const double* X, double* norms,
                         double* work, int64_t work_len) {
  if (n < COLSTAT_SHORT) {
    hipLaunchKernelGGL(colnorm_kernel, dim3(R), dim3(256), 0, s, n, R, X, norms);
    return hipGetLastError();
  }
  return colstat(s, n, R, X, norms, nullptr, work, work_len);
}

hipError_t rec_col_norms4(hipStream_t s, int64_t nA, int64_t nB, int R, const double* Ac,
                          const double* Ap, const double* Bc, const double* Bp, double* norms,
                          double* work, int64_t work_len) {
  if (nA < COLSTAT_SHORT && nB < COLSTAT_SHORT) {
    hipLaunchKernelGGL(colnorm4_kernel, dim3(4 * R), dim3(256), 0, s, nA, nB, R, Ac, Ap, Bc, Bp,
                       norms);
    return hipGetLastError();
  }
  hipError_t e = rec_col_norms(s, nA, R, Ac, norms, work, work_len);
  if (e == hipSuccess) e = rec_col_norms(s, nA, R, Ap, norms + R, work, work_len);
  if (e == hipSuccess) e = rec_col_norms(s, nB, R, Bc, norms + 2 * R, work, work_len);
  if (e == hipSuccess) e = rec_col_norms(s, nB, R, Bp, norms + 3 * R, work, work_len);
  return e;
}

hipError_t rec_canon2(hipStream_t s, int64_t nA, int64_t nB, int R, const double* XA,
                      double* outA, double* kA, const double* XB, double* outB, double* kB,
                      double* work, int64_t work_len) {
  if (nA < COLSTAT_SHORT && nB < COLSTAT_SHORT) {
    hipLaunchKernelGGL(canon2_kernel, dim3(2 * R), dim3(256), 0, s, nA, nB, R, XA, outA, kA, XB,
                       outB, kB);
    return hipGetLastError();
  }
  hipError_t e = rec_canon(s, nA, R, XA, outA, kA, work, work_len);
  if (e == hipSuccess) e = rec_canon(s, nB, R, XB, outB, kB, work, work_len);
  return e;
}

hipError_t rec_copy3(hipStream_t s, double* d1, const double* s1, int64_t n1, double* d2,
                     const double* s2, int64_t n2, double* d3, const double* s3, int64_t n3) {
  int64_t n = n1 > n2 ? n1 : n2;
  if (n3 > n) n = n3;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(copy3_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d1, s1, n1, d2, s2,
                     n2, d3, s3, n3);
  return hipGetLastError();
}

hipError_t rec_tmatch(hipStream_t s, int R, const double* cross, const double* norms, int* tperm,
                      double* tsign, double* tmargin) {
  if (R > MAXR) return hipErrorInvalidValue;
  if (R * R <= 256)
    hipLaunchKernelGGL(tmatch_kernel<4>, dim3(1), dim3(64), 0, s, R, cross, norms, tperm, tsign,
                       tmargin);
  else if (R * R <= 512)
    hipLaunchKernelGGL(tmatch_kernel<8>, dim3(1), dim3(64), 0, s, R, cross, norms, tperm, tsign,
                       tmargin);
  else
    hipLaunchKernelGGL(tmatch_kernel<16>, dim3(1), dim3(64), 0, s, R, cross, norms, tperm, tsign,
                       tmargin);
  return hipGetLastError();
}

hipError_t rec_temporal_prep(hipStream_t s, int M1, int R, const double* H, const int* tperm,
                             const double* tsign, const double* ka, const double* kb, double* kappa,
                             double* Hcur, const double* rhs2, double* rhs_c, int have_prev) {
  hipLaunchKernelGGL(temporal_prep_kernel, dim3(grid_for((int64_t)M1 * R)), dim3(256), 0, s, M1, R,
                     H, tperm, tsign, ka, kb, kappa, Hcur, rhs2, rhs_c, have_prev);
  return hipGetLastError();
}

hipError_t rec_temporal_finish(hipStream_t s, int R, int64_t Kold, int64_t t, const double* kappa,
                               const int* tperm, const double* tsign, double* Cnew, double* Chist,
                               double* tmp, int have_prev) {
  const int64_t big = (Kold + t) * R;
  hipLaunchKernelGGL(temporal_finish_kernel, dim3(grid_for(big)), dim3(256), 0, s, R, Kold, t,
                     kappa, tperm, tsign, Cnew, Chist, tmp, have_prev, 0);
  hipLaunchKernelGGL(temporal_finish_kernel, dim3(grid_for(big)), dim3(256), 0, s, R, Kold, t,
                     kappa, tperm, tsign, Cnew, Chist, tmp, have_prev, 1);
  return hipGetLastError();
}

hipError_t rec_weights(hipStream_t s, int M1, int S, int P, double* w, double* w2) {
  hipLaunchKernelGGL(weights_kernel, dim3(grid_for(M1)), dim3(256), 0, s, M1, S, P, w, w2);
  return hipGetLastError();
}

}  // namespace octen
