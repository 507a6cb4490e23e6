// The N-mode extension (supplement, "Extending to Higher-Order Tensors"):
// kernels for an N-mode tensor growing in its last mode, FP64 throughout.
//
// Layouts: a batch X is [t][I_1]...[I_{N-1}] (time first, the last mode
// fastest); a replica summary is [Q]^N with the temporal index last; replica
// factors are [P][N][Q][R], mode N-1 temporal.
//
// Compression (supplement, compressed cubes): the last non-temporal mode is
// contracted with all M1 compression columns at once (one GEMM, outside
// these kernels), the columns of each replica are gathered, the remaining
// non-temporal modes are contracted one by one (nm_ttm_kernel), and the
// temporal mode last (nm_temporal_kernel, which flags non-finite values).
// ALS: one workgroup per replica (nm_als_kernel).  Matching and stacking:
// nm_align_kernel, nm_stack_kernel; pairing with the previous batch:
// nm_tmatch_kernel.  Fit: nm_fit_kernel + nm_fit_reduce.
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int NM_NT = 256;

__device__ __forceinline__ int rep_col(int p, int q, int Q, int S) {
  return q < S ? q : S + p * (Q - S) + (q - S);
}

// out[p][row][q] = T[row][col_p(q)]
__global__ void nm_gather_kernel(const double* __restrict__ T, int64_t rows, int M1, int P, int Q,
                                 int S, double* __restrict__ out) {
  const int p = blockIdx.y;
  const int64_t n = rows * Q;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / Q;
    const int q = (int)(e - row * Q);
    out[(int64_t)p * n + e] = T[row * M1 + rep_col(p, q, Q, S)];
  }
}

// out[p][pre][q][post] = sum_i in[p][pre][i][post] U[i][col_p(q)]
__global__ void nm_ttm_kernel(const double* __restrict__ in, int64_t in_stride, int64_t pre,
                              int64_t d, int64_t post, const double* __restrict__ U, int M1, int P,
                              int Q, int S, double* __restrict__ out, int64_t out_stride) {
  const int p = blockIdx.y;
  const int64_t n = pre * Q * post;
  const double* src = in + (int64_t)p * in_stride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / (Q * post);
    const int64_t rem = e - a * Q * post;
    const int q = (int)(rem / post);
    const int64_t b = rem - (int64_t)q * post;
    const int col = rep_col(p, q, Q, S);
    const double* x = src + a * d * post + b;
    double s = 0.0;
    for (int64_t i = 0; i < d; ++i) s = fma(x[i * post], U[i * M1 + col], s);
    out[(int64_t)p * out_stride + e] = s;
  }
}

// Z[p][x][c] = sum_k T[p][k][x] W[k][col_p(c)], x < L; non-finite results
// flag the replica
__global__ void nm_temporal_kernel(const double* __restrict__ T, int64_t t_stride, int64_t t,
                                   int64_t L, const double* __restrict__ W, int M1, int P, int Q,
                                   int S, double* __restrict__ Z, int* __restrict__ zbad) {
  const int p = blockIdx.y;
  const int64_t n = L * Q;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = e / Q;
    const int c = (int)(e - x * Q);
    const int col = rep_col(p, c, Q, S);
    const double* src = T + (int64_t)p * t_stride + x;
    double s = 0.0;
    for (int64_t k = 0; k < t; ++k) s = fma(src[k * L], W[k * M1 + col], s);
    bad |= isfinite(s) ? 0 : 1;
    Z[(int64_t)p * n + e] = s;
  }
  if (bad) atomicOr(zbad + p, 1);
}

struct NmAlsArgs {
  const double* Y;      // [P][Q^N]
  const double* init;   // [P][N][Q][R]
  double* F;            // [P][N][Q][R]
  double* lam;          // [P][R]
  int* flags;           // [P]: bit0 non-positive pivot, bit2 not finite
  int N, Q, R, iters;
  int64_t QN, QN1;      // Q^N, Q^(N-1)
};

// Rank-R CP of each replica by Gauss-Seidel ALS (the N-mode form of the
// replica ALS, Sec. 4.1): per mode the MTTKRP (each output summed over the
// other N-1 indices in fixed chunks, the chunks then added in order), the
// Hadamard product of the other Grams, the solve F = M G^-1 by Gauss-Jordan
// on [G | M^T] (one barrier per pivot, no pivoting: G is SPD; a
// non-positive pivot is flagged), unit columns, lambda from the last mode.
__global__ __launch_bounds__(NM_NT) void nm_als_kernel(NmAlsArgs g) {
  extern __shared__ double sm[];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int N = g.N, Q = g.Q, R = g.R, QR = Q * R, RR = R * R;
  double* Fl = sm;                       // [N][Q][R]
  double* M = Fl + N * QR;               // [Q][R]
  double* Gr = M + QR;                   // [N][R][R] Grams
  double* aug = Gr + N * RR;             // [R][R + Q]
  double* part = aug + R * (R + Q);      // [NM_NT] chunk sums
  double* nrm = part + NM_NT;            // [R]
  __shared__ int s_bad;
  const double* Y = g.Y + (int64_t)p * g.QN;
  for (int e = tid; e < N * QR; e += NM_NT) Fl[e] = g.init[(int64_t)p * N * QR + e];
  if (tid == 0) s_bad = 0;
  if (tid < R) nrm[tid] = 1.0;
  __syncthreads();
  for (int m = 0; m < N; ++m)
    for (int e = tid; e < RR; e += NM_NT) {
      const int r1 = e / R, r2 = e - r1 * R;
      double s = 0.0;
      for (int q = 0; q < Q; ++q) s = fma(Fl[m * QR + q * R + r1], Fl[m * QR + q * R + r2], s);
      Gr[m * RR + e] = s;
    }
  __syncthreads();
  const int nchunk = QR >= NM_NT ? 1 : NM_NT / QR;
  const int64_t clen = (g.QN1 + nchunk - 1) / nchunk;
  for (int it = 0; it < g.iters; ++it) {
    for (int n = 0; n < N; ++n) {
      // MTTKRP: output o = (q, r), chunk ch of the other indices
      for (int base = 0; base < QR * nchunk; base += NM_NT) {
        const int w = base + tid;
        double s = 0.0;
        if (w < QR * nchunk) {
          const int o = w % QR, ch = w / QR;
          const int q = o / R, r = o - q * R;
          const int64_t e0 = (int64_t)ch * clen;
          const int64_t e1 = e0 + clen < g.QN1 ? e0 + clen : g.QN1;
          for (int64_t e = e0; e < e1; ++e) {
            // digits of the other modes (mode N-1 fastest), offset in Y
            int64_t rem = e, off = 0, stride = 1;
            double pr = 1.0;
            for (int m = N - 1; m >= 0; --m) {
              int dgt;
              if (m == n) {
                dgt = q;
              } else {
                const int64_t nx = rem / Q;
                dgt = (int)(rem - nx * Q);
                rem = nx;
                pr *= Fl[m * QR + dgt * R + r];
              }
              off += dgt * stride;
              stride *= Q;
            }
            s = fma(Y[off], pr, s);
          }
        }
        part[tid] = s;
        __syncthreads();
        if (tid < QR && base == 0) {
          double t = 0.0;
          for (int ch = 0; ch < nchunk; ++ch) t += part[ch * QR + tid];
          M[tid] = t;
        } else if (w < QR * nchunk && nchunk == 1) {
          M[w] = s;
        }
        __syncthreads();
      }
      // [G | M^T] with G the Hadamard product of the other Grams
      for (int e = tid; e < R * (R + Q); e += NM_NT) {
        const int i = e / (R + Q), c = e - i * (R + Q);
        double v;
        if (c < R) {
          v = 1.0;
          for (int m = 0; m < N; ++m)
            if (m != n) v *= Gr[m * RR + i * R + c];
        } else {
          v = M[(c - R) * R + i];
        }
        aug[e] = v;
      }
      __syncthreads();
      for (int j = 0; j < R; ++j) {
        double piv = aug[j * (R + Q) + j];
        if (!(piv > 0.0)) {
          if (tid == 0) s_bad = 1;
          piv = 1e-300;
        }
        const double rp = 1.0 / piv;
        // every thread reads the pivot row and its own column's factors
        // before the barrier, then writes
        double vals[4];
        int cnt = 0;
        for (int e = tid; e < R * (R + Q); e += NM_NT) {
          const int i = e / (R + Q), c = e - i * (R + Q);
          const double pj = aug[j * (R + Q) + c] * rp;
          vals[cnt < 4 ? cnt : 3] = (i == j) ? pj : aug[e] - aug[i * (R + Q) + j] * pj;
          ++cnt;
        }
        __syncthreads();
        cnt = 0;
        for (int e = tid; e < R * (R + Q); e += NM_NT) {
          aug[e] = vals[cnt < 4 ? cnt : 3];
          ++cnt;
        }
        __syncthreads();
      }
      // F_n = (M G^-1), unit columns
      double* Fn = Fl + n * QR;
      for (int e = tid; e < QR; e += NM_NT) {
        const int q = e / R, r = e - q * R;
        Fn[e] = aug[r * (R + Q) + R + q];
      }
      __syncthreads();
      if (tid < R) {
        double s = 0.0;
        for (int q = 0; q < Q; ++q) s = fma(Fn[q * R + tid], Fn[q * R + tid], s);
        const double v = sqrt(s);
        nrm[tid] = v > 0.0 ? v : 1.0;
      }
      __syncthreads();
      for (int e = tid; e < QR; e += NM_NT) Fn[e] /= nrm[e % R];
      __syncthreads();
      for (int e = tid; e < RR; e += NM_NT) {
        const int r1 = e / R, r2 = e - r1 * R;
        double s = 0.0;
        for (int q = 0; q < Q; ++q) s = fma(Fn[q * R + r1], Fn[q * R + r2], s);
        Gr[n * RR + e] = s;
      }
      __syncthreads();
    }
  }
  int nf = 0;
  for (int e = tid; e < N * QR; e += NM_NT) {
    const double v = Fl[e];
    nf |= isfinite(v) ? 0 : 1;
    g.F[(int64_t)p * N * QR + e] = v;
  }
  if (tid < R) {
    g.lam[(int64_t)p * R + tid] = nrm[tid];
    nf |= isfinite(nrm[tid]) ? 0 : 1;
  }
  if (nf) atomicOr(g.flags + p, 4);
  if (tid == 0 && s_bad) atomicOr(g.flags + p, 1);
}

// Exclusive greedy assignment on sim (R x R, LDS) by one thread: the largest
// free entry, ties to the smallest column then row (column-major scan with
// strict improvement); margin = smallest gap to the best free rival in the
// chosen row or column.
__device__ void greedy_one(const double* sim, int R, int* perm, double* margin, int* rowf,
                           int* colf) {
  for (int r = 0; r < R; ++r) { rowf[r] = 1; colf[r] = 1; perm[r] = -1; }
  double mg = INFINITY;
  for (int round = 0; round < R; ++round) {
    double best = -INFINITY;
    int br = -1, bc = -1;
    for (int c = 0; c < R; ++c) {
      if (!colf[c]) continue;
      for (int r = 0; r < R; ++r) {
        if (!rowf[r]) continue;
        if (sim[r * R + c] > best) { best = sim[r * R + c]; br = r; bc = c; }
      }
    }
    double rival = -INFINITY;
    for (int c = 0; c < R; ++c)
      if (colf[c] && c != bc) rival = fmax(rival, sim[br * R + c]);
    for (int r = 0; r < R; ++r)
      if (rowf[r] && r != br) rival = fmax(rival, sim[r * R + bc]);
    if (isfinite(rival)) mg = fmin(mg, best - rival);
    perm[br] = bc;
    rowf[br] = 0;
    colf[bc] = 0;
  }
  *margin = mg;
}

// lambda^(1/N) on every mode, then replica p >= 1 matched to replica 0 on the
// product over the N modes of |cos| between anchor columns (first S rows),
// with the per-mode least-squares scale; replica 0 is copied.  One
// workgroup per replica; aligned [P][N][Q][R].
__global__ __launch_bounds__(NM_NT) void nm_align_kernel(const double* __restrict__ F,
                                                         const double* __restrict__ lam, int P,
                                                         int N, int Q, int R, int S,
                                                         double* __restrict__ aligned,
                                                         int* __restrict__ perm,
                                                         double* __restrict__ margin) {
  extern __shared__ double sm[];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int QR = Q * R;
  double* sim = sm;                 // [R][R]
  double* root = sim + R * R;       // [2][R]: lambda^(1/N) of p and of 0
  __shared__ int s_perm[32], s_rowf[32], s_colf[32];
  __shared__ double s_margin;
  if (tid < R) {
    root[tid] = pow(lam[(int64_t)p * R + tid], 1.0 / N);
    root[R + tid] = pow(lam[tid], 1.0 / N);
  }
  __syncthreads();
  const double* Fp = F + (int64_t)p * N * QR;
  const double* F0 = F;
  if (p == 0) {
    for (int e = tid; e < N * QR; e += NM_NT) aligned[e] = Fp[e] * root[e % R];
    if (tid < R) perm[tid] = tid;
    if (tid == 0) margin[0] = INFINITY;
    return;
  }
  for (int e = tid; e < R * R; e += NM_NT) {
    const int r = e / R, c = e - r * R;
    double v = 1.0;
    for (int n = 0; n < N; ++n) {
      double ab = 0.0, aa = 0.0, bb = 0.0;
      for (int q = 0; q < S; ++q) {
        const double a = Fp[n * QR + q * R + r] * root[r];
        const double b = F0[n * QR + q * R + c] * root[R + c];
        ab = fma(a, b, ab);
        aa = fma(a, a, aa);
        bb = fma(b, b, bb);
      }
      const double den = sqrt(aa) * sqrt(bb);
      v *= den > 0.0 ? fabs(ab) / den : 0.0;
    }
    sim[e] = v;
  }
  __syncthreads();
  if (tid == 0) greedy_one(sim, R, s_perm, &s_margin, s_rowf, s_colf);
  __syncthreads();
  for (int e = tid; e < N * R; e += NM_NT) {
    const int n = e / R, r = e - n * R;
    const int rr = s_perm[r];
    double ab = 0.0, aa = 0.0;
    for (int q = 0; q < S; ++q) {
      const double a = Fp[n * QR + q * R + r] * root[r];
      const double b = F0[n * QR + q * R + rr] * root[R + rr];
      ab = fma(b, a, ab);
      aa = fma(a, a, aa);
    }
    const double d = aa > 0.0 ? ab / aa : 0.0;
    for (int q = 0; q < Q; ++q)
      aligned[(int64_t)p * N * QR + n * QR + q * R + rr] = d * Fp[n * QR + q * R + r] * root[r];
  }
  if (tid < R) perm[(int64_t)p * R + tid] = s_perm[tid];
  if (tid == 0) margin[p] = s_margin;
}

// rhs[n][M1][R]: the anchor rows averaged over the replicas, then each
// replica's own rows (the deduplicated stack of Eq. 5)
__global__ void nm_stack_kernel(const double* __restrict__ aligned, int P, int N, int Q, int R,
                                int S, double* __restrict__ rhs) {
  const int M1 = S + P * (Q - S);
  const int64_t n_all = (int64_t)N * M1 * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_all;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / ((int64_t)M1 * R));
    const int rem = (int)(e - (int64_t)n * M1 * R);
    const int row = rem / R, r = rem - row * R;
    double v;
    if (row < S) {
      v = 0.0;
      for (int p = 0; p < P; ++p) v += aligned[(((int64_t)p * N + n) * Q + row) * R + r];
      v /= P;
    } else {
      const int p = (row - S) / (Q - S), q = S + (row - S) - p * (Q - S);
      v = aligned[(((int64_t)p * N + n) * Q + q) * R + r];
    }
    rhs[e] = v;
  }
}

// kappa[r] = product over the non-temporal modes of k[n][r]; ones[r] = 1
__global__ void nm_kappa_kernel(const double* __restrict__ k, int nm, int R,
                                double* __restrict__ kappa, double* __restrict__ ones) {
  const int r = threadIdx.x;
  if (r < R) {
    double v = 1.0;
    for (int n = 0; n < nm; ++n) v *= k[n * R + r];
    kappa[r] = v;
    ones[r] = 1.0;
  }
}

// Pairing with the previous batch over the nm non-temporal modes:
// sim = prod_n |cross_n| / (norm_cur norm_prev), greedy; sign = prod_n
// sign(cross_n).  cross [nm][R][R] (current x previous), norms [nm][2][R].
__global__ void nm_tmatch_kernel(const double* __restrict__ cross, const double* __restrict__ norms,
                                 int nm, int R, int* __restrict__ tperm,
                                 double* __restrict__ tsign, double* __restrict__ tmargin) {
  __shared__ double sim[32 * 32];
  __shared__ int s_perm[32], s_rowf[32], s_colf[32];
  __shared__ double s_margin;
  const int tid = threadIdx.x;
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int r = e / R, c = e - r * R;
    double v = 1.0;
    for (int n = 0; n < nm; ++n) {
      const double den = norms[(n * 2) * R + r] * norms[(n * 2 + 1) * R + c];
      v *= fabs(cross[n * R * R + e]) / (den > 0.0 ? den : 1.0);
    }
    sim[e] = v;
  }
  __syncthreads();
  if (tid == 0) greedy_one(sim, R, s_perm, &s_margin, s_rowf, s_colf);
  __syncthreads();
  if (tid < R) {
    const int c = s_perm[tid];
    double sg = 1.0;
    for (int n = 0; n < nm; ++n) {
      const double x = cross[n * R * R + tid * R + c];
      sg *= x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0);
    }
    tperm[tid] = c;
    tsign[tid] = sg == 0.0 ? 1.0 : sg;
  }
  if (tid == 0) *tmargin = s_margin;
}

struct NmFitArgs {
  const double* X;               // [t][I_1]...[I_{N-1}]
  const double* A[5];            // non-temporal factors [I_n][R]
  const double* C;               // [K][R]
  int64_t dims[5];
  int nm, R;
  int64_t t, k0, per;            // per = elements of one slice
  double* partials;              // [2][nblocks]
};

__global__ __launch_bounds__(NM_NT) void nm_fit_kernel(NmFitArgs g) {
  __shared__ double s_a[NM_NT], s_b[NM_NT];
  const int64_t n = g.t * g.per;
  double sse = 0.0, nx = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)NM_NT + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * NM_NT) {
    const int64_t k = e / g.per;
    int64_t rem = e - k * g.per;
    int64_t idx[5];
    for (int m = g.nm - 1; m >= 0; --m) {
      const int64_t nx2 = rem / g.dims[m];
      idx[m] = rem - nx2 * g.dims[m];
      rem = nx2;
    }
    double xh = 0.0;
    for (int r = 0; r < g.R; ++r) {
      double pr = g.C[(g.k0 + k) * g.R + r];
      for (int m = 0; m < g.nm; ++m) pr *= g.A[m][idx[m] * g.R + r];
      xh += pr;
    }
    const double x = g.X[e];
    sse = fma(x - xh, x - xh, sse);
    nx = fma(x, x, nx);
  }
  s_a[threadIdx.x] = sse;
  s_b[threadIdx.x] = nx;
  __syncthreads();
  for (int st = NM_NT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s_a[threadIdx.x] += s_a[threadIdx.x + st];
      s_b[threadIdx.x] += s_b[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    g.partials[blockIdx.x] = s_a[0];
    g.partials[gridDim.x + blockIdx.x] = s_b[0];
  }
}

__global__ void nm_fit_reduce(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nb; ++i) { a += partials[i]; b += partials[nb + i]; }
    out[0] = a;
    out[1] = b;
  }
}

unsigned grid_of(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t nm_gather(hipStream_t s, const double* T, int64_t rows, int M1, int P, int Q, int S,
                     double* out) {
  hipLaunchKernelGGL(nm_gather_kernel, dim3(grid_of(rows * Q), P), dim3(256), 0, s, T, rows, M1, P,
                     Q, S, out);
  return hipGetLastError();
}

hipError_t nm_ttm(hipStream_t s, const double* in, int64_t in_stride, int64_t pre, int64_t d,
                  int64_t post, const double* U, int M1, int P, int Q, int S, double* out,
                  int64_t out_stride) {
  hipLaunchKernelGGL(nm_ttm_kernel, dim3(grid_of(pre * Q * post), P), dim3(256), 0, s, in,
                     in_stride, pre, d, post, U, M1, P, Q, S, out, out_stride);
  return hipGetLastError();
}

hipError_t nm_temporal(hipStream_t s, const double* T, int64_t t_stride, int64_t t, int64_t L,
                       const double* W, int M1, int P, int Q, int S, double* Z, int* zbad) {
  hipLaunchKernelGGL(nm_temporal_kernel, dim3(grid_of(L * Q), P), dim3(256), 0, s, T, t_stride, t,
                     L, W, M1, P, Q, S, Z, zbad);
  return hipGetLastError();
}

size_t nm_als_lds_bytes(int N, int Q, int R) {
  return (size_t)((size_t)N * Q * R + (size_t)Q * R + (size_t)N * R * R + (size_t)R * (R + Q) +
                  NM_NT + R) * 8;
}

hipError_t nm_als(hipStream_t s, const double* Y, int P, int N, int Q, int R, const double* init,
                  double* F, double* lam, int* flags, int iters) {
  NmAlsArgs a;
  a.Y = Y; a.init = init; a.F = F; a.lam = lam; a.flags = flags;
  a.N = N; a.Q = Q; a.R = R; a.iters = iters;
  int64_t qn = 1;
  for (int n = 0; n < N - 1; ++n) qn *= Q;
  a.QN1 = qn;
  a.QN = qn * Q;
  const size_t lds = nm_als_lds_bytes(N, Q, R);
  if (lds > 160 * 1024 || (int64_t)R * (R + Q) > 4 * NM_NT) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nm_als_kernel, dim3(P), dim3(NM_NT), lds, s, a);
  return hipGetLastError();
}

hipError_t nm_align(hipStream_t s, const double* F, const double* lam, int P, int N, int Q, int R,
                    int S, double* aligned, int* perm, double* margin) {
  if (R > 32) return hipErrorInvalidValue;
  const size_t lds = (size_t)(R * R + 2 * R) * 8;
  hipLaunchKernelGGL(nm_align_kernel, dim3(P), dim3(NM_NT), lds, s, F, lam, P, N, Q, R, S, aligned,
                     perm, margin);
  return hipGetLastError();
}

hipError_t nm_stack(hipStream_t s, const double* aligned, int P, int N, int Q, int R, int S,
                    double* rhs) {
  const int M1 = S + P * (Q - S);
  hipLaunchKernelGGL(nm_stack_kernel, dim3(grid_of((int64_t)N * M1 * R)), dim3(256), 0, s, aligned,
                     P, N, Q, R, S, rhs);
  return hipGetLastError();
}

hipError_t nm_kappa(hipStream_t s, const double* k, int nm, int R, double* kappa, double* ones) {
  hipLaunchKernelGGL(nm_kappa_kernel, dim3(1), dim3(64), 0, s, k, nm, R, kappa, ones);
  return hipGetLastError();
}

hipError_t nm_tmatch(hipStream_t s, const double* cross, const double* norms, int nm, int R,
                     int* tperm, double* tsign, double* tmargin) {
  if (R > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nm_tmatch_kernel, dim3(1), dim3(256), 0, s, cross, norms, nm, R, tperm, tsign,
                     tmargin);
  return hipGetLastError();
}

hipError_t nm_fit(hipStream_t s, const double* X, int64_t t, const int64_t* dims, int nm,
                  const double* const* A, const double* C, int R, int64_t k0, double* partials,
                  int nparts, double* out2) {
  if (nm > 5 || nm < 1) return hipErrorInvalidValue;
  NmFitArgs g;
  g.X = X; g.C = C; g.nm = nm; g.R = R; g.t = t; g.k0 = k0; g.partials = partials;
  int64_t per = 1;
  for (int m = 0; m < 5; ++m) {
    g.A[m] = m < nm ? A[m] : nullptr;
    g.dims[m] = m < nm ? dims[m] : 1;
    if (m < nm) per *= dims[m];
  }
  g.per = per;
  int64_t nb = (t * per + NM_NT - 1) / NM_NT;
  if (nb > nparts) nb = nparts;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(nm_fit_kernel, dim3((unsigned)nb), dim3(NM_NT), 0, s, g);
  hipLaunchKernelGGL(nm_fit_reduce, dim3(1), dim3(64), 0, s, partials, (int)nb, out2);
  return hipGetLastError();
}

}  // namespace octen
