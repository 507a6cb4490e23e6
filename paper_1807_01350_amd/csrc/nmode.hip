// The N-mode extension (supplement, "Extending to Higher-Order Tensors"):
// kernels for an N-mode tensor growing in its last mode, FP64 throughout.
//
// Layouts: a batch X is [t][I_1]...[I_{N-1}] (time first, the last mode
// fastest); a replica summary is [Q]^N with the temporal index last; replica
// factors are [P][N][Q][R], mode N-1 temporal.
//
// Compression (supplement, compressed cubes): the last non-temporal mode is
// contracted with all M1 compression columns at once (one GEMM, outside
// these kernels), the remaining non-temporal modes one by one on FP64 matrix
// cores (nm_ttm_mfma_kernel, the first reading each replica's columns of the
// GEMM output in place), and the temporal mode last (nm_temporal_kernel,
// which flags non-finite values).
// ALS: one workgroup per replica (nm_als_kernel).  Matching and stacking:
// nm_align_kernel, nm_stack_kernel; pairing with the previous batch:
// nm_tmatch_kernel.  Fit: nm_fit_kernel + nm_fit_reduce.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int NM_NT = 512;
constexpr int OCTEN_NM_MAX_MODES_K = 6;

__device__ __forceinline__ int rep_col(int p, int q, int Q, int S) {
  return q < S ? q : S + p * (Q - S) + (q - S);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Mode product on FP64 matrix cores: out[p][a][q][b] = sum_i
// in(p, a, i, b) U[i][col_p(q)] for a < pre, q < Q, b < post, i < d.  One
// wavefront per 16 x 16 tile of (q, b) of one (p, a), K steps of 4 on
// v_mfma_f64_16x16x4f64 (lane l supplies A[l%16][l/16] = U[i][col_p(q)] and
// B[l/16][l%16] = in(p, a, i, b); element k of the result is
// D[l/16 + 4k][l%16]); indexes past Q, post or d read zero.  in(p, a, i, b)
// is in[(a d + i) M1 + col_p(b)] when `cols` (the product of X with all M1
// compression columns of the next mode, shared by the replicas), else
// in[p in_stride + (a d + i) post + b].
__global__ __launch_bounds__(256) void nm_ttm_mfma_kernel(
    const double* __restrict__ in, int64_t in_stride, bool cols, int64_t pre, int d, int post,
    const double* __restrict__ U, int M1, int P, int Q, int S, double* __restrict__ out,
    int64_t out_stride, int nqb, int nbb, int64_t ntiles) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const int bb = (int)(tile % nbb);
  int64_t rest = tile / nbb;
  const int qb = (int)(rest % nqb);
  rest /= nqb;
  const int64_t a = rest % pre;
  const int p = (int)(rest / pre);
  const int li = lane >> 4, lj = lane & 15;
  const int qa = qb * 16 + lj;                 // A row (q) of this lane
  const int bn = bb * 16 + lj;                 // B column (b) of this lane
  const bool qok = qa < Q, bok = bn < post;
  const int ucol = qok ? rep_col(p, qa, Q, S) : 0;
  const double* src;
  int64_t istep;
  if (cols) {
    src = in + (a * d) * (int64_t)M1 + (bok ? rep_col(p, bn, Q, S) : 0);
    istep = M1;
  } else {
    src = in + (int64_t)p * in_stride + (a * d) * (int64_t)post + (bok ? bn : 0);
    istep = post;
  }
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < d; i0 += 4) {
    const int i = i0 + li;
    const bool iok = i < d;
    const double av = (iok && qok) ? U[(int64_t)i * M1 + ucol] : 0.0;
    const double bv = (iok && bok) ? src[(int64_t)i * istep] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  if (bok) {
    double* dst = out + (int64_t)p * out_stride + (a * Q) * (int64_t)post + bn;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = qb * 16 + li + 4 * k;
      if (q < Q) dst[(int64_t)q * post] = acc[k];
    }
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

constexpr unsigned NM_SPIN_LIMIT = 1u << 22;

struct NmAlsArgs {
  const double* Y;      // [P][Q^N]
  const double* init;   // [P][N][Q][R]
  double* F;            // [P][N][Q][R]
  double* lam;          // [P][R]
  int* flags;           // [P]: bit0 non-positive pivot, bit1 barrier timed out, bit2 not finite
  double* work;         // [P][work_stride]: T_L, T_R, then the workgroups' intermediates
  int64_t work_stride;
  unsigned* ctr;        // [P] barrier counters (zero at launch)
  int* err;             // [1] a barrier timed out
  int N, Q, R, iters, W;
  int QN1;              // Q^(N-1)
  int inter_lds;        // intermediates in LDS, else in the work buffer
  int SA, SB;           // doubles of the two intermediate buffers of a workgroup
  int t_lds;            // the contracted summary T copied to LDS before the mode updates
  int TMAX;             // doubles of T at most (RC * max(Q^nL, Q^(N-nL)))
};

typedef __attribute__((address_space(3))) double lds_f64;
// An LDS pointer as a wave-uniform (scalar) LDS address.
__device__ __forceinline__ lds_f64* lds_uniform(const double* p) {
  const unsigned a = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(const lds_f64*)p);
  return (lds_f64*)(uintptr_t)a;
}

// Orders the LDS accesses of one wavefront (its LDS operations complete in
// order; the fence keeps the compiler from moving accesses across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Value of x held by lane j (j uniform).
__device__ __forceinline__ double lane_value(double x, int j) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), j);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), j);
  return __hiloint2double(hi, lo);
}

// 1 / p for p > 0: the hardware estimate refined by two Newton steps
// r <- r + r (1 - p r) (a few units in the last place).
__device__ __forceinline__ double recip(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  r = fma(r, fma(-p, r, 1.0), r);
  return r;
}

// Barrier of the W workgroups of one replica: every wave waits for its own
// stores, one thread makes them visible to the other XCDs (agent-scope
// release), bumps the counter, polls it, and takes the others' stores
// (agent-scope acquire: the CU's L1 and the XCD's L2 drop stale lines).  A
// poll that runs past NM_SPIN_LIMIT sets *err; a workgroup that sees *err
// leaves.  Returns false then.
__device__ bool nm_barrier(unsigned* ctr, unsigned target, int* err, int* s_ok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (++spins > NM_SPIN_LIMIT) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// out[(a L + l) Bo + b] = sum_i in[a sa + i si + l sl + b] F(i, r) for
// a < pre, l < L, b < Bo, i < Q (i ascending).  `first`: in is the summary
// itself (no r index), one thread per (a, l, b) output computing all RC
// columns; otherwise in and out carry a trailing [RC] index and one thread
// computes one (a, l, b, r) output.  The loads of up to 16 consecutive i are
// issued before any is used (the contraction waits on memory latency
// otherwise); indexes past Q are clamped and their terms skipped.
template <int RC>
__device__ void nm_contract(const double* in, bool first, int pre, int L, int Bo, int sa, int si,
                            int sl, int Q, const double* Fm, double* out) {
  constexpr int IB = 16;
  const int LB = L * Bo;
  if (first) {
    const int n = pre * LB;
    for (int o = threadIdx.x; o < n; o += NM_NT) {
      const int a = o / LB, rem = o - a * LB, l = rem / Bo, b = rem - l * Bo;
      double acc[RC];
#pragma unroll
      for (int r = 0; r < RC; ++r) acc[r] = 0.0;
      const double* src = in + a * sa + l * sl + b;
      for (int i0 = 0; i0 < Q; i0 += IB) {
        double y[IB];
#pragma unroll
        for (int k = 0; k < IB; ++k) y[k] = src[min(i0 + k, Q - 1) * si];
#pragma unroll
        for (int k = 0; k < IB; ++k) {
          if (i0 + k < Q) {
            const double* f = Fm + (i0 + k) * RC;
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[r] = fma(y[k], f[r], acc[r]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RC; ++r) out[o * RC + r] = acc[r];
    }
  } else {
    const int n = pre * LB * RC;
    for (int o = threadIdx.x; o < n; o += NM_NT) {
      const int alb = o / RC, r = o - alb * RC;
      const int a = alb / LB, rem = alb - a * LB, l = rem / Bo, b = rem - l * Bo;
      const double* src = in + (a * sa + l * sl + b) * RC + r;
      double acc = 0.0;
      for (int i0 = 0; i0 < Q; i0 += IB) {
        double v[IB];
#pragma unroll
        for (int k = 0; k < IB; ++k) v[k] = src[min(i0 + k, Q - 1) * si * RC];
#pragma unroll
        for (int k = 0; k < IB; ++k)
          if (i0 + k < Q) acc = fma(v[k], Fm[(i0 + k) * RC + r], acc);
      }
      out[o] = acc;
    }
  }
}

// MTTKRP of mode n (b0 <= n < b1) from T, the summary contracted with the
// factors of every mode outside the block [b0, b1) ([Q^(b1-b0)][RC], mode b0
// slowest): M(q, r) = sum over the other modes of the block (at most two:
// blocks hold at most three modes) of T times their factors.  All threads:
// each output's terms are split into up to NM_NT / (Q R) chunks, summed in
// order per chunk and the chunks added in order.  part: NM_NT doubles of LDS.
template <int RC>
__device__ void nm_mttkrp_block(const double* T, const double* Fl, double* M, double* part, int n,
                                int b0, int b1, int Q, int R) {
  const int tid = threadIdx.x, QR = Q * R, QRC = Q * RC;
  int o0 = -1, o1 = -1, no = 0;
  for (int m = b0; m < b1; ++m)
    if (m != n) {
      if (no == 0) o0 = m; else o1 = m;
      ++no;
    }
  int st_n = 1, st0 = 0, st1 = 0, ncomb = 1;
  for (int m = b1 - 1, st = 1; m >= b0; --m, st *= Q) {
    if (m == n) st_n = st;
    if (m == o0) st0 = st;
    if (m == o1) st1 = st;
  }
  for (int k = 0; k < no; ++k) ncomb *= Q;
  int nchunk = NM_NT / QR;
  if (nchunk < 1) nchunk = 1;
  if (nchunk > ncomb) nchunk = ncomb;
  const int clen = (ncomb + nchunk - 1) / nchunk;
  for (int base = 0; base < QR * nchunk; base += NM_NT) {
    const int w = base + tid;
    double s = 0.0;
    if (w < QR * nchunk) {
      const int o = w % QR, ch = w / QR;
      const int q = o / R, r = o - q * R;
      const int u0 = ch * clen;
      const int u1 = u0 + clen < ncomb ? u0 + clen : ncomb;
      const double* t = T + q * st_n * RC + r;
      const double* f0 = Fl + (o0 >= 0 ? o0 : 0) * QRC + r;
      const double* f1 = Fl + (o1 >= 0 ? o1 : 0) * QRC + r;
      for (int u = u0; u < u1; ++u) {
        const int d0 = no > 1 ? u / Q : u;
        const int d1 = no > 1 ? u - d0 * Q : 0;
        double pr = 1.0;
        if (no > 0) pr *= f0[d0 * RC];
        if (no > 1) pr *= f1[d1 * RC];
        s = fma(t[(d0 * st0 + d1 * st1) * RC], pr, s);
      }
    }
    if (nchunk > 1) {
      part[tid] = s;
      __syncthreads();
      if (tid < QR) {
        double v = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) v += part[ch * QR + tid];
        M[tid] = v;
      }
    } else if (w < QR) {
      M[w] = s;
    }
    __syncthreads();
  }
}

// One wavefront: the update of mode n from its MTTKRP M [Q][R]:
//  - G = Hadamard product of the other modes' Grams;
//  - F^T = G^-1 M^T by Gauss-Jordan without pivoting on [G | M^T] held by
//    columns in the lanes: lane c < RMAX keeps column c of G (padded to
//    RMAX x RMAX with the identity, so the padding adds exact zeros), lane
//    RMAX + q keeps row q of M; after the RMAX steps lane RMAX + q holds row
//    q of F (Q + RMAX <= 64);
//  - the Gram of F, the norms from its diagonal, unit columns and their Gram.
// work: R^2 doubles of LDS.  *bad = 1 when a pivot is not positive.
template <int RMAX>
__device__ __forceinline__ void nm_mode_wave(const double* M_, double* Fl_, double* Gr_,
                                             double* work_, double* nrm_, int n_, int N_, int Q_,
                                             int R_, int* bad) {
  constexpr int RC = RMAX;
  const int lane = threadIdx.x & 63;
  const int R = __builtin_amdgcn_readfirstlane(R_);
  const int Q = __builtin_amdgcn_readfirstlane(Q_);
  const int N = __builtin_amdgcn_readfirstlane(N_);
  const int n = __builtin_amdgcn_readfirstlane(n_);
  lds_f64* Fl = lds_uniform(Fl_);
  lds_f64* Gr = lds_uniform(Gr_);
  const lds_f64* M = lds_uniform(M_);
  lds_f64* G = lds_uniform(work_);
  lds_f64* nrm = lds_uniform(nrm_);
  const int RR = R * R, QRC = Q * RC;
  for (int e = lane; e < RR; e += 64) {
    double v = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != n) v *= Gr[m * RR + e];
    G[e] = v;
  }
  wave_sync();
  const int q = lane - RMAX;              // row of M / F held by this lane
  const bool frow = q >= 0 && q < Q;
  double a[RMAX];
#pragma unroll
  for (int i = 0; i < RMAX; ++i) {
    double v = 0.0;
    if (lane < RMAX) {
      if (i < R && lane < R) v = G[i * R + lane];
      else if (i == lane) v = 1.0;
    } else if (frow && i < R) {
      v = M[q * R + i];
    }
    a[i] = v;
  }
  int badl = 0;
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    double col[RMAX];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) col[i] = lane_value(a[i], j);
    double piv = col[j];
    badl |= !(piv > 0.0);
    piv = piv > 0.0 ? piv : 1e-300;
    const double rj = a[j] * recip(piv);
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i != j) a[i] = fma(-col[i], rj, a[i]);
    a[j] = rj;
  }
  if (lane == 0 && badl) *bad = 1;
  lds_f64* Fn = Fl + n * QRC;
  if (frow) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < R) Fn[q * RC + i] = a[i];
  }
  wave_sync();
  // Gram of F, the norms from its diagonal, unit columns and their Gram
  for (int e = lane; e < RR; e += 64) {
    const int r1 = e / R, r2 = e - r1 * R;
    double s = 0.0;
#pragma unroll 8
    for (int qq = 0; qq < Q; ++qq) s = fma(Fn[qq * RC + r1], Fn[qq * RC + r2], s);
    G[e] = s;
  }
  wave_sync();
  if (lane < R) {
    const double v = sqrt(G[lane * R + lane]);
    nrm[lane] = v > 0.0 ? v : 1.0;
  }
  wave_sync();
  if (frow) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < R) Fn[q * RC + i] = a[i] / nrm[i];
  }
  lds_f64* Gn = Gr + n * RR;
  for (int e = lane; e < RR; e += 64) {
    const int r1 = e / R, r2 = e - r1 * R;
    Gn[e] = G[e] / (nrm[r1] * nrm[r2]);
  }
  wave_sync();
}

template <int RMAX>
__device__ __noinline__ void nm_mode_call(const double* M, double* Fl, double* Gr, double* work,
                                          double* nrm, int n, int N, int Q, int R, int* bad) {
  nm_mode_wave<RMAX>(M, Fl, Gr, work, nrm, n, N, Q, R, bad);
}

// The first contraction (in = the summary) on FP64 matrix cores, used for
// RC >= 16 (at RC = 8 half of every 16-wide tile would be padding and the
// VALU form above is faster): outputs o = (a L + l) Bo + b in tiles of 16 per
// wavefront, A[o][i] = in[a sa + i si + l sl + b], B[i][r] = F(i, r) (zero
// past Q and RC), v_mfma_f64_16x16x4f64 over i in steps of 4 (lane t supplies
// A[t%16][t/16] and B[t/16][t%16]; element k of the result is
// D[t/16 + 4k][t%16]); all Q / 4 operand loads of a tile are issued before
// its products (Q <= 32).
template <int RC>
__device__ void nm_contract_first_mfma(const double* in, int pre, int L, int Bo, int sa, int si,
                                       int sl, int Q, const double* Fm, double* out) {
  constexpr int NT = (RC + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int LB = L * Bo, n = pre * LB, ntile = (n + 15) / 16;
  const int m = lane & 15, kq = lane >> 4;
  for (int tile = wave; tile < ntile; tile += NM_NT / 64) {
    const int o = tile * 16 + m;
    const bool ook = o < n;
    const int oc = ook ? o : n - 1;
    const int a = oc / LB, rem = oc - a * LB, l = rem / Bo, b = rem - l * Bo;
    const double* src = in + a * sa + l * sl + b;
    double av[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = 4 * u + kq;
      av[u] = (4 * u < Q && ook && i < Q) ? src[i * si] : 0.0;
    }
    f64x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (4 * u < Q) {
        const int i = 4 * u + kq;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int col = t * 16 + m;
          const double bv = (i < Q && col < RC) ? Fm[i * RC + col] : 0.0;
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv, acc[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 16 + m;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o2 = tile * 16 + kq + 4 * k;
        if (o2 < n && col < RC) out[o2 * RC + col] = acc[t][k];
      }
    }
  }
}

// Rank-R CP of each replica by Gauss-Seidel ALS over the N modes (the N-mode
// form of the replica ALS, Sec. 4.1), W workgroups per replica (a
// cooperative launch when W > 1).  The MTTKRPs follow a dimension tree
// split after mode nL = N/2: the summary contracted with the factors of
// modes nL..N-1, one mode at a time, gives T_L [Q^nL][R], from which the
// MTTKRPs of modes 0..nL-1 are short sums; after those modes are updated,
// the summary contracted with their factors gives T_R [Q^(N-nL)][R] for
// modes nL..N-1.  The workgroups of a replica split each contraction (T_L
// by its rows, T_R by its columns; the partial contractions of a workgroup
// stay its own), meet at one barrier per half-sweep, and then every one of
// them runs the same mode updates on the same data (one wavefront,
// nm_mode_wave), so that all keep identical factors.  lambda: the norms of
// the last mode.
template <int RC>
__global__ __launch_bounds__(NM_NT) void nm_als_kernel(NmAlsArgs g) {
  extern __shared__ double sm[];
  const int W = g.W;
  const int p = blockIdx.x / W, w = blockIdx.x - p * W, tid = threadIdx.x;
  const int N = g.N, Q = g.Q, R = g.R, QRC = Q * RC, RR = R * R, QR = Q * R;
  double* Fl = sm;                       // [N][Q][RC], zero beyond R
  double* Gr = Fl + N * QRC;             // [N][R][R] Grams
  double* Mb = Gr + N * RR;              // [Q][R] MTTKRP of the mode being updated
  double* wk = Mb + QR;                  // [R^2] mode-update workspace
  double* part = wk + RR;                // [NM_NT] chunk sums of the MTTKRP
  double* nrm = part + NM_NT;            // [R]
  double* Tl = nrm + R;                  // [TMAX] if t_lds
  double* ldsA = Tl + (g.t_lds ? g.TMAX : 0);
  __shared__ int s_bad, s_ok;
  const double* Y = g.Y + (int64_t)p * g.QN1 * Q;
  const int nL = N / 2;
  int qpow[OCTEN_NM_MAX_MODES_K + 1];
  qpow[0] = 1;
  for (int k = 1; k <= OCTEN_NM_MAX_MODES_K; ++k) qpow[k] = qpow[k - 1] * Q;
  double* TLg = g.work + (int64_t)p * g.work_stride;          // [Q^nL][RC]
  double* TRg = TLg + (int64_t)qpow[nL] * RC;                 // [Q^(N-nL)][RC]
  double* bufA;
  if (g.inter_lds) {
    bufA = ldsA;
  } else {
    bufA = TRg + (int64_t)qpow[N - nL] * RC + (int64_t)w * (g.SA + g.SB);
  }
  double* bufB = bufA + g.SA;
  // this workgroup's rows of T_L and columns of T_R
  const int nrow = qpow[nL], ncol = qpow[N - nL];
  const int a0 = (int)((int64_t)nrow * w / W), a1 = (int)((int64_t)nrow * (w + 1) / W);
  const int c0 = (int)((int64_t)ncol * w / W), c1 = (int)((int64_t)ncol * (w + 1) / W);
  for (int e = tid; e < N * QRC; e += NM_NT) {
    const int m = e / QRC, rem = e - m * QRC, q = rem / RC, r = rem - q * RC;
    Fl[e] = r < R ? g.init[(int64_t)p * N * QR + m * QR + q * R + r] : 0.0;
  }
  if (tid == 0) s_bad = 0;
  if (tid < R) nrm[tid] = 1.0;
  __syncthreads();
  for (int m = 0; m < N; ++m)
    for (int e = tid; e < RR; e += NM_NT) {
      const int r1 = e / R, r2 = e - r1 * R;
      double s = 0.0;
      for (int q = 0; q < Q; ++q) s = fma(Fl[m * QRC + q * RC + r1], Fl[m * QRC + q * RC + r2], s);
      Gr[m * RR + e] = s;
    }
  __syncthreads();
  bool alive = true;
  unsigned nbar = 0;
  for (int it = 0; it < g.iters && alive; ++it) {
    for (int side = 0; side < 2 && alive; ++side) {
      const int b0 = side == 0 ? 0 : nL, b1 = side == 0 ? nL : N;
      double* Tg = side == 0 ? TLg : TRg;
      if (side == 0) {
        // modes nL..N-1 contracted, the first remaining one each time, on
        // rows [a0, a1) of T_L
        const int cnt = a1 - a0;
        const double* src = Y;
        double* dst = bufA;
        for (int m = nL; m < N; ++m) {
          const int post = qpow[N - 1 - m];
          const bool first = m == nL;
          if (m == N - 1) dst = TLg + (int64_t)a0 * RC;
          if (RC >= 16 && first)
            nm_contract_first_mfma<RC>(Y + (int64_t)a0 * Q * post, cnt, 1, post, Q * post, post, 0,
                                       Q, Fl + m * QRC, dst);
          else
            nm_contract<RC>(first ? Y + (int64_t)a0 * Q * post : src, first, cnt, 1, post,
                            Q * post, post, 0, Q, Fl + m * QRC, dst);
          __syncthreads();
          src = dst;
          dst = dst == bufA ? bufB : bufA;
        }
      } else {
        // modes 0..nL-1 contracted on columns [c0, c1) of T_R
        const int cnt = c1 - c0;
        const double* src = Y;
        double* dst = bufA;
        for (int m = 0; m < nL; ++m) {
          const int Lk = qpow[nL - 1 - m];
          const bool first = m == 0;
          if (m == nL - 1) dst = TRg + (int64_t)c0 * RC;
          if (RC >= 16 && first)
            nm_contract_first_mfma<RC>(Y + c0, 1, Lk, cnt, 0, Lk * ncol, ncol, Q, Fl + m * QRC,
                                       dst);
          else if (first)
            nm_contract<RC>(Y + c0, true, 1, Lk, cnt, 0, Lk * ncol, ncol, Q, Fl + m * QRC, dst);
          else
            nm_contract<RC>(src, false, 1, Lk, cnt, 0, Lk * cnt, cnt, Q, Fl + m * QRC, dst);
          __syncthreads();
          src = dst;
          dst = dst == bufA ? bufB : bufA;
        }
      }
      if (W > 1) {
        nbar += (unsigned)W;
        alive = nm_barrier(g.ctr + p, nbar, g.err, &s_ok);
        if (!alive) break;
      }
      const int tlen = qpow[b1 - b0] * RC;
      const double* T = Tg;
      if (g.t_lds) {
        for (int e0 = tid; e0 < tlen; e0 += 4 * NM_NT) {
          double v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = e0 + k * NM_NT < tlen ? Tg[e0 + k * NM_NT] : 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (e0 + k * NM_NT < tlen) Tl[e0 + k * NM_NT] = v[k];
        }
        __syncthreads();
        T = Tl;
      }
      for (int n = b0; n < b1; ++n) {
        nm_mttkrp_block<RC>(T, Fl, Mb, part, n, b0, b1, Q, R);
        if (tid < 64) {
          if constexpr (RC >= 16)
            nm_mode_call<RC>(Mb, Fl, Gr, wk, nrm, n, N, Q, R, &s_bad);
          else
            nm_mode_wave<RC>(Mb, Fl, Gr, wk, nrm, n, N, Q, R, &s_bad);
        }
        __syncthreads();
      }
    }
  }
  if (w != 0) return;
  int nf = 0;
  for (int e = tid; e < N * QR; e += NM_NT) {
    const int m = e / QR, rem = e - m * QR, q = rem / R, r = rem - q * R;
    const double v = Fl[m * QRC + q * RC + r];
    nf |= isfinite(v) ? 0 : 1;
    g.F[(int64_t)p * N * QR + e] = v;
  }
  if (tid < R) {
    g.lam[(int64_t)p * R + tid] = nrm[tid];
    nf |= isfinite(nrm[tid]) ? 0 : 1;
  }
  if (nf) atomicOr(g.flags + p, 4);
  if (tid == 0 && s_bad) atomicOr(g.flags + p, 1);
  if (tid == 0 && !alive) atomicOr(g.flags + p, 2);
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

// out = (sum of partials[0..nb), sum of partials[nb..2 nb)), a fixed order:
// strided per-thread sums, then a tree
__global__ __launch_bounds__(256) void nm_fit_reduce(const double* __restrict__ partials, int nb,
                                                     double* __restrict__ out) {
  __shared__ double s_a[256], s_b[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += partials[i];
    b += partials[nb + i];
  }
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s_a[threadIdx.x] += s_a[threadIdx.x + st];
      s_b[threadIdx.x] += s_b[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_a[0];
    out[1] = s_b[0];
  }
}

unsigned grid_of(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t nm_ttm_mfma(hipStream_t s, const double* in, int64_t in_stride, bool cols, int64_t pre,
                       int d, int post, const double* U, int M1, int P, int Q, int S, double* out,
                       int64_t out_stride) {
  const int nqb = (Q + 15) / 16, nbb = (post + 15) / 16;
  const int64_t ntiles = (int64_t)P * pre * nqb * nbb;
  const int64_t blocks = (ntiles + 3) / 4;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nm_ttm_mfma_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, in_stride,
                     cols, pre, d, post, U, M1, P, Q, S, out, out_stride, nqb, nbb, ntiles);
  return hipGetLastError();
}

hipError_t nm_temporal(hipStream_t s, const double* T, int64_t t_stride, int64_t t, int64_t L,
                       const double* W, int M1, int P, int Q, int S, double* Z, int* zbad) {
  hipLaunchKernelGGL(nm_temporal_kernel, dim3(grid_of(L * Q), P), dim3(256), 0, s, T, t_stride, t,
                     L, W, M1, P, Q, S, Z, zbad);
  return hipGetLastError();
}

static int nm_rc(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : 32); }

namespace {
struct NmAlsPlan {
  int W, inter_lds, t_lds, SA, SB, TMAX;
  size_t lds;
  int64_t work;   // doubles per replica
};

int64_t ipow64(int64_t b, int e) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}

// Workgroups per replica and the place of the intermediates for one launch.
NmAlsPlan nm_plan(int N, int Q, int R, int W) {
  NmAlsPlan pl{};
  const int RC = nm_rc(R);
  const int nL = N / 2;
  const int64_t nrow = ipow64(Q, nL), ncol = ipow64(Q, N - nL);
  pl.W = W;
  const int64_t crow = (nrow + W - 1) / W, ccol = (ncol + W - 1) / W;
  // first and second contraction of either half, for the largest share
  const int64_t sa = std::max(crow * ipow64(Q, N - 1 - nL), ipow64(Q, nL - 1) * ccol) * RC;
  const int64_t sb = std::max(N - nL >= 3 ? crow * ipow64(Q, N - 2 - nL) : 0,
                              nL >= 3 ? ipow64(Q, nL - 2) * ccol : 0) * RC;
  pl.SA = (int)sa;
  pl.SB = (int)sb;
  pl.TMAX = (int)(std::max(nrow, ncol) * RC);
  const size_t base = ((size_t)N * Q * RC + (size_t)N * R * R + (size_t)Q * R +
                       (size_t)R * R + NM_NT + R) * 8;
  const size_t cap = 160 * 1024 - 64;
  size_t lds = base;
  pl.t_lds = (lds + (size_t)pl.TMAX * 8 <= cap) ? 1 : 0;
  if (pl.t_lds) lds += (size_t)pl.TMAX * 8;
  pl.inter_lds = (lds + (size_t)(sa + sb) * 8 <= cap) ? 1 : 0;
  if (pl.inter_lds) lds += (size_t)(sa + sb) * 8;
  pl.lds = lds;
  pl.work = (nrow + ncol) * RC + (pl.inter_lds ? 0 : (int64_t)W * (sa + sb));
  return pl;
}

// Workgroups per replica: up to 8, at most one workgroup per CU over all
// replicas, no more than the rows of T_L or the columns of T_R.
int nm_pick_w(int P, int N, int Q) {
  const int nL = N / 2;
  int W = 256 / (P > 0 ? P : 1);
  W = W < 8 ? W : 8;
  const int64_t nrow = ipow64(Q, nL);
  if (W > nrow) W = (int)nrow;
  return W < 2 ? 1 : W;
}
}  // namespace

size_t nm_als_lds_bytes(int N, int Q, int R) { return nm_plan(N, Q, R, 1).lds; }

int64_t nm_als_work_len(int N, int Q, int R, int P) {
  const int W = nm_pick_w(P, N, Q);
  return std::max(nm_plan(N, Q, R, W).work, nm_plan(N, Q, R, 1).work);
}

hipError_t nm_als(hipStream_t s, const double* Y, int P, int N, int Q, int R, const double* init,
                  double* F, double* lam, int* flags, int iters, double* work, unsigned* ctr,
                  int* err) {
  if (N < 3 || N > OCTEN_NM_MAX_MODES_K || ipow64(Q, N) > (1LL << 22) || R > 32 || R > Q || R < 1)
    return hipErrorInvalidValue;
  NmAlsArgs a;
  a.Y = Y; a.init = init; a.F = F; a.lam = lam; a.flags = flags; a.work = work;
  a.ctr = ctr; a.err = err;
  a.N = N; a.Q = Q; a.R = R; a.iters = iters;
  a.QN1 = (int)ipow64(Q, N - 1);
  a.work_stride = nm_als_work_len(N, Q, R, P);
  const int rc = nm_rc(R);
  const void* fn = rc == 8 ? (const void*)nm_als_kernel<8>
                           : (rc == 16 ? (const void*)nm_als_kernel<16> : (const void*)nm_als_kernel<32>);
  int W = nm_pick_w(P, N, Q);
  if (W > 1) {
    const NmAlsPlan pl = nm_plan(N, Q, R, W);
    a.W = W; a.inter_lds = pl.inter_lds; a.t_lds = pl.t_lds; a.SA = pl.SA; a.SB = pl.SB;
    a.TMAX = pl.TMAX;
    hipError_t e = fill_i32(s, (int*)ctr, P, 0);
    if (e == hipSuccess) e = fill_i32(s, err, 1, 0);
    if (e == hipSuccess && pl.lds <= 160 * 1024 - 64)
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    if (e == hipSuccess && pl.lds <= 160 * 1024 - 64) {
      void* args[] = {&a};
      e = hipLaunchCooperativeKernel(fn, dim3(P * W), dim3(NM_NT), args, (unsigned)pl.lds, s);
      if (e == hipSuccess) return hipSuccess;
    }
    (void)hipGetLastError();   // no cooperative launch here: one workgroup per replica
  }
  const NmAlsPlan pl = nm_plan(N, Q, R, 1);
  if (pl.lds > 160 * 1024 - 64) return hipErrorInvalidValue;
  a.W = 1; a.inter_lds = pl.inter_lds; a.t_lds = pl.t_lds; a.SA = pl.SA; a.SB = pl.SB;
  a.TMAX = pl.TMAX;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3(P), dim3(NM_NT), args, pl.lds, s);
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
  hipLaunchKernelGGL(nm_fit_reduce, dim3(1), dim3(256), 0, s, partials, (int)nb, out2);
  return hipGetLastError();
}

}  // namespace octen
