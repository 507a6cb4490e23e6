// Sparse batches given by their nonzeros (COO sorted by k, then i, then j).
//
// Compression (Sec. 4.1; the summaries of a sparse tensor are dense and Eq. 1
// applies to the sum over nonzeros).  Integer bookkeeping first, exact:
//   segment s = one distinct (k, i) pair, in input order;
//   seg_start[s] = its first nonzero (seg_start[nseg] = nnz),
//   seg_row[s] = its i, seg_slice[s] = its k,
//   slice_seg[k] .. slice_seg[k+1] = the segments of slice k.
// Then per slice k and replica p (one workgroup each):
//   r_s(b) = sum_{n in s} v_n V_p(j_n, b)        lanes over b (gather); a
//                                                 segment of more than 32
//                                                 nonzeros is cut into
//                                                 chunks summed separately
//   M_k^p  = sum_s U_p(i_s, :)^T r_s              32 rows per pass;
//                                                 MFMA 32x32x2 for f32,
//                                                 plain FMAs for f64
// and the mode-3 product of the dense path produces Z_p.
//
// Fitness (Sec. 5.1) of a sparse tensor through
//   ||X - Xh||^2 = ||X||^2 - 2 <X, Xh> + sum((A^T A) * (B^T B) * (C^T C)).
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

typedef float f32x4c __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = NT * SCAN_ITEMS;

inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

// bad |= 1: a coordinate out of range; bad |= 2: not sorted by (k, i, j)
__global__ void coo_check_kernel(int64_t nnz, const int* __restrict__ k, const int* __restrict__ i,
                                 const int* __restrict__ j, int64_t t, int64_t I, int64_t J,
                                 int check_order, int* __restrict__ bad) {
  int b = 0;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < nnz;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int kk = k[n], ii = i[n], jj = j[n];
    if (kk < 0 || kk >= t || ii < 0 || ii >= I || jj < 0 || jj >= J) b |= 1;
    if (check_order && n > 0) {
      const int k0 = k[n - 1], i0 = i[n - 1], j0 = j[n - 1];
      if (kk < k0 || (kk == k0 && (ii < i0 || (ii == i0 && jj < j0)))) b |= 2;
    }
  }
  if (b) atomicOr(bad, b);
}

__device__ __forceinline__ int seg_head(int64_t n, const int* __restrict__ k,
                                        const int* __restrict__ i) {
  return (n == 0 || k[n] != k[n - 1] || i[n] != i[n - 1]) ? 1 : 0;
}

// Inclusive scan of the segment-head flags, pass 1: scan within tiles of
// SCAN_TILE nonzeros, tile totals to sums.
__global__ __launch_bounds__(NT) void scan_tile_kernel(int64_t nnz, const int* __restrict__ k,
                                                       const int* __restrict__ i,
                                                       int* __restrict__ out,
                                                       int* __restrict__ sums) {
  __shared__ int sm[NT];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS], run = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    const int64_t n = base + q;
    run += n < nnz ? seg_head(n, k, i) : 0;
    v[q] = run;
  }
  sm[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const int add = threadIdx.x >= off ? sm[threadIdx.x - off] : 0;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  const int prefix = threadIdx.x > 0 ? sm[threadIdx.x - 1] : 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < nnz) out[base + q] = v[q] + prefix;
  if (threadIdx.x == NT - 1) sums[blockIdx.x] = sm[NT - 1];
}

// pass 2, one workgroup: exclusive scan of the tile totals in place; the
// grand total (the segment count) goes to sums[nb]
__global__ __launch_bounds__(NT) void scan_sums_kernel(int nb, int* __restrict__ sums) {
  __shared__ int sm[NT];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += NT) {
    const int x = b0 + threadIdx.x;
    const int v = x < nb ? sums[x] : 0;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
      const int add = threadIdx.x >= off ? sm[threadIdx.x - off] : 0;
      __syncthreads();
      sm[threadIdx.x] += add;
      __syncthreads();
    }
    if (x < nb) sums[x] = carry + sm[threadIdx.x] - v;
    carry += sm[NT - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

// pass 3: add the tile offsets and scatter the segment heads
__global__ __launch_bounds__(NT) void seg_fill_kernel(int64_t nnz, const int* __restrict__ k,
                                                      const int* __restrict__ i,
                                                      const int* __restrict__ scan,
                                                      const int* __restrict__ sums,
                                                      int* __restrict__ seg_start,
                                                      int* __restrict__ seg_row,
                                                      int* __restrict__ seg_slice) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  const int off = sums[blockIdx.x];
  for (int q = threadIdx.x; q < SCAN_TILE; q += NT) {
    const int64_t n = base + q;
    if (n < nnz && seg_head(n, k, i)) {
      const int s = scan[n] + off - 1;
      seg_start[s] = (int)n;
      seg_row[s] = i[n];
      seg_slice[s] = k[n];
    }
  }
}

// slice_seg[x] = first segment whose slice is >= x, x in [0, t]; closes
// seg_start with nnz.  nseg is read from the device.
__global__ void slice_range_kernel(const int* __restrict__ nseg_p, int64_t t, int64_t nnz,
                                   const int* __restrict__ seg_slice, int* __restrict__ slice_seg,
                                   int* __restrict__ seg_start) {
  const int nseg = *nseg_p;
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x <= t) {
    int lo = 0, hi = nseg;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (seg_slice[mid] < x) lo = mid + 1; else hi = mid;
    }
    slice_seg[x] = lo;
  }
  if (x == 0) seg_start[nseg] = (int)nnz;
}

template <typename T>
struct CooTraits;
template <>
struct CooTraits<float> {
  static constexpr int SC = 32;  // segments per pass (16 MFMA k-steps of 2)
};
template <>
struct CooTraits<double> {
  static constexpr int SC = 16;
};

// One workgroup per (slice k, replica p); blockIdx is mapped so that the P
// workgroups of one slice run on the same XCD (they read the same nonzeros
// and the same rows of U and V).  The FP32 kernels for Q <= 96 are held to
// 128 registers (four workgroups per CU instead of three, no spills): the
// gathers are latency-bound, and a 16-replica batch of 100 slices then runs
// in two waves of workgroups instead of three.
template <typename T, int QT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 && QT <= 3 ? 4 : 1))) void coo_compress_kernel(
    const int* __restrict__ seg_start, const int* __restrict__ seg_row,
    const int* __restrict__ slice_seg, const int* __restrict__ jj, const float* __restrict__ vv,
    const T* __restrict__ Vm, const T* __restrict__ Um, int64_t t, int M1, int P, int Q, int S,
    int per_xcd, T* __restrict__ Mout) {
  constexpr int SC = CooTraits<T>::SC;
  // the SC + 1 segment starts of a pass are read by the lanes of one wavefront
  static_assert(SC < 64, "segments per pass must fit one wavefront");
  constexpr int QP = QT * 32;
  constexpr int NX = QT > 2 ? 2 : 1;   // columns gathered per lane
  __shared__ T Ub[SC][QP];
  __shared__ T Rb[SC][QP];
  const int64_t u = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (u >= t * P) return;
  const int64_t k = u / P;
  const int p = (int)(u % P);
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int s0 = slice_seg[k], s1 = slice_seg[k + 1];

  int colx[NX];
  bool okx[NX];
#pragma unroll
  for (int x = 0; x < NX; ++x) {
    const int b = lane + 64 * x;
    okx[x] = b < Q;
    colx[x] = b < S ? b : S + p * (Q - S) + (b - S);
  }
  // padding columns stay zero
  for (int e = tid; e < SC * QP; e += NT) {
    const int b = e % QP;
    if (b >= Q) { Ub[e / QP][b] = T(0); Rb[e / QP][b] = T(0); }
  }

  // FP32: 16 x 16 output tiles (Q = 80 is five of them, no padded work),
  // dealt to the four wavefronts; at most (2 QT)^2 / 4 = QT^2 per wavefront
  constexpr int TPW = QT * QT;
  const int Q16 = (Q + 15) / 16;
  const int ntile = Q16 * Q16;
  // tile t -> (t / Q16, t % Q16) by a multiply-high: exact for t < 64, Q16 <= 8
  const unsigned q16inv = (65536u + (unsigned)Q16 - 1u) / (unsigned)Q16;
  constexpr int NOUT = (QP * QP + NT - 1) / NT;
  f32x4c acc[sizeof(T) == 4 ? TPW : 1];
  double accd[sizeof(T) == 8 ? NOUT : 1];
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int q = 0; q < TPW; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[q][e] = 0.f;
  } else {
#pragma unroll
    for (int q = 0; q < NOUT; ++q) accd[q] = 0.0;
  }

  // Passes over the slice's segments.  A pass is either up to SC consecutive
  // segments of at most CH nonzeros (one row each), or one longer segment cut
  // into SC chunks of its nonzeros (one row per chunk, each with the same U
  // row): a few rows of a Zipf-skewed slice hold thousands of nonzeros and
  // would otherwise serialise one wavefront.  Each wavefront walks its SPW
  // rows together, one nonzero of each per step, so their loads overlap.
  constexpr int CH = 32;
  constexpr int SPW = SC / 4;
  // segment starts c0 .. c0 + SC of a pass (one per lane, clamped to s1;
  // seg_start holds nseg + 1 entries); the next pass's are loaded while the
  // current pass's outer products run
  int c0 = s0;
  int st_next = seg_start[c0 + lane <= s1 ? c0 + lane : s1];
  while (c0 < s1) {
    // this pass's segment starts, their lengths and the long ones
    const int st = st_next;
    const int st1 = __shfl_down(st, 1, 64);
    const bool is_long = lane < SC && c0 + lane < s1 && st1 - st > CH;
    const unsigned long long longm = __ballot(is_long);
    const int n_first = __builtin_amdgcn_readfirstlane(st);
    const bool long_pass = (longm & 1ull) != 0;
    int ns = 1;
    if (!long_pass) {
      ns = longm ? __builtin_ctzll(longm) : SC;
      if (ns > s1 - c0) ns = s1 - c0;
      if (ns > SC) ns = SC;
    }
    const int n_last = long_pass ? __builtin_amdgcn_readlane(st, 1) : 0;
    const int chunk = long_pass ? (n_last - n_first + SC - 1) / SC : 0;
    const int64_t irow_long = long_pass ? (int64_t)seg_row[c0] * M1 : 0;

    int nb[SPW], ne[SPW];
    int64_t irow[SPW];
    bool rowok[SPW];
    int maxlen = 0;
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
      const int r = wave + 4 * q;
      if (long_pass) {
        nb[q] = n_first + r * chunk;
        ne[q] = nb[q] + chunk < n_last ? nb[q] + chunk : n_last;
        if (ne[q] < nb[q]) ne[q] = nb[q];
        irow[q] = irow_long;
        rowok[q] = true;
      } else {
        rowok[q] = r < ns;
        nb[q] = __builtin_amdgcn_readlane(st, r);
        ne[q] = rowok[q] ? __builtin_amdgcn_readlane(st, r + 1) : nb[q];
        irow[q] = rowok[q] ? (int64_t)seg_row[c0 + r] * M1 : 0;
      }
      maxlen = ne[q] - nb[q] > maxlen ? ne[q] - nb[q] : maxlen;
    }
    T r[SPW][NX], uu[SPW][NX];
#pragma unroll
    for (int q = 0; q < SPW; ++q)
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        r[q][x] = T(0);
        uu[q][x] = (okx[x] && rowok[q]) ? Um[irow[q] + colx[x]] : T(0);
      }
    // the value and row index of step m + 1 are loaded while the rows of
    // step m are in flight (scalar loads, a separate counter)
    T vn[SPW];
    const T* rn[SPW];
    auto load_idx = [&](int m) {
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        const int n = nb[q] + m;
        const bool ok = n < ne[q];
        const int nn = ok ? n : n_first;   // a valid index; its value is not used
        vn[q] = ok ? (T)vv[nn] : T(0);
        rn[q] = Vm + (int64_t)jj[nn] * M1;
      }
    };
    if (maxlen > 0) load_idx(0);
    for (int m = 0; m < maxlen; ++m) {
      T v[SPW], val[SPW][NX];
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        v[q] = vn[q];
#pragma unroll
        for (int x = 0; x < NX; ++x) val[q][x] = okx[x] ? rn[q][colx[x]] : T(0);
      }
      if (m + 1 < maxlen) load_idx(m + 1);
#pragma unroll
      for (int q = 0; q < SPW; ++q)
#pragma unroll
        for (int x = 0; x < NX; ++x) r[q][x] = fma(v[q], val[q][x], r[q][x]);
    }
    const int c0n = c0 + (long_pass ? 1 : ns);
    st_next = seg_start[c0n + lane <= s1 ? c0n + lane : s1];
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
      const int sg = wave + 4 * q;
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        if (okx[x]) {
          Ub[sg][lane + 64 * x] = uu[q][x];
          Rb[sg][lane + 64 * x] = r[q][x];
        }
      }
    }
    c0 = c0n;
    __syncthreads();
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const int tt = wave + 4 * q;
        if (tt < ntile) {
          const int ti = (int)(((unsigned)tt * q16inv) >> 16), tj = tt - ti * Q16;
          // A = U^T (lane: column ti*16 + lane%16 of segment row kk), B = R
#pragma unroll
          for (int ks = 0; ks < SC / 4; ++ks) {
            const int kk = 4 * ks + lane / 16;
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                (float)Ub[kk][ti * 16 + lane % 16], (float)Rb[kk][tj * 16 + lane % 16], acc[q], 0,
                0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NOUT; ++q) {
        const int e = tid + NT * q;
        if (e < Q * Q) {
          const int a = e / Q, b = e % Q;
          double sacc = accd[q];
#pragma unroll
          for (int sg = 0; sg < SC; ++sg) sacc = fma((double)Ub[sg][a], (double)Rb[sg][b], sacc);
          accd[q] = sacc;
        }
      }
    }
    __syncthreads();
  }

  T* out = Mout + ((int64_t)k * P + p) * Q * Q;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int tt = wave + 4 * q;
      if (tt < ntile) {
        const int ti = (int)(((unsigned)tt * q16inv) >> 16), tj = tt - ti * Q16;
        const int bcol = tj * 16 + lane % 16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int arow = ti * 16 + 4 * (lane / 16) + e;
          if (arow < Q && bcol < Q) out[arow * Q + bcol] = acc[q][e];
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < NOUT; ++q) {
      const int e = tid + NT * q;
      if (e < Q * Q) out[e] = (T)accd[q];
    }
  }
}

// sum over the given nonzeros of v^2 and v * Xh(i, j, k0 + k), FP64
__global__ __launch_bounds__(NT) void fit_coo_kernel(int64_t nnz, const int* __restrict__ k,
                                                     const int* __restrict__ i,
                                                     const int* __restrict__ j,
                                                     const float* __restrict__ v, int64_t k0,
                                                     int R, const double* __restrict__ A,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ C,
                                                     double* __restrict__ partials) {
  __shared__ double r1[NT], r2[NT];
  double nx = 0.0, inner = 0.0;
  for (int64_t n = blockIdx.x * (int64_t)NT + threadIdx.x; n < nnz; n += (int64_t)gridDim.x * NT) {
    const double* a = A + (int64_t)i[n] * R;
    const double* b = B + (int64_t)j[n] * R;
    const double* c = C + (k0 + k[n]) * R;
    double xh = 0.0;
    for (int r = 0; r < R; ++r) xh = fma(a[r] * b[r], c[r], xh);
    const double x = (double)v[n];
    nx = fma(x, x, nx);
    inner = fma(x, xh, inner);
  }
  r1[threadIdx.x] = nx;
  r2[threadIdx.x] = inner;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = r1[0];
    partials[2 * blockIdx.x + 1] = r2[0];
  }
}

// out[0], out[1] = sums of the partials; out[2] = sum of GA * GB * GC
__global__ __launch_bounds__(NT) void fit_coo_reduce(const double* __restrict__ partials, int np,
                                                     const double* __restrict__ G, int R,
                                                     double* __restrict__ out) {
  __shared__ double r1[NT], r2[NT], r3[NT];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int e = threadIdx.x; e < np; e += NT) { a += partials[2 * e]; b += partials[2 * e + 1]; }
  for (int e = threadIdx.x; e < R * R; e += NT) c += G[e] * G[R * R + e] * G[2 * R * R + e];
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  r3[threadIdx.x] = c;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
      r3[threadIdx.x] += r3[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = r1[0]; out[1] = r2[0]; out[2] = r3[0]; }
}

template <typename T>
hipError_t launch_coo_compress(hipStream_t s, int64_t t, int P, int Q, int S, int M1,
                               const int* seg_start, const int* seg_row, const int* slice_seg,
                               const int* j, const float* v, const T* Vm, const T* Um, T* Mout) {
  const int64_t nblk = t * P;
  const int per = (int)((nblk + 7) / 8);
  const dim3 grid((unsigned)(8 * (int64_t)per));
  switch ((Q + 31) / 32) {
#define OCTEN_COO_CASE(QT)                                                                  \
  case QT:                                                                                  \
    hipLaunchKernelGGL((coo_compress_kernel<T, QT>), grid, dim3(NT), 0, s, seg_start, seg_row, \
                       slice_seg, j, v, Vm, Um, t, M1, P, Q, S, per, Mout);                 \
    break;
    OCTEN_COO_CASE(1)
    OCTEN_COO_CASE(2)
    OCTEN_COO_CASE(3)
    OCTEN_COO_CASE(4)
#undef OCTEN_COO_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t coo_work_ints(int64_t nnz) {
  const int64_t nb = (nnz + SCAN_TILE - 1) / SCAN_TILE;
  return (size_t)(nnz + nb + 1);
}

hipError_t coo_check(hipStream_t s, int64_t nnz, const int* k, const int* i, const int* j,
                     int64_t t, int64_t I, int64_t J, bool check_order, int* bad) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(coo_check_kernel, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, k, i, j, t, I, J,
                     check_order ? 1 : 0, bad);
  return hipGetLastError();
}

hipError_t coo_segments(hipStream_t s, int64_t nnz, const int* k, const int* i, int64_t t,
                        int* work, int* seg_start, int* seg_row, int* seg_slice, int* slice_seg,
                        int* nseg_dev) {
  const int64_t nb = (nnz + SCAN_TILE - 1) / SCAN_TILE;
  int* scan = work;
  int* sums = work + nnz;
  if (nnz > 0) {
    hipLaunchKernelGGL(scan_tile_kernel, dim3((unsigned)nb), dim3(NT), 0, s, nnz, k, i, scan, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(NT), 0, s, (int)nb, sums);
    hipLaunchKernelGGL(seg_fill_kernel, dim3((unsigned)nb), dim3(NT), 0, s, nnz, k, i, scan, sums,
                       seg_start, seg_row, seg_slice);
    hipLaunchKernelGGL(slice_range_kernel, dim3(grid_for(t + 1)), dim3(256), 0, s, sums + nb, t,
                       nnz, seg_slice, slice_seg, seg_start);
    hipError_t e = hipMemcpyAsync(nseg_dev, sums + nb, sizeof(int), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  } else {
    hipError_t e = fill_i32(s, slice_seg, t + 1, 0);
    if (e == hipSuccess) e = fill_i32(s, seg_start, 1, 0);
    if (e == hipSuccess) e = fill_i32(s, nseg_dev, 1, 0);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t coo_compress(hipStream_t s, bool f64, int64_t t, int P, int Q, int S, int M1,
                        const int* seg_start, const int* seg_row, const int* slice_seg,
                        const int* j, const float* v, const void* Vm, const void* Um, void* Mout) {
  if (f64)
    return launch_coo_compress<double>(s, t, P, Q, S, M1, seg_start, seg_row, slice_seg, j, v,
                                       (const double*)Vm, (const double*)Um, (double*)Mout);
  return launch_coo_compress<float>(s, t, P, Q, S, M1, seg_start, seg_row, slice_seg, j, v,
                                    (const float*)Vm, (const float*)Um, (float*)Mout);
}

hipError_t fit_coo(hipStream_t s, int64_t nnz, const int* k, const int* i, const int* j,
                   const float* v, int64_t k0, int64_t I, int64_t J, int64_t kc, int R,
                   const double* A, const double* B, const double* C, double* G, double* partials,
                   int nparts, double* out3) {
  // Gram matrices of the three factors (C over its first kc rows)
  hipError_t e = rowdot(s, R, R, I, A, 1, R, A, R, 1, nullptr, 1.0, 0.0, G, R);
  if (e == hipSuccess) e = rowdot(s, R, R, J, B, 1, R, B, R, 1, nullptr, 1.0, 0.0, G + R * R, R);
  if (e == hipSuccess)
    e = rowdot(s, R, R, kc, C, 1, R, C, R, 1, nullptr, 1.0, 0.0, G + 2 * R * R, R);
  if (e != hipSuccess) return e;
  int np = 1;
  if (nnz > 0) {
    np = grid_for(nnz);
    if (np > nparts) np = nparts;
    hipLaunchKernelGGL(fit_coo_kernel, dim3(np), dim3(NT), 0, s, nnz, k, i, j, v, k0, R, A, B, C,
                       partials);
  } else {
    e = fill_f64(s, partials, 2, 0.0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fit_coo_reduce, dim3(1), dim3(NT), 0, s, partials, np, G, R, out3);
  return hipGetLastError();
}

}  // namespace octen
