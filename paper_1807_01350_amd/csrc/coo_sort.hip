// Stable sort of a sparse batch by (k, i, j), for batches that do not
// arrive in that order (the sparse input of Sec. 4.1; the segments of the
// compression are runs of equal (k, i)).
//
// Least-significant-digit radix sort of packed keys
//   key = k << (bi + bj) | i << bj | j      (bk + bi + bj <= 64 bits)
// with the value carried along, 8-bit digits, one pass per digit:
//   1. per tile of RS_TILE entries, a 256-bin digit histogram, stored
//      bin-major: hist[d * ntile + tile];
//   2. an exclusive scan of hist gives every (digit, tile) its first output
//      position;
//   3. each tile scatters its entries in input order: every wavefront owns a
//      contiguous quarter of the tile, takes its offset per digit from the
//      waves before it, and walks its quarter 64 entries at a time, an
//      entry's rank among the equal digits of its group of 64 coming from
//      eight ballots.  Equal keys keep their input order (stable), so the
//      result is unique, and so is the whole pass sequence.
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

namespace {

constexpr int RS_NT = 256;
constexpr int RS_WAVES = RS_NT / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_NT * RS_ITEMS;   // 4096 entries per tile
constexpr int RS_QUARTER = RS_TILE / RS_WAVES;
constexpr int RS_BINS = 256;
constexpr int SC_CHUNK = 2048;              // scan: entries per block

__global__ void pack_kernel(int64_t n, const int* __restrict__ k, const int* __restrict__ i,
                            const int* __restrict__ j, const float* __restrict__ v, int sh_k,
                            int sh_i, unsigned long long* __restrict__ key,
                            float* __restrict__ val) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    key[e] = ((unsigned long long)(unsigned)k[e] << sh_k) |
             ((unsigned long long)(unsigned)i[e] << sh_i) | (unsigned long long)(unsigned)j[e];
    val[e] = v[e];
  }
}

__global__ void unpack_kernel(int64_t n, const unsigned long long* __restrict__ key,
                              const float* __restrict__ val, int sh_k, int sh_i,
                              int* __restrict__ k, int* __restrict__ i, int* __restrict__ j,
                              float* __restrict__ v) {
  const unsigned long long mi = (1ull << (sh_k - sh_i)) - 1ull, mj = (1ull << sh_i) - 1ull;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long x = key[e];
    k[e] = (int)(sh_k < 64 ? x >> sh_k : 0ull);
    i[e] = (int)((x >> sh_i) & mi);
    j[e] = (int)(x & mj);
    v[e] = val[e];
  }
}

__global__ __launch_bounds__(RS_NT) void hist_kernel(int64_t n, const unsigned long long* __restrict__ key,
                                                     int shift, int ntile, int* __restrict__ hist) {
  __shared__ int h[RS_BINS];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
  for (int u = 0; u < RS_ITEMS; ++u) {
    const int64_t e = base + u * RS_NT + threadIdx.x;
    if (e < n) atomicAdd(&h[(int)((key[e] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan, pass 1: each block scans SC_CHUNK entries in place and
// writes its total to sums[block].
__global__ __launch_bounds__(RS_NT) void scan_chunk_kernel(int64_t len, int* __restrict__ a,
                                                           int* __restrict__ sums) {
  __shared__ int sm[RS_NT];
  constexpr int PER = SC_CHUNK / RS_NT;
  const int64_t base = (int64_t)blockIdx.x * SC_CHUNK + threadIdx.x * PER;
  int x[PER], run = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    x[u] = base + u < len ? a[base + u] : 0;
    const int t = x[u];
    x[u] = run;
    run += t;
  }
  sm[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < RS_NT; off <<= 1) {
    const int y = threadIdx.x >= (unsigned)off ? sm[threadIdx.x - off] : 0;
    __syncthreads();
    sm[threadIdx.x] += y;
    __syncthreads();
  }
  const int before = threadIdx.x > 0 ? sm[threadIdx.x - 1] : 0;
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (base + u < len) a[base + u] = x[u] + before;
  if (threadIdx.x == RS_NT - 1) sums[blockIdx.x] = sm[RS_NT - 1];
}

// Pass 2: one block turns the chunk totals into exclusive chunk offsets.
__global__ __launch_bounds__(RS_NT) void scan_sums_kernel2(int nch, int* __restrict__ sums) {
  __shared__ int sm[RS_NT];
  const int per = (nch + RS_NT - 1) / RS_NT;
  const int b0 = threadIdx.x * per;
  int run = 0;
  for (int u = 0; u < per; ++u)
    if (b0 + u < nch) run += sums[b0 + u];
  sm[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < RS_NT; off <<= 1) {
    const int y = threadIdx.x >= (unsigned)off ? sm[threadIdx.x - off] : 0;
    __syncthreads();
    sm[threadIdx.x] += y;
    __syncthreads();
  }
  int acc = threadIdx.x > 0 ? sm[threadIdx.x - 1] : 0;
  for (int u = 0; u < per; ++u)
    if (b0 + u < nch) {
      const int t = sums[b0 + u];
      sums[b0 + u] = acc;
      acc += t;
    }
}

// Pass 3: chunk offsets added.
__global__ __launch_bounds__(RS_NT) void scan_add_kernel(int64_t len, int* __restrict__ a,
                                                         const int* __restrict__ sums) {
  const int64_t e = (int64_t)blockIdx.x * RS_NT + threadIdx.x;
  if (e < len) a[e] += sums[e / SC_CHUNK];
}

__global__ __launch_bounds__(RS_NT) void scatter_kernel(int64_t n, const unsigned long long* __restrict__ key,
                                                        const float* __restrict__ val, int shift,
                                                        int ntile, const int* __restrict__ hist,
                                                        unsigned long long* __restrict__ okey,
                                                        float* __restrict__ oval) {
  __shared__ int gbase[RS_BINS];
  __shared__ int woff[RS_WAVES][RS_BINS];   // per-wave counts, then offsets
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  gbase[tid] = hist[(int64_t)tid * ntile + blockIdx.x];
#pragma unroll
  for (int w = 0; w < RS_WAVES; ++w) woff[w][tid] = 0;
  __syncthreads();
  const int64_t qbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)wave * RS_QUARTER;
  // counts of every digit in each wave's quarter
  for (int c = 0; c < RS_QUARTER; c += 64) {
    const int64_t e = qbase + c + lane;
    if (e < n) atomicAdd(&woff[wave][(int)((key[e] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  // offsets of each wave within the tile's run of a digit: the tile's first
  // position plus the counts of the waves before it
  {
    int acc = gbase[tid];
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
      const int cnt = woff[w][tid];
      woff[w][tid] = acc;
      acc += cnt;
    }
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int c = 0; c < RS_QUARTER; c += 64) {
    const int64_t e = qbase + c + lane;
    const bool ok = e < n;
    const unsigned long long x = ok ? key[e] : 0ull;
    const float y = ok ? val[e] : 0.f;
    const int d = (int)((x >> shift) & 255ull);
    unsigned long long same = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long bb = __ballot((d >> b) & 1);
      same &= ((d >> b) & 1) ? bb : ~bb;
    }
    const int pos = woff[wave][d] + __popcll(same & below);
    if (ok) {
      okey[pos] = x;
      oval[pos] = y;
    }
    // the highest lane of each digit moves that digit's offset past the group
    if (ok && (same >> lane) == 1ull) woff[wave][d] += __popcll(same);
    __builtin_amdgcn_wave_barrier();
  }
}

int bits_for(int64_t extent) {
  int b = 0;
  while (b < 63 && (1ll << b) < extent) ++b;
  return b;
}

}  // namespace

size_t coo_sort_work_bytes(int64_t nnz) {
  const int64_t ntile = (nnz + RS_TILE - 1) / RS_TILE;
  const int64_t hlen = (int64_t)RS_BINS * ntile;
  const int64_t nch = (hlen + SC_CHUNK - 1) / SC_CHUNK;
  return (size_t)nnz * 2 * (8 + 4) + (size_t)(hlen + nch + 64) * 4 + 256;
}

int coo_sort_key_bits(int64_t t, int64_t I, int64_t J) {
  return bits_for(t) + bits_for(I) + bits_for(J);
}

hipError_t coo_sort(hipStream_t s, int64_t nnz, const int* k, const int* i, const int* j,
                    const float* v, int64_t t, int64_t I, int64_t J, void* work, int* ko, int* io,
                    int* jo, float* vo) {
  if (nnz <= 0) return hipSuccess;
  const int bj = bits_for(J), bi = bits_for(I), bk = bits_for(t);
  if (bk + bi + bj > 64 || nnz >= 0x7fffffffLL) return hipErrorInvalidValue;
  const int sh_i = bj, sh_k = bi + bj;
  const int64_t ntile = (nnz + RS_TILE - 1) / RS_TILE;
  const int64_t hlen = (int64_t)RS_BINS * ntile;
  const int64_t nch = (hlen + SC_CHUNK - 1) / SC_CHUNK;
  if (ntile > 0x7fffffffLL) return hipErrorInvalidValue;
  unsigned char* w = (unsigned char*)work;
  unsigned long long* key[2] = {(unsigned long long*)w, (unsigned long long*)w + nnz};
  float* val[2] = {(float*)(key[1] + nnz), (float*)(key[1] + nnz) + nnz};
  int* hist = (int*)(val[1] + nnz);
  int* sums = hist + hlen;
  const unsigned g = (unsigned)((nnz + 255) / 256 < 65536 ? (nnz + 255) / 256 : 65536);
  hipLaunchKernelGGL(pack_kernel, dim3(g), dim3(256), 0, s, nnz, k, i, j, v, sh_k, sh_i, key[0],
                     val[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int cur = 0;
  for (int shift = 0; shift < bk + bi + bj; shift += 8) {
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)ntile), dim3(RS_NT), 0, s, nnz, key[cur], shift,
                       (int)ntile, hist);
    hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)nch), dim3(RS_NT), 0, s, hlen, hist, sums);
    hipLaunchKernelGGL(scan_sums_kernel2, dim3(1), dim3(RS_NT), 0, s, (int)nch, sums);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((hlen + RS_NT - 1) / RS_NT)), dim3(RS_NT),
                       0, s, hlen, hist, sums);
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)ntile), dim3(RS_NT), 0, s, nnz, key[cur],
                       val[cur], shift, (int)ntile, hist, key[cur ^ 1], val[cur ^ 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cur ^= 1;
  }
  hipLaunchKernelGGL(unpack_kernel, dim3(g), dim3(256), 0, s, nnz, key[cur], val[cur], sh_k, sh_i,
                     ko, io, jo, vo);
  return hipGetLastError();
}

}  // namespace octen
