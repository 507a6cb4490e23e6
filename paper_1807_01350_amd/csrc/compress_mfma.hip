// Dense compression on gfx950 matrix cores (Sec. 4.1, Eq. 1: every replica
// is X x1 U_p^T x2 V_p^T x3 W_p^T of the batch).
//
// The two non-temporal products are one fused kernel per (slice k, block of
// BM rows i, column block cb):
//   stage 1  T = X_k[rows, :] V[:, cols(cb)]      (BM x 256, K = J)
//   stage 2  M_p += U_p[rows, :]^T T[:, cols(p)]  (Q x Q for each replica p in cb)
// A column block holds the S shared columns and G replicas' own columns, so
// both stages finish inside one workgroup.  Stage 1 streams X once from HBM
// (f32 rows, converted on the fly to the MFMA input type with the optional
// per-slice power-of-two scale), takes V from a pre-packed fragment image that
// stays in L2, and double-buffers both operands through LDS.  Stage 2 reads T
// back from LDS (transposed) and U from a pre-packed fragment image.  Partial
// M of each row block go to a workspace; a second kernel sums them and applies
// the mode-3 product with the batch's W rows (FP64 accumulation).
//
// Tile order is XCD-aware: workgroup x runs on XCD x % 8, and the column
// blocks that share one X tile are consecutive on the same XCD so that the
// second and third reads of the tile hit that XCD's L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "octen_internal.h"

namespace octen {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BN = 256;   // stage-1 columns per tile (shared + G replicas)
constexpr int KC = 32;    // j per pipeline chunk

// Rows per tile and threads per workgroup: the BF16 kernels take 256 rows
// with eight wavefronts (4 x 2 over the tile), so V is streamed from L2 once
// per 256 rows of X and half as many row-block partials are written; the
// FP32 kernels keep 128 rows and four wavefronts (their transposed stage-2
// tile would not fit in LDS at 256 rows).
template <int KIND>
struct Tile;
template <>
struct Tile<1> {
  static constexpr int BM = 128, NT = 256;
};
template <>
struct Tile<2> {
  static constexpr int BM = 256, NT = 512;
};

// Input kinds: 1 = f32 MFMA (32x32x2), 2 = bf16 MFMA (32x32x16).
template <int KIND> struct Kind;
template <> struct Kind<1> {
  using T = float;
  using Frag = float;
  static constexpr int KSTEP = 2;                  // k per MFMA
  static constexpr int EPL = 1;                    // elements per lane per fragment
  __device__ static Frag ld(const T* p) { return *p; }
  __device__ static f32x16 mma(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Kind<2> {
  using T = __bf16;
  using Frag = bf16x8;
  static constexpr int KSTEP = 16;
  static constexpr int EPL = 8;
  __device__ static Frag ld(const T* p) { return *(const bf16x8*)p; }
  __device__ static f32x16 mma(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// Fragment image of one KC chunk: [ks][tile][lane][EPL]
template <int KIND>
__host__ __device__ constexpr int chunk_elems(int tiles) {
  return (KC / Kind<KIND>::KSTEP) * tiles * 64 * Kind<KIND>::EPL;
}

template <int KIND>
__device__ __forceinline__ typename Kind<KIND>::T cvt(float x) {
  return (typename Kind<KIND>::T)x;
}

// Position of k index kk (0..KC) of row r inside the A fragment image.
template <int KIND>
__device__ __forceinline__ int a_pos(int r, int kk) {
  constexpr int KS = Kind<KIND>::KSTEP, E = Kind<KIND>::EPL;
  constexpr int BM = Tile<KIND>::BM;
  const int ks = kk / KS, kin = kk % KS;
  const int lane = (r % 32) + 32 * (kin / E);
  return ((ks * (BM / 32) + r / 32) * 64 + lane) * E + (kin % E);
}

struct Args {
  const float* X;
  const float* scale;       // [t] or null
  const void* Vpack;        // [ncb][nchunk][chunk image]
  const void* Upack;        // [nrb][P][BM/KSTEP][QT][64][EPL]
  const int* tilecol;       // [ncb][G][QT*32] -> column of T (BN = zero row)
  float* Mpart;             // [t][nrb][P][Q][Q]
  int64_t I, J;
  int t, P, Q, G, ncb, nrb, nchunk, tiles;
};

// Stage 2 of the two-term form, shared by the bfloat16 kernels: T (the
// float32 stage-1 accumulators of a BM x BN tile, in the 32x32 MFMA output
// layout of a 4 x 2 grid of wavefronts) goes through the LDS buffer T2t twice,
// first as T_hi = bf16(T), then as T_lo = bf16(T - T_hi); each work item (one
// 32-row tile of one replica's Q x Q output) accumulates both passes.  T_lo
// is formed with T_hi and kept packed (two values per register) until the
// second pass, so the float32 accumulators die after the first write.
template <int QT, int SPLIT>
__device__ __forceinline__ void stage2_split(const Args& g, const f32x16 (&acc)[2][4], __bf16* T2t,
                                             int k, int rb, int cb, float sc) {
  constexpr int BM = Tile<2>::BM, NT = Tile<2>::NT, E = 8;
  constexpr int T2LD = BM + 8;
  using T = __bf16;
  using Frag = bf16x8;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int p0 = cb * g.G;
  const int gcount = (g.P - p0) < g.G ? (g.P - p0) : g.G;
  const int nitems = gcount * QT;
  const float inv = 1.0f / sc;
  constexpr int KS = 16;
  bf16x4 lo[2][4][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn * 128 + j * 32 + lane % 32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 32 + 8 * q + 4 * (lane / 32);
        bf16x4 hi;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float v = acc[i][j][4 * q + e];
          hi[e] = (T)v;
          lo[i][j][q][e] = (T)(v - (float)hi[e]);
        }
        *(bf16x4*)(T2t + col * T2LD + r) = hi;
      }
    }
  f32x16 m[SPLIT][QT];
#pragma unroll
  for (int it = 0; it < SPLIT; ++it)
#pragma unroll
    for (int j = 0; j < QT; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) m[it][j][e] = 0.f;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = wn * 128 + j * 32 + lane % 32;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = wm * 64 + i * 32 + 8 * q + 4 * (lane / 32);
            *(bf16x4*)(T2t + col * T2LD + r) = lo[i][j][q];
          }
        }
    }
    for (int e = tid; e < T2LD; e += NT) T2t[BN * T2LD + e] = (T)0.f;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SPLIT; ++it) {
      const int item = wave + it * (NT / 64);
      if (item >= nitems) continue;
      const int gg = item / QT, i = item % QT;
      const int p = p0 + gg;
      const T* Up = (const T*)g.Upack + ((int64_t)rb * g.P + p) * (BM / KS) * QT * 64 * E;
      const int* tc = g.tilecol + ((int64_t)cb * g.G + gg) * QT * 32;
      int colrow[QT];
#pragma unroll
      for (int j = 0; j < QT; ++j) colrow[j] = tc[j * 32 + lane % 32];
#pragma unroll 2
      for (int ks = 0; ks < BM / KS; ++ks) {
        const Frag af = *(const Frag*)(Up + ((int64_t)(ks * QT + i) * 64 + lane) * E);
#pragma unroll
        for (int j = 0; j < QT; ++j) {
          const Frag bf = *(const Frag*)(T2t + colrow[j] * T2LD + ks * KS + (lane / 32) * E);
          m[it][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf, m[it][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < SPLIT; ++it) {
    const int item = wave + it * (NT / 64);
    if (item >= nitems) continue;
    const int gg = item / QT, i = item % QT;
    const int p = p0 + gg;
    float* out = g.Mpart + (((int64_t)k * g.nrb + rb) * g.P + p) * g.Q * g.Q;
#pragma unroll
    for (int j = 0; j < QT; ++j) {
      const int bcol = j * 32 + lane % 32;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int arow = i * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
        if (arow < g.Q && bcol < g.Q) out[arow * g.Q + bcol] = m[it][j][e] * inv;
      }
    }
  }
}

// SPLIT > 0 (bfloat16 only): the two-term form of compress_pipe2, with the
// hi and lo images of each X chunk side by side in LDS.
template <int KIND, int QT, bool VEC, int SPLIT>
__global__ __launch_bounds__(Tile<KIND>::NT) void compress_fused(Args g) {
  constexpr int BM = Tile<KIND>::BM, NT = Tile<KIND>::NT;
  using T = typename Kind<KIND>::T;
  using Frag = typename Kind<KIND>::Frag;
  constexpr int KS = Kind<KIND>::KSTEP, E = Kind<KIND>::EPL;
  constexpr int A_EL = chunk_elems<KIND>(BM / 32);   // A chunk image elements
  constexpr int B_EL = chunk_elems<KIND>(BN / 32);   // B chunk image elements
  constexpr int T2LD = BM + 16 / (int)sizeof(T);     // padded row of T^T
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NPART = SPLIT > 0 ? 2 : 1;
  T* As = (T*)smem;                 // [2][NPART][A_EL]
  T* Bs = As + 2 * NPART * A_EL;    // [2][B_EL]
  T* T2t = (T*)smem;                // [BN + 1][T2LD], reuses the staging buffers

  // XCD-aware tile index
  const int per = (g.tiles + 7) / 8;
  const int u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= g.tiles) return;
  const int cb = u % g.ncb;
  const int rb = (u / g.ncb) % g.nrb;
  const int k = u / (g.ncb * g.nrb);

  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const float sc = g.scale ? g.scale[k] : 1.0f;
  const int64_t row0 = (int64_t)rb * BM;
  const float* Xk = g.X + (int64_t)k * g.I * g.J;
  const T* Vc = (const T*)g.Vpack + (int64_t)cb * g.nchunk * B_EL;

  // global -> register staging: thread loads 16 consecutive floats of one row
  const int lr = tid / 2, lh = tid % 2;
  const int64_t gi = row0 + lr;
  const bool row_ok = gi < g.I;
  const float* xrow = Xk + gi * g.J;
  float xr[16];
  constexpr int VB = B_EL * (int)sizeof(T) / NT / 16;   // 16-byte words per thread for B
  u32x4 vr[VB];

#define OCTEN_LOAD_CHUNK(c)                                                          \
  do {                                                                               \
    const int64_t j0 = (int64_t)(c) * KC + lh * 16;                                  \
    if (VEC) {                                                                       \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                \
        f32x4 v = {0.f, 0.f, 0.f, 0.f};                                              \
        if (row_ok && j0 + 4 * q < g.J) v = *(const f32x4*)(xrow + j0 + 4 * q);      \
        xr[4 * q] = v[0]; xr[4 * q + 1] = v[1]; xr[4 * q + 2] = v[2]; xr[4 * q + 3] = v[3]; \
      }                                                                              \
    } else if (row_ok && j0 + 16 <= g.J) {                                           \
      /* the 16 floats lie inside the row: four 16-byte loads from a 4-byte */       \
      /* aligned address (the unaligned access mode of the target) */                \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                \
        f32x4 v;                                                                     \
        __builtin_memcpy(&v, xrow + j0 + 4 * q, sizeof(v));                          \
        xr[4 * q] = v[0]; xr[4 * q + 1] = v[1]; xr[4 * q + 2] = v[2]; xr[4 * q + 3] = v[3]; \
      }                                                                              \
    } else {                                                                         \
      _Pragma("unroll") for (int q = 0; q < 16; ++q)                                 \
        xr[q] = (row_ok && j0 + q < g.J) ? xrow[j0 + q] : 0.f;                       \
    }                                                                                \
    const u32x4* vsrc = (const u32x4*)(Vc + (int64_t)(c) * B_EL);                    \
    _Pragma("unroll") for (int q = 0; q < VB; ++q) vr[q] = vsrc[q * NT + tid];       \
  } while (0)

#define OCTEN_STORE_CHUNK(buf)                                                       \
  do {                                                                               \
    T* a_ = As + (buf) * NPART * A_EL;                                               \
    if constexpr (KIND == 2) {                                                       \
      bf16x8 h0, h1, l0, l1;                                                         \
      _Pragma("unroll") for (int q = 0; q < 8; ++q) {                                \
        const float x0 = xr[q] * sc, x1 = xr[8 + q] * sc;                            \
        h0[q] = (__bf16)x0;                                                          \
        h1[q] = (__bf16)x1;                                                          \
        if constexpr (SPLIT > 0) {                                                   \
          l0[q] = (__bf16)(x0 - (float)h0[q]);                                       \
          l1[q] = (__bf16)(x1 - (float)h1[q]);                                       \
        }                                                                            \
      }                                                                              \
      *(bf16x8*)(a_ + a_pos<KIND>(lr, lh * 16)) = h0;                                \
      *(bf16x8*)(a_ + a_pos<KIND>(lr, lh * 16 + 8)) = h1;                            \
      if constexpr (SPLIT > 0) {                                                     \
        *(bf16x8*)(a_ + A_EL + a_pos<KIND>(lr, lh * 16)) = l0;                       \
        *(bf16x8*)(a_ + A_EL + a_pos<KIND>(lr, lh * 16 + 8)) = l1;                   \
      }                                                                              \
    } else {                                                                         \
      _Pragma("unroll") for (int q = 0; q < 16; ++q)                                 \
        a_[a_pos<KIND>(lr, lh * 16 + q)] = cvt<KIND>(xr[q] * sc);                    \
    }                                                                                \
    u32x4* b_ = (u32x4*)(Bs + (buf) * B_EL);                                         \
    _Pragma("unroll") for (int q = 0; q < VB; ++q) b_[q * NT + tid] = vr[q];         \
  } while (0)

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  OCTEN_LOAD_CHUNK(0);
  OCTEN_STORE_CHUNK(0);
  __syncthreads();
  for (int c = 0; c < g.nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < g.nchunk) OCTEN_LOAD_CHUNK(c + 1);
    const T* a = As + buf * NPART * A_EL;
    const T* b = Bs + buf * B_EL;
#pragma unroll
    for (int ks = 0; ks < KC / KS; ++ks) {
      Frag af[2], al[2], bfr[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = Kind<KIND>::ld(a + ((ks * (BM / 32) + wm * 2 + i) * 64 + lane) * E);
        if constexpr (SPLIT > 0)
          al[i] = Kind<KIND>::ld(a + A_EL + ((ks * (BM / 32) + wm * 2 + i) * 64 + lane) * E);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bfr[j] = Kind<KIND>::ld(b + ((ks * (BN / 32) + wn * 4 + j) * 64 + lane) * E);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = Kind<KIND>::mma(af[i], bfr[j], acc[i][j]);
          if constexpr (SPLIT > 0) acc[i][j] = Kind<KIND>::mma(al[i], bfr[j], acc[i][j]);
        }
    }
    if (c + 1 < g.nchunk) OCTEN_STORE_CHUNK(buf ^ 1);
    __syncthreads();
  }

#undef OCTEN_LOAD_CHUNK
#undef OCTEN_STORE_CHUNK

  if constexpr (SPLIT > 0) {
    stage2_split<QT, SPLIT>(g, acc, (__bf16*)smem, k, rb, cb, sc);
    return;
  }
  // ---- stage 2: T^T into LDS (in the MFMA input type), zero row at BN
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn * 128 + j * 32 + lane % 32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 32 + 8 * q + 4 * (lane / 32);
        T* dst = T2t + col * T2LD + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = cvt<KIND>(acc[i][j][4 * q + e]);
      }
    }
  for (int e = tid; e < T2LD; e += NT) T2t[BN * T2LD + e] = cvt<KIND>(0.f);
  __syncthreads();

  const int p0 = cb * g.G;
  const int gcount = (g.P - p0) < g.G ? (g.P - p0) : g.G;
  const float inv = 1.0f / sc;
  // each replica's Q x Q output is split between two wavefronts by tile rows
  constexpr int QH = (QT + 1) / 2;
  for (int item = wave; item < 2 * gcount; item += NT / 64) {
    const int gg = item >> 1, ih = item & 1;
    const int p = p0 + gg;
    f32x16 m[QH][QT];
#pragma unroll
    for (int i = 0; i < QH; ++i)
#pragma unroll
      for (int j = 0; j < QT; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) m[i][j][e] = 0.f;
    const T* Up = (const T*)g.Upack + ((int64_t)rb * g.P + p) * (BM / KS) * QT * 64 * E;
    const int* tc = g.tilecol + ((int64_t)cb * g.G + gg) * QT * 32;
    int colrow[QT];
#pragma unroll
    for (int j = 0; j < QT; ++j) colrow[j] = tc[j * 32 + lane % 32];
    for (int ks = 0; ks < BM / KS; ++ks) {
      Frag af[QH];
#pragma unroll
      for (int ii = 0; ii < QH; ++ii) {
        const int i = ih * QH + ii < QT ? ih * QH + ii : QT - 1;
        af[ii] = Kind<KIND>::ld(Up + ((int64_t)(ks * QT + i) * 64 + lane) * E);
      }
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const Frag bf = Kind<KIND>::ld(T2t + colrow[j] * T2LD + ks * KS + (lane / 32) * E);
#pragma unroll
        for (int ii = 0; ii < QH; ++ii) m[ii][j] = Kind<KIND>::mma(af[ii], bf, m[ii][j]);
      }
    }
    float* out = g.Mpart + (((int64_t)k * g.nrb + rb) * g.P + p) * g.Q * g.Q;
#pragma unroll
    for (int ii = 0; ii < QH; ++ii) {
      const int i = ih * QH + ii;
      if (i >= QT) continue;
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const int bcol = j * 32 + lane % 32;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int arow = i * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
          if (arow < g.Q && bcol < g.Q) out[arow * g.Q + bcol] = m[ii][j][e] * inv;
        }
      }
    }
  }
}

// s_waitcnt immediate that waits until at most n vector-memory operations of
// this wave are outstanding (lgkm and exp counters left unconstrained).
__host__ __device__ constexpr unsigned vmcnt_imm(unsigned n) {
  return (n & 0xFu) | ((n >> 4) << 14) | (0x7u << 4) | (0xFu << 8);
}

typedef __attribute__((address_space(3))) void* lds_vptr;
typedef __attribute__((address_space(1))) void* gbl_vptr;

// Same tile and output as compress_fused, with a deeper pipeline: NSTAGE LDS
// stages filled by direct global->LDS loads (16 bytes per lane) issued
// NSTAGE-1 chunks ahead, so that enough bytes are in flight to cover the
// memory latency.  X is staged as raw f32 rows (16-byte slots XOR-swizzled by
// row to spread LDS banks) and converted to the MFMA input type when the A
// fragments are formed; V is staged as its fragment image.  Rows past I and
// columns past J read clamped in-bounds addresses; they meet zero rows of the
// U image or zero rows of the V image, so they add nothing.  Needs J % 4 == 0
// and 16-byte aligned X.
template <int KIND, int QT, int NSTAGE>
__global__ __launch_bounds__(Tile<KIND>::NT) void compress_pipe(Args g) {
  constexpr int BM = Tile<KIND>::BM, NT = Tile<KIND>::NT;
  using T = typename Kind<KIND>::T;
  using Frag = typename Kind<KIND>::Frag;
  constexpr int KS = Kind<KIND>::KSTEP, E = Kind<KIND>::EPL;
  constexpr int B_EL = chunk_elems<KIND>(BN / 32);
  constexpr int XBYTES = BM * KC * 4;                       // raw f32 X chunk
  constexpr int VBYTES = B_EL * (int)sizeof(T);
  constexpr int STAGE = XBYTES + VBYTES;
  constexpr int XL = XBYTES / (NT * 16);                    // X loads per thread per chunk
  constexpr int VL = VBYTES / (NT * 16);                    // V loads per thread per chunk
  constexpr int LPC = XL + VL;
  constexpr int T2LD = BM + 16 / (int)sizeof(T);
  extern __shared__ __align__(16) unsigned char smem[];
  T* T2t = (T*)smem;

  const int per = (g.tiles + 7) / 8;
  const int u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= g.tiles) return;
  const int cb = u % g.ncb;
  const int rb = (u / g.ncb) % g.nrb;
  const int k = u / (g.ncb * g.nrb);

  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const float sc = g.scale ? g.scale[k] : 1.0f;
  const int64_t row0 = (int64_t)rb * BM;
  const float* Xk = g.X + (int64_t)k * g.I * g.J;
  const unsigned char* Vc = (const unsigned char*)g.Vpack + (int64_t)cb * g.nchunk * VBYTES;

  // per-thread X source rows (clamped) and swizzled segments, fixed per tile
  const float* xsrc[XL];
  int xseg[XL];
#pragma unroll
  for (int q = 0; q < XL; ++q) {
    const int r = (wave * XL + q) * 8 + lane / 8;
    int64_t gr = row0 + r;
    if (gr > g.I - 1) gr = g.I - 1;
    xsrc[q] = Xk + gr * g.J;
    xseg[q] = (lane % 8) ^ (r % 8);
  }

  auto issue = [&](int c, int st) {
    unsigned char* base = smem + st * STAGE;
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      int64_t j = (int64_t)c * KC + xseg[q] * 4;
      if (j > g.J - 4) j = g.J - 4;
      __builtin_amdgcn_global_load_lds((gbl_vptr)(xsrc[q] + j),
                                       (lds_vptr)(base + (wave * XL + q) * 1024), 16, 0, 0);
    }
    const unsigned char* vs = Vc + (int64_t)c * VBYTES;
#pragma unroll
    for (int q = 0; q < VL; ++q)
      __builtin_amdgcn_global_load_lds((gbl_vptr)(vs + (q * NT + tid) * 16),
                                       (lds_vptr)(base + XBYTES + (q * NT + wave * 64) * 16), 16, 0,
                                       0);
  };

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int nchunk = g.nchunk;
#pragma unroll
  for (int c = 0; c < NSTAGE - 1; ++c)
    if (c < nchunk) issue(c, c);
  for (int c = 0; c < nchunk; ++c) {
    const int ahead = (nchunk - 1 - c) < (NSTAGE - 2) ? (nchunk - 1 - c) : (NSTAGE - 2);
    if (ahead >= 2) __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * LPC));
    else if (ahead == 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(LPC));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    // bare barrier: the explicit wait above already covers this chunk's loads;
    // a full __syncthreads would also wait for the prefetches still in flight
    __builtin_amdgcn_s_barrier();
    if (c + NSTAGE - 1 < nchunk) issue(c + NSTAGE - 1, (c + NSTAGE - 1) % NSTAGE);
    const unsigned char* base = smem + (c % NSTAGE) * STAGE;
    const float* xs = (const float*)base;
    const T* b = (const T*)(base + XBYTES);
#pragma unroll
    for (int ks = 0; ks < KC / KS; ++ks) {
      Frag af[2], bfr[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int m = (wm * 2 + i) * 32 + lane % 32;
        const float* xrow = xs + m * KC;
        if constexpr (KIND == 2) {
          const int s0 = ks * 4 + 2 * (lane / 32);
          const f32x4 lo = *(const f32x4*)(xrow + 4 * (s0 ^ (m % 8)));
          const f32x4 hi = *(const f32x4*)(xrow + 4 * ((s0 + 1) ^ (m % 8)));
          bf16x8 f;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            f[e] = (__bf16)(lo[e] * sc);
            f[4 + e] = (__bf16)(hi[e] * sc);
          }
          af[i] = f;
        } else {
          const int kk = ks * 2 + lane / 32;
          af[i] = xrow[4 * ((kk / 4) ^ (m % 8)) + kk % 4] * sc;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bfr[j] = Kind<KIND>::ld(b + ((ks * (BN / 32) + wn * 4 + j) * 64 + lane) * E);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Kind<KIND>::mma(af[i], bfr[j], acc[i][j]);
    }
  }
  __syncthreads();

  // ---- stage 2 (as in compress_fused)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn * 128 + j * 32 + lane % 32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 32 + 8 * q + 4 * (lane / 32);
        T* dst = T2t + col * T2LD + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = cvt<KIND>(acc[i][j][4 * q + e]);
      }
    }
  for (int e = tid; e < T2LD; e += NT) T2t[BN * T2LD + e] = cvt<KIND>(0.f);
  __syncthreads();

  const int p0 = cb * g.G;
  const int gcount = (g.P - p0) < g.G ? (g.P - p0) : g.G;
  const float inv = 1.0f / sc;
  // each replica's Q x Q output is split between two wavefronts by tile rows
  constexpr int QH = (QT + 1) / 2;
  for (int item = wave; item < 2 * gcount; item += NT / 64) {
    const int gg = item >> 1, ih = item & 1;
    const int p = p0 + gg;
    f32x16 m[QH][QT];
#pragma unroll
    for (int i = 0; i < QH; ++i)
#pragma unroll
      for (int j = 0; j < QT; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) m[i][j][e] = 0.f;
    const T* Up = (const T*)g.Upack + ((int64_t)rb * g.P + p) * (BM / KS) * QT * 64 * E;
    const int* tc = g.tilecol + ((int64_t)cb * g.G + gg) * QT * 32;
    int colrow[QT];
#pragma unroll
    for (int j = 0; j < QT; ++j) colrow[j] = tc[j * 32 + lane % 32];
    for (int ks = 0; ks < BM / KS; ++ks) {
      Frag af[QH];
#pragma unroll
      for (int ii = 0; ii < QH; ++ii) {
        const int i = ih * QH + ii < QT ? ih * QH + ii : QT - 1;
        af[ii] = Kind<KIND>::ld(Up + ((int64_t)(ks * QT + i) * 64 + lane) * E);
      }
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const Frag bf = Kind<KIND>::ld(T2t + colrow[j] * T2LD + ks * KS + (lane / 32) * E);
#pragma unroll
        for (int ii = 0; ii < QH; ++ii) m[ii][j] = Kind<KIND>::mma(af[ii], bf, m[ii][j]);
      }
    }
    float* out = g.Mpart + (((int64_t)k * g.nrb + rb) * g.P + p) * g.Q * g.Q;
#pragma unroll
    for (int ii = 0; ii < QH; ++ii) {
      const int i = ih * QH + ii;
      if (i >= QT) continue;
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const int bcol = j * 32 + lane % 32;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int arow = i * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
          if (arow < g.Q && bcol < g.Q) out[arow * g.Q + bcol] = m[ii][j][e] * inv;
        }
      }
    }
  }
}

// BF16 only: the tile and output of compress_pipe with half-size chunks (16
// columns of X, one MFMA k step) in NS2 = 6 LDS stages, and the fragments of
// chunk c + 1 read into registers while the MFMAs of chunk c run.  With one
// barrier per chunk and the reads issued right after it, the wavefronts of a
// workgroup otherwise move between all-LDS and all-MFMA phases in lockstep;
// here each wavefront overlaps its own LDS reads with its matrix work.  Global
// loads are issued NS2 - 2 chunks ahead of their first use.  X rows are 64
// bytes per stage, their four 16-byte slots XOR-swizzled by ((m >> 1) ^
// (m >> 2)) & 3, which keeps the A-fragment reads free of bank conflicts for
// both 8 and 16 lanes per LDS cycle.  The V image is the one of the other
// kernels: a 32-column chunk holds two k steps, i.e. two half chunks.
constexpr int NS2 = 6;
constexpr int KC2 = 16;

__device__ __forceinline__ int swz4(int m) { return ((m >> 1) ^ (m >> 2)) & 3; }

//
// SPLIT > 0 selects the two-term form: every X value x (after the scale) is
// the pair hi = bf16(x), lo = bf16(x - hi), both multiplied by the same V
// fragment into the same float32 accumulators, so stage 1 sees x to 16
// significant bits.  Stage 2 then takes T as the pair T_hi, T_lo in two
// passes through the same LDS buffer, accumulating into the same output
// tiles.  The V and U images must hold the compression matrices exactly
// (they are on the bfloat16 grid; checked when the plan is made).  In this
// form a work item is one 32-row tile of one replica's output, and SPLIT is
// the number of items per wavefront (their accumulators stay live across
// both passes).
template <int QT, bool SCALED, int SPLIT>
__global__ __launch_bounds__(Tile<2>::NT) void compress_pipe2(Args g) {
  constexpr int BM = Tile<2>::BM, NT = Tile<2>::NT;
  using T = __bf16;
  using Frag = bf16x8;
  constexpr int E = 8;
  constexpr int XBYTES = BM * KC2 * 4;                 // 16 KB of raw f32 X
  constexpr int VBYTES = (BN / 32) * 64 * E * 2;       // 8 KB: one k step of the V image
  constexpr int STAGE = XBYTES + VBYTES;
  constexpr int XL = XBYTES / (NT * 16);               // X loads per thread per chunk
  constexpr int VL = VBYTES / (NT * 16);               // V loads per thread per chunk
  constexpr int LPC = XL + VL;
  constexpr int T2LD = BM + 16 / (int)sizeof(T);
  static_assert(XL * NT * 16 == XBYTES && VL * NT * 16 == VBYTES, "whole 16-byte loads");
  extern __shared__ __align__(16) unsigned char smem[];
  T* T2t = (T*)smem;

  const int per = (g.tiles + 7) / 8;
  const int u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= g.tiles) return;
  const int cb = u % g.ncb;
  const int rb = (u / g.ncb) % g.nrb;
  const int k = u / (g.ncb * g.nrb);

  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const float sc = SCALED ? g.scale[k] : 1.0f;
  const int64_t row0 = (int64_t)rb * BM;
  const float* Xk = g.X + (int64_t)k * g.I * g.J;
  const unsigned char* Vc = (const unsigned char*)g.Vpack + (int64_t)cb * g.nchunk * 2 * VBYTES;
  const int n2 = 2 * g.nchunk;

  // per-thread X source rows (clamped) and swizzled 16-byte segments
  const float* xsrc[XL];
  int xseg[XL];
#pragma unroll
  for (int q = 0; q < XL; ++q) {
    const int r = (wave * XL + q) * 16 + lane / 4;
    int64_t gr = row0 + r;
    if (gr > g.I - 1) gr = g.I - 1;
    xsrc[q] = Xk + gr * g.J;
    xseg[q] = (lane % 4) ^ swz4(r);
  }

  auto issue = [&](int c) {
    unsigned char* base = smem + (c % NS2) * STAGE;
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      int64_t j = (int64_t)c * KC2 + xseg[q] * 4;
      if (j > g.J - 4) j = g.J - 4;
      __builtin_amdgcn_global_load_lds((gbl_vptr)(xsrc[q] + j),
                                       (lds_vptr)(base + (wave * XL + q) * 1024), 16, 0, 0);
    }
    const unsigned char* vs = Vc + (int64_t)c * VBYTES;
#pragma unroll
    for (int q = 0; q < VL; ++q)
      __builtin_amdgcn_global_load_lds((gbl_vptr)(vs + (q * NT + tid) * 16),
                                       (lds_vptr)(base + XBYTES + (q * NT + wave * 64) * 16), 16, 0,
                                       0);
  };
  // waits until at most `ahead` chunks of this thread's loads are outstanding
  auto wait_ahead = [&](int ahead) {
    if (ahead >= 3) __builtin_amdgcn_s_waitcnt(vmcnt_imm(3 * LPC));
    else if (ahead == 2) __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * LPC));
    else if (ahead == 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(LPC));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
  };

  struct Frags {
    f32x4 a[2][2];
    Frag b[4];
  };
  auto read_frags = [&](int c, Frags& f) {
    const unsigned char* base = smem + (c % NS2) * STAGE;
    const float* xs = (const float*)base;
    const T* bimg = (const T*)(base + XBYTES);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = (wm * 2 + i) * 32 + lane % 32;
      const float* xrow = xs + m * KC2;
      const int s0 = 2 * (lane / 32);
      f.a[i][0] = *(const f32x4*)(xrow + 4 * (s0 ^ swz4(m)));
      f.a[i][1] = *(const f32x4*)(xrow + 4 * ((s0 + 1) ^ swz4(m)));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) f.b[j] = *(const Frag*)(bimg + ((wn * 4 + j) * 64 + lane) * E);
  };

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  auto mfmas = [&](const Frags& f) {
    Frag af[2], al[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      bf16x8 v, w;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = e < 4 ? f.a[i][0][e] : f.a[i][1][e - 4];
        const float xs = SCALED ? x * sc : x;
        v[e] = (__bf16)xs;
        if constexpr (SPLIT > 0) w[e] = (__bf16)(xs - (float)v[e]);
      }
      af[i] = v;
      if constexpr (SPLIT > 0) al[i] = w;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], f.b[j], acc[i][j], 0, 0, 0);
        if constexpr (SPLIT > 0)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], f.b[j], acc[i][j], 0, 0, 0);
      }
  };

  // prologue: chunks 0 .. NS2 - 1 in flight; chunks 0 and 1 landed
  const int pro = n2 < NS2 ? n2 : NS2;
  for (int c = 0; c < pro; ++c) issue(c);
  wait_ahead(pro - 2 > 0 ? (pro - 2 > 3 ? 3 : pro - 2) : 0);
  if (pro - 2 > 3) __builtin_amdgcn_s_waitcnt(vmcnt_imm(4 * LPC));
  __builtin_amdgcn_s_barrier();

  // one chunk: read the next chunk's fragments, run this chunk's MFMAs, wait
  // for chunk c + 2, barrier, refill the stage of chunk c with chunk c + NS2
  auto step = [&](int c, Frags& cur, Frags& nxt) {
    if (c + 1 < n2) read_frags(c + 1, nxt);
    mfmas(cur);
    const int last = (c + NS2 - 1 < n2 - 1 ? c + NS2 - 1 : n2 - 1);   // last chunk issued
    const int ahead = last - (c + 2);
    wait_ahead(ahead < 0 ? 0 : (ahead > 3 ? 3 : ahead));
    __builtin_amdgcn_s_barrier();
    if (c + NS2 < n2) issue(c + NS2);
  };
  Frags f0, f1;
  read_frags(0, f0);
  int c = 0;
  for (; c + 1 < n2; c += 2) {
    step(c, f0, f1);
    step(c + 1, f1, f0);
  }
  if (c < n2) step(c, f0, f1);
  __syncthreads();

  if constexpr (SPLIT > 0) {
    stage2_split<QT, SPLIT>(g, acc, T2t, k, rb, cb, sc);
  } else {
  // ---- stage 2 (as in compress_pipe)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn * 128 + j * 32 + lane % 32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 32 + 8 * q + 4 * (lane / 32);
        T* dst = T2t + col * T2LD + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = (T)acc[i][j][4 * q + e];
      }
    }
  for (int e = tid; e < T2LD; e += NT) T2t[BN * T2LD + e] = (T)0.f;
  __syncthreads();

  const int p0 = cb * g.G;
  const int gcount = (g.P - p0) < g.G ? (g.P - p0) : g.G;
  const float inv = 1.0f / sc;
  constexpr int KS = 16;
  constexpr int QH = (QT + 1) / 2;
  for (int item = wave; item < 2 * gcount; item += NT / 64) {
    const int gg = item >> 1, ih = item & 1;
    const int p = p0 + gg;
    f32x16 m[QH][QT];
#pragma unroll
    for (int i = 0; i < QH; ++i)
#pragma unroll
      for (int j = 0; j < QT; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) m[i][j][e] = 0.f;
    const T* Up = (const T*)g.Upack + ((int64_t)rb * g.P + p) * (BM / KS) * QT * 64 * E;
    const int* tc = g.tilecol + ((int64_t)cb * g.G + gg) * QT * 32;
    int colrow[QT];
#pragma unroll
    for (int j = 0; j < QT; ++j) colrow[j] = tc[j * 32 + lane % 32];
    for (int ks = 0; ks < BM / KS; ++ks) {
      Frag af[QH];
#pragma unroll
      for (int ii = 0; ii < QH; ++ii) {
        const int i = ih * QH + ii < QT ? ih * QH + ii : QT - 1;
        af[ii] = *(const Frag*)(Up + ((int64_t)(ks * QT + i) * 64 + lane) * E);
      }
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const Frag bf = *(const Frag*)(T2t + colrow[j] * T2LD + ks * KS + (lane / 32) * E);
#pragma unroll
        for (int ii = 0; ii < QH; ++ii)
          m[ii][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ii], bf, m[ii][j], 0, 0, 0);
      }
    }
    float* out = g.Mpart + (((int64_t)k * g.nrb + rb) * g.P + p) * g.Q * g.Q;
#pragma unroll
    for (int ii = 0; ii < QH; ++ii) {
      const int i = ih * QH + ii;
      if (i >= QT) continue;
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const int bcol = j * 32 + lane % 32;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int arow = i * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
          if (arow < g.Q && bcol < g.Q) out[arow * g.Q + bcol] = m[ii][j][e] * inv;
        }
      }
    }
  }
  }
}

// V image: [cb][chunk][ks][nt][lane][E]; element V[j][col] with
// j = c*KC + ks*KS + (lane/32)*E + e (KS = 16) or c*KC + ks*2 + lane/32 (KS = 2).
template <int KIND>
__global__ void pack_v(const double* __restrict__ V, int64_t J, int M1, const int* __restrict__ colmap,
                       int ncb, int nchunk, typename Kind<KIND>::T* __restrict__ out) {
  constexpr int KS = Kind<KIND>::KSTEP, E = Kind<KIND>::EPL;
  const int64_t per_chunk = chunk_elems<KIND>(BN / 32);
  const int64_t tot = (int64_t)ncb * nchunk * per_chunk;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = x;
    const int e = (int)(r % E); r /= E;
    const int lane = (int)(r % 64); r /= 64;
    const int nt = (int)(r % (BN / 32)); r /= (BN / 32);
    const int ks = (int)(r % (KC / KS)); r /= (KC / KS);
    const int c = (int)(r % nchunk); r /= nchunk;
    const int cb = (int)r;
    const int64_t j = (int64_t)c * KC + ks * KS + (lane / 32) * E + e;
    const int col = colmap[cb * BN + nt * 32 + lane % 32];
    float v = (j < J && col >= 0) ? (float)V[j * M1 + col] : 0.f;
    out[x] = (typename Kind<KIND>::T)v;
  }
}

// U image: [rb][p][ks][mt][lane][E]; element U[i][col_p(a)] with
// i = rb*BM + ks*KS + (lane/32)*E + e, a = mt*32 + lane%32.
template <int KIND>
__global__ void pack_u(const double* __restrict__ U, int64_t I, int M1, int P, int Q, int S,
                       int QT, int nrb, typename Kind<KIND>::T* __restrict__ out) {
  constexpr int KS = Kind<KIND>::KSTEP, E = Kind<KIND>::EPL;
  constexpr int BM = Tile<KIND>::BM;
  const int64_t tot = (int64_t)nrb * P * (BM / KS) * QT * 64 * E;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = x;
    const int e = (int)(r % E); r /= E;
    const int lane = (int)(r % 64); r /= 64;
    const int mt = (int)(r % QT); r /= QT;
    const int ks = (int)(r % (BM / KS)); r /= (BM / KS);
    const int p = (int)(r % P); r /= P;
    const int rb = (int)r;
    const int64_t i = (int64_t)rb * BM + ks * KS + (lane / 32) * E + e;
    const int a = mt * 32 + lane % 32;
    float v = 0.f;
    if (i < I && a < Q) {
      const int col = a < S ? a : S + p * (Q - S) + (a - S);
      v = (float)U[i * M1 + col];
    }
    out[x] = (typename Kind<KIND>::T)v;
  }
}

inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

template <int KIND, int QT, bool VEC, int SPLIT = 0>
hipError_t launch_fused(hipStream_t s, const Args& a, size_t lds) {
  auto fn = compress_fused<KIND, QT, VEC, SPLIT>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int per = (a.tiles + 7) / 8;
  hipLaunchKernelGGL(fn, dim3(8 * per), dim3(Tile<KIND>::NT), lds, s, a);
  return hipGetLastError();
}

template <int KIND, int QT>
hipError_t launch_pipe(hipStream_t s, const Args& a) {
  constexpr int NS = 3;
  constexpr int BM = Tile<KIND>::BM;
  constexpr size_t stage = (size_t)BM * KC * 4 + (size_t)chunk_elems<KIND>(BN / 32) *
                                                     sizeof(typename Kind<KIND>::T);
  const size_t t2 = (size_t)(BN + 1) * (BM + 16 / sizeof(typename Kind<KIND>::T)) *
                    sizeof(typename Kind<KIND>::T);
  const size_t lds = NS * stage > t2 ? NS * stage : t2;
  auto fn = compress_pipe<KIND, QT, NS>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int per = (a.tiles + 7) / 8;
  hipLaunchKernelGGL(fn, dim3(8 * per), dim3(Tile<KIND>::NT), lds, s, a);
  return hipGetLastError();
}

template <int QT, bool SCALED, int SPLIT>
hipError_t launch_pipe2(hipStream_t s, const Args& a) {
  constexpr int BM = Tile<2>::BM;
  constexpr size_t stage = (size_t)BM * KC2 * 4 + (size_t)(BN / 32) * 64 * 8 * 2;
  const size_t t2 = (size_t)(BN + 1) * (BM + 8) * 2;
  const size_t lds = NS2 * stage > t2 ? NS2 * stage : t2;
  auto fn = compress_pipe2<QT, SCALED, SPLIT>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int per = (a.tiles + 7) / 8;
  hipLaunchKernelGGL(fn, dim3(8 * per), dim3(Tile<2>::NT), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_pipe2_q(hipStream_t s, const Args& a, int QT) {
  switch (QT) {
    case 1: return a.scale ? launch_pipe2<1, true, 0>(s, a) : launch_pipe2<1, false, 0>(s, a);
    case 2: return a.scale ? launch_pipe2<2, true, 0>(s, a) : launch_pipe2<2, false, 0>(s, a);
    case 3: return a.scale ? launch_pipe2<3, true, 0>(s, a) : launch_pipe2<3, false, 0>(s, a);
    case 4: return a.scale ? launch_pipe2<4, true, 0>(s, a) : launch_pipe2<4, false, 0>(s, a);
  }
  return hipErrorInvalidValue;
}

template <int QT, int SPLIT>
hipError_t launch_split(hipStream_t s, const Args& a, bool vec, size_t lds) {
  if (!vec) return launch_fused<2, QT, false, SPLIT>(s, a, lds);
  return a.scale ? launch_pipe2<QT, true, SPLIT>(s, a) : launch_pipe2<QT, false, SPLIT>(s, a);
}

// Two-term form: ceil(G * QT / 8) work items per wavefront, each holding QT
// accumulator tiles; plans keep items * QT <= 4.
int split_items(int G, int QT) { return (G * QT + 7) / 8; }

hipError_t launch_split_q(hipStream_t s, const Args& a, int QT, bool vec, size_t lds) {
  const int items = split_items(a.G, QT);
  if (items * QT > 4) return hipErrorInvalidValue;
  switch (QT) {
    case 1:
      if (items <= 1) return launch_split<1, 1>(s, a, vec, lds);
      if (items <= 2) return launch_split<1, 2>(s, a, vec, lds);
      return launch_split<1, 4>(s, a, vec, lds);
    case 2:
      if (items <= 1) return launch_split<2, 1>(s, a, vec, lds);
      return launch_split<2, 2>(s, a, vec, lds);
    case 3: return launch_split<3, 1>(s, a, vec, lds);
    case 4: return launch_split<4, 1>(s, a, vec, lds);
  }
  return hipErrorInvalidValue;
}

template <int KIND>
hipError_t launch_pipe_q(hipStream_t s, const Args& a, int QT) {
  switch (QT) {
    case 1: return launch_pipe<KIND, 1>(s, a);
    case 2: return launch_pipe<KIND, 2>(s, a);
    case 3: return launch_pipe<KIND, 3>(s, a);
    case 4: return launch_pipe<KIND, 4>(s, a);
  }
  return hipErrorInvalidValue;
}

template <int KIND, bool VEC>
hipError_t launch_q(hipStream_t s, const Args& a, int QT, size_t lds) {
  switch (QT) {
    case 1: return launch_fused<KIND, 1, VEC>(s, a, lds);
    case 2: return launch_fused<KIND, 2, VEC>(s, a, lds);
    case 3: return launch_fused<KIND, 3, VEC>(s, a, lds);
    case 4: return launch_fused<KIND, 4, VEC>(s, a, lds);
  }
  return hipErrorInvalidValue;
}

}  // namespace

struct MfmaPlan {
  CompressShape sh;
  int kind = 0;   // 1 f32, 2 bf16, 3 two-term bf16
  int variant = 0;  // 0 pipelined, 1 register-staged 16-byte loads, 2 scalar loads,
                    // 3 half chunks with register double buffering (bf16 only)
  int G = 0, ncb = 0, nrb = 0, nchunk = 0, QT = 0;
  void* Vpack = nullptr;
  void* Upack = nullptr;
  int* tilecol = nullptr;
  int* colmap = nullptr;
  size_t lds = 0;
};

int mfma_plan_max_G(const CompressShape& sh, int kind) {
  int G = (BN - sh.S) / (sh.Q - sh.S);
  if (kind == 3) {
    // the two-term stage 2 keeps its work items' accumulators live across
    // both passes: items per wavefront * QT <= 4
    const int QT = (sh.Q + 31) / 32;
    const int gmax = QT == 1 ? 32 : (QT == 2 ? 8 : 2);
    if (G > gmax) G = gmax;
  }
  return G > sh.P ? sh.P : G;
}

// Counts entries of A (n doubles) that are not bfloat16 values.
__global__ void off_bf16_grid_kernel(const double* __restrict__ A, int64_t n, int* __restrict__ count) {
  int c = 0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const double v = A[x];
    const __bf16 b = (__bf16)(float)v;
    c += ((double)(float)b != v) ? 1 : 0;
  }
  if (c) atomicAdd(count, c);
}

int mfma_plan_G(const MfmaPlan* p) { return p->G; }
void mfma_plan_set_variant(MfmaPlan* p, int variant) { p->variant = variant; }
int mfma_plan_variant(const MfmaPlan* p) { return p->variant; }

hipError_t mfma_plan_create(const CompressShape& sh, int in_kind, const double* U, const double* V,
                            hipStream_t s, MfmaPlan** out, int G_request) {
  *out = nullptr;
  if (in_kind != 1 && in_kind != 2 && in_kind != 3) return hipErrorInvalidValue;
  const int P = sh.P, Q = sh.Q, S = sh.S, M1 = sh.M1;
  if (Q > 128 || S + (Q - S) > BN) return hipErrorNotSupported;
  if (in_kind == 3) {
    // the two-term form multiplies the images of U and V as they are: they
    // must hold the compression matrices exactly
    int* cnt = nullptr;
    hipError_t e = hipMalloc(&cnt, sizeof(int));
    if (e != hipSuccess) return e;
    int h = 0;
    e = hipMemsetAsync(cnt, 0, sizeof(int), s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(off_bf16_grid_kernel, dim3(grid_for(sh.I * M1)), dim3(256), 0, s, U,
                         sh.I * (int64_t)M1, cnt);
      hipLaunchKernelGGL(off_bf16_grid_kernel, dim3(grid_for(sh.J * M1)), dim3(256), 0, s, V,
                         sh.J * (int64_t)M1, cnt);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, cnt, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(cnt);
    if (e != hipSuccess) return e;
    if (h != 0) return hipErrorInvalidValue;
  }
  MfmaPlan* p = new MfmaPlan();
  p->sh = sh;
  p->kind = in_kind;
  int G = mfma_plan_max_G(sh, in_kind);
  if (G_request > 0 && G_request < G) G = G_request;
  if (G < 1) { delete p; return hipErrorNotSupported; }
  p->G = G;
  p->ncb = (P + G - 1) / G;
  const int BM = in_kind != 1 ? Tile<2>::BM : Tile<1>::BM;
  p->nrb = (int)((sh.I + BM - 1) / BM);
  p->nchunk = (int)((sh.J + KC - 1) / KC);
  p->QT = (Q + 31) / 32;
  std::vector<int> colmap((size_t)p->ncb * BN, -1);
  std::vector<int> tilecol((size_t)p->ncb * G * p->QT * 32, BN);
  for (int cb = 0; cb < p->ncb; ++cb) {
    for (int c = 0; c < S; ++c) colmap[(size_t)cb * BN + c] = c;
    for (int gg = 0; gg < G; ++gg) {
      const int pr = cb * G + gg;
      if (pr >= P) break;
      for (int c = 0; c < Q - S; ++c)
        colmap[(size_t)cb * BN + S + gg * (Q - S) + c] = S + pr * (Q - S) + c;
      for (int b = 0; b < Q; ++b)
        tilecol[((size_t)cb * G + gg) * p->QT * 32 + b] = b < S ? b : S + gg * (Q - S) + (b - S);
    }
  }
  const size_t esz = in_kind == 1 ? 4 : 2;
  const int64_t vcount = (int64_t)p->ncb * p->nchunk *
                         (in_kind == 1 ? chunk_elems<1>(BN / 32) : chunk_elems<2>(BN / 32));
  const int KS = in_kind == 1 ? 2 : 16, E = in_kind == 1 ? 1 : 8;
  const int64_t ucount = (int64_t)p->nrb * P * (BM / KS) * p->QT * 64 * E;
  hipError_t e;
  if ((e = hipMalloc(&p->Vpack, vcount * esz)) != hipSuccess ||
      (e = hipMalloc(&p->Upack, ucount * esz)) != hipSuccess ||
      (e = hipMalloc(&p->colmap, colmap.size() * sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&p->tilecol, tilecol.size() * sizeof(int))) != hipSuccess) {
    mfma_plan_destroy(p);
    return e;
  }
  hipMemcpy(p->colmap, colmap.data(), colmap.size() * sizeof(int), hipMemcpyHostToDevice);
  hipMemcpy(p->tilecol, tilecol.data(), tilecol.size() * sizeof(int), hipMemcpyHostToDevice);
  if (in_kind == 1) {
    hipLaunchKernelGGL(pack_v<1>, dim3(grid_for(vcount)), dim3(256), 0, s, V, sh.J, M1, p->colmap,
                       p->ncb, p->nchunk, (float*)p->Vpack);
    hipLaunchKernelGGL(pack_u<1>, dim3(grid_for(ucount)), dim3(256), 0, s, U, sh.I, M1, P, Q, S,
                       p->QT, p->nrb, (float*)p->Upack);
  } else {
    hipLaunchKernelGGL(pack_v<2>, dim3(grid_for(vcount)), dim3(256), 0, s, V, sh.J, M1, p->colmap,
                       p->ncb, p->nchunk, (__bf16*)p->Vpack);
    hipLaunchKernelGGL(pack_u<2>, dim3(grid_for(ucount)), dim3(256), 0, s, U, sh.I, M1, P, Q, S,
                       p->QT, p->nrb, (__bf16*)p->Upack);
  }
  if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
    mfma_plan_destroy(p);
    return e;
  }
  const int T2LD = BM + (in_kind == 1 ? 4 : 8);
  const int npart = in_kind == 3 ? 2 : 1;   // hi and lo X images of the two-term form
  const size_t stage = 2 * (size_t)(npart * (in_kind == 1 ? chunk_elems<1>(BM / 32) : chunk_elems<2>(BM / 32)) +
                                    (in_kind == 1 ? chunk_elems<1>(BN / 32) : chunk_elems<2>(BN / 32))) * esz;
  const size_t t2 = (size_t)(BN + 1) * T2LD * esz;
  p->lds = stage > t2 ? stage : t2;
  *out = p;
  return hipSuccess;
}

void mfma_plan_destroy(MfmaPlan* p) {
  if (!p) return;
  if (p->Vpack) hipFree(p->Vpack);
  if (p->Upack) hipFree(p->Upack);
  if (p->colmap) hipFree(p->colmap);
  if (p->tilecol) hipFree(p->tilecol);
  delete p;
}

size_t mfma_workspace_bytes(const MfmaPlan* p, int64_t t) {
  return (size_t)t * p->nrb * p->sh.P * p->sh.Q * p->sh.Q * sizeof(float);
}

hipError_t compress_mfma_main(hipStream_t s, const MfmaPlan* p, const float* X, int64_t t,
                              const float* slice_scale, void* work) {
  Args a;
  a.X = X;
  a.scale = slice_scale;
  a.Vpack = p->Vpack;
  a.Upack = p->Upack;
  a.tilecol = p->tilecol;
  a.Mpart = (float*)work;
  a.I = p->sh.I;
  a.J = p->sh.J;
  a.t = (int)t;
  a.P = p->sh.P;
  a.Q = p->sh.Q;
  a.G = p->G;
  a.ncb = p->ncb;
  a.nrb = p->nrb;
  a.nchunk = p->nchunk;
  const int64_t tiles = t * p->nrb * p->ncb;
  if (tiles > (int64_t)1 << 30) return hipErrorInvalidValue;
  a.tiles = (int)tiles;
  const bool vec = (p->sh.J % 4 == 0) && (((uintptr_t)X & 15) == 0);
  hipError_t e;
  // the 16-byte load paths need J % 4 == 0 and an aligned X
  const int v = vec ? p->variant : 2;
  if (p->kind == 3)
    e = launch_split_q(s, a, p->QT, vec, p->lds);
  else if (v == 3 && p->kind == 2)
    e = launch_pipe2_q(s, a, p->QT);
  else if (v == 0 || v == 3)
    e = p->kind == 1 ? launch_pipe_q<1>(s, a, p->QT) : launch_pipe_q<2>(s, a, p->QT);
  else if (v == 1)
    e = p->kind == 1 ? launch_q<1, true>(s, a, p->QT, p->lds) : launch_q<2, true>(s, a, p->QT, p->lds);
  else
    e = p->kind == 1 ? launch_q<1, false>(s, a, p->QT, p->lds) : launch_q<2, false>(s, a, p->QT, p->lds);
  return e;
}

hipError_t compress_mfma_mode3(hipStream_t s, const MfmaPlan* p, int64_t t, const double* W,
                               const void* work, float* Z, int* zbad) {
  return compress_mode3_partials(s, p->sh, t, p->nrb, (const float*)work, W, Z, zbad);
}

}  // namespace octen
