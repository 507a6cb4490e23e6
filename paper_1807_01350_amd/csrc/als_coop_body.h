// Device code of the cooperative replica ALS, shared by the launch of one
// handle (als_coop.hip) and the grouped launch of several handles
// (als_coop_group.hip).
//
// Per-replica CP-ALS across many workgroups (Sec. 4.1: each replica summary
// is decomposed on its own; the model and unfoldings are those of Sec. 2).
//
// Each replica is cut along mode 1 into NW slabs of rows a; a workgroup keeps
// its slab of the summary X_p in LDS for the whole sweep loop, plus the small
// factor state, all in FP64.  One sweep:
//   mode 1  T(a,b,:) = sum_c X(a,b,c) C(c,:)                  slab-local, MFMA
//           A(a,:)   = [sum_b T(a,b,:) * B(b,:)] G1^{-1},  G1 = B'B * C'C
//   mode 2  M2(b,:)  = sum_a T(a,b,:) * A(a,:),  and A'A      slab partials
//           -- reduction 1 over the replica's workgroups --
//           normalise A (norms from diag(A'A)); B = M2 G2^{-1}; normalise B
//   mode 3  M3(c,:)  = sum_{a,b} X(a,b,c) A(a,:) * B(b,:)     slab partial, MFMA
//           -- reduction 2 --
//           C = M3 G3^{-1}; normalise; lambda = column norms of C
// B and C (Q x R) are solved redundantly by every workgroup of the replica, so
// only two reductions per sweep cross workgroups.  Reductions add the slab
// partials in slab order: results do not depend on timing.
//
// The R x R normal matrices are inverted by one wavefront (Gauss-Jordan on
// the identity-padded SPD matrix, one column per lane, pivot columns read
// with lane reads) while the others work: in mode 1 beside the slab
// contraction T on v_mfma_f64_16x16x4 (run by the six wavefronts that do not
// share its SIMD: FP64 MFMA there slows the inverse's FP64 arithmetic down),
// in modes 2 and 3 beside the sums of the slab partials.
//
// Workgroups of a replica synchronise through a monotonically increasing
// counter (relaxed bump and polling); every wait is bounded and raises an
// error flag when exceeded, after which all workgroups skip to the end.  The
// launch is cooperative, so all workgroups are resident.  Replica p is placed
// on XCD p % 8 (workgroup x runs on XCD x % 8) so that its counter and
// partial sums stay in one L2; when the XCC ids recorded at launch confirm
// that, the barriers need no cache maintenance beyond device-coherent loads
// of the partials, otherwise they add an agent-scope release and acquire.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "octen_internal.h"

namespace octen {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4a __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8a __attribute__((ext_vector_type(8)));

namespace {

constexpr int NT = 512;            // eight wavefronts: two per SIMD
constexpr int MAXR = 32;
constexpr unsigned SPIN_LIMIT = 1u << 22;

struct CoopArgs {
  const void* Y;          // [P][Q][Q][Q]
  const double* init;     // [P][3][Q][R]
  double* F;              // [P][3][Q][R]
  double* lam;            // [P][R]
  int* iters;             // [P]
  int* flags;             // [P]
  double* slots;          // [2][P][NW][slot_len]
  unsigned* counters;     // [2][P]: barrier counts, then masks of XCDs
  int* err;               // [1]
  int P, Q, R, NW, na_max, npair_pad, per_xcd, slot_len, max_iters;
  int allow_local;        // 0: device-wide cache maintenance at every barrier
  double tol;
};

// D(16 x 16) += A(16 x 4) B(4 x 16); lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element i of lane l holds D[l/16 + 4 i][l%16].
__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Two-term bfloat16 form of the contractions (SPLIT kernels).  An operand
// value v (float) is the pair hi = bf16(v), lo = bf16(v - hi); a product of
// two operands is taken as hi*hi + lo*hi + hi*lo (the lo*lo term, of relative
// size 2^-16, is dropped), every product exact in float32 and summed into
// float32 accumulators.  D(16 x 16) += A(16 x 32) B(32 x 16) on
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8 (l/16) + j] and
// B[8 (l/16) + j][l%16], j = 0..7; element i of lane l holds D[4 (l/16) + i][l%16].
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8a& hi, bf16x8a& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    hi[j] = (__bf16)v[j];
    lo[j] = (__bf16)(v[j] - (float)hi[j]);
  }
}
__device__ __forceinline__ f32x4a mma3(bf16x8a ah, bf16x8a al, bf16x8a bh, bf16x8a bl, f32x4a c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return c;
}

typedef __attribute__((address_space(3))) double lds_f64;
// An LDS pointer argument as a wave-uniform (scalar) LDS address.
__device__ __forceinline__ lds_f64* lds_uniform(const double* p) {
  const unsigned a = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(const lds_f64*)p);
  return (lds_f64*)(uintptr_t)a;
}

// Index of the accelerator complex die (XCD) the calling wavefront runs on.
__device__ __forceinline__ unsigned xcd_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(v));
  return v;
}

// Barrier of the NW workgroups of one replica.  Every wave first waits for
// its own global stores to complete (a plain workgroup barrier does not), then
// one thread bumps the counter and polls it with relaxed loads (no cache
// invalidation per poll).  Completed stores sit in the L2 of the writer's XCD;
// readers take slot data with device-coherent loads (slot_load), which miss
// in the CU's L1, where a copy from two barriers earlier may still live.
//  - across XCDs (local false): one agent-scope release before the bump
//    writes the L2 back and one agent-scope acquire after the poll
//    invalidates the reader's L2;
//  - within one XCD (local true): the L2 is shared by writer and reader and
//    neither is needed.
__device__ bool replica_barrier(unsigned* ctr, unsigned target, int* err, int* s_ok,
                                bool local) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (++spins > SPIN_LIMIT) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Slot entry written by another workgroup of the replica (see above).
__device__ __forceinline__ double slot_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value of x held by lane j (j uniform), through two scalar lane reads.
__device__ __forceinline__ double lane_value(double x, int j) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), j);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), j);
  return __hiloint2double(hi, lo);
}

// Orders the LDS accesses of one wavefront: what a lane wrote before is seen
// by every lane after (LDS operations of a wavefront complete in order; this
// keeps the compiler from moving memory operations across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// 1 / p for p > 0 (normal): the hardware reciprocal estimate refined by two
// Newton steps r <- r + r (1 - p r), each of which squares the relative
// error, to within a few units in the last place (not the correctly rounded
// quotient an IEEE division sequence gives, and about a third of its
// latency).
__device__ __forceinline__ double recip(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  r = fma(r, fma(-p, r, 1.0), r);
  return r;
}

// Inverse of the SPD matrix G (R x R, LDS) by Gauss-Jordan elimination
// without pivoting, run by one wavefront on [G | I] stored by columns: lane
// c keeps column c in registers.  G is padded to RMAX x RMAX with the
// identity (lanes 0..RMAX-1 hold its columns, lanes RMAX..RMAX+R-1 the
// inverse's), so all RMAX steps run as straight-line code; the padding only
// adds exact zeros to the real entries.  At step j every lane needs the pivot
// column, which lives in lane j: its RMAX entries are read with scalar lane
// reads, all before the updates so that the reads are not serialised behind
// them (no LDS traffic, no cross-lane permutes).  Writes Ginv (LDS) and sets
// *bad when a pivot is not positive.
template <int RMAX>
__device__ __forceinline__ void spd_inverse_wave(const double* G_, double* Ginv_, int R_, int* bad) {
  static_assert(2 * RMAX <= 64, "one wavefront holds [G | I]");
  const int lane = threadIdx.x & 63;
  // LDS operands, uniform rank (scalar branches when called out of line)
  const lds_f64* G = lds_uniform(G_);
  lds_f64* Ginv = lds_uniform(Ginv_);
  const int R = __builtin_amdgcn_readfirstlane(R_);
  double a[RMAX];
#pragma unroll
  for (int i = 0; i < RMAX; ++i) {
    double v = 0.0;
    if (lane < RMAX) {
      if (i < R && lane < R) v = G[i * R + lane];
      else if (i == lane) v = 1.0;
    } else if (lane == RMAX + i) {
      v = 1.0;
    }
    a[i] = v;
  }
  int badl = 0;
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    double col[RMAX];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) col[i] = lane_value(a[i], j);
    __builtin_amdgcn_sched_barrier(0);
    double piv = col[j];
    badl |= !(piv > 0.0);
    piv = piv > 0.0 ? piv : 1e-300;
    const double rj = a[j] * recip(piv);
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i != j) a[i] = fma(-col[i], rj, a[i]);
    a[j] = rj;
  }
  if (lane >= RMAX && lane < RMAX + R) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < R) Ginv[i * R + (lane - RMAX)] = a[i];
  }
  if (lane == 0 && badl) *bad = 1;
}

// The inverse as called by the ALS kernel: inline for the smallest ranks; for
// RMAX >= 8 out of line, so that the registers of its straight-line code
// do not add to those of the kernel's MFMA phases (it would spill there).
template <int RMAX>
__device__ __noinline__ void spd_inverse_call(const double* G, double* Ginv, int R, int* bad) {
  spd_inverse_wave<RMAX>(G, Ginv, R, bad);
}
template <int RMAX>
__device__ __forceinline__ void spd_inverse(const double* G, double* Ginv, int R, int* bad) {
  if constexpr (RMAX >= 8) spd_inverse_call<RMAX>(G, Ginv, R, bad);
  else spd_inverse_wave<RMAX>(G, Ginv, R, bad);
}

// Quotient of e by a fixed divisor d through a 64-bit product with
// m = ceil(2^32 / d) (2^32 itself for d = 1): exact for e * d < 2^32 (here
// e < 2^20, d <= 128); the divisors are runtime values, and a general integer
// division is a long instruction sequence on the GPU.
struct FastDiv {
  unsigned long long m;
  int d;
  __device__ explicit FastDiv(int dd) : m(0xFFFFFFFFull / (unsigned)dd + 1ull), d(dd) {}
  __device__ __forceinline__ int div(int e) const {
    return (int)(((unsigned long long)(unsigned)e * m) >> 32);
  }
  __device__ __forceinline__ int mod(int e) const { return e - div(e) * d; }
};

// G = F^T F (F: n x R in LDS, row stride R) by one wavefront on MFMA; R <= 32.
__device__ void gram_wave(const double* Fm, int n, int R, double* G) {
  const int lane = threadIdx.x & 63;
  const int ntile = (R + 15) / 16;
  for (int ti = 0; ti < ntile; ++ti)
    for (int tj = 0; tj < ntile; ++tj) {
      f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
      const int r1 = ti * 16 + lane % 16, r2 = tj * 16 + lane % 16;
      const double* f1 = Fm + (r1 < R ? r1 : R - 1);
      const double* f2 = Fm + (r2 < R ? r2 : R - 1);
#pragma unroll 4
      for (int k0 = 0; k0 < n; k0 += 8) {
        const int q = k0 + lane / 16, q2 = q + 4;
        const int qc = q < n ? q : n - 1, qc2 = q2 < n ? q2 : n - 1;
        const double a0 = f1[qc * R], b0 = f2[qc * R], a1 = f1[qc2 * R], b1 = f2[qc2 * R];
        acc0 = mfma64(q < n ? a0 : 0.0, b0, acc0);
        acc1 = mfma64(q2 < n ? a1 : 0.0, b1, acc1);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + lane / 16 + 4 * i, col = r2;
        if (row < R && col < R) G[row * R + col] = acc0[i] + acc1[i];
      }
    }
}

// G = F^T F (F: n x R in LDS) by all threads: four lanes per entry split the
// rows (two accumulators each), then the four partial sums are added across
// lanes in a fixed order.
__device__ void gram_all(const double* Fm, int n, int R, double* G) {
  const int RR = R * R;
  for (int base = 0; base < RR * 4; base += NT) {
    const int idx = base + (int)threadIdx.x;
    const int e = idx >> 2, sub = idx & 3;
    double s0 = 0.0, s1 = 0.0;
    if (e < RR) {
      const FastDiv fr(R);
      const double* f1 = Fm + fr.div(e);
      const double* f2 = Fm + fr.mod(e);
      int q = sub;
      for (; q + 4 < n; q += 8) {
        s0 = fma(f1[q * R], f2[q * R], s0);
        s1 = fma(f1[(q + 4) * R], f2[(q + 4) * R], s1);
      }
      if (q < n) s0 = fma(f1[q * R], f2[q * R], s0);
    }
    double s = s0 + s1;
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (e < RR && sub == 0) G[e] = s;
  }
}

// out(q, :) = M(q, :) Ginv for q < n (all threads; the few rows of a
// workgroup's slab in mode 1).  The sum over k runs in blocks of 8 whose
// sixteen loads are issued together (indices clamped, the terms past R
// skipped); even and odd k go to two accumulators.
__device__ void apply_inverse(const double* M, const double* Ginv, double* out, int n, int R) {
  const FastDiv fr(R);
  for (int e = threadIdx.x; e < n * R; e += NT) {
    const int q = fr.div(e), r = e - q * R;
    const double* m = M + q * R;
    double s0 = 0.0, s1 = 0.0;
    for (int k0 = 0; k0 < R; k0 += 8) {
      double mv[8], gv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + u < R ? k0 + u : R - 1;
        mv[u] = m[k];
        gv[u] = Ginv[k * R + r];
      }
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        if (k0 + u < R) s0 = fma(mv[u], gv[u], s0);
        if (k0 + u + 1 < R) s1 = fma(mv[u + 1], gv[u + 1], s1);
      }
    }
    out[e] = s0 + s1;
  }
}

// F = M Ginv (n x R, all in LDS) on v_mfma_f64_16x16x4f64: wavefront w takes
// the 16-row tiles w, w + 8, ..., each with every column tile (R <= 32).
// With part set, the wavefront also forms its rows' share of F^T F straight
// from the accumulators (element s of a 16 x 16 result fragment is, lane for
// lane, both operand fragments of k-step s of that tile's F_t^T F_t) and
// writes it to part[w] (R x R) when it had a tile: part[0 .. min(8, tiles))
// then sum to F^T F.  Rows past n and columns past R are exact zeros.  Out
// of line (its registers stay out of the kernel's MFMA phases); the
// pointers are LDS ones, cast so that the accesses are LDS instructions.
__device__ __noinline__ void apply_gram(const double* M_, const double* Gi_, double* F_, int n_,
                                       int R_, double* part_) {
  // the arguments are the same in every lane: say so, so that the loops
  // below are scalar branches and not masked ones
  const lds_f64* M = lds_uniform(M_);
  const lds_f64* Ginv = lds_uniform(Gi_);
  lds_f64* F = lds_uniform(F_);
  const bool with_part = __builtin_amdgcn_readfirstlane(part_ != nullptr ? 1 : 0) != 0;
  lds_f64* part = with_part ? lds_uniform(part_) : nullptr;
  const int n = __builtin_amdgcn_readfirstlane(n_), R = __builtin_amdgcn_readfirstlane(R_);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int RT = (R + 15) >> 4, ks = (R + 3) >> 2, ntr = (n + 15) >> 4;
  f64x4 g00 = {0.0, 0.0, 0.0, 0.0}, g01 = g00, g11 = g00;
  for (int rt = wave; rt < ntr; rt += NT / 64) {
    f64x4 d[2];
    const int row = rt * 16 + (lane & 15);
    const int rowc = row < n ? row : n - 1;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      if (ct < RT) {
        const int col = ct * 16 + (lane & 15);
        const int colc = col < R ? col : R - 1;
        // operands of four k-steps first (indices clamped), then their MFMAs
        for (int s0 = 0; s0 < ks; s0 += 4) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = 4 * (s0 + u) + (lane >> 4);
            const int kc = k < R ? k : R - 1;
            av[u] = M[rowc * R + kc];
            bv[u] = Ginv[kc * R + colc];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = 4 * (s0 + u) + (lane >> 4);
            if (s0 + u < ks)
              acc = mfma64((row < n && k < R) ? av[u] : 0.0, col < R ? bv[u] : 0.0, acc);
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rt * 16 + (lane >> 4) + 4 * i;
          if (r < n && col < R) F[r * R + col] = acc[i];
        }
      }
      d[ct] = acc;
    }
    if (with_part) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        g00 = mfma64(d[0][s4], d[0][s4], g00);
        if (RT > 1) {
          g01 = mfma64(d[0][s4], d[1][s4], g01);
          g11 = mfma64(d[1][s4], d[1][s4], g11);
        }
      }
    }
  }
  if (with_part && wave < ntr) {
    lds_f64* pw = part + wave * R * R;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r1 = (lane >> 4) + 4 * i, r2 = lane & 15;
      if (r1 < R && r2 < R) pw[r1 * R + r2] = g00[i];
      if (RT > 1) {
        // the lower-left block is the transpose of the upper-right one
        if (r1 < R && r2 + 16 < R) {
          pw[r1 * R + r2 + 16] = g01[i];
          pw[(r2 + 16) * R + r1] = g01[i];
        }
        if (r1 + 16 < R && r2 + 16 < R) pw[(r1 + 16) * R + r2 + 16] = g11[i];
      }
    }
  }
}

// 1 / sqrt(d) for d > 0 (normal): the hardware estimate refined by two
// Newton steps r <- r + r (1 - d r^2) / 2, each squaring the relative error.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = fma(0.5 * r, fma(-d * r, r, 1.0), r);
  r = fma(0.5 * r, fma(-d * r, r, 1.0), r);
  return r;
}

// From the nslot partial Grams of an unnormalised factor F: lam[r] = the
// 2-norm of column r (0 replaced by 1), rlam[r] = 1 / lam[r], and the Gram
// of the normalised factor FtF(r1, r2) = (F^T F)(r1, r2) rlam[r1] rlam[r2];
// the partials are added in slot order; 1 / lam from rsqrt_nr (a few units
// in the last place).
__device__ void norm_gram(const double* part, int nslot, int R, double* FtF, double* lam,
                          double* rlam) {
  const int RR = R * R;
  const FastDiv fr(R);
  for (int e = threadIdx.x; e < RR; e += NT) {
    const int r1 = fr.div(e), r2 = e - r1 * R;
    double sv = 0.0, d1 = 0.0, d2 = 0.0;
    for (int w = 0; w < nslot; ++w) {
      sv += part[w * RR + e];
      d1 += part[w * RR + r1 * (R + 1)];
      d2 += part[w * RR + r2 * (R + 1)];
    }
    // a zero column keeps lambda = 1
    const double q1 = d1 > 0.0 ? rsqrt_nr(d1) : 1.0, q2 = d2 > 0.0 ? rsqrt_nr(d2) : 1.0;
    FtF[e] = sv * q1 * q2;
    if (r1 == r2) {
      lam[r1] = d1 > 0.0 ? d1 * q1 : 1.0;
      rlam[r1] = q1;
    }
  }
}

// Column 2-norms of F (n x R): lam[r] (0 replaced by 1) and rlam[r] =
// 1 / lam[r]; sixteen lanes per column split the rows (two accumulators),
// then a butterfly within the sixteen; all columns in one round (R <= 32).
__device__ void col_norms(const double* Fm, int n, int R, double* lam, double* rlam) {
  const int grp = threadIdx.x / 16, sub = threadIdx.x & 15;
  for (int r = grp; r < R; r += NT / 16) {
    double s0 = 0.0, s1 = 0.0;
    int q = sub;
    for (; q + 16 < n; q += 32) {
      const double a = Fm[q * R + r], b = Fm[(q + 16) * R + r];
      s0 = fma(a, a, s0);
      s1 = fma(b, b, s1);
    }
    if (q < n) s0 = fma(Fm[q * R + r], Fm[q * R + r], s0);
    double s = s0 + s1;
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (sub == 0) {
      const double nr = sqrt(s);
      const double l = nr > 0.0 ? nr : 1.0;
      lam[r] = l;
      rlam[r] = 1.0 / l;
    }
  }
}

// Sum over the NW slab partials of element e, slab order; loads are issued
// sixteen at a time before they are added, so that they are in flight together.
__device__ __forceinline__ double sum_slots(const double* base, int64_t stride, int NW) {
  double s = 0.0;
  for (int w0 = 0; w0 < NW; w0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = w0 + u < NW ? slot_load(base + (w0 + u) * stride) : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (w0 + u < NW) s += v[u];
  }
  return s;
}

// GX: the slab is read from the summary in global memory on every use (it
// stays in L2: the replicas of one XCD total a few MB) instead of being held
// in LDS; for replicas whose slab does not fit next to the factor state.
// SPLIT (float summaries only): the two contractions T and M3 take their
// operands in the two-term bfloat16 form above; the factor C and the rows W
// are kept in that form in LDS as B-operand fragments (Cb, Wb).
// The ALS of workgroup `bid` of a launch over the replicas of one handle.
template <typename T, int RMAX, bool GX, bool SPLIT>
__device__ __forceinline__ void als_coop_body(const CoopArgs& g, const int bid) {
  static_assert(!SPLIT || sizeof(T) == 4, "the two-term form takes float summaries");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_ok, s_bad, s_stop, s_local;
  __shared__ double s_nx2, s_fit_old;
  __shared__ int s_have_old;

  // placement: workgroup x -> XCD x % 8; replicas p = x % 8 + 8 k live there
  const int xcd = bid % 8, loc = bid / 8;
  const int p = xcd + 8 * (loc / g.NW);
  const int w = loc % g.NW;
  if (p >= g.P) return;

  const int Q = g.Q, R = g.R, NW = g.NW, QR = Q * R, RR = R * R;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid & 63;
  const int a0 = (int)((int64_t)w * Q / NW), a1 = (int)((int64_t)(w + 1) * Q / NW);
  const int na = a1 - a0;
  const int npair = na * Q;                   // rows (a, b) of the slab
  // LDS slab: rows padded to npair_pad and columns to QPAD (a multiple of
  // 32) with zeros, plus one column against bank conflicts, so that the MFMA
  // loops run whole groups of 32 without clamping (Cf carries QPAD rows, Ts
  // npair_pad rows, zero past the data)
  const int QPAD = ((Q + 31) / 32) * 32;
  const int QP = GX ? Q : QPAD + 1;           // slab row stride
  const int RT = (R + 15) / 16;               // 16-wide tiles over r
  const FastDiv fR(R), fQ(Q);
  const int64_t Q2 = (int64_t)Q * Q;

  double* Ts = (double*)smem;                 // [npair_pad][R]  T, then W
  double* Bf = Ts + (int64_t)g.npair_pad * R; // [Q][R]
  double* Cf = Bf + QR;                       // [QPAD][R]
  double* Mf = Cf + QPAD * R;                 // reduced M2 / M3
  double* Ml = Mf + QR;                       // [Q][R] scratch (M1 rows)
  double* Al = Ml + QR;                       // [na_max][R]
  double* G = Al + g.na_max * R;              // [R][R]
  double* Gi = G + RR;                        // inverse
  double* AtA = Gi + RR;
  double* BtB = AtA + RR;
  double* CtC = BtB + RR;
  double* lamv = CtC + RR;                    // [MAXR]
  double* rlam = lamv + MAXR;                 // [MAXR] 1 / lamv
  double* scr = rlam + MAXR;                  // [NT]
  // the mode-2/3 solves on MFMA with the partial Grams from the result
  // fragments, which go where T is (T is dead from the end of mode 2 to the
  // next sweep), when they fit there and the factors have enough rows to
  // pay for it (below 40 rows the all-thread solve, column norms and Gram
  // are faster)
  const int nslot = min(NT / 64, (Q + 15) / 16);
  const bool pg = Q >= 40 && nslot * RR <= g.npair_pad * R;
  // SPLIT: B-operand fragments, [r tile][k chunk of 32][hi, lo][lane][8],
  // 16-byte aligned; those of W take the place of T when they fit there (T
  // is dead from the end of mode 2 to the next sweep)
  const int nkc = QPAD / 32, npc = g.npair_pad / 32;
  const bool walias = SPLIT && R >= 8 * RT;
  __bf16* Cb = (__bf16*)(SPLIT ? ((uintptr_t)(scr + NT) + 15) & ~(uintptr_t)15
                               : (uintptr_t)(scr + NT));                      // C: k = c
  __bf16* Wb = walias ? (__bf16*)Ts : Cb + (SPLIT ? (int64_t)RT * nkc * 2 * 512 : 0);   // W: k = pair
  unsigned char* after_frag = (unsigned char*)(
      Cb + (SPLIT ? (int64_t)RT * nkc * 2 * 512 + (walias ? 0 : (int64_t)RT * npc * 2 * 512) : 0));
  // fragments of C (after every update of C); with scale, C is first
  // normalised in place (each element of C belongs to exactly one fragment
  // entry, so the thread that scales it is the one that reads it)
  auto build_cb = [&](bool scale) {
    for (int e = tid; e < RT * nkc * 64; e += NT) {
      const int ln = e & 63, kc = (e >> 6) % nkc, rt = (e >> 6) / nkc;
      const int r = rt * 16 + (ln & 15);
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = kc * 32 + 8 * (ln >> 4) + j;
        double x = 0.0;
        if (c < Q && r < R) {
          x = Cf[c * R + r];
          if (scale) {
            x *= rlam[r];
            Cf[c * R + r] = x;
          }
        }
        v[j] = (float)x;
      }
      bf16x8a hi, lo;
      split8(v, hi, lo);
      __bf16* dst = Cb + ((int64_t)(rt * nkc + kc) * 2 * 64 + ln) * 8;
      *(bf16x8a*)dst = hi;
      *(bf16x8a*)(dst + 512) = lo;
    }
  };
  const T* Xp = (const T*)g.Y + (int64_t)p * Q2 * Q;
  const T* Xs;                                // [na * Q][QP] (LDS: [npair_pad][QP])
  if constexpr (GX) {
    Xs = Xp + (int64_t)a0 * Q2;
  } else {
    T* xl = (T*)after_frag;
    const FastDiv fQP(QP);
    for (int e = tid; e < g.npair_pad * QP; e += NT) {
      const int row = fQP.div(e), col = e - row * QP;
      xl[e] = (row < npair && col < Q) ? Xp[(int64_t)a0 * Q2 + (int64_t)row * Q + col] : (T)0;
    }
    Xs = xl;
  }
  for (int e = npair * R + tid; e < g.npair_pad * R; e += NT) Ts[e] = 0.0;
  for (int e = QR + tid; e < QPAD * R; e += NT) Cf[e] = 0.0;
  const double* F0 = g.init + (int64_t)p * 3 * QR;
  for (int e = tid; e < na * R; e += NT) Al[e] = F0[a0 * R + e];
  for (int e = tid; e < QR; e += NT) { Bf[e] = F0[QR + e]; Cf[e] = F0[2 * QR + e]; }
  if (tid == 0) { s_bad = 0; s_stop = 0; s_have_old = 0; s_fit_old = 0.0; s_nx2 = 0.0; }
  __syncthreads();

  unsigned* ctr = g.counters + p;
  unsigned nbar = 0;
  bool alive = true;
  // a replica whose workgroups all landed on one XCD synchronises through
  // that XCD's L2 (the placement above asks for this; the mask checks it)
  bool local = false;
  if (NW > 1) {
    unsigned* xmask = g.counters + g.P + p;
    if (tid == 0)
      __hip_atomic_fetch_or(xmask, 1u << xcd_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    alive = replica_barrier(ctr, (++nbar) * NW, g.err, &s_ok, false);
    if (tid == 0)
      s_local = __popc(__hip_atomic_load(xmask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 1;
    __syncthreads();
    local = alive && s_local && g.allow_local;
  }
  const int slot_len = g.slot_len;
  // the slot set alternates with the barrier count: a set is rewritten two
  // barriers later, when every workgroup has finished reading it
  auto slot = [&](int set, int ww) {
    return g.slots + (((int64_t)set * g.P + p) * NW + ww) * slot_len;
  };

  if (g.tol > 0.0) {
    double s = 0.0;
    for (int64_t e = tid; e < (int64_t)npair * Q; e += NT) {
      const double v = (double)Xs[(e / Q) * QP + e % Q];
      s = fma(v, v, s);
    }
    scr[tid] = s;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
      if (tid < st) scr[tid] += scr[tid + st];
      __syncthreads();
    }
    if (NW > 1) {
      const int bs = (nbar + 1) & 1;
      if (tid == 0) slot(bs, w)[0] = scr[0];
      alive = replica_barrier(ctr, (++nbar) * NW, g.err, &s_ok, local) && alive;
      if (alive && tid == 0) {
        double t = 0.0;
        for (int ww = 0; ww < NW; ++ww) t += slot_load(slot(bs, ww));
        s_nx2 = t;
      }
    } else if (tid == 0) {
      s_nx2 = scr[0];
    }
    __syncthreads();
  }
  if (wave == 0) gram_wave(Bf, Q, R, BtB);
  if (wave == 1) gram_wave(Cf, Q, R, CtC);
  if constexpr (SPLIT) build_cb(false);
  __syncthreads();


  int done = 0;
  for (int it = 0; it < g.max_iters && alive; ++it) {
    // ------------------------------------------------ mode 1 (rows of A)
    // wavefront 0 forms G1 = B'B o C'C itself (both complete: the sweep
    // before ended with a barrier) while the others start on T
    if (wave == 0) {
      for (int e = lane; e < RR; e += 64) G[e] = BtB[e] * CtC[e];
      wave_sync();
      spd_inverse<RMAX>(G, Gi, R, &s_bad);
    }
    {
      // T(pair, r) = sum_c X(pair, c) C(c, r) on MFMA, tiles over pairs x r,
      // dealt to the six wavefronts that do not share a SIMD with the
      // inverting wavefront 0 (wavefront w runs on SIMD w % 4: wavefront 4
      // stays idle, so the inverse's FP64 arithmetic does not compete with
      // FP64 MFMA on its SIMD); when one tile is left over after at least
      // two whole rounds, wavefront 0 takes it after the inverse
      constexpr int NMW = NT / 64 - 2;
      const int mw = wave < 4 ? wave - 1 : wave - 2;     // 0..5 for the MFMA wavefronts
      const int ntile = (npair + 15) / 16 * RT;
      const bool w0_tile = ntile % NMW == 1 && ntile > 2 * NMW;
      const int t_first = wave == 0 ? (w0_tile ? ntile - 1 : ntile) : (wave == 4 ? ntile : mw);
      const int t_end = wave == 0 || !w0_tile ? ntile : ntile - 1;
      const int t_step = wave == 0 ? 1 : NMW;
      for (int tt = t_first; tt < t_end; tt += t_step) {
        const int pt = tt / RT, rt = tt % RT;
        const int pr = pt * 16 + lane % 16;
        const int rr = rt * 16 + lane % 16;
        if constexpr (SPLIT) {
          f32x4a acc = {0.f, 0.f, 0.f, 0.f};
          const __bf16* cb = Cb + ((int64_t)rt * nkc * 2 * 64 + lane) * 8;
          for (int kc = 0; kc < nkc; ++kc) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int c = kc * 32 + 8 * (lane >> 4) + j;
              if constexpr (GX) v[j] = (pr < npair && c < Q) ? (float)Xs[(int64_t)pr * QP + c] : 0.f;
              else v[j] = (float)Xs[pr * QP + c];
            }
            bf16x8a ah, al;
            split8(v, ah, al);
            const bf16x8a bh = *(const bf16x8a*)(cb + (int64_t)kc * 2 * 512);
            const bf16x8a bl = *(const bf16x8a*)(cb + (int64_t)kc * 2 * 512 + 512);
            acc = mma3(ah, al, bh, bl, acc);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = pt * 16 + 4 * (lane >> 4) + i;
            if (row < npair && rr < R) Ts[row * R + rr] = (double)acc[i];
          }
          continue;
        }
        f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        const bool okc = rr < R;
        const double* cr = Cf + (okc ? rr : R - 1);
        if constexpr (!GX) {
          // LDS slab padded with zeros (rows and columns) and Cf with zero
          // rows: groups of 32 columns (four steps of 8), all sixteen loads,
          // then the conversions, then the eight MFMAs (a VALU instruction
          // issued between MFMAs of one wavefront waits for them)
          const T* xp = Xs + pr * QP + lane / 16;
          const double* cp = cr + (lane / 16) * R;
          for (int c0 = 0; c0 < Q; c0 += 32) {
            T xv[8];
            double bv[8], xd[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) { xv[u] = xp[4 * u]; bv[u] = cp[4 * u * R]; }
#pragma unroll
            for (int u = 0; u < 8; ++u) xd[u] = (double)xv[u];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
              acc0 = mfma64(xd[u], bv[u], acc0);
              acc1 = mfma64(xd[u + 1], bv[u + 1], acc1);
            }
            __builtin_amdgcn_sched_barrier(0);
            xp += 32;
            cp += 32 * R;
          }
        } else {
          const T* xr = Xs + (pr < npair ? pr : npair - 1) * QP;
          // whole groups of 32 columns: all sixteen loads first, then the
          // conversions, then the eight MFMAs (a VALU instruction issued
          // between MFMAs of one wavefront waits for them); same order of
          // accumulation as the step loop below
          int c0 = 0;
          {
            const T* xp = xr + lane / 16;
            const double* cp = cr + (lane / 16) * R;
            for (; c0 + 32 <= Q; c0 += 32) {
              T xv[8];
              double bv[8], xd[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) { xv[u] = xp[4 * u]; bv[u] = cp[4 * u * R]; }
#pragma unroll
              for (int u = 0; u < 8; ++u) xd[u] = (double)xv[u];
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int u = 0; u < 8; u += 2) {
                acc0 = mfma64(xd[u], bv[u], acc0);
                acc1 = mfma64(xd[u + 1], bv[u + 1], acc1);
              }
              __builtin_amdgcn_sched_barrier(0);
              xp += 32;
              cp += 32 * R;
            }
          }
          // the rest: indices clamped into range and the k tail zeroed after
          // the load (no branches around the loads)
          for (; c0 < Q; c0 += 8) {
            const int c = c0 + lane / 16, c2 = c + 4;
            const int cc = c < Q ? c : Q - 1, cc2 = c2 < Q ? c2 : Q - 1;
            const double x0 = (double)xr[cc], x1 = (double)xr[cc2];
            const double b0 = cr[cc * R], b1 = cr[cc2 * R];
            acc0 = mfma64(c < Q ? x0 : 0.0, b0, acc0);
            acc1 = mfma64(c2 < Q ? x1 : 0.0, b1, acc1);
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = pt * 16 + lane / 16 + 4 * i;
          if (row < npair && okc) Ts[row * R + rr] = acc0[i] + acc1[i];
        }
      }
    }
    __syncthreads();
    // M1(la, r) = sum_b T(la, b, r) B(b, r): eight lanes per entry split b,
    // their partial sums are added across lanes in a fixed order
    for (int base = 0; base < na * R * 8; base += NT) {
      const int idx = base + tid, e = idx >> 3, sub = idx & 7;
      double s0 = 0.0, s1 = 0.0;
      if (e < na * R) {
        const int la = fR.div(e), r = e - la * R;
        const double* tr = Ts + (int64_t)la * QR + r;
        const double* br = Bf + r;
        int b = sub;
        for (; b + 8 < Q; b += 16) {
          s0 = fma(tr[b * R], br[b * R], s0);
          s1 = fma(tr[(b + 8) * R], br[(b + 8) * R], s1);
        }
        if (b < Q) s0 = fma(tr[b * R], br[b * R], s0);
      }
      double sm = s0 + s1;
      sm += __shfl_xor(sm, 1, 64);
      sm += __shfl_xor(sm, 2, 64);
      sm += __shfl_xor(sm, 4, 64);
      if (e < na * R && sub == 0) Ml[e] = sm;
    }
    __syncthreads();
    apply_inverse(Ml, Gi, Al, na, R);
    __syncthreads();
    // ------------------------------------------------ mode 2 partials
    const int set1 = (nbar + 1) & 1;
    double* sl = NW > 1 ? slot(set1, w) : nullptr;
    for (int e = tid; e < QR + RR; e += NT) {
      double s = 0.0;
      if (e < QR) {
        const int b = fR.div(e), r = e - b * R;
        for (int la = 0; la < na; ++la) s = fma(Ts[((int64_t)la * Q + b) * R + r], Al[la * R + r], s);
      } else {
        const int r1 = fR.div(e - QR), r2 = e - QR - r1 * R;
        for (int la = 0; la < na; ++la) s = fma(Al[la * R + r1], Al[la * R + r2], s);
      }
      if (NW > 1) sl[e] = s;
      else if (e < QR) Mf[e] = s;
      else AtA[e - QR] = s;
    }
    // sums of the partials: wavefront 0 takes A'A and goes on to lambda_A
    // (norms from diag(A'A)), the normalised A'A, G2 and its inverse, while
    // the other wavefronts sum M2
    if (NW > 1) {
      alive = replica_barrier(ctr, (++nbar) * NW, g.err, &s_ok, local);
      if (!alive) break;
      if (wave == 0) {
        // two entries per lane, both sets of loads in flight together
        for (int e = lane; e < RR; e += 128) {
          const double* b0 = slot(set1, 0) + QR + e;
          const bool two = e + 64 < RR;
          double v0[16], v1[16];
          double a0 = 0.0, a1 = 0.0;
          for (int w0 = 0; w0 < NW; w0 += 16) {
#pragma unroll
            for (int u2 = 0; u2 < 16; ++u2) {
              v0[u2] = w0 + u2 < NW ? slot_load(b0 + (int64_t)(w0 + u2) * slot_len) : 0.0;
              v1[u2] = (two && w0 + u2 < NW) ? slot_load(b0 + (int64_t)(w0 + u2) * slot_len + 64) : 0.0;
            }
#pragma unroll
            for (int u2 = 0; u2 < 16; ++u2)
              if (w0 + u2 < NW) { a0 += v0[u2]; a1 += v1[u2]; }
          }
          AtA[e] = a0;
          if (two) AtA[e + 64] = a1;
        }
      } else {
        for (int e = tid - 64; e < QR; e += NT - 64) Mf[e] = sum_slots(slot(set1, 0) + e, slot_len, NW);
      }
    } else {
      __syncthreads();
    }
    if (wave == 0) {
      wave_sync();
      if (lane < R) {
        const double n = sqrt(AtA[lane * R + lane]);
        const double l = n > 0.0 ? n : 1.0;
        lamv[lane] = l;
        rlam[lane] = 1.0 / l;
      }
      wave_sync();
      for (int e = lane; e < RR; e += 64) {
        AtA[e] *= rlam[fR.div(e)] * rlam[fR.mod(e)];
        G[e] = AtA[e] * CtC[e];
      }
      wave_sync();
      // ---------------------------------------------- mode 2 solve (B)
      spd_inverse<RMAX>(G, Gi, R, &s_bad);
      // M2 was formed with the unnormalised A: B = (M2 / lambda_A) G2^{-1},
      // so row k of the inverse takes the factor 1 / lambda_A(k)
      wave_sync();
      for (int e = lane; e < RR; e += 64) Gi[e] *= rlam[fR.div(e)];
    }
    __syncthreads();
    for (int e = tid; e < na * R; e += NT) Al[e] *= rlam[fR.mod(e)];
    if (pg) apply_gram(Mf, Gi, Bf, Q, R, Ts);
    else apply_inverse(Mf, Gi, Bf, Q, R);
    __syncthreads();
    // lambda_B and B'B of the normalised B from the partial Grams
    if (pg) norm_gram(Ts, nslot, R, BtB, lamv, rlam);
    else col_norms(Bf, Q, R, lamv, rlam);
    __syncthreads();
    for (int e = tid; e < QR; e += NT) Bf[e] *= rlam[fR.mod(e)];
    __syncthreads();
    // W(pair, r) = A(a, r) B(b, r) into Ts (B'B here when it was not formed
    // above)
    if (!pg) gram_all(Bf, Q, R, BtB);
    if constexpr (SPLIT) {
      // W(pair, r) = A(a, r) B(b, r) as B-operand fragments (k = pair)
      for (int e = tid; e < RT * npc * 64; e += NT) {
        const int ln = e & 63, pc = (e >> 6) % npc, rt = (e >> 6) / npc;
        const int r = rt * 16 + (ln & 15);
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int pr = pc * 32 + 8 * (ln >> 4) + j;
          const int a = fQ.div(pr), b = pr - a * Q;
          v[j] = (pr < npair && r < R) ? (float)(Al[a * R + r] * Bf[b * R + r]) : 0.f;
        }
        bf16x8a hi, lo;
        split8(v, hi, lo);
        __bf16* dst = Wb + ((int64_t)(rt * npc + pc) * 2 * 64 + ln) * 8;
        *(bf16x8a*)dst = hi;
        *(bf16x8a*)(dst + 512) = lo;
      }
    } else {
      for (int e = tid; e < npair * R; e += NT) {
        const int pr = fR.div(e), r = e - pr * R;
        const int a = fQ.div(pr), b = pr - a * Q;
        Ts[e] = Al[a * R + r] * Bf[b * R + r];
      }
    }
    __syncthreads();
    // ------------------------------------------------ mode 3 partial
    {
      const int set2 = (nbar + 1) & 1;
      double* dst = NW > 1 ? slot(set2, w) : Mf;
      // M3(c, r) = sum_pair X(pair, c) W(pair, r): tiles over c x r; when the
      // tiles are fewer than half the MFMA wavefronts, the pair range is cut
      // in two and the second halves are added through LDS (fixed order)
      const int ctiles = (Q + 15) / 16, ntl = ctiles * RT;
      // when the tiles (and halves) fit on wavefronts 1-7, wavefront 0 forms
      // and inverts G3 meanwhile; otherwise all eight wavefronts take tiles
      // and the inverse waits until after the reduction below, where it
      // overlaps the sum of the partials
      const bool early = ntl * (2 * ntl <= NT / 64 - 1 ? 2 : 1) <= NT / 64 - 1;
      const int NMW = early ? NT / 64 - 1 : NT / 64;
      const int ksp = 2 * ntl <= NMW ? 2 : 1;
      // pair range: padded to a multiple of 32 in LDS (zero rows), halves
      // cut at a multiple of 32; from global memory, the exact range
      const int npp = (GX && !SPLIT) ? npair : ((npair + 31) / 32) * 32;
      const int kh = ksp == 1 ? npp
                              : ((GX && !SPLIT) ? ((npair + 15) / 16) * 8 : ((npp / 32 + 1) / 2) * 32);
      f64x4 keep = {0.0, 0.0, 0.0, 0.0};
      int keep_tile = -1;
      if (early && wave == 0) {
        for (int e = lane; e < RR; e += 64) G[e] = AtA[e] * BtB[e];
        wave_sync();
        spd_inverse<RMAX>(G, Gi, R, &s_bad);
      } else {
        for (int item = early ? wave - 1 : wave; item < ntl * ksp; item += NMW) {
          const int tt = item % ntl, part = item / ntl;
          const int kb = part * kh, ke = kb + kh < npp ? kb + kh : npp;
          const int ct = tt / RT, rt = tt % RT;
          const int c = ct * 16 + lane % 16;
          const int rr = rt * 16 + lane % 16;
          if constexpr (SPLIT) {
            // M3(c, r) = sum over pairs of X(pair, c) W(pair, r): A = X^T
            f32x4a acc = {0.f, 0.f, 0.f, 0.f};
            const __bf16* wb = Wb + ((int64_t)rt * npc * 2 * 64 + lane) * 8;
            for (int k0 = kb; k0 < ke; k0 += 32) {
              float v[8];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                const int pr = k0 + 8 * (lane >> 4) + j;
                if constexpr (GX) v[j] = (pr < npair && c < Q) ? (float)Xs[(int64_t)pr * QP + c] : 0.f;
                else v[j] = (float)Xs[pr * QP + c];
              }
              bf16x8a ah, al;
              split8(v, ah, al);
              const int pc = k0 >> 5;
              const bf16x8a bh = *(const bf16x8a*)(wb + (int64_t)pc * 2 * 512);
              const bf16x8a bl = *(const bf16x8a*)(wb + (int64_t)pc * 2 * 512 + 512);
              acc = mma3(ah, al, bh, bl, acc);
            }
            f64x4 accd;
#pragma unroll
            for (int i = 0; i < 4; ++i) accd[i] = (double)acc[i];
            if (ksp == 2 && part == 0) {
              keep = accd;
              keep_tile = tt;
              continue;
            }
            double* o = ksp == 2 ? Ml : dst;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = ct * 16 + 4 * (lane >> 4) + i;
              if (row < Q && rr < R) o[row * R + rr] = accd[i];
            }
            continue;
          }
          f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
          const bool okr = rr < R;
          const double* wc = Ts + (okr ? rr : R - 1);
          if constexpr (!GX) {
            // zero-padded LDS slab and W: groups of 32 pairs as for T
            const T* xp = Xs + c + (kb + lane / 16) * QP;
            const double* wp = wc + (kb + lane / 16) * R;
            for (int k0 = kb; k0 < ke; k0 += 32) {
              T xv[8];
              double bv[8], xd[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) { xv[u] = xp[4 * u * QP]; bv[u] = wp[4 * u * R]; }
#pragma unroll
              for (int u = 0; u < 8; ++u) xd[u] = (double)xv[u];
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int u = 0; u < 8; u += 2) {
                acc0 = mfma64(xd[u], bv[u], acc0);
                acc1 = mfma64(xd[u + 1], bv[u + 1], acc1);
              }
              __builtin_amdgcn_sched_barrier(0);
              xp += 32 * QP;
              wp += 32 * R;
            }
          } else {
            const T* xc = Xs + (c < Q ? c : Q - 1);
            // whole groups of 32 pairs as for T above, then the clamped steps
            int k0 = kb;
            {
              const T* xp = xc + (kb + lane / 16) * QP;
              const double* wp = wc + (kb + lane / 16) * R;
              for (; k0 + 32 <= ke; k0 += 32) {
                T xv[8];
                double bv[8], xd[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) { xv[u] = xp[4 * u * QP]; bv[u] = wp[4 * u * R]; }
#pragma unroll
                for (int u = 0; u < 8; ++u) xd[u] = (double)xv[u];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                  acc0 = mfma64(xd[u], bv[u], acc0);
                  acc1 = mfma64(xd[u + 1], bv[u + 1], acc1);
                }
                __builtin_amdgcn_sched_barrier(0);
                xp += 32 * QP;
                wp += 32 * R;
              }
            }
            for (; k0 < ke; k0 += 8) {
              const int pr = k0 + lane / 16, pr2 = pr + 4;
              const int pc = pr < ke ? pr : ke - 1, pc2 = pr2 < ke ? pr2 : ke - 1;
              const double x0 = (double)xc[pc * QP], x1 = (double)xc[pc2 * QP];
              const double b0 = wc[pc * R], b1 = wc[pc2 * R];
              acc0 = mfma64(pr < ke ? x0 : 0.0, b0, acc0);
              acc1 = mfma64(pr2 < ke ? x1 : 0.0, b1, acc1);
            }
          }
          const f64x4 acc = acc0 + acc1;
          if (ksp == 2 && part == 0) {
            keep = acc;
            keep_tile = tt;
            continue;
          }
          double* o = ksp == 2 ? Ml : dst;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = ct * 16 + lane / 16 + 4 * i;
            if (row < Q && okr) o[row * R + rr] = acc[i];
          }
        }
      }
      if (ksp == 2) {
        __syncthreads();
        if (keep_tile >= 0) {
          const int ct = keep_tile / RT, rt = keep_tile % RT;
          const int rr = rt * 16 + lane % 16;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = ct * 16 + (SPLIT ? 4 * (lane / 16) + i : lane / 16 + 4 * i);
            if (row < Q && rr < R) dst[row * R + rr] = keep[i] + Ml[row * R + rr];
          }
        }
      }
      if (NW > 1) {
        alive = replica_barrier(ctr, (++nbar) * NW, g.err, &s_ok, local);
        if (!alive) break;
        if (early)
          for (int e = tid; e < QR; e += NT) Mf[e] = sum_slots(slot(set2, 0) + e, slot_len, NW);
        else if (wave != 0)
          for (int e = tid - 64; e < QR; e += NT - 64) Mf[e] = sum_slots(slot(set2, 0) + e, slot_len, NW);
      }
      if (wave == 0 && !early) {
        // G3 = A'A o B'B (both complete) by wavefront 0 while the others
        // sum the partials of M3
        for (int e = lane; e < RR; e += 64) G[e] = AtA[e] * BtB[e];
        wave_sync();
        spd_inverse<RMAX>(G, Gi, R, &s_bad);
      }
    }
    __syncthreads();
    // ------------------------------------------------ mode 3 solve (C)
    if (pg) apply_gram(Mf, Gi, Cf, Q, R, Ts);
    else apply_inverse(Mf, Gi, Cf, Q, R);
    __syncthreads();
    if (pg) norm_gram(Ts, nslot, R, CtC, lamv, rlam);
    else col_norms(Cf, Q, R, lamv, rlam);
    __syncthreads();
    // C normalised (and, two-term, its fragments)
    if constexpr (SPLIT) build_cb(true);
    else
      for (int e = tid; e < QR; e += NT) Cf[e] *= rlam[fR.mod(e)];
    __syncthreads();
    if (!pg) {
      gram_all(Cf, Q, R, CtC);
      __syncthreads();
    }
    ++done;
    if (g.tol > 0.0) {
      // replica fit from the Gram identity, summed by wavefront 0 in a fixed
      // order (every workgroup of the replica reaches the same decision)
      if (wave == 0) {
        double inner = 0.0, nh = 0.0;
        for (int e = lane; e < QR; e += 64) inner = fma(Mf[e] * lamv[fR.mod(e)], Cf[e], inner);
        for (int e = lane; e < RR; e += 64)
          nh += lamv[fR.div(e)] * (AtA[e] * BtB[e] * CtC[e]) * lamv[fR.mod(e)];
        for (int off = 32; off > 0; off >>= 1) {
          inner += __shfl_xor(inner, off, 64);
          nh += __shfl_xor(nh, off, 64);
        }
        if (lane == 0) {
          double res = s_nx2 - 2.0 * inner + nh;
          if (res < 0.0) res = 0.0;
          const double fit = s_nx2 > 0.0 ? 1.0 - sqrt(res) / sqrt(s_nx2) : 0.0;
          s_stop = (s_have_old && fabs(fit - s_fit_old) < g.tol) ? 1 : 0;
          s_fit_old = fit;
          s_have_old = 1;
        }
      }
      __syncthreads();
      if (s_stop) break;
    }
  }
  // write back: slab rows of A from every workgroup; B, C, lambda from slab 0
  double* Fo = g.F + (int64_t)p * 3 * QR;
  for (int e = tid; e < na * R; e += NT) Fo[a0 * R + e] = Al[e];
  if (w == 0) {
    for (int e = tid; e < QR; e += NT) { Fo[QR + e] = Bf[e]; Fo[2 * QR + e] = Cf[e]; }
    if (tid < R) g.lam[(int64_t)p * R + tid] = lamv[tid];
    if (tid == 0) {
      g.iters[p] = done;
      if (s_bad) g.flags[p] |= 1;
      if (!alive) g.flags[p] |= 2;
    }
  } else if (tid == 0 && s_bad) {
    atomicOr(g.flags + p, 1);
  }
}


inline int pad_pairs(int Q, int NW) {
  const int na_max = (Q + NW - 1) / NW;
  return ((na_max * Q + 31) / 32) * 32;
}

// Launch arguments of one handle's cooperative ALS; false when the sizes are
// outside what the kernel supports.
inline bool coop_args(const AlsCoopItem& it, CoopArgs& a, size_t& lds) {
  const int P = it.P, Q = it.Q, R = it.R, NW = it.NW;
  if (R > MAXR || Q > 128 || NW < 1 || NW > Q || NW > 32) return false;
  if (it.split && it.y_f64) return false;
  a.Y = it.Y; a.init = it.init; a.F = it.F; a.lam = it.lam; a.iters = it.iters;
  a.flags = it.flags; a.slots = it.slots; a.counters = it.counters; a.err = it.err;
  a.P = P; a.Q = Q; a.R = R; a.NW = NW;
  a.na_max = (Q + NW - 1) / NW;
  a.npair_pad = pad_pairs(Q, NW);
  a.per_xcd = (P + 7) / 8;
  a.slot_len = als_coop_slot_len(Q, R);
  a.max_iters = it.max_iters; a.tol = it.tol; a.allow_local = it.allow_local ? 1 : 0;
  lds = als_coop_lds_bytes(Q, R, NW, it.y_f64, it.slab_global, it.split);
  return lds <= 160 * 1024;
}

// The inverse runs RMAX straight-line steps: exact fits for the common ranks.
inline int rmax_class(int R) {
  return R <= 6 ? 6 : R <= 8 ? 8 : R <= 10 ? 10 : R <= 12 ? 12 : R <= 16 ? 16 : R <= 20 ? 20
         : R <= 24 ? 24 : 32;
}

inline int coop_grid(const CoopArgs& a) { return 8 * a.per_xcd * a.NW; }

}  // namespace
}  // namespace octen
