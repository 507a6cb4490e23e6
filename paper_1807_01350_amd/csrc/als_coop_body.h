// Types and device helpers of the cooperative replica ALS kernel, shared by
// the launch of one handle (als_coop.hip) and the grouped launch of several
// handles (als_coop_group.hip); the kernel's statements are in
// als_coop_kernel_body.inc.
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
__host__ __device__ inline int rmax_class(int R) {
  return R <= 6 ? 6 : R <= 8 ? 8 : R <= 10 ? 10 : R <= 12 ? 12 : R <= 16 ? 16 : R <= 20 ? 20
         : R <= 24 ? 24 : 32;
}

inline int coop_grid(const CoopArgs& a) { return 8 * a.per_xcd * a.NW; }

}  // namespace
}  // namespace octen
