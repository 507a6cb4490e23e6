// Internal declarations shared by the HIP translation units of libocten.
// Every launcher enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace octen {

// ---------------------------------------------------------------- linalg ---
// C[b] = alpha * opA[b] * diag(d) * opB[b] + beta * C[b]   (f64 accumulate)
// A element (m, k) at A[b*sab + m*sam + k*sak]; B element (k, n) at
// B[b*sbb + k*sbk + n*sbn]; C element (m, n) at C[b*scb + m*scm + n*scn].
// d may be null (identity).  beta == 0 never reads C.
hipError_t gemm_f64(hipStream_t s, int M, int N, int K, int batch,
                    const double* A, int64_t sam, int64_t sak, int64_t sab,
                    const double* B, int64_t sbk, int64_t sbn, int64_t sbb,
                    double* C, int64_t scm, int64_t scn, int64_t scb,
                    const double* d, double alpha, double beta);
hipError_t gemm_f32in_f64(hipStream_t s, int M, int N, int K, int batch,
                          const float* A, int64_t sam, int64_t sak, int64_t sab,
                          const double* B, int64_t sbk, int64_t sbn, int64_t sbb,
                          double* C, int64_t scm, int64_t scn, int64_t scb,
                          const double* d, double alpha, double beta);

// In-place inverse of an n x n symmetric positive definite matrix (leading
// dimension n) by Gauss-Jordan elimination without pivoting; work: 2n doubles.
// info (device int) is set to k+1 if pivot k is not positive.
hipError_t spd_invert(hipStream_t s, double* A, int n, double* work, int* info);

// out(i, r) = alpha * sum_k A(i,k) d(k) B(k,r) + beta * out(i, r), i < nrows,
// r < ncols; A(i,k) = A[i*sai + k*sak], B(k,r) = B[k*sbk + r*sbr]; d may be
// null.  Tall products with unit inner strides (sak = sbr = 1, no d, at least
// 16384 rows, ncols <= 32) run on FP64 MFMA with A streamed once; small
// Gram-type products (sai = sbr = 1, no d, nrows and ncols <= 32, K >= 8192,
// work given) as k-blocked partials in LDS summed in block order; otherwise
// one wavefront per row and block of 32 columns (small outputs, long k).
// work (optional, work_len doubles): partial sums for splitting K when there
// are few rows; without it, one wavefront covers all of K.
hipError_t rowdot(hipStream_t s, int64_t nrows, int ncols, int64_t K, const double* A, int64_t sai,
                  int64_t sak, const double* B, int64_t sbk, int64_t sbr, const double* d,
                  double alpha, double beta, double* out, int64_t ldo, double* work = nullptr,
                  int64_t work_len = 0);
// The arguments of one rowdot product.
struct RowdotArgs {
  int64_t nrows;
  int ncols;
  int64_t K;
  const double* A;
  int64_t sai, sak;
  const double* B;
  int64_t sbk, sbr;
  const double* d;
  double alpha, beta;
  double* out;
  int64_t ldo;
};
// Two independent rowdot products (neither writes what the other reads) in
// one launch of the row kernel and at most one of the split reduction, each
// with half of work; products the tall or Gram-type kernels take run one
// after the other.
hipError_t rowdot_pair(hipStream_t s, const RowdotArgs& x, const RowdotArgs& y, double* work,
                       int64_t work_len);

// One-workgroup solve of N X = Bm for SPD N (N: n x n, Bm: n x nrhs, both
// row-major; Bm is overwritten by the solution, N by its Cholesky factor for
// n > 96 or nrhs > 32, else left as it was: Gauss-Jordan in LDS); work: n doubles.
hipError_t spd_solve_small(hipStream_t s, double* N, int n, double* Bm, int nrhs, double* work,
                           int* info);

hipError_t fill_f64(hipStream_t s, double* p, int64_t n, double v);
// Set-up of one ALS call in one launch: F0[0, nf) = src, lam0[0, nl) = lam_src
// (ones if null), flags[0, P) = 0, ctr[0, nctr) = 0 and *err = 0 (either
// skipped if null).
hipError_t als_prep(hipStream_t s, int64_t nf, double* F0, const double* src, int64_t nl,
                    double* lam0, const double* lam_src, int P, int* flags, unsigned* ctr,
                    int nctr, int* err);
hipError_t fill_i32(hipStream_t s, int* p, int64_t n, int v);
hipError_t convert_f64_to_f32(hipStream_t s, const double* in, float* out, int64_t n);
// y[i] += x[i]
// Eq. 2 update: Y_p += Z_p for every replica p whose zbad[p] is zero (n
// values per replica); a replica left out sets bit 0 of *health.
hipError_t update_masked(hipStream_t s, void* Y, const void* Z, int P, int64_t n, bool f64,
                         const int* zbad, int* health);
// ALS commit: a replica whose flags show a failed solve or barrier, or whose
// factors or weights are not finite, gets its starting factors F0 / lam0 back
// (flags bits 2 and 3 as documented in octen.h) and sets bit 1 of *health.
hipError_t als_commit(hipStream_t s, int P, int QR3, int R, double* F, double* lam,
                      const double* F0, const double* lam0, int* flags, int* health);
// X[i][j] *= v[j] (rows x cols)
hipError_t scale_cols(hipStream_t s, double* X, int64_t rows, int64_t cols, const double* v);
// X[i][j] *= v[i] * v[j] (n x n)
hipError_t scale_rows_cols(hipStream_t s, double* X, int64_t n, const double* v);
// X[i][j] *= v[i] (rows x cols)
hipError_t scale_rows(hipStream_t s, double* X, int64_t rows, int64_t cols, const double* v);

// ----------------------------------------------------------- compression ---
struct CompressShape {
  int64_t I, J;
  int P, Q, S, M1;
};
// Generic FP64-accumulating compression (reference path, any dtype of X):
// M[k][p][Q][Q] for k in [0, t) via T2 = X V (chunked), then
// Z[p] = sum_k M[k][p] (x) W_p(k, :).
hipError_t compress_reference(hipStream_t s, const CompressShape& sh, const void* X, bool x_f64,
                              int64_t t, const double* U, const double* V, const double* W,
                              double* T2work, int64_t t2_rows_cap, double* Mwork, void* Z,
                              bool z_f64, int* zbad);

// Mode-3 product and store: Z[p][a][b][c] = sum_k M[k][p][a][b] * W[k][col_p(c)].
// M is f32 or f64 ([t][P][Q][Q]); Z f32 or f64.  zbad[p] |= 1 when replica p
// receives a non-finite value (zbad is not cleared here).
hipError_t compress_mode3(hipStream_t s, const CompressShape& sh, int64_t t, const void* M,
                          bool m_f64, const double* W, void* Z, bool z_f64, int* zbad);

// Same with per-row-block partials Mpart [t][nrb][P][Q][Q] f32 summed first.
hipError_t compress_mode3_partials(hipStream_t s, const CompressShape& sh, int64_t t, int nrb,
                                  const float* Mpart, const double* W, float* Z, int* zbad);

// MFMA path (f32 or bf16 inputs, f32 accumulate) for dense f32 slices.
struct MfmaPlan;
// G_request: replicas per column block (<= 0: as many as fit, the default)
hipError_t mfma_plan_create(const CompressShape& sh, int in_kind /*1=f32, 2=bf16, 3=bf16x2*/, const double* U,
                            const double* V, hipStream_t s, MfmaPlan** out, int G_request = 0);
int mfma_plan_max_G(const CompressShape& sh, int in_kind);
int mfma_plan_G(const MfmaPlan* p);
// kernel variant: 0 pipelined (direct-to-LDS loads), 1 register-staged with
// 16-byte loads, 2 register-staged scalar loads (any J, any alignment)
void mfma_plan_set_variant(MfmaPlan* p, int variant);
int mfma_plan_variant(const MfmaPlan* p);
void mfma_plan_destroy(MfmaPlan* p);
size_t mfma_workspace_bytes(const MfmaPlan* p, int64_t t);
// Modes 1 and 2: partial M per row block into work.
hipError_t compress_mfma_main(hipStream_t s, const MfmaPlan* plan, const float* X, int64_t t,
                              const float* slice_scale, void* work);
// Sum of partials and mode 3 into Z.
hipError_t compress_mfma_mode3(hipStream_t s, const MfmaPlan* plan, int64_t t, const double* W,
                               const void* work, float* Z, int* zbad);

// ------------------------------------------------------------------- ALS ---
// One workgroup per replica; Y is [P][Q][Q][Q] (f32 or f64).
hipError_t als_reference(hipStream_t s, const void* Y, bool y_f64, int P, int Q, int R,
                         const double* init, double* F, double* lam, int* iters, int* flags,
                         int max_iters, double tol);

// Many workgroups per replica, slabs of X_p in LDS, cooperative launch.
// slots: [2][P][NW][als_coop_slot_len] f64; counters: [2][P]; err: [1].
inline int als_coop_slot_len(int Q, int R) { return Q * R + R * R + 8; }
// slab_global: the slab is read from Y in global memory instead of LDS.
// allow_local: replicas whose workgroups all run on one XCD synchronise
// through its L2 without device-wide write-back and invalidation.
// split (float summaries): the contractions on two-term bfloat16 operands.
size_t als_coop_lds_bytes(int Q, int R, int NW, bool x_f64, bool slab_global, bool split);
// cleared: counters and err are already zero (als_prep), else cleared here.
hipError_t als_coop(hipStream_t s, const void* Y, bool y_f64, int P, int Q, int R, int NW,
                    bool slab_global, const double* init, double* F, double* lam, int* iters,
                    int* flags, double* slots, unsigned* counters, int* err, int max_iters,
                    double tol, bool allow_local, bool split, bool cleared = false);
// One handle's cooperative ALS (the arguments of als_coop), for als_coop_group.
struct AlsCoopItem {
  const void* Y;
  bool y_f64;
  int P, Q, R, NW;
  bool slab_global;
  const double* init;
  double* F;
  double* lam;
  int* iters;
  int* flags;
  double* slots;
  unsigned* counters;
  int* err;
  int max_iters;
  double tol;
  bool allow_local, split;
};
// The cooperative ALS of n handles (counters and err already zero): handles
// of the same kernel form (any rank) share a launch while all their
// workgroups fit on the device at once, up to 16 per launch.
// launches: NULL or the number of cooperative launches made.
hipError_t als_coop_group(hipStream_t s, const AlsCoopItem* items, int n, int* launches);

// -------------------------------------------------------------- recovery ---
// lambda^(1/3), anchor similarity, exclusive greedy matching, scale alignment.
hipError_t rec_align(hipStream_t s, int P, int Q, int R, int S, const double* F,
                     const double* lam, double* aligned, int* perm, double* margin);
// rhs[n][M1][R] from aligned [P][3][Q][R].
hipError_t rec_stack(hipStream_t s, int P, int Q, int R, int S, const double* aligned, double* rhs);
// Canonical columns: out = X / (norm * sign of largest-magnitude entry);
// kfac[r] = norm * sign.  X, out: [n][R].
hipError_t rec_canon(hipStream_t s, int64_t n, int R, const double* X, double* out, double* kfac,
                     double* work, int64_t work_len);
// Pairing with the previous canonical factors: cross [2][R][R] = (Ac^T Ap, Bc^T Bp),
// norms [4][R] = column norms of Ac, Ap, Bc, Bp.  Writes tperm, tsign.
hipError_t rec_col_norms(hipStream_t s, int64_t n, int R, const double* X, double* norms,
                         double* work, int64_t work_len);
// Column norms of Ac, Ap ([nA][R]) and Bc, Bp ([nB][R]) into norms [4][R],
// one launch when all columns are short.
hipError_t rec_col_norms4(hipStream_t s, int64_t nA, int64_t nB, int R, const double* Ac,
                          const double* Ap, const double* Bc, const double* Bp, double* norms,
                          double* work, int64_t work_len);
// rec_canon of (XA [nA][R] -> outA, kA) and (XB [nB][R] -> outB, kB), one
// launch when both are short.
hipError_t rec_canon2(hipStream_t s, int64_t nA, int64_t nB, int R, const double* XA,
                      double* outA, double* kA, const double* XB, double* outB, double* kB,
                      double* work, int64_t work_len);
// Three device-to-device copies of n1, n2, n3 doubles in one launch.
hipError_t rec_copy3(hipStream_t s, double* d1, const double* s1, int64_t n1, double* d2,
                     const double* s2, int64_t n2, double* d3, const double* s3, int64_t n3);
hipError_t rec_tmatch(hipStream_t s, int R, const double* cross, const double* norms, int* tperm,
                      double* tsign, double* tmargin);
// Hcur = H[:, tperm] * tsign; rhs_c = rhs2 - Hcur / kappa; kappa = ka * kb.
hipError_t rec_temporal_prep(hipStream_t s, int M1, int R, const double* H, const int* tperm,
                             const double* tsign, const double* ka, const double* kb, double* kappa,
                             double* Hcur, const double* rhs2, double* rhs_c, int have_prev);
// Cnew *= kappa (column scaling), Chist rows [0, Kold) permuted/sign-fixed via
// tmp, Cnew appended at row Kold.
hipError_t rec_temporal_finish(hipStream_t s, int R, int64_t Kold, int64_t t, const double* kappa,
                               const int* tperm, const double* tsign, double* Cnew, double* Chist,
                               double* tmp, int have_prev);
// Row weights of the deduplicated stack: sqrt(P) on the first S rows.
hipError_t rec_weights(hipStream_t s, int M1, int S, int P, double* w, double* w2);

// ---------------------------------------------------------------- sparse ---
// COO batches by (k, i, j).  bad |= 1 for a coordinate outside
// [0,t) x [0,I) x [0,J), |= 2 for an order violation (if check_order).
hipError_t coo_check(hipStream_t s, int64_t nnz, const int* k, const int* i, const int* j,
                     int64_t t, int64_t I, int64_t J, bool check_order, int* bad);
// Ints of scratch needed by coo_segments.
size_t coo_work_ints(int64_t nnz);
// Stable sort of a COO batch by (k, i, j) into ko, io, jo, vo (equal
// coordinates keep their input order).  Coordinates must be in range (see
// coo_check); the packed key needs coo_sort_key_bits(t, I, J) <= 64 bits,
// else hipErrorInvalidValue.  work: coo_sort_work_bytes(nnz) bytes.
size_t coo_sort_work_bytes(int64_t nnz);
int coo_sort_key_bits(int64_t t, int64_t I, int64_t J);
hipError_t coo_sort(hipStream_t s, int64_t nnz, const int* k, const int* i, const int* j,
                    const float* v, int64_t t, int64_t I, int64_t J, void* work, int* ko, int* io,
                    int* jo, float* vo);
// Segments = distinct (k, i) pairs in input order: seg_start [nseg + 1]
// (last = nnz), seg_row, seg_slice [nseg], slice_seg [t + 1]; nseg_dev gets
// the count.  Arrays sized for nseg = nnz.
hipError_t coo_segments(hipStream_t s, int64_t nnz, const int* k, const int* i, int64_t t,
                        int* work, int* seg_start, int* seg_row, int* seg_slice, int* slice_seg,
                        int* nseg_dev);
// M[k][p][Q][Q] (f64 or f32, with U, V of the same type, [n][M1]) from the
// segments; one workgroup per (slice, replica).
hipError_t coo_compress(hipStream_t s, bool f64, int64_t t, int P, int Q, int S, int M1,
                        const int* seg_start, const int* seg_row, const int* slice_seg,
                        const int* j, const float* v, const void* Vm, const void* Um, void* Mout);
// out3 = (sum v^2, sum v * Xh, sum (A^T A)*(B^T B)*(C[0:kc]^T C[0:kc])); G: 3 R^2
// doubles, partials: 2 * nparts doubles.
hipError_t fit_coo(hipStream_t s, int64_t nnz, const int* k, const int* i, const int* j,
                   const float* v, int64_t k0, int64_t I, int64_t J, int64_t kc, int R,
                   const double* A, const double* B, const double* C, double* G, double* partials,
                   int nparts, double* out3);

// ------------------------------------------------------------ warm start ---
// Offsets of the MLP parameters in the flat FP32 buffer:
// W1 [nh][nin], b1 [nh], W2 [nh][nh], b2 [nh], W3 [nout][nh], b3 [nout].
struct MlpLayout {
  int nin, nh, nout;
  int64_t W1, b1, W2, b2, W3, b3, total;
};
int64_t mlp_param_count(int nin, int nh, int nout);
MlpLayout mlp_layout(int nin, int nh, int nout);
// Y = X[:, :nout] + W3 relu(W2 relu(W1 X + b1) + b2) + b3; H1, H2: [n][nh]
hipError_t mlp_forward(hipStream_t s, const MlpLayout& L, const float* w, const float* X, int64_t n,
                       float* H1, float* H2, float* Y);
// gradients of a loss with dL/dY given (activations from mlp_forward)
hipError_t mlp_backward(hipStream_t s, const MlpLayout& L, const float* w, const float* X,
                        int64_t n, const float* H1, const float* H2, const float* dY, float* dZ2,
                        float* dZ1, float* grad);
// loss = mean (Y - T)^2 (device double), dY = 2 (Y - T) / cnt
hipError_t mlp_mse(hipStream_t s, const float* Y, const float* T, int64_t cnt, float* dY,
                   double* partials, int nparts, double* loss);
hipError_t mlp_adam(hipStream_t s, float* w, const float* g, float* m, float* v, int64_t n,
                    float lr, float beta1, float beta2, float eps, int64_t step);
// sketch sk[p] = G vec(Z_p) / ||Z_p||, G: [D][Q^3] f32, D <= 32
int64_t ws_sketch_part_len(int P, int Q, int D);
hipError_t ws_sketch(hipStream_t s, const void* Z, bool z_f64, int P, int Q, const float* G, int D,
                     double* part, int64_t part_cap, float* sk);
// u [P*R][Q]: change of each mode-3 column caused by the batch Z with the
// mode-1 and mode-2 columns held (lambda^(1/3)-scaled factors)
hipError_t ws_mode3_change(hipStream_t s, const void* Z, bool z_f64, const double* F,
                           const double* lam, int P, int Q, int R, double* u);
// features [P*R][4Q + D] (targets = false; writes signs [P*R][2] and the
// plain scaled start [P][3][Q][R]) or targets [P*R][3Q] (targets = true;
// reads signs) of every column
hipError_t ws_columns(hipStream_t s, const double* F, const double* lam, int P, int Q, int R,
                      const float* sk, const double* u, int D, bool targets, float* out,
                      double* signs, double* plain);
hipError_t ws_candidate(hipStream_t s, const float* Y, const double* signs, int P, int Q, int R,
                        double* cand);
// judge: part [P][2][ws_judge_splits(Q)][2], fits [P][2], keep [P], init [P][3][Q][R]
int ws_judge_splits(int Q);
hipError_t ws_judge(hipStream_t s, const void* Y, bool y_f64, int P, int Q, int R,
                    const double* plain, const double* cand, double* part, double* fits,
                    int* keep, double* init);

// ------------------------------------------------------------------- fit ---
hipError_t fit_dense(hipStream_t s, const void* X, bool x_f64, int64_t t, int64_t I, int64_t J,
                     int R, int64_t k0, const double* A, const double* B, const double* C,
                     double* partials, int nparts, double* out2);

// ---------------------------------------------------------------- N-mode ---
// Kernels of the N-mode extension (layouts in octen_nmode.h), FP64.
// out[p][a][q][b] = sum_i in(p, a, i, b) U[i][col_p(q)], a < pre, i < d,
// b < post, on FP64 matrix cores (d, post < 2^31): in(p, a, i, b) is
// in[p in_stride + (a d + i) post + b], or with `cols`
// in[(a d + i) M1 + col_p(b)] (the product of X with all compression
// columns of the next mode, shared by the replicas).
hipError_t nm_ttm_mfma(hipStream_t s, const double* in, int64_t in_stride, bool cols, int64_t pre,
                       int d, int post, const double* U, int M1, int P, int Q, int S, double* out,
                       int64_t out_stride);
// Z[p][x][c] = sum_k T[p][k][x] W[k][col_p(c)], x < L; zbad[p] |= 1 on a
// non-finite value
hipError_t nm_temporal(hipStream_t s, const double* T, int64_t t_stride, int64_t t, int64_t L,
                       const double* W, int M1, int P, int Q, int S, double* Z, int* zbad);
// Replica ALS, fixed sweeps, several workgroups per replica (cooperative
// launch; one workgroup per replica where that launch is not possible);
// hipErrorInvalidValue when the LDS image does not fit.  work:
// P * nm_als_work_len(N, Q, R, P) doubles (contracted summaries and partial
// contractions); ctr: [P] barrier counters, err: [1] (both cleared here).
size_t nm_als_lds_bytes(int N, int Q, int R);
int64_t nm_als_work_len(int N, int Q, int R, int P);
hipError_t nm_als(hipStream_t s, const double* Y, int P, int N, int Q, int R, const double* init,
                  double* F, double* lam, int* flags, int iters, double* work, unsigned* ctr,
                  int* err);
// lambda^(1/N) on every mode and the anchor matching to replica 0
hipError_t nm_align(hipStream_t s, const double* F, const double* lam, int P, int N, int Q, int R,
                    int S, double* aligned, int* perm, double* margin);
// rhs [N][M1][R] from aligned [P][N][Q][R]
hipError_t nm_stack(hipStream_t s, const double* aligned, int P, int N, int Q, int R, int S,
                    double* rhs);
// kappa[r] = prod_n k[n][r] over nm modes; ones[r] = 1
hipError_t nm_kappa(hipStream_t s, const double* k, int nm, int R, double* kappa, double* ones);
// pairing with the previous batch: cross [nm][R][R], norms [nm][2][R]
hipError_t nm_tmatch(hipStream_t s, const double* cross, const double* norms, int nm, int R,
                     int* tperm, double* tsign, double* tmargin);
// out2 = (sum of squared residuals, sum of squares) of t slices;
// partials: 2 * nparts doubles
hipError_t nm_fit(hipStream_t s, const double* X, int64_t t, const int64_t* dims, int nm,
                  const double* const* A, const double* C, int R, int64_t k0, double* partials,
                  int nparts, double* out2);

}  // namespace octen
