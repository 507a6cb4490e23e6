/*
 * octen.h - C ABI of the MI355X (gfx950) online compressed CP decomposition.
 *
 * The library implements, for a 3-mode tensor that grows along mode 3 in
 * batches of frontal slices, the update of OCTen (Gujral et al., "OCTen:
 * Online Compression-based Tensor Decomposition"):
 *   Sec. 4.1 / Eq. 1   compress the batch into P replicas with random
 *                      multi-mode products sharing S anchor columns,
 *   Sec. 4.1 / Eq. 2   add the compressed batch onto the stored summaries,
 *   Sec. 4.1           fit every replica by rank-R CP-ALS,
 *   Sec. 4.2 / Eq. 5   match replica components through the anchor rows,
 *   Sec. 4.3 / Eq. 6-7 recover the full factors by least squares,
 *   Sec. 5.1           and measure the fitness of the recovered model.
 * Algorithm 1 (supplement) gives the loop these calls make up:
 *   octen_compress_batch -> octen_update_replicas -> octen_cp_als_replicas
 *   -> octen_recover_factors, repeated per batch; octen_fit on demand.
 *
 * Conventions for every call:
 *  - Bulk arrays are DEVICE pointers owned by the caller (row-major, C order).
 *    Arrays named "_host" are host pointers.
 *  - Calls enqueue work on the stream given to octen_init and return without
 *    waiting, except the ones that write a host result (they synchronise the
 *    stream first).  Caller inputs must stay valid until the stream reaches
 *    the call.
 *  - Arguments are validated before anything is launched; on error nothing
 *    is enqueued and the handle state is unchanged.  No exception crosses the
 *    ABI.  octen_last_error() gives a text for the last failure of a handle.
 *  - One handle is used by one host thread at a time.
 *
 * Notation: M1 = S + P*(Q - S) distinct compression columns per mode.
 * Replica p uses compression columns [0, S) (shared anchors, Eq. 1) and
 * [S + p*(Q-S), S + (p+1)*(Q-S)) (its own).
 */
#ifndef OCTEN_H
#define OCTEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCTEN_ABI_VERSION 1

typedef struct octen_ctx* octen_t;

typedef enum {
  OCTEN_OK = 0,
  OCTEN_ERR_ARG = 1,         /* invalid argument (null pointer, bad size) */
  OCTEN_ERR_STATE = 2,       /* call out of order (e.g. update before compress) */
  OCTEN_ERR_HIP = 3,         /* HIP runtime error; see octen_last_error */
  OCTEN_ERR_NOMEM = 4,       /* device allocation failed */
  OCTEN_ERR_NUMERIC = 5,     /* non-finite values or a failed solve */
  OCTEN_ERR_UNSUPPORTED = 6  /* valid request the library does not implement */
} octen_status;

/* Element and arithmetic types.  OCTEN_BF16X2 is the two-term bfloat16 form
 * of the compression: every slice value x enters the matrix cores as
 * hi = bf16(x) and lo = bf16(x - hi) (16 significant bits), both multiplied
 * into float32 accumulators, and the intermediate mode-2 product is carried
 * into the mode-1 product the same way; it needs compression matrices whose
 * entries are bfloat16 values.  (Value 3 is not used.) */
typedef enum {
  OCTEN_F64 = 0,
  OCTEN_F32 = 1,
  OCTEN_BF16 = 2,
  OCTEN_BF16X2 = 4
} octen_dtype;

/* ALS starting point (octen_cp_als_replicas). */
enum { OCTEN_INIT_GIVEN = 0, OCTEN_INIT_PREV = 1, OCTEN_INIT_LEARNED = 2 };

/* Internal arrays readable through octen_get_state (for tests). */
enum {
  OCTEN_STATE_Y = 0,        /* [P][Q][Q][Q] summaries, accumulation type      */
  OCTEN_STATE_Z = 1,        /* [P][Q][Q][Q] last compressed batch             */
  OCTEN_STATE_FACTORS = 2,  /* [P][3][Q][R] f64 replica factors, unit columns */
  OCTEN_STATE_LAMBDA = 3,   /* [P][R] f64 replica weights                     */
  OCTEN_STATE_PERM = 4,     /* [P][R] int32: replica column r -> reference    */
  OCTEN_STATE_ALIGNED = 5,  /* [P][3][Q][R] f64 aligned replica factors       */
  OCTEN_STATE_RHS = 6,      /* [3][M1][R] f64 deduplicated stacked factors    */
  OCTEN_STATE_H = 7,        /* [M1][R] f64 temporal carry W_old^T C_old       */
  OCTEN_STATE_TPERM = 8,    /* [R] int32 column pairing with previous batch   */
  OCTEN_STATE_ITERS = 9,    /* [P] int32 ALS sweeps done                      */
  OCTEN_STATE_MARGIN = 10,  /* [P] f64 matching margin (replica 0: +inf)      */
  OCTEN_STATE_FLAGS = 11,   /* [P] int32 replica flags of the last ALS call:
                               bit0 a normal-equation solve met a
                               non-positive pivot, bit1 a barrier between the
                               replica's workgroups timed out, bit2 factors or
                               weights not finite, bit3 the replica was not
                               committed (its starting factors were kept)   */
  /* bookkeeping of the last sparse batch (octen_compress_batch_coo); a
   * segment is one distinct (k, i) pair, numbered in input order */
  OCTEN_STATE_COO_SIZES = 12,     /* [2] int32: nseg, t                      */
  OCTEN_STATE_COO_SEG_START = 13, /* [nseg+1] int32 first nonzero of each
                                     segment, then nnz                       */
  OCTEN_STATE_COO_SEG_ROW = 14,   /* [nseg] int32 row i of each segment      */
  OCTEN_STATE_COO_SLICE_SEG = 15, /* [t+1] int32 first segment of each slice,
                                     then nseg                               */
  /* last learned warm start (OCTEN_INIT_LEARNED) */
  OCTEN_STATE_WARM_KEEP = 16,     /* [P] int32: 1 = network start kept       */
  OCTEN_STATE_WARM_FITS = 17      /* [P][2] f64 replica fit of the plain and
                                     of the network start                    */
};

/* Flags (octen_config.flags). */
#define OCTEN_FLAG_REFERENCE_PATH 0x2ull /* plain FP64 kernels, no MFMA       */
#define OCTEN_FLAG_TIMING 0x4ull         /* record HIP events around stages   */
#define OCTEN_FLAG_ALS_ONE_WG 0x8ull     /* ALS: one workgroup per replica, no
                                            cooperative launch (group steps
                                            always run this way)              */
#define OCTEN_FLAG_ALS_DEVICE_SYNC 0x10ull /* ALS: the barriers between the
                                            workgroups of a replica always
                                            write back and invalidate the L2,
                                            also where all of them run on one
                                            XCD (same results, slower)        */
#define OCTEN_FLAG_ALS_FEW_WG 0x20ull    /* ALS: the fewest workgroups per
                                            replica whose slab fits in LDS
                                            (default: enough to spread about
                                            2e5 FMAs per workgroup and sweep);
                                            for handles of a group, whose
                                            cooperative ALS then share launches
                                            with more handles;
                                            octen_autotune_als replaces the
                                            choice by its timed one         */

/* Stages timed with OCTEN_FLAG_TIMING (octen_stage_time). */
enum {
  OCTEN_STAGE_COMPRESS_MAIN = 0,   /* modes 1 and 2 of the compression kernel */
  OCTEN_STAGE_COMPRESS_MODE3 = 1,  /* mode-3 product (and partial sums)       */
  OCTEN_STAGE_UPDATE = 2,
  OCTEN_STAGE_ALS = 3,
  OCTEN_STAGE_RECOVER = 4,
  OCTEN_STAGE_COO_INDEX = 5,       /* checks and segments of a sparse batch   */
  OCTEN_NUM_STAGES = 6
};

typedef struct {
  int32_t abi_version;     /* must be OCTEN_ABI_VERSION                        */
  int32_t R;               /* CP rank (Sec. 2), 1 <= R <= 32                   */
  int32_t P;               /* number of replicas p (Sec. 4.1), P >= 1          */
  int32_t Q;               /* replica side Q (Sec. 4.1), S < Q <= 128, R <= Q  */
  int32_t S;               /* shared anchor columns (Eq. 1), S >= 1            */
  int32_t x_dtype;         /* element type of X: OCTEN_F64 or OCTEN_F32        */
  int32_t compress_dtype;  /* compression arithmetic: F64, F32, BF16 or BF16X2
                              inputs; accumulation is F64 for F64, else F32;
                              BF16X2 needs U and V on the bfloat16 grid
                              (OCTEN_ERR_ARG otherwise); any other value
                              gives OCTEN_ERR_UNSUPPORTED                     */
  int32_t als_dtype;       /* arithmetic of the two slab contractions of the
                              replica ALS (Sec. 4.1; Y x3 C and the mode-3
                              MTTKRP): OCTEN_F64, or OCTEN_BF16X2 = both
                              operands as two-term bfloat16 expansions,
                              products hi*hi + lo*hi + hi*lo, float32 sums
                              (needs a narrow compress_dtype, so the
                              summaries are float32, and the cooperative ALS:
                              not with OCTEN_FLAG_ALS_ONE_WG or
                              OCTEN_FLAG_REFERENCE_PATH);
                              anything else gives OCTEN_ERR_UNSUPPORTED.
                              R x R solves and recovery are always F64        */
  int64_t I;               /* mode-1 size I (problem statement, Sec. 3)        */
  int64_t J;               /* mode-2 size J                                    */
  uint64_t flags;          /* OCTEN_FLAG_*                                     */
} octen_config;

/* Create a handle.  U: [I][M1] f64, V: [J][M1] f64 device arrays, the fixed
 * mode-1 and mode-2 compression matrices in deduplicated layout (shared
 * columns first, then each replica's own; Eq. 1).  They are copied; the
 * least-squares operators of Eq. 7 for modes 1 and 2 are built here once.
 * stream: a hipStream_t (NULL = default stream).  Summaries start at zero. */
octen_status octen_init(const octen_config* cfg, const double* U, const double* V,
                        void* stream, octen_t* out);

/* Sec. 4.1 compression of one batch: Z_p = X x1 U_p^T x2 V_p^T x3 W_p^T.
 * X: [t][I][J] in cfg.x_dtype (frontal slices, j fastest).  W: [t][M1] f64,
 * the batch's mode-3 compression rows.  slice_scale: NULL or [t] f32 powers of
 * two applied to slice k before rounding to a narrow type and undone exactly
 * after the contraction (needed for F16 range; no effect on F32/F64).
 * Replaces the previous batch's Z. */
octen_status octen_compress_batch(octen_t h, const void* X, int64_t t, const double* W,
                                  const float* slice_scale);

/* Sec. 4.1 compression of the next batch, overlapped with the current one
 * (same arguments and result as octen_compress_batch).  The kernels run on a
 * second stream of the handle (default priority, created on first use) once
 * everything enqueued on the handle stream before this call has finished, so
 * work enqueued after it (the ALS and recovery of the batch added just
 * before) runs concurrently on the CUs the cooperative ALS leaves free.  The
 * handle stream waits for the compression at the next call that reads or
 * rewrites Z, W or the compression workspace (octen_update_replicas, the
 * compress calls, octen_get_state, octen_autotune, octen_compress_variant,
 * the learned warm start).  Replaces the previous batch's Z: call it after
 * octen_update_replicas of that batch.  Stage times of the compression are
 * taken on the second stream.  Errors as octen_compress_batch, plus
 * OCTEN_ERR_HIP when the stream or its events cannot be created. */
octen_status octen_compress_batch_async(octen_t h, const void* X, int64_t t, const double* W,
                                        const float* slice_scale);

/* Same for a sparse batch given as COO with slice indices k in [0, t)
 * relative to the batch.  k, i, j: [nnz] int32, v: [nnz] f32, all device
 * arrays (read only); 0 <= nnz < 2^31.  Duplicated coordinates add up.  The
 * coordinates are checked on the device first (synchronises): OCTEN_ERR_ARG
 * if one is out of range.  A batch not ordered by k, then i, then j is
 * sorted on the device into arrays of the handle (a stable radix sort:
 * equal coordinates keep their order; OCTEN_ERR_UNSUPPORTED if the packed
 * key ceil(log2 t) + ceil(log2 I) + ceil(log2 J) exceeds 64 bits).  The
 * summaries are dense (Sec. 4.1): f64 arithmetic for compress_dtype F64,
 * f32 gathers and MFMA f32 accumulation otherwise (also for BF16). */
octen_status octen_compress_batch_coo(octen_t h, int64_t nnz, const int32_t* k,
                                      const int32_t* i, const int32_t* j, const float* v,
                                      int64_t t, const double* W);

/* Eq. 2: Y_p += Z_p for every replica; the slice count K grows by t. */
octen_status octen_update_replicas(octen_t h);

/* Conditions a handle records on the device (asynchronous calls cannot
 * return them) until a synchronising call reports them:
 *  OCTEN_HEALTH_NONFINITE_BATCH  a compressed batch held non-finite values
 *      (a NaN or Inf slice value): octen_update_replicas left the summaries
 *      of the replicas concerned unchanged (the slices still count in K);
 *  OCTEN_HEALTH_ALS_FAILED       octen_cp_als_replicas met a failed solve,
 *      a barrier time-out or non-finite factors in some replica: that
 *      replica keeps its starting factors (OCTEN_STATE_FLAGS bit 3).
 * octen_cp_als_replicas with iters_done_host, octen_recover_factors with
 * K_out_host and octen_health return OCTEN_ERR_NUMERIC when any bit is set,
 * and clear the bits. */
#define OCTEN_HEALTH_NONFINITE_BATCH 0x1
#define OCTEN_HEALTH_ALS_FAILED 0x2

/* Waits for the handle's work, writes the health bits recorded since the
 * last report to *bits_host (may be NULL) and clears them: OCTEN_OK when
 * none is set, OCTEN_ERR_NUMERIC otherwise. */
octen_status octen_health(octen_t h, int32_t* bits_host);

/* Sec. 4.1: rank-R CP-ALS of every replica summary.  Gauss-Seidel sweeps
 * over modes 1, 2, 3; each mode solves the R x R normal equations in f64
 * (Cholesky) and scales the columns to unit 2-norm; lambda = norms of mode 3.
 * max_iters >= 1 sweeps, or fewer when tol > 0 and the replica fit changes by
 * less than tol in one sweep.  init_mode OCTEN_INIT_GIVEN: init is
 * [P][3][Q][R] f64 (device); OCTEN_INIT_PREV: start from the factors of the
 * previous call (init ignored); OCTEN_INIT_LEARNED: start from the network
 * set by octen_warmstart_set where its start fits the updated summary at
 * least as well as the previous factors do, else from those (init ignored;
 * the choice per replica is readable as OCTEN_STATE_WARM_KEEP).
 * iters_done_host: NULL or [P] host int32 (synchronises, and then reports
 * the health bits: OCTEN_ERR_NUMERIC if a replica failed).  A replica whose
 * solve meets a non-positive pivot, whose barrier times out or whose factors
 * are not finite is not committed: it keeps its starting factors. */
octen_status octen_cp_als_replicas(octen_t h, int32_t max_iters, double tol, int32_t init_mode,
                                   const double* init, int32_t* iters_done_host);

/* Sec. 4.2 and 4.3 / Eq. 5-7: distribute lambda^(1/3), align every replica
 * to replica 0 through the anchor rows, stack, and solve for the factors in
 * f64 (minimum-norm least squares).  Outputs, all f64 device arrays:
 * A: [I][R], B: [J][R] with unit-norm columns whose largest-magnitude entry is
 * positive, and C: [K][R] (all slices seen so far; the columns of earlier
 * rows follow the current A, B).  c_capacity: rows available in C (>= K).
 * K_out_host: NULL or host int64 (synchronises, and then reports the health
 * bits as octen_health does). */
octen_status octen_recover_factors(octen_t h, double* A, double* B, double* C,
                                   int64_t c_capacity, int64_t* K_out_host);

/* Sec. 5.1 fitness terms over the slices X [t][I][J] (cfg.x_dtype) with global
 * slice index k0..k0+t-1: out_host[0] += sum (X - [[A,B,C]])^2,
 * out_host[1] += sum X^2, accumulated in f64 (synchronises).
 * fit = 1 - sqrt(out[0] / out[1]) over all slices. */
octen_status octen_fit(octen_t h, const void* X, int64_t t, int64_t k0, const double* A,
                       const double* B, const double* C, double* out_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the dense
 * fitness terms of octen_fit without a handle and without any allocation,
 * through the same kernels.  X: [t][I][J] device array of x_dtype
 * (OCTEN_F64 or OCTEN_F32); A: [I][R], B: [J][R], C: [k0 + t][R] f64 device
 * arrays (slice k of X is row k0 + k of C); stream: a hipStream_t of the
 * current device (NULL = default stream).  out_host[0] += sum (X - [[A,B,C]])^2,
 * out_host[1] += sum X^2 (synchronises the stream).  The block partial sums
 * live in a fixed device array of 2 * 2048 + 2 doubles (32 KiB) that the
 * library keeps on every device it has run on until the process ends (at
 * most 2048 blocks are launched, so no input size overflows it); calls that
 * overlap on one device race on that array.  OCTEN_ERR_ARG for null
 * pointers, t, I or J < 1, k0 < 0, R outside [1, 32], t * I >= 2^40 or
 * another x_dtype; OCTEN_ERR_HIP when the array's address cannot be taken
 * or a launch or copy fails. */
octen_status octen_fit_noalloc(const void* X, int32_t x_dtype, int64_t t, int64_t I, int64_t J,
                               int32_t R, int64_t k0, const double* A, const double* B,
                               const double* C, void* stream, double* out_host);

/* Sec. 5.1 fitness of a sparse tensor through
 * ||X - Xh||^2 = ||X||^2 - 2 <X, Xh> + sum((A^T A) * (B^T B) * (C^T C)).
 * Nonzeros as in octen_compress_batch_coo (bounds are checked, order is not),
 * slice k of the nonzeros is row k0 + k of C, k0 + k < kc.  out_host (f64,
 * synchronises): [0] += sum v^2, [1] += sum v * Xh over the given nonzeros;
 * [2] = sum of (A^T A) * (B^T B) * (C^T C) with C over its rows [0, kc)
 * (set, not accumulated).  Over all nonzeros of the tensor:
 * fit = 1 - sqrt(max(out[0] - 2 out[1] + out[2], 0) / out[0]). */
octen_status octen_fit_coo(octen_t h, int64_t nnz, const int32_t* k, const int32_t* i,
                           const int32_t* j, const float* v, int64_t k0, const double* A,
                           const double* B, const double* C, int64_t kc, double* out_host);

/* Copy one internal array (OCTEN_STATE_*) into dst (device), bytes must be
 * at least its size. */
octen_status octen_get_state(octen_t h, int32_t what, void* dst, size_t bytes);

/* Host-only identifiability verdicts (Eq. 4, Eq. 8): bit0 Eq. 8 holds,
 * bit1 M1 >= I, bit2 M1 >= J, bit3 M1 >= t, bit4 Eq. 4 with generic Kruskal
 * ranks.  A violation is not an error: recovery is then minimum-norm. */
octen_status octen_check_identifiable(const octen_config* cfg, int64_t K, int64_t t,
                                      int32_t* bits_host, double* p_min_host);

/* Durations in milliseconds of the most recent runs of one stage, from HIP
 * events recorded on the handle's stream around the stage's kernels (needs
 * OCTEN_FLAG_TIMING; the last OCTEN_TIMING_RING runs are kept, no
 * synchronisation happens while they are recorded).  Writes at most n values,
 * oldest first, into ms_host and their number into count_host; synchronises. */
#define OCTEN_TIMING_RING 256
octen_status octen_stage_times(octen_t h, int32_t stage, double* ms_host, int32_t n,
                               int32_t* count_host);

/* Release every device buffer of the handle (synchronises its stream). */
octen_status octen_destroy(octen_t h);

const char* octen_status_str(octen_status s);
const char* octen_last_error(octen_t h);
int32_t octen_abi_version(void);

/* ---- Tuning and batched steps (not in the paper).
 *
 * octen_autotune: times the compression kernel variants on the batch X
 * ([t][I][J] f32, as octen_compress_batch) -- 0 pipelined direct-to-LDS
 * loads, 1 register-staged 16-byte loads, 2 register-staged scalar loads,
 * 3 (BF16 only) half chunks with the next chunk's fragments read during the
 * current chunk's MFMAs -- for the default and for half the replicas per
 * column block, and keeps the fastest for this handle.  choice_host: NULL or
 * 10 * replicas_per_block + variant.
 * Only handles with F32 or BF16 compression are tuned (else
 * OCTEN_ERR_UNSUPPORTED).  Synchronises. */
octen_status octen_autotune(octen_t h, const void* X, int64_t t, int32_t* choice_host);

/* octen_compress_variant: selects one of the compression kernel variants
 * above (0..3) for this handle without timing (for callers that know their
 * shapes, and for checking the variants against each other).  A variant
 * that needs 16-byte rows falls back to 2 on a batch with J % 4 != 0 or an
 * unaligned X.  OCTEN_ERR_ARG for a variant outside [0, 3];
 * OCTEN_ERR_UNSUPPORTED for a handle without F32 or BF16 compression, or
 * variant 3 on a handle without BF16 compression. */
octen_status octen_compress_variant(octen_t h, int32_t variant);

/* Times the cooperative ALS for `sweeps` sweeps on the current summaries with
 * each workgroups-per-replica count that is the smallest one for its slab
 * height ceil(Q / count) (at most the CUs of one XCD per replica), with the
 * replica slab in LDS or in global memory, starting from the current factors;
 * three interleaved rounds, the best time of each candidate counts; keeps the
 * fastest and restores the factors afterwards.  choice_host: NULL or
 * 10 * workgroups + (1 if the slab is in global memory).  Needs factors from
 * an earlier ALS call.  Synchronises. */
octen_status octen_autotune_als(octen_t h, int32_t sweeps, int32_t* choice_host);

/* A group runs one update step (compress, update, ALS) of many handles as
 * one captured HIP graph: each handle's launches form a parallel branch.
 * The first step with given descriptors captures the graph; later steps
 * with the same descriptors (pointers and depths), the same ALS settings and
 * the same handle state replay it, otherwise the graph is captured again.
 * The caller rewrites the batch buffers in place between steps.  Every
 * handle must share one stream and hold replica factors already (its first
 * batch goes through its own calls).  Handles
 * whose ALS is a cooperative grid run it after the branches join (no
 * cooperative grid shares the GPU with other work of the step): handles
 * whose ALS runs the same kernel form (summary precision, contraction form
 * and slab placement; any rank) share one cooperative launch, up to 16
 * handles, while all their workgroups fit on the device at once.  The others
 * (OCTEN_FLAG_ALS_ONE_WG, or replicas too large) run it in their branch, one
 * workgroup per replica.
 * Recovery stays outside the graph: per handle, or for all handles at once
 * with octen_group_recover. */
typedef struct octen_group* octen_group_t;
typedef struct {
  const void* X;            /* [t][I][J] in the handle's x_dtype (device)      */
  int64_t t;                /* slices in the batch                              */
  const double* W;          /* [t][M1] f64 mode-3 compression rows (device)     */
  const float* slice_scale; /* NULL or [t] f32 powers of two                    */
} octen_batch_desc;

/* handles: n distinct handles (1 <= n <= 4096) on one stream.  A handle
 * with als_dtype OCTEN_BF16X2 needs its cooperative ALS after the join (a
 * step whose capture falls back to the branch ALS fails with
 * OCTEN_ERR_UNSUPPORTED for it). */
octen_status octen_group_create(const octen_t* handles, int32_t n, octen_group_t* out);
/* init_mode: OCTEN_INIT_PREV or OCTEN_INIT_LEARNED (every handle then needs
 * a network, octen_warmstart_set).  replayed_host: NULL or 1 when the
 * captured graph was replayed. */
octen_status octen_group_step(octen_group_t g, const octen_batch_desc* desc, int32_t max_iters,
                              double tol, int32_t init_mode, int32_t* replayed_host);
/* Recovery of every handle of the group after a step: octen_recover_factors
 * of handle i with A[i], B[i], C[i], c_capacity[i] (host arrays of n device
 * pointers and n row capacities) and no row count, each handle on a stream
 * of its own that starts after the work already on the handles' stream and
 * is joined back into it, so the handles' recoveries run concurrently.  The
 * results are those of the handle-by-handle calls.  On an error the handles
 * before it have recovered and the error names the handle; the rest have
 * not. */
octen_status octen_group_recover(octen_group_t g, double* const* A, double* const* B,
                                 double* const* C, const int64_t* c_capacity);
/* Number of cooperative ALS launches in the graph of the latest captured
 * step (0 before the first step, or when the ALS runs in the branches). */
octen_status octen_group_als_launches(octen_group_t g, int32_t* out_host);
octen_status octen_group_destroy(octen_group_t g);
const char* octen_group_last_error(octen_group_t g);

/* ---- Learned warm start of the replica ALS (an addition to the method of
 * the paper, whose Algorithm 1 restarts ALS from the previous factors).
 * A residual MLP maps the features of one replica column,
 *   x = [s_a a ; s_b b ; s_a s_b (c + u) ; s_a s_b u ; sketch_p]  (4Q + D)
 * with a, b, c the previous unit columns times lambda^(1/3) (Sec. 4.2),
 * s_a, s_b the signs of the entries of largest magnitude of a and b (first
 * on ties), u = (Z_p x1 a x2 b) / (||a||^2 ||b||^2) the change of the mode-3
 * least-squares column caused by the new batch Z_p with a, b held, and
 * sketch_p = G vec(Z_p) / ||Z_p|| (G: D x Q^3), to
 * y = x[0:3Q] + W3 relu(W2 relu(W1 x + b1) + b2) + b3, a predicted column
 * after ALS.  Products run on BF16 MFMA with FP32 accumulation; parameters,
 * gradients and Adam moments are FP32. */
typedef struct octen_mlp* octen_mlp_t;

/* Number of FP32 parameters; layout W1 [H][In], b1 [H], W2 [H][H], b2 [H],
 * W3 [Out][H], b3 [Out] (weights as [out][in], row-major).  -1 if invalid
 * (needs Out <= In). */
int64_t octen_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out);

/* Create a network from params (device, FP32, the layout above; copied).
 * Adam moments start at zero.  stream: hipStream_t or NULL. */
octen_status octen_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, const float* params,
                              void* stream, octen_mlp_t* out);
octen_status octen_mlp_destroy(octen_mlp_t m);
const char* octen_mlp_last_error(octen_mlp_t m);

/* Y [n][Out] = network(X [n][In]), device FP32, 1 <= n <= 2^24. */
octen_status octen_mlp_forward(octen_mlp_t m, const float* X, int64_t n, float* Y);

/* Gradients of loss = mean over all n * Out entries of (Y - T)^2 with
 * respect to every parameter, into grads (device, the parameter layout);
 * loss_host: NULL or the loss (synchronises). */
octen_status octen_mlp_gradients(octen_mlp_t m, const float* X, const float* T, int64_t n,
                                 float* grads, double* loss_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * given gradients (device, parameter layout). */
octen_status octen_mlp_adam(octen_mlp_t m, const float* grads, float lr);

/* Gradients of the loss above on (X, T), then one Adam step; loss_host: NULL
 * or the loss before the step (synchronises). */
octen_status octen_mlp_train_step(octen_mlp_t m, const float* X, const float* T, int64_t n,
                                  float lr, double* loss_host);

/* Hidden activations relu(W1 x + b1), relu(W2 h1 + b2) [n][H] of the first
 * n rows of the last forward pass (forward, gradients or training step). */
octen_status octen_mlp_last_activations(octen_mlp_t m, int64_t n, float* H1, float* H2);

/* Copy the FP32 parameters into dst (device). */
octen_status octen_mlp_get_params(octen_mlp_t m, float* dst);

/* Attach a network (In = 4Q + D, Out = 3Q; not copied: it must outlive its
 * use by the handle; NULL: features and targets only, for collecting
 * training pairs) and a sketch matrix G [D][Q^3] (device FP32, copied),
 * 1 <= D <= 32; at most 32 replicas (else OCTEN_ERR_UNSUPPORTED). */
octen_status octen_warmstart_set(octen_t h, octen_mlp_t m, const float* G, int32_t D);

/* Features of every replica column (rows ordered replica-major) from the
 * current replica factors and the last compressed batch: X [P*R][4Q+D]
 * device FP32 (NULL: only kept inside the handle).  The signs are kept for
 * octen_warmstart_targets. */
octen_status octen_warmstart_features(octen_t h, float* X);

/* Training targets: the current replica factors (after ALS) as columns
 * lambda^(1/3)-scaled with the signs of the last features: T [P*R][3Q]. */
octen_status octen_warmstart_targets(octen_t h, float* T);

#ifdef __cplusplus
}
#endif
#endif /* OCTEN_H */
