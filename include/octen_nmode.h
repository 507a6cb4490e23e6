/*
 * octen_nmode.h - C ABI of the N-mode extension (supplement of the OCTen
 * paper, "Extending to Higher-Order Tensors"): an N-mode tensor
 * X in R^{I_1 x ... x I_{N-1} x T} growing in its last (temporal) mode, with
 * N - 1 fixed compression matrices for the non-temporal modes and fresh
 * temporal rows per batch.  The steps are those of octen.h written for N
 * modes:
 *   compression     Z_p = X x_1 U1_p^T ... x_{N-1} U(N-1)_p^T x_N W_p^T
 *                   (the compressed cubes of the supplement),
 *   update          Y_p += Z_p (a replica whose Z_p is not finite is left out),
 *   replica CP      Gauss-Seidel ALS over the N modes,
 *   matching        lambda^(1/N) on each mode, anchor similarity over the N
 *                   modes (Sec. 4.2 for N modes),
 *   recovery        the stacked update rule of the supplement: each
 *                   non-temporal mode by the weighted minimum-norm solve of
 *                   its deduplicated stack (Eq. 7 per mode), the temporal
 *                   rows appended with the carried history removed,
 *   fit             Sec. 5.1.
 * Arithmetic: FP64 throughout.  Conventions as in octen.h (device arrays
 * owned by the caller, row-major; calls enqueue on the handle's stream;
 * arguments validated before anything is launched).
 *
 * Layouts: a batch X is [t][I_1]...[I_{N-1}] f64 (the last mode fastest);
 * U_n: [I_n][M1] f64 with M1 = S + P*(Q - S) columns in the deduplicated
 * layout of octen.h; W: [t][M1] f64; replica summaries [P][Q]^N with the
 * temporal index last; replica factors [P][N][Q][R], mode N-1 temporal;
 * recovered factors A_n: [I_n][R], C: [K][R].
 */
#ifndef OCTEN_NMODE_H
#define OCTEN_NMODE_H

#include <stddef.h>
#include <stdint.h>

#include "octen.h"

#ifdef __cplusplus
extern "C" {
#endif

#define OCTEN_NM_MAX_MODES 6

typedef struct octen_nm_ctx* octen_nm_t;

typedef struct {
  int32_t abi_version;   /* OCTEN_ABI_VERSION                                  */
  int32_t N;             /* number of modes, 3 <= N <= OCTEN_NM_MAX_MODES      */
  int32_t R;             /* CP rank, 1 <= R <= 32, R <= Q                      */
  int32_t P;             /* replicas, P >= 1                                   */
  int32_t Q;             /* replica side, S < Q <= 32, Q^N <= 2^22             */
  int32_t S;             /* shared anchor columns, S >= 1                      */
  int64_t dims[OCTEN_NM_MAX_MODES - 1]; /* I_1 .. I_{N-1}, each >= 1          */
} octen_nm_config;

/* Create a handle.  U: host array of N - 1 device pointers, U[n] is
 * [I_{n+1}][M1] f64 (copied).  The least-squares operators of Eq. 7 for the
 * N - 1 non-temporal modes are built here (OCTEN_ERR_NUMERIC when a U[n]
 * lacks full rank).  OCTEN_ERR_ARG for a bad argument,
 * OCTEN_ERR_UNSUPPORTED for sizes outside the limits above (the replica ALS
 * keeps a replica's factors and Grams in the LDS of one workgroup),
 * OCTEN_ERR_NOMEM when device memory runs out.  Device memory: the summaries
 * Y, Z (16 P Q^N bytes), the ALS's partial contractions (about
 * 8 P Q^(N-1) RC (1 + 1/Q) bytes, RC = R rounded up to 8, 16 or 32) and the
 * compression workspace, which grows with the batch: about
 * 8 (t I_1 ... I_{N-2} (M1 + 2 P Q)) bytes. */
octen_status octen_nm_init(const octen_nm_config* cfg, const double* const* U, void* stream,
                           octen_nm_t* out);
/* Compression of one batch: X [t][I_1]...[I_{N-1}] f64, W [t][M1] f64
 * (copied).  t >= 1 and t I_1 ... I_{N-2} < 2^31.  The mode products are
 * taken from the last non-temporal mode to the first, then the temporal
 * mode. */
octen_status octen_nm_compress_batch(octen_nm_t h, const double* X, int64_t t, const double* W);
/* Y_p += Z_p (a replica whose compressed batch holds a non-finite value is
 * not updated; reported as OCTEN_ERR_NUMERIC by octen_nm_recover_factors). */
octen_status octen_nm_update_replicas(octen_nm_t h);
/* iters ALS sweeps per replica (Gauss-Seidel over the N modes; one
 * cooperative launch with up to 8 workgroups per replica, or one workgroup
 * per replica where that launch is not possible).  init_mode
 * OCTEN_INIT_GIVEN with init [P][N][Q][R] f64 (device), or OCTEN_INIT_PREV
 * (the previous factors).  A replica whose solve meets a non-positive pivot,
 * whose barrier timed out or whose factors are not finite keeps its starting
 * factors (OCTEN_STATE_FLAGS bits 0-3 as in octen.h) and is reported as
 * OCTEN_ERR_NUMERIC by the next synchronising octen_nm_recover_factors.
 * OCTEN_ERR_STATE before the first update or without previous factors. */
octen_status octen_nm_cp_als_replicas(octen_nm_t h, int32_t iters, int32_t init_mode,
                                      const double* init);
/* Matching and recovery.  A: host array of N - 1 device pointers
 * ([I_n][R] f64, canonical columns: unit 2-norm, largest-magnitude entry
 * positive), C: [c_capacity][R] f64 receiving all K rows so far.
 * K_out_host: NULL or the number of rows (then the call synchronises and
 * reports OCTEN_ERR_NUMERIC for a non-finite batch or a flagged replica). */
octen_status octen_nm_recover_factors(octen_nm_t h, double* const* A, double* C,
                                      int64_t c_capacity, int64_t* K_out_host);
/* Fitness terms of t slices (global index k0..k0+t-1): out_host[0] += sum of
 * squared residuals, out_host[1] += sum of squares of X (synchronises). */
octen_status octen_nm_fit(octen_nm_t h, const double* X, int64_t t, int64_t k0,
                          const double* const* A, const double* C, double* out_host);
/* Copy an internal array into dst (device), bytes at least its size:
 * OCTEN_STATE_Y, _Z ([P][Q]^N f64), _FACTORS, _ALIGNED ([P][N][Q][R] f64),
 * _LAMBDA ([P][R] f64), _PERM ([P][R] int32), _RHS ([N][M1][R] f64, the
 * deduplicated stack of every mode), _H ([M1][R] f64), _TPERM ([R] int32),
 * _MARGIN ([P] f64), _FLAGS ([P] int32, bits as in octen.h).
 * OCTEN_ERR_ARG for another id or a short destination. */
octen_status octen_nm_get_state(octen_nm_t h, int32_t what, void* dst, size_t bytes);
octen_status octen_nm_destroy(octen_nm_t h);
const char* octen_nm_last_error(octen_nm_t h);

#ifdef __cplusplus
}
#endif

#endif
