// C ABI of libocten: argument validation, handle state and the sequence of
// kernel launches for each step of the online update (Algorithm 1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/octen.h"
#include "mlp_ctx.h"
#include "octen_internal.h"

using namespace octen;

struct octen_ctx {
  octen_config cfg;
  int64_t I = 0, J = 0;
  int R = 0, P = 0, Q = 0, S = 0, M1 = 0;
  hipStream_t stream = nullptr;
  // overlapped compression (octen_compress_batch_async): a second stream of
  // the default priority; ev_z marks the end of the latest compression there
  hipStream_t side = nullptr;
  hipEvent_t ev_main = nullptr, ev_z = nullptr;
  bool z_async = false;       // a compression on the side stream is not joined yet
  bool acc_f64 = true;  // summaries (Y, Z) in f64, else f32
  std::string err;

  // state machine
  bool z_ready = false;       // a compressed batch waits for octen_update_replicas
  int64_t t_z = 0;            // depth of that batch
  int64_t t_pend = 0;         // slices added since the last recovery
  bool have_factors = false;  // replica factors exist
  bool factors_fresh = false; // ALS ran after the last update
  bool have_prev = false;     // a previous recovery exists (canonical A, B)
  int64_t K = 0;              // slices recovered so far (rows of C)

  // fixed operators
  double *U = nullptr, *V = nullptr;       // [I][M1], [J][M1]
  double *OpA = nullptr, *OpB = nullptr;   // [I][M1], [J][M1] least-squares operators
  double *w = nullptr, *w2 = nullptr;      // [M1] row weights
  MfmaPlan* plan = nullptr;

  // summaries
  void *Y = nullptr, *Z = nullptr;         // [P][Q][Q][Q]
  // batch workspace
  double* Wz = nullptr;   int64_t Wz_cap = 0;    // W of the compressed, not yet added batch
  double* Wp = nullptr;   int64_t Wp_cap = 0;    // W rows of slices added since last recovery
  double* T2 = nullptr;   int64_t T2_rows = 0;   // reference path workspace
  double* Mk = nullptr;   int64_t Mk_cap = 0;    // [t][P][Q][Q] f64
  void* mfma_work = nullptr; size_t mfma_work_bytes = 0;

  // ALS
  double *F = nullptr, *lam = nullptr;     // [P][3][Q][R], [P][R]
  int *iters = nullptr, *flags = nullptr;  // [P]
  double *F0 = nullptr, *lam0 = nullptr;   // starting factors of the running ALS call
  int* zbad = nullptr;                     // [P] non-finite entries in replica p's Z
  int* health = nullptr;                   // [1] OCTEN_HEALTH_* bits since the last report
  int als_nw = 0;                          // workgroups per replica (0: reference kernel)
  bool als_gx = false;                     // slab read from global memory, not LDS
  bool als_split = false;                  // contractions on two-term bfloat16 operands
  double* als_slots = nullptr;
  unsigned* als_ctr = nullptr;
  int* als_err = nullptr;
  // recovery
  double *aligned = nullptr, *margin = nullptr, *rhs = nullptr, *rhs_c = nullptr;
  int* perm = nullptr;
  double *Araw = nullptr, *Braw = nullptr, *Ac = nullptr, *Bc = nullptr;
  double *Aprev = nullptr, *Bprev = nullptr;
  double *ka = nullptr, *kb = nullptr, *kappa = nullptr, *tsign = nullptr, *tmargin = nullptr;
  int* tperm = nullptr;
  double *cross = nullptr, *norms = nullptr;
  double *H = nullptr, *Hcur = nullptr;
  double *Chist = nullptr, *Ctmp = nullptr; int64_t C_cap = 0;
  double *Nt = nullptr; int64_t Nt_cap = 0;      // temporal normal matrix
  double *bt = nullptr; int64_t bt_cap = 0;      // temporal rhs / solution
  int* info = nullptr;
  // fit
  double* partials = nullptr;
  double* fit_out = nullptr;
  double* gj_work = nullptr;
  double* rd_work = nullptr;                     // partial sums of split products
  static constexpr int64_t RD_WORK = 1 << 18;
  // sparse batches
  int* coo_work = nullptr;  int64_t coo_work_cap = 0;
  int* seg_start = nullptr; int64_t seg_start_cap = 0;
  int* seg_row = nullptr;   int64_t seg_row_cap = 0;
  int* seg_slice = nullptr; int64_t seg_slice_cap = 0;
  int* slice_seg = nullptr; int64_t slice_seg_cap = 0;
  int* coo_small = nullptr;          // [4]: error bits, nseg, t, unused
  // an unsorted batch, sorted: coordinates, values, radix-sort scratch
  int *coo_ks = nullptr, *coo_is = nullptr, *coo_js = nullptr;
  int64_t coo_ks_cap = 0, coo_is_cap = 0, coo_js_cap = 0;
  float* coo_vs = nullptr;           int64_t coo_vs_cap = 0;
  double* coo_sort_work = nullptr;   int64_t coo_sort_work_cap = 0;
  int coo_nseg = -1;                 // segments of the last sparse batch
  int64_t coo_t = 0;
  float *Uf = nullptr, *Vf = nullptr;            // f32 copies for sparse gathers
  float* Mkf = nullptr; int64_t Mkf_cap = 0;     // [t][P][Q][Q] f32
  double* fitG = nullptr;                        // [3][R][R] Gram matrices
  bool z_any = false;                            // some batch has been compressed
  // learned warm start
  octen_mlp_t ws_mlp = nullptr;
  float* ws_G = nullptr;  int ws_D = 0;          // sketch matrix [D][Q^3]
  float* ws_sk = nullptr;                        // [P][D]
  double* ws_part = nullptr; int64_t ws_part_len = 0;
  double* ws_signs = nullptr;                    // [P*R][2]
  double* ws_u = nullptr;                        // [P*R][Q] mode-3 changes
  double *ws_plain = nullptr, *ws_cand = nullptr, *ws_init = nullptr;   // [P][3][Q][R]
  float* ws_X = nullptr;                         // [P*R][3Q+D]
  float* ws_Y = nullptr;                         // [P*R][3Q]
  double* ws_jpart = nullptr;                    // judge partials
  double* ws_fits = nullptr;                     // [P][2]
  int* ws_keep = nullptr;                        // [P]
  bool ws_signs_ok = false;

  std::vector<void*> allocs;
  bool group_mode = false;       // inside a group step: one workgroup per replica ALS
  AlsCoopItem* als_defer = nullptr;  // set: the cooperative ALS launch is left to the caller

  // stage timing (OCTEN_FLAG_TIMING): ring of event pairs per stage
  std::vector<hipEvent_t> ev[OCTEN_NUM_STAGES];   // 2 * OCTEN_TIMING_RING
  int64_t ev_count[OCTEN_NUM_STAGES] = {};
  bool timing = false;
};

namespace {
struct StageTimer {
  octen_t h;
  int stage;
  int slot;
  StageTimer(octen_t hh, int st) : h(hh), stage(st), slot(0) {
    if (h->timing) {
      slot = (int)(h->ev_count[stage] % OCTEN_TIMING_RING);
      hipEventRecord(h->ev[stage][2 * slot], h->stream);
    }
  }
  ~StageTimer() {
    if (h->timing) {
      hipEventRecord(h->ev[stage][2 * slot + 1], h->stream);
      ++h->ev_count[stage];
    }
  }
};
}  // namespace

namespace {

constexpr int FIT_PARTS = 2048;

octen_status fail(octen_t h, octen_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

#define HIPCHK(h, expr)                                                             \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail((h), OCTEN_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
octen_status dalloc(octen_t h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(h, OCTEN_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = (T*)q;
  return OCTEN_OK;
}

void dfree(octen_t h, void* p) {
  if (!p) return;
  for (auto& a : h->allocs)
    if (a == p) { hipFree(p); a = nullptr; return; }
}

// grow a device array to at least `count` elements (contents discarded)
template <typename T>
octen_status dgrow(octen_t h, T** p, int64_t* cap, int64_t count) {
  if (*p && *cap >= count) return OCTEN_OK;
  if (*p) { hipStreamSynchronize(h->stream); dfree(h, *p); *p = nullptr; }
  int64_t n = count < 1 ? 1 : count;
  octen_status st = dalloc(h, p, (size_t)n);
  if (st == OCTEN_OK) *cap = n;
  return st;
}

#define OKCHK(expr)                      \
  do {                                   \
    octen_status s_ = (expr);            \
    if (s_ != OCTEN_OK) return s_;       \
  } while (0)

// Makes the handle stream wait for an overlapped compression (Z, Wz and the
// compression workspace are then safe to read or rewrite on it).
static octen_status join_side(octen_t h) {
  if (h->z_async) {
    h->z_async = false;
    if (hipStreamWaitEvent(h->stream, h->ev_z, 0) != hipSuccess)
      return fail(h, OCTEN_ERR_HIP, "join of the overlapped compression failed");
  }
  return OCTEN_OK;
}

bool valid_dtype_x(int d) { return d == OCTEN_F64 || d == OCTEN_F32; }

// Matrix-core input kind of a compression type (see mfma_plan_create).
int mfma_kind(int compress_dtype) {
  return compress_dtype == OCTEN_BF16 ? 2 : (compress_dtype == OCTEN_BF16X2 ? 3 : 1);
}

octen_status validate(const octen_config* c, std::string* msg) {
  if (!c) { *msg = "config is NULL"; return OCTEN_ERR_ARG; }
  if (c->abi_version != OCTEN_ABI_VERSION) { *msg = "ABI version mismatch"; return OCTEN_ERR_ARG; }
  if (c->I < 1 || c->J < 1) { *msg = "I and J must be >= 1"; return OCTEN_ERR_ARG; }
  if (c->I > (1LL << 30) || c->J > (1LL << 30)) { *msg = "I or J too large"; return OCTEN_ERR_ARG; }
  if (c->R < 1 || c->R > 32) { *msg = "R must be in [1, 32]"; return OCTEN_ERR_ARG; }
  if (c->P < 1) { *msg = "P must be >= 1"; return OCTEN_ERR_ARG; }
  if (c->S < 1) { *msg = "S must be >= 1 (anchor rows are needed for matching)"; return OCTEN_ERR_ARG; }
  if (c->Q <= c->S || c->Q > 128) { *msg = "Q must satisfy S < Q <= 128"; return OCTEN_ERR_ARG; }
  if (c->R > c->Q) { *msg = "R must be <= Q"; return OCTEN_ERR_ARG; }
  if (!valid_dtype_x(c->x_dtype)) { *msg = "x_dtype must be F64 or F32"; return OCTEN_ERR_ARG; }
  if (c->compress_dtype != OCTEN_F64 && c->compress_dtype != OCTEN_F32 &&
      c->compress_dtype != OCTEN_BF16 && c->compress_dtype != OCTEN_BF16X2) {
    *msg = "compress_dtype must be F64, F32, BF16 or BF16X2";
    return OCTEN_ERR_UNSUPPORTED;
  }
  if (c->compress_dtype == OCTEN_F64 && c->x_dtype != OCTEN_F64) {
    // f32 slices with f64 arithmetic are allowed (exact upcast)
  }
  if (c->compress_dtype != OCTEN_F64 && c->x_dtype == OCTEN_F64) {
    *msg = "narrow compression needs f32 slices";
    return OCTEN_ERR_UNSUPPORTED;
  }
  if (c->als_dtype != OCTEN_F64 && c->als_dtype != OCTEN_BF16X2) {
    *msg = "als_dtype must be F64 or BF16X2";
    return OCTEN_ERR_UNSUPPORTED;
  }
  if (c->als_dtype == OCTEN_BF16X2 &&
      (c->compress_dtype == OCTEN_F64 || (c->flags & (OCTEN_FLAG_ALS_ONE_WG | OCTEN_FLAG_REFERENCE_PATH)))) {
    // the two-term contractions exist in the cooperative ALS on float summaries only
    *msg = "als_dtype BF16X2 needs float summaries (compress_dtype F32, BF16 or BF16X2) and the "
           "cooperative ALS";
    return OCTEN_ERR_UNSUPPORTED;
  }
  int64_t M1 = (int64_t)c->S + (int64_t)c->P * (c->Q - c->S);
  if (M1 > (1 << 20)) { *msg = "too many compression columns"; return OCTEN_ERR_ARG; }
  const uint64_t known = OCTEN_FLAG_REFERENCE_PATH | OCTEN_FLAG_TIMING | OCTEN_FLAG_ALS_ONE_WG |
                         OCTEN_FLAG_ALS_DEVICE_SYNC | OCTEN_FLAG_ALS_FEW_WG;
  if (c->flags & ~known) { *msg = "unknown flag bits"; return OCTEN_ERR_ARG; }
  return OCTEN_OK;
}

// Least-squares operator of Eq. 7 for a fixed deduplicated compression matrix
// Pt (n x M1): the minimum-norm solution of the sqrt(P)-weighted stack is
// x = Op * rhs with Op (n x M1) built once here.
octen_status build_operator(octen_t h, const double* Pt, int64_t n, double* Op) {
  hipStream_t s = h->stream;
  const int M1 = h->M1;
  double* N = nullptr;
  if (n <= M1) {
    OKCHK(dalloc(h, &N, (size_t)(n * n)));
    HIPCHK(h, gemm_f64(s, (int)n, (int)n, M1, 1, Pt, M1, 1, 0, Pt, 1, M1, 0, N, n, 1, 0, h->w2,
                       1.0, 0.0));
    HIPCHK(h, spd_invert(s, N, (int)n, h->gj_work, h->info));
    HIPCHK(h, gemm_f64(s, (int)n, M1, (int)n, 1, N, n, 1, 0, Pt, M1, 1, 0, Op, M1, 1, 0, nullptr,
                       1.0, 0.0));
    HIPCHK(h, scale_cols(s, Op, n, M1, h->w2));
  } else {
    OKCHK(dalloc(h, &N, (size_t)M1 * M1));
    HIPCHK(h, gemm_f64(s, M1, M1, (int)n, 1, Pt, 1, M1, 0, Pt, M1, 1, 0, N, M1, 1, 0, nullptr, 1.0,
                       0.0));
    HIPCHK(h, scale_rows_cols(s, N, M1, h->w));
    HIPCHK(h, spd_invert(s, N, M1, h->gj_work, h->info));
    HIPCHK(h, gemm_f64(s, (int)n, M1, M1, 1, Pt, M1, 1, 0, N, M1, 1, 0, Op, M1, 1, 0, h->w, 1.0,
                       0.0));
    HIPCHK(h, scale_cols(s, Op, n, M1, h->w));
  }
  HIPCHK(h, hipStreamSynchronize(s));
  dfree(h, N);
  return OCTEN_OK;
}

// Waits for the handle's stream, reads and clears the health bits (the
// OCTEN_HEALTH_* conditions since the last report): OCTEN_ERR_NUMERIC when
// any is set.
octen_status report_health(octen_t h, int32_t* bits_host = nullptr) {
  int v = 0;
  HIPCHK(h, hipMemcpyAsync(&v, h->health, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (bits_host) *bits_host = v;
  if (v == 0) return OCTEN_OK;
  HIPCHK(h, fill_i32(h->stream, h->health, 1, 0));
  std::string what;
  if (v & OCTEN_HEALTH_NONFINITE_BATCH) what += "non-finite compressed batch (summaries not updated)";
  if (v & OCTEN_HEALTH_ALS_FAILED) {
    if (!what.empty()) what += "; ";
    what += "replica fit failed (starting factors kept, see OCTEN_STATE_FLAGS)";
  }
  return fail(h, OCTEN_ERR_NUMERIC, what);
}

int host_info(octen_t h) {
  int v = 0;
  hipMemcpyAsync(&v, h->info, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  hipStreamSynchronize(h->stream);
  return v;
}

}  // namespace

// Smallest workgroup count with the same slab height ceil(Q / nw) as nw: the
// slowest workgroup of a replica sets the pace, so extra workgroups that do
// not lower the tallest slab only add barrier participants.
static int balanced_nw(int Q, int nw) {
  if (nw < 1) return 1;
  const int na = (Q + nw - 1) / nw;
  return (Q + na - 1) / na;
}

extern "C" {

int32_t octen_abi_version(void) { return OCTEN_ABI_VERSION; }

const char* octen_status_str(octen_status s) {
  switch (s) {
    case OCTEN_OK: return "ok";
    case OCTEN_ERR_ARG: return "invalid argument";
    case OCTEN_ERR_STATE: return "call out of order";
    case OCTEN_ERR_HIP: return "HIP runtime error";
    case OCTEN_ERR_NOMEM: return "out of device memory";
    case OCTEN_ERR_NUMERIC: return "numerical failure";
    case OCTEN_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* octen_last_error(octen_t h) { return h ? h->err.c_str() : "null handle"; }

octen_status octen_health(octen_t h, int32_t* bits_host) {
  if (!h) return OCTEN_ERR_ARG;
  OKCHK(join_side(h));
  return report_health(h, bits_host);
}

octen_status octen_check_identifiable(const octen_config* cfg, int64_t K, int64_t t,
                                      int32_t* bits_host, double* p_min_host) {
  std::string msg;
  octen_status st = validate(cfg, &msg);
  if (st != OCTEN_OK) return st;
  if (K < 0 || t < 0 || !bits_host) return OCTEN_ERR_ARG;
  const double I = (double)cfg->I, J = (double)cfg->J, Q = cfg->Q, S = cfg->S;
  // Eq. 8 as printed: p >= max((I - shared)/(Q - shared), J/Q, K/Q)
  double pmin = (I - S) / (Q - S);
  if (J / Q > pmin) pmin = J / Q;
  if ((double)K / Q > pmin) pmin = (double)K / Q;
  const int64_t M1 = (int64_t)cfg->S + (int64_t)cfg->P * (cfg->Q - cfg->S);
  int32_t bits = 0;
  if ((double)cfg->P >= ceil(pmin - 1e-12)) bits |= 1;
  if (M1 >= cfg->I) bits |= 2;
  if (M1 >= cfg->J) bits |= 4;
  if (M1 >= t) bits |= 8;
  auto mn = [](int64_t a, int64_t b) { return a < b ? a : b; };
  const int64_t R = cfg->R;
  const int64_t kr = mn(cfg->Q, mn(cfg->I, R)) + mn(cfg->Q, mn(cfg->J, R)) + mn(cfg->Q, mn(K, R));
  if (kr >= 2 * R + 2) bits |= 16;
  *bits_host = bits;
  if (p_min_host) *p_min_host = pmin;
  return OCTEN_OK;
}

octen_status octen_init(const octen_config* cfg, const double* U, const double* V, void* stream,
                        octen_t* out) {
  if (!out) return OCTEN_ERR_ARG;
  *out = nullptr;
  std::string msg;
  octen_status st = validate(cfg, &msg);
  if (st != OCTEN_OK) return st;
  if (!U || !V) return OCTEN_ERR_ARG;
  octen_t h = new octen_ctx();
  h->cfg = *cfg;
  h->I = cfg->I; h->J = cfg->J; h->R = cfg->R; h->P = cfg->P; h->Q = cfg->Q; h->S = cfg->S;
  h->M1 = h->S + h->P * (h->Q - h->S);
  h->stream = (hipStream_t)stream;
  h->acc_f64 = cfg->compress_dtype == OCTEN_F64;
  const int64_t I = h->I, J = h->J, M1 = h->M1, P = h->P, Q = h->Q, R = h->R;
  const int64_t Q3 = Q * Q * Q;
  const size_t accsz = h->acc_f64 ? 8 : 4;
  auto bail = [&](octen_status s2) { octen_destroy(h); return s2; };
#define IOK(expr)                       \
  do {                                  \
    octen_status s_ = (expr);           \
    if (s_ != OCTEN_OK) return bail(s_); \
  } while (0)
  IOK(dalloc(h, &h->U, I * M1));
  IOK(dalloc(h, &h->V, J * M1));
  IOK(dalloc(h, &h->OpA, I * M1));
  IOK(dalloc(h, &h->OpB, J * M1));
  IOK(dalloc(h, &h->w, M1));
  IOK(dalloc(h, &h->w2, M1));
  IOK(dalloc(h, (char**)&h->Y, P * Q3 * accsz));
  IOK(dalloc(h, (char**)&h->Z, P * Q3 * accsz));
  IOK(dalloc(h, &h->F, P * 3 * Q * R));
  IOK(dalloc(h, &h->lam, P * R));
  IOK(dalloc(h, &h->iters, P));
  IOK(dalloc(h, &h->flags, P));
  IOK(dalloc(h, &h->F0, P * 3 * Q * R));
  IOK(dalloc(h, &h->lam0, P * R));
  IOK(dalloc(h, &h->zbad, P));
  IOK(dalloc(h, &h->health, 1));
  IOK(dalloc(h, &h->aligned, P * 3 * Q * R));
  IOK(dalloc(h, &h->margin, P));
  IOK(dalloc(h, &h->perm, P * R));
  IOK(dalloc(h, &h->rhs, 3 * M1 * R));
  IOK(dalloc(h, &h->rhs_c, M1 * R));
  IOK(dalloc(h, &h->Araw, I * R));
  IOK(dalloc(h, &h->Braw, J * R));
  IOK(dalloc(h, &h->Ac, I * R));
  IOK(dalloc(h, &h->Bc, J * R));
  IOK(dalloc(h, &h->Aprev, I * R));
  IOK(dalloc(h, &h->Bprev, J * R));
  IOK(dalloc(h, &h->ka, R));
  IOK(dalloc(h, &h->kb, R));
  IOK(dalloc(h, &h->kappa, R));
  IOK(dalloc(h, &h->tsign, R));
  IOK(dalloc(h, &h->tmargin, 1));
  IOK(dalloc(h, &h->tperm, R));
  IOK(dalloc(h, &h->cross, 2 * R * R));
  IOK(dalloc(h, &h->norms, 4 * R));
  IOK(dalloc(h, &h->H, M1 * R));
  IOK(dalloc(h, &h->Hcur, M1 * R));
  IOK(dalloc(h, &h->info, 1));
  IOK(dalloc(h, &h->partials, 2 * FIT_PARTS));
  IOK(dalloc(h, &h->fit_out, 3));
  IOK(dalloc(h, &h->rd_work, (size_t)octen_ctx::RD_WORK));
  IOK(dalloc(h, &h->coo_small, 4));
  IOK(dalloc(h, &h->fitG, 3 * R * R));
  IOK(dalloc(h, &h->gj_work, 2 * (I > J ? (I > M1 ? I : M1) : (J > M1 ? J : M1))));
  hipStream_t s = h->stream;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) { h->err = std::string(what) + ": " + hipGetErrorString(e); return false; }
    return true;
  };
  if (!hip_ok(hipMemcpyAsync(h->U, U, I * M1 * 8, hipMemcpyDeviceToDevice, s), "copy U") ||
      !hip_ok(hipMemcpyAsync(h->V, V, J * M1 * 8, hipMemcpyDeviceToDevice, s), "copy V") ||
      !hip_ok(hipMemsetAsync(h->Y, 0, P * Q3 * accsz, s), "zero Y") ||
      !hip_ok(hipMemsetAsync(h->Z, 0, P * Q3 * accsz, s), "zero Z") ||
      !hip_ok(hipMemsetAsync(h->H, 0, M1 * R * 8, s), "zero H") ||
      !hip_ok(hipMemsetAsync(h->info, 0, sizeof(int), s), "zero info") ||
      !hip_ok(hipMemsetAsync(h->flags, 0, P * sizeof(int), s), "zero flags") ||
      !hip_ok(hipMemsetAsync(h->zbad, 0, P * sizeof(int), s), "zero zbad") ||
      !hip_ok(hipMemsetAsync(h->health, 0, sizeof(int), s), "zero health") ||
      !hip_ok(rec_weights(s, (int)M1, h->S, (int)P, h->w, h->w2), "weights")) {
    octen_destroy(h);
    return OCTEN_ERR_HIP;
  }
  {
    std::vector<int> ident(R);
    std::vector<double> ones(R, 1.0);
    for (int r = 0; r < R; ++r) ident[r] = r;
    if (!hip_ok(hipMemcpy(h->tperm, ident.data(), R * sizeof(int), hipMemcpyHostToDevice), "tperm") ||
        !hip_ok(hipMemcpy(h->tsign, ones.data(), R * sizeof(double), hipMemcpyHostToDevice), "tsign")) {
      octen_destroy(h);
      return OCTEN_ERR_HIP;
    }
  }
  if (!(cfg->flags & OCTEN_FLAG_REFERENCE_PATH)) {
    // workgroups per replica for the cooperative ALS: enough to spread ~2e5
    // FMAs per workgroup per sweep, at most the CUs of one XCD per replica,
    // and few enough that the slab fits in LDS; if no count lets it fit, the
    // slab stays in global memory and the most workgroups are used
    const int per_xcd = (int)((P + 7) / 8);
    const bool split = cfg->als_dtype == OCTEN_BF16X2;
    int max_nw = per_xcd > 0 ? 32 / per_xcd : 0;
    if (max_nw > Q) max_nw = (int)Q;
    if (max_nw >= 1) {
      const size_t lds_cap = 160 * 1024;
      const double work = 4.0 * (double)Q * Q * Q * R;
      int nw = (cfg->flags & OCTEN_FLAG_ALS_FEW_WG) ? 1 : (int)ceil(work / 2.0e5);
      if (nw < 1) nw = 1;
      if (nw > max_nw) nw = max_nw;
      bool gx = false;
      while (nw < max_nw && als_coop_lds_bytes((int)Q, (int)R, nw, h->acc_f64, false, split) > lds_cap) ++nw;
      if (als_coop_lds_bytes((int)Q, (int)R, nw, h->acc_f64, false, split) > lds_cap) {
        nw = max_nw;
        gx = true;
      }
      nw = balanced_nw((int)Q, nw);   // same slab height, so the same LDS size
      if (als_coop_lds_bytes((int)Q, (int)R, nw, h->acc_f64, gx, split) <= lds_cap) {
        h->als_nw = nw;
        h->als_gx = gx;
        h->als_split = split;
        IOK(dalloc(h, &h->als_slots, (size_t)2 * P * nw * als_coop_slot_len((int)Q, (int)R)));
        IOK(dalloc(h, &h->als_ctr, 2 * (size_t)P));
        IOK(dalloc(h, &h->als_err, 1));
      }
    }
  }
  if (cfg->als_dtype == OCTEN_BF16X2 && !h->als_split) {
    octen_destroy(h);
    return OCTEN_ERR_UNSUPPORTED;   // no cooperative ALS configuration fits
  }
  if (cfg->flags & OCTEN_FLAG_TIMING) {
    for (int st2 = 0; st2 < OCTEN_NUM_STAGES; ++st2) {
      h->ev[st2].assign(2 * OCTEN_TIMING_RING, nullptr);
      for (auto& e2 : h->ev[st2])
        if (!hip_ok(hipEventCreate(&e2), "event")) { octen_destroy(h); return OCTEN_ERR_HIP; }
    }
    h->timing = true;
  }
  IOK(build_operator(h, h->U, I, h->OpA));
  IOK(build_operator(h, h->V, J, h->OpB));
  if (host_info(h) != 0) {
    octen_destroy(h);
    return OCTEN_ERR_NUMERIC;
  }
  if (h->cfg.compress_dtype != OCTEN_F64 && !(h->cfg.flags & OCTEN_FLAG_REFERENCE_PATH)) {
    CompressShape sh{I, J, (int)P, (int)Q, h->S, (int)M1};
    hipError_t e = mfma_plan_create(sh, mfma_kind(h->cfg.compress_dtype), h->U, h->V, s, &h->plan);
    if (e != hipSuccess) {
      octen_destroy(h);
      if (e == hipErrorInvalidValue && cfg->compress_dtype == OCTEN_BF16X2) return OCTEN_ERR_ARG;
      return e == hipErrorNotSupported ? OCTEN_ERR_UNSUPPORTED : OCTEN_ERR_HIP;
    }
  }
#undef IOK
  *out = h;
  return OCTEN_OK;
}

octen_status octen_destroy(octen_t h) {
  if (!h) return OCTEN_ERR_ARG;
  hipStreamSynchronize(h->stream);
  if (h->side) {
    hipStreamSynchronize(h->side);
    hipStreamDestroy(h->side);
  }
  if (h->ev_main) hipEventDestroy(h->ev_main);
  if (h->ev_z) hipEventDestroy(h->ev_z);
  if (h->plan) mfma_plan_destroy(h->plan);
  for (int st = 0; st < OCTEN_NUM_STAGES; ++st)
    for (auto e : h->ev[st])
      if (e) hipEventDestroy(e);
  for (void* p : h->allocs)
    if (p) hipFree(p);
  delete h;
  return OCTEN_OK;
}

octen_status octen_compress_batch(octen_t h, const void* X, int64_t t, const double* W,
                                  const float* slice_scale) {
  if (!h) return OCTEN_ERR_ARG;
  if (!X || !W || t < 1) return fail(h, OCTEN_ERR_ARG, "X, W must be non-null and t >= 1");
  if (t > (1 << 24)) return fail(h, OCTEN_ERR_ARG, "t too large");
  OKCHK(join_side(h));
  hipStream_t s = h->stream;
  const int64_t I = h->I, J = h->J, M1 = h->M1;
  CompressShape sh{I, J, h->P, h->Q, h->S, h->M1};
  OKCHK(dgrow(h, &h->Wz, &h->Wz_cap, t * M1));
  HIPCHK(h, hipMemcpyAsync(h->Wz, W, t * M1 * 8, hipMemcpyDeviceToDevice, s));
  const bool x_f64 = h->cfg.x_dtype == OCTEN_F64;
  if (h->plan) {
    size_t need = mfma_workspace_bytes(h->plan, t);
    if (need > h->mfma_work_bytes) {
      if (h->mfma_work) { hipStreamSynchronize(s); dfree(h, h->mfma_work); h->mfma_work = nullptr; }
      OKCHK(dalloc(h, (char**)&h->mfma_work, need));
      h->mfma_work_bytes = need;
    }
    HIPCHK(h, fill_i32(s, h->zbad, h->P, 0));
    {
      StageTimer tm(h, OCTEN_STAGE_COMPRESS_MAIN);
      HIPCHK(h, compress_mfma_main(s, h->plan, (const float*)X, t, slice_scale, h->mfma_work));
    }
    {
      StageTimer tm(h, OCTEN_STAGE_COMPRESS_MODE3);
      HIPCHK(h, compress_mfma_mode3(s, h->plan, t, h->Wz, h->mfma_work, (float*)h->Z, h->zbad));
    }
  } else {
    // reference path: T2 chunk of at most ~64 Mi doubles
    int64_t rows_cap = (int64_t)1 << 26;
    rows_cap /= M1;
    if (rows_cap < I) rows_cap = I;
    int64_t want = rows_cap < t * I ? rows_cap : t * I;
    want = (want / I) * I;
    OKCHK(dgrow(h, &h->T2, &h->T2_rows, want * M1));
    OKCHK(dgrow(h, &h->Mk, &h->Mk_cap, t * h->P * h->Q * h->Q));
    HIPCHK(h, fill_i32(s, h->zbad, h->P, 0));
    StageTimer tm(h, OCTEN_STAGE_COMPRESS_MAIN);
    HIPCHK(h, compress_reference(s, sh, X, x_f64, t, h->U, h->V, h->Wz, h->T2, h->T2_rows / M1,
                                 h->Mk, h->Z, h->acc_f64, h->zbad));
  }
  h->z_ready = true;
  h->z_any = true;
  h->t_z = t;
  return OCTEN_OK;
}

octen_status octen_compress_batch_async(octen_t h, const void* X, int64_t t, const double* W,
                                        const float* slice_scale) {
  if (!h) return OCTEN_ERR_ARG;
  if (!h->side) {
    hipStream_t side = nullptr;
    hipEvent_t em = nullptr, ez = nullptr;
    if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&em, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ez, hipEventDisableTiming) != hipSuccess) {
      if (ez) hipEventDestroy(ez);
      if (em) hipEventDestroy(em);
      if (side) hipStreamDestroy(side);
      return fail(h, OCTEN_ERR_HIP, "side stream for the overlapped compression");
    }
    h->side = side;
    h->ev_main = em;
    h->ev_z = ez;
  }
  // everything enqueued on the handle stream so far (the producer of X, the
  // update that consumed the previous batch) precedes the compression
  HIPCHK(h, hipEventRecord(h->ev_main, h->stream));
  HIPCHK(h, hipStreamWaitEvent(h->side, h->ev_main, 0));
  hipStream_t keep = h->stream;
  h->stream = h->side;
  const octen_status st = octen_compress_batch(h, X, t, W, slice_scale);
  h->stream = keep;
  if (st != OCTEN_OK) return st;
  HIPCHK(h, hipEventRecord(h->ev_z, h->side));
  h->z_async = true;
  return OCTEN_OK;
}

octen_status octen_compress_batch_coo(octen_t h, int64_t nnz, const int32_t* k, const int32_t* i,
                                      const int32_t* j, const float* v, int64_t t, const double* W) {
  if (!h) return OCTEN_ERR_ARG;
  if (!W || t < 1) return fail(h, OCTEN_ERR_ARG, "W must be non-null and t >= 1");
  if (t > (1 << 24)) return fail(h, OCTEN_ERR_ARG, "t too large");
  if (nnz < 0 || nnz >= 0x7fffffffLL) return fail(h, OCTEN_ERR_ARG, "nnz must be in [0, 2^31 - 1)");
  if (nnz > 0 && (!k || !i || !j || !v)) return fail(h, OCTEN_ERR_ARG, "k, i, j, v must be non-null");
  OKCHK(join_side(h));
  hipStream_t s = h->stream;
  const int64_t M1 = h->M1, P = h->P, Q = h->Q;
  OKCHK(dgrow(h, &h->coo_work, &h->coo_work_cap, (int64_t)coo_work_ints(nnz)));
  OKCHK(dgrow(h, &h->seg_start, &h->seg_start_cap, nnz + 1));
  OKCHK(dgrow(h, &h->seg_row, &h->seg_row_cap, nnz));
  OKCHK(dgrow(h, &h->seg_slice, &h->seg_slice_cap, nnz));
  OKCHK(dgrow(h, &h->slice_seg, &h->slice_seg_cap, t + 1));
  {
    StageTimer tm(h, OCTEN_STAGE_COO_INDEX);
    HIPCHK(h, fill_i32(s, h->coo_small, 4, 0));
    HIPCHK(h, coo_check(s, nnz, k, i, j, t, h->I, h->J, true, h->coo_small));
    HIPCHK(h, coo_segments(s, nnz, k, i, t, h->coo_work, h->seg_start, h->seg_row, h->seg_slice,
                           h->slice_seg, h->coo_small + 1));
    HIPCHK(h, fill_i32(s, h->coo_small + 2, 1, (int)t));
  }
  int hs[2] = {0, 0};
  HIPCHK(h, hipMemcpyAsync(hs, h->coo_small, sizeof(hs), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (hs[0] & 1) return fail(h, OCTEN_ERR_ARG, "COO coordinate out of range");
  if (hs[0] & 2) {
    // not in (k, i, j) order: a stable device sort into the handle's
    // arrays, then the segments of the sorted batch
    if (coo_sort_key_bits(t, h->I, h->J) > 64)
      return fail(h, OCTEN_ERR_UNSUPPORTED,
                  "unsorted COO batch whose packed (k, i, j) key exceeds 64 bits");
    OKCHK(dgrow(h, &h->coo_ks, &h->coo_ks_cap, nnz));
    OKCHK(dgrow(h, &h->coo_is, &h->coo_is_cap, nnz));
    OKCHK(dgrow(h, &h->coo_js, &h->coo_js_cap, nnz));
    OKCHK(dgrow(h, &h->coo_vs, &h->coo_vs_cap, nnz));
    OKCHK(dgrow(h, &h->coo_sort_work, &h->coo_sort_work_cap,
                (int64_t)(coo_sort_work_bytes(nnz) + 7) / 8));
    {
      StageTimer tm(h, OCTEN_STAGE_COO_INDEX);
      HIPCHK(h, coo_sort(s, nnz, k, i, j, v, t, h->I, h->J, h->coo_sort_work, h->coo_ks,
                         h->coo_is, h->coo_js, h->coo_vs));
      k = h->coo_ks;
      i = h->coo_is;
      j = h->coo_js;
      v = h->coo_vs;
      HIPCHK(h, fill_i32(s, h->coo_small, 4, 0));
      HIPCHK(h, coo_segments(s, nnz, k, i, t, h->coo_work, h->seg_start, h->seg_row,
                             h->seg_slice, h->slice_seg, h->coo_small + 1));
      HIPCHK(h, fill_i32(s, h->coo_small + 2, 1, (int)t));
    }
    HIPCHK(h, hipMemcpyAsync(hs, h->coo_small, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  h->coo_nseg = hs[1];
  h->coo_t = t;
  OKCHK(dgrow(h, &h->Wz, &h->Wz_cap, t * M1));
  HIPCHK(h, hipMemcpyAsync(h->Wz, W, t * M1 * 8, hipMemcpyDeviceToDevice, s));
  CompressShape sh{h->I, h->J, h->P, h->Q, h->S, h->M1};
  const bool f64 = h->cfg.compress_dtype == OCTEN_F64;
  const void *Um = h->U, *Vm = h->V;
  void* Mk = nullptr;
  if (f64) {
    OKCHK(dgrow(h, &h->Mk, &h->Mk_cap, t * P * Q * Q));
    Mk = h->Mk;
  } else {
    if (!h->Uf) {
      OKCHK(dalloc(h, &h->Uf, (size_t)(h->I * M1)));
      OKCHK(dalloc(h, &h->Vf, (size_t)(h->J * M1)));
      HIPCHK(h, convert_f64_to_f32(s, h->U, h->Uf, h->I * M1));
      HIPCHK(h, convert_f64_to_f32(s, h->V, h->Vf, h->J * M1));
    }
    OKCHK(dgrow(h, &h->Mkf, &h->Mkf_cap, t * P * Q * Q));
    Um = h->Uf;
    Vm = h->Vf;
    Mk = h->Mkf;
  }
  {
    StageTimer tm(h, OCTEN_STAGE_COMPRESS_MAIN);
    HIPCHK(h, coo_compress(s, f64, t, h->P, h->Q, h->S, h->M1, h->seg_start, h->seg_row,
                           h->slice_seg, j, v, Vm, Um, Mk));
  }
  HIPCHK(h, fill_i32(s, h->zbad, h->P, 0));
  {
    StageTimer tm(h, OCTEN_STAGE_COMPRESS_MODE3);
    HIPCHK(h, compress_mode3(s, sh, t, Mk, f64, h->Wz, h->Z, h->acc_f64, h->zbad));
  }
  h->z_ready = true;
  h->z_any = true;
  h->t_z = t;
  return OCTEN_OK;
}

octen_status octen_update_replicas(octen_t h) {
  if (h) OKCHK(join_side(h));
  if (!h) return OCTEN_ERR_ARG;
  if (!h->z_ready) return fail(h, OCTEN_ERR_STATE, "update before compress");
  hipStream_t s = h->stream;
  const int64_t n = (int64_t)h->P * h->Q * h->Q * h->Q;
  {
    StageTimer tm(h, OCTEN_STAGE_UPDATE);
    HIPCHK(h, update_masked(s, h->Y, h->Z, h->P, n / h->P, h->acc_f64, h->zbad, h->health));
  }
  // append this batch's W rows to the pending temporal block
  const int64_t M1 = h->M1;
  if (h->t_pend + h->t_z > h->Wp_cap / (M1 > 0 ? M1 : 1)) {
    double* nw = nullptr;
    const int64_t cap = (h->t_pend + h->t_z) * 2 * M1;
    OKCHK(dalloc(h, &nw, cap));
    if (h->t_pend > 0)
      HIPCHK(h, hipMemcpyAsync(nw, h->Wp, h->t_pend * M1 * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));
    dfree(h, h->Wp);
    h->Wp = nw;
    h->Wp_cap = cap;
  }
  HIPCHK(h, hipMemcpyAsync(h->Wp + h->t_pend * M1, h->Wz, h->t_z * M1 * 8,
                           hipMemcpyDeviceToDevice, s));
  h->t_pend += h->t_z;
  h->z_ready = false;
  h->factors_fresh = false;
  return OCTEN_OK;
}

namespace {

octen_status ws_features(octen_t h) {
  OKCHK(join_side(h));
  if (!h->have_factors) return fail(h, OCTEN_ERR_STATE, "no previous replica factors");
  if (!h->z_any) return fail(h, OCTEN_ERR_STATE, "no compressed batch to sketch");
  hipStream_t s = h->stream;
  HIPCHK(h, ws_sketch(s, h->Z, h->acc_f64, h->P, h->Q, h->ws_G, h->ws_D, h->ws_part,
                      h->ws_part_len, h->ws_sk));
  HIPCHK(h, ws_mode3_change(s, h->Z, h->acc_f64, h->F, h->lam, h->P, h->Q, h->R, h->ws_u));
  HIPCHK(h, ws_columns(s, h->F, h->lam, h->P, h->Q, h->R, h->ws_sk, h->ws_u, h->ws_D, false,
                       h->ws_X, h->ws_signs, h->ws_plain));
  h->ws_signs_ok = true;
  return OCTEN_OK;
}

// After the replica ALS: a replica whose fit failed gets its starting factors
// back; the factors are current.
octen_status als_finish(octen_t h) {
  HIPCHK(h, als_commit(h->stream, h->P, 3 * h->Q * h->R, h->R, h->F, h->lam, h->F0, h->lam0,
                       h->flags, h->health));
  h->have_factors = true;
  h->factors_fresh = true;
  return OCTEN_OK;
}

// features -> network -> candidate -> judge; the chosen start goes to ws_init
octen_status learned_init(octen_t h) {
  OKCHK(ws_features(h));
  octen_mlp_t m = h->ws_mlp;
  const int64_t n = (int64_t)h->P * h->R;
  octen_status st = octen_mlp_ensure_rows(m, n);
  if (st != OCTEN_OK) return fail(h, st, "warm-start network buffers: " + m->err);
  hipStream_t s = h->stream;
  HIPCHK(h, mlp_forward(s, m->L, m->w, h->ws_X, n, m->H1, m->H2, h->ws_Y));
  HIPCHK(h, ws_candidate(s, h->ws_Y, h->ws_signs, h->P, h->Q, h->R, h->ws_cand));
  HIPCHK(h, ws_judge(s, h->Y, h->acc_f64, h->P, h->Q, h->R, h->ws_plain, h->ws_cand, h->ws_jpart,
                     h->ws_fits, h->ws_keep, h->ws_init));
  return OCTEN_OK;
}

}  // namespace

octen_status octen_cp_als_replicas(octen_t h, int32_t max_iters, double tol, int32_t init_mode,
                                   const double* init, int32_t* iters_done_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (max_iters < 1) return fail(h, OCTEN_ERR_ARG, "max_iters must be >= 1");
  if (!(tol >= 0.0)) return fail(h, OCTEN_ERR_ARG, "tol must be >= 0");
  if (h->K + h->t_pend == 0) return fail(h, OCTEN_ERR_STATE, "no summaries yet");
  const double* src;
  if (init_mode == OCTEN_INIT_GIVEN) {
    if (!init) return fail(h, OCTEN_ERR_ARG, "init is NULL with OCTEN_INIT_GIVEN");
    src = init;
  } else if (init_mode == OCTEN_INIT_PREV) {
    if (!h->have_factors) return fail(h, OCTEN_ERR_STATE, "no previous factors");
    src = h->F;
  } else if (init_mode == OCTEN_INIT_LEARNED) {
    if (!h->ws_mlp) return fail(h, OCTEN_ERR_STATE, "no warm-start network set");
    OKCHK(learned_init(h));
    src = h->ws_init;
  } else {
    return fail(h, OCTEN_ERR_ARG, "unknown init_mode");
  }
  hipStream_t s = h->stream;
  const int64_t QR3 = (int64_t)3 * h->Q * h->R;
  {
    StageTimer tm(h, OCTEN_STAGE_ALS);
    hipError_t e = hipErrorNotSupported;
    // group branches run concurrently: no cooperative grid there
    const bool in_branch = h->group_mode;
    if (h->cfg.als_dtype == OCTEN_BF16X2 && (in_branch || h->als_nw <= 0))
      return fail(h, OCTEN_ERR_UNSUPPORTED,
                  "the two-term contractions run in the cooperative ALS only");
    const bool coop = h->als_nw > 0 && !in_branch && !(h->cfg.flags & OCTEN_FLAG_ALS_ONE_WG);
    // one launch: the starting point (given back to a replica whose fit
    // fails) and its weights, the replica flags, and the cooperative
    // launch's barrier words
    const bool fresh = init_mode == OCTEN_INIT_GIVEN || !h->have_factors;
    HIPCHK(h, als_prep(s, (int64_t)h->P * QR3, h->F0, src, (int64_t)h->P * h->R, h->lam0,
                       fresh ? nullptr : h->lam, h->P, h->flags, coop ? h->als_ctr : nullptr,
                       2 * h->P, coop ? h->als_err : nullptr));
    if (coop && h->als_defer) {
      // a group step launches it with other handles' ALS, then calls als_finish
      *h->als_defer = AlsCoopItem{h->Y, h->acc_f64, h->P, h->Q, h->R, h->als_nw, h->als_gx, src,
                                  h->F, h->lam, h->iters, h->flags, h->als_slots, h->als_ctr,
                                  h->als_err, max_iters, tol,
                                  !(h->cfg.flags & OCTEN_FLAG_ALS_DEVICE_SYNC), h->als_split};
      return OCTEN_OK;
    }
    if (coop) {
      e = als_coop(s, h->Y, h->acc_f64, h->P, h->Q, h->R, h->als_nw, h->als_gx, src, h->F,
                   h->lam, h->iters, h->flags, h->als_slots, h->als_ctr, h->als_err, max_iters,
                   tol, !(h->cfg.flags & OCTEN_FLAG_ALS_DEVICE_SYNC), h->als_split, true);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        h->als_nw = 0;   // cooperative launch not possible here: use the reference kernel
        if (h->als_split)
          return fail(h, OCTEN_ERR_UNSUPPORTED,
                      "cooperative ALS launch failed (the two-term contractions need it)");
      }
    }
    if (e != hipSuccess)
      HIPCHK(h, als_reference(s, h->Y, h->acc_f64, h->P, h->Q, h->R, src, h->F, h->lam, h->iters,
                              h->flags, max_iters, tol));
    OKCHK(als_finish(h));
  }
  if (iters_done_host) {
    HIPCHK(h, hipMemcpyAsync(iters_done_host, h->iters, h->P * sizeof(int), hipMemcpyDeviceToHost, s));
    return report_health(h);
  }
  return OCTEN_OK;
}

octen_status octen_recover_factors(octen_t h, double* A, double* B, double* C, int64_t c_capacity,
                                   int64_t* K_out_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (!A || !B || !C) return fail(h, OCTEN_ERR_ARG, "A, B, C must be non-null");
  if (!h->factors_fresh || h->t_pend == 0)
    return fail(h, OCTEN_ERR_STATE, "recover needs ALS after the latest update");
  const int64_t Knew = h->K + h->t_pend;
  if (c_capacity < Knew) return fail(h, OCTEN_ERR_ARG, "C capacity smaller than K");
  hipStream_t s = h->stream;
  const int P = h->P, Q = h->Q, R = h->R, S = h->S, M1 = h->M1;
  const int64_t I = h->I, J = h->J, t = h->t_pend;
  StageTimer tm(h, OCTEN_STAGE_RECOVER);
  // Sec. 4.2: align replicas; Eq. 5 stack
  HIPCHK(h, rec_align(s, P, Q, R, S, h->F, h->lam, h->aligned, h->perm, h->margin));
  HIPCHK(h, rec_stack(s, P, Q, R, S, h->aligned, h->rhs));
  // Eq. 7 for modes 1 and 2
  HIPCHK(h, rowdot_pair(s, {I, R, M1, h->OpA, M1, 1, h->rhs, R, 1, nullptr, 1.0, 0.0, h->Araw, R},
                        {J, R, M1, h->OpB, M1, 1, h->rhs + (int64_t)M1 * R, R, 1, nullptr, 1.0,
                         0.0, h->Braw, R},
                        h->rd_work, octen_ctx::RD_WORK));
  HIPCHK(h, rec_canon2(s, I, J, R, h->Araw, h->Ac, h->ka, h->Braw, h->Bc, h->kb, h->rd_work,
                       octen_ctx::RD_WORK));
  if (h->have_prev) {
    HIPCHK(h, rowdot_pair(s, {R, R, I, h->Ac, 1, R, h->Aprev, R, 1, nullptr, 1.0, 0.0, h->cross, R},
                          {R, R, J, h->Bc, 1, R, h->Bprev, R, 1, nullptr, 1.0, 0.0,
                           h->cross + R * R, R},
                          h->rd_work, octen_ctx::RD_WORK));
    HIPCHK(h, rec_col_norms4(s, I, J, R, h->Ac, h->Aprev, h->Bc, h->Bprev, h->norms, h->rd_work,
                             octen_ctx::RD_WORK));
    HIPCHK(h, rec_tmatch(s, R, h->cross, h->norms, h->tperm, h->tsign, h->tmargin));
  }
  // temporal rows (reading: incremental solve with the carried history removed)
  const double* rhs2 = h->rhs + 2 * (int64_t)M1 * R;
  HIPCHK(h, rec_temporal_prep(s, M1, R, h->H, h->tperm, h->tsign, h->ka, h->kb, h->kappa, h->Hcur,
                              rhs2, h->rhs_c, h->have_prev ? 1 : 0));
  OKCHK(dgrow(h, &h->bt, &h->bt_cap, (t > M1 ? t : (int64_t)M1) * R));
  if (t <= M1) {
    OKCHK(dgrow(h, &h->Nt, &h->Nt_cap, t * t));
    HIPCHK(h, rowdot_pair(s, {t, (int)t, M1, h->Wp, M1, 1, h->Wp, 1, M1, h->w2, 1.0, 0.0, h->Nt, t},
                          {t, R, M1, h->Wp, M1, 1, h->rhs_c, R, 1, h->w2, 1.0, 0.0, h->bt, R},
                          h->rd_work, octen_ctx::RD_WORK));
    HIPCHK(h, spd_solve_small(s, h->Nt, (int)t, h->bt, R, h->gj_work, h->info));
  } else {
    OKCHK(dgrow(h, &h->Nt, &h->Nt_cap, (int64_t)M1 * M1 + (int64_t)M1 * R));
    double* y = h->Nt + (int64_t)M1 * M1;
    HIPCHK(h, gemm_f64(s, M1, M1, (int)t, 1, h->Wp, 1, M1, 0, h->Wp, M1, 1, 0, h->Nt, M1, 1, 0,
                       nullptr, 1.0, 0.0));
    HIPCHK(h, scale_rows_cols(s, h->Nt, M1, h->w));
    HIPCHK(h, hipMemcpyAsync(y, h->rhs_c, (size_t)M1 * R * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, scale_rows(s, y, M1, R, h->w));
    HIPCHK(h, spd_solve_small(s, h->Nt, M1, y, R, h->gj_work, h->info));
    HIPCHK(h, gemm_f64(s, (int)t, R, M1, 1, h->Wp, M1, 1, 0, y, R, 1, 0, h->bt, R, 1, 0, h->w, 1.0,
                       0.0));
  }
  if (h->C_cap < Knew * R) {
    int64_t cap = Knew * R * 2;
    double *nc = nullptr, *nt = nullptr;
    OKCHK(dalloc(h, &nc, cap));
    OKCHK(dalloc(h, &nt, cap));
    if (h->K > 0)
      HIPCHK(h, hipMemcpyAsync(nc, h->Chist, h->K * R * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));
    dfree(h, h->Chist);
    dfree(h, h->Ctmp);
    h->Chist = nc;
    h->Ctmp = nt;
    h->C_cap = cap;
  }
  HIPCHK(h, rec_temporal_finish(s, R, h->K, t, h->kappa, h->tperm, h->tsign, h->bt, h->Chist,
                                h->Ctmp, h->have_prev ? 1 : 0));
  // H = Hcur + W^T C_new (canonical convention): the buffers trade places
  std::swap(h->H, h->Hcur);
  HIPCHK(h, rowdot(s, M1, R, t, h->Wp, 1, M1, h->bt, R, 1, nullptr, 1.0, 1.0, h->H, R, h->rd_work, octen_ctx::RD_WORK));
  // outputs in one launch; the canonical factors become the previous ones
  HIPCHK(h, rec_copy3(s, A, h->Ac, I * R, B, h->Bc, J * R, C, h->Chist, Knew * R));
  std::swap(h->Ac, h->Aprev);
  std::swap(h->Bc, h->Bprev);
  h->K = Knew;
  h->t_pend = 0;
  h->have_prev = true;
  h->factors_fresh = false;
  if (K_out_host) {
    *K_out_host = h->K;
    return report_health(h);
  }
  return OCTEN_OK;
}

octen_status octen_fit(octen_t h, const void* X, int64_t t, int64_t k0, const double* A,
                       const double* B, const double* C, double* out_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (!X || !A || !B || !C || !out_host || t < 1 || k0 < 0)
    return fail(h, OCTEN_ERR_ARG, "bad fit arguments");
  hipStream_t s = h->stream;
  int64_t rows = t * h->I;
  int parts = rows < FIT_PARTS ? (int)rows : FIT_PARTS;
  HIPCHK(h, fit_dense(s, X, h->cfg.x_dtype == OCTEN_F64, t, h->I, h->J, h->R, k0, A, B, C,
                      h->partials, parts, h->fit_out));
  double o[2];
  HIPCHK(h, hipMemcpyAsync(o, h->fit_out, sizeof(o), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  out_host[0] += o[0];
  out_host[1] += o[1];
  return OCTEN_OK;
}

octen_status octen_fit_coo(octen_t h, int64_t nnz, const int32_t* k, const int32_t* i,
                           const int32_t* j, const float* v, int64_t k0, const double* A,
                           const double* B, const double* C, int64_t kc, double* out_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (!A || !B || !C || !out_host || k0 < 0 || kc < 1 || nnz < 0 || nnz >= 0x7fffffffLL)
    return fail(h, OCTEN_ERR_ARG, "bad sparse fit arguments");
  if (nnz > 0 && (!k || !i || !j || !v)) return fail(h, OCTEN_ERR_ARG, "k, i, j, v must be non-null");
  if (nnz > 0 && k0 >= kc) return fail(h, OCTEN_ERR_ARG, "k0 must be < kc");
  hipStream_t s = h->stream;
  HIPCHK(h, fill_i32(s, h->coo_small, 1, 0));
  HIPCHK(h, coo_check(s, nnz, k, i, j, kc - k0, h->I, h->J, false, h->coo_small));
  int bad = 0;
  HIPCHK(h, hipMemcpyAsync(&bad, h->coo_small, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bad) return fail(h, OCTEN_ERR_ARG, "COO coordinate out of range");
  HIPCHK(h, fit_coo(s, nnz, k, i, j, v, k0, h->I, h->J, kc, h->R, A, B, C, h->fitG, h->partials,
                    FIT_PARTS, h->fit_out));
  double o[3];
  HIPCHK(h, hipMemcpyAsync(o, h->fit_out, sizeof(o), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  out_host[0] += o[0];
  out_host[1] += o[1];
  out_host[2] = o[2];
  return OCTEN_OK;
}

octen_status octen_stage_times(octen_t h, int32_t stage, double* ms_host, int32_t n,
                               int32_t* count_host) {
  if (!h || !ms_host || !count_host || n < 0) return OCTEN_ERR_ARG;
  if (stage < 0 || stage >= OCTEN_NUM_STAGES) return fail(h, OCTEN_ERR_ARG, "unknown stage");
  if (!h->timing) return fail(h, OCTEN_ERR_STATE, "handle created without OCTEN_FLAG_TIMING");
  const int64_t total = h->ev_count[stage];
  int64_t avail = total < OCTEN_TIMING_RING ? total : OCTEN_TIMING_RING;
  if (avail > n) avail = n;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int64_t q = 0; q < avail; ++q) {
    const int64_t run = total - avail + q;
    const int slot = (int)(run % OCTEN_TIMING_RING);
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev[stage][2 * slot], h->ev[stage][2 * slot + 1]));
    ms_host[q] = ms;
  }
  *count_host = (int32_t)avail;
  return OCTEN_OK;
}

octen_status octen_warmstart_set(octen_t h, octen_mlp_t m, const float* G, int32_t D) {
  if (!h) return OCTEN_ERR_ARG;
  if (!G) return fail(h, OCTEN_ERR_ARG, "sketch matrix must be non-null");
  if (D < 1 || D > 32) return fail(h, OCTEN_ERR_ARG, "sketch length must be in [1, 32]");
  const int Q = h->Q, R = h->R, P = h->P;
  if (P > 32) return fail(h, OCTEN_ERR_UNSUPPORTED, "the learned warm start takes at most 32 replicas");
  if (m && (m->L.nin != 4 * Q + D || m->L.nout != 3 * Q))
    return fail(h, OCTEN_ERR_ARG, "network must map 4Q + D inputs to 3Q outputs");
  const int64_t Q3 = (int64_t)Q * Q * Q;
  if (!h->ws_G || h->ws_D != D) {
    if (h->ws_G) { hipStreamSynchronize(h->stream); dfree(h, h->ws_G); dfree(h, h->ws_sk); dfree(h, h->ws_part); dfree(h, h->ws_X); }
    OKCHK(dalloc(h, &h->ws_G, (size_t)(D * Q3)));
    OKCHK(dalloc(h, &h->ws_sk, (size_t)P * D));
    h->ws_part_len = ws_sketch_part_len(P, Q, D);
    OKCHK(dalloc(h, &h->ws_part, (size_t)h->ws_part_len));
    OKCHK(dalloc(h, &h->ws_X, (size_t)P * R * (4 * Q + D)));
  }
  if (!h->ws_signs) {
    OKCHK(dalloc(h, &h->ws_signs, (size_t)P * R * 2));
    OKCHK(dalloc(h, &h->ws_u, (size_t)P * R * Q));
    OKCHK(dalloc(h, &h->ws_plain, (size_t)P * 3 * Q * R));
    OKCHK(dalloc(h, &h->ws_cand, (size_t)P * 3 * Q * R));
    OKCHK(dalloc(h, &h->ws_init, (size_t)P * 3 * Q * R));
    OKCHK(dalloc(h, &h->ws_Y, (size_t)P * R * 3 * Q));
    OKCHK(dalloc(h, &h->ws_jpart, (size_t)P * 2 * ws_judge_splits(Q) * 2));
    OKCHK(dalloc(h, &h->ws_fits, (size_t)P * 2));
    OKCHK(dalloc(h, &h->ws_keep, (size_t)P));
  }
  h->ws_D = D;
  HIPCHK(h, hipMemcpyAsync(h->ws_G, G, (size_t)D * Q3 * 4, hipMemcpyDeviceToDevice, h->stream));
  h->ws_mlp = m;
  h->ws_signs_ok = false;
  return OCTEN_OK;
}

octen_status octen_warmstart_features(octen_t h, float* X) {
  if (!h) return OCTEN_ERR_ARG;
  if (!h->ws_G) return fail(h, OCTEN_ERR_STATE, "octen_warmstart_set first");
  OKCHK(ws_features(h));
  if (X)
    HIPCHK(h, hipMemcpyAsync(X, h->ws_X, (size_t)h->P * h->R * (4 * h->Q + h->ws_D) * 4,
                             hipMemcpyDeviceToDevice, h->stream));
  return OCTEN_OK;
}

octen_status octen_warmstart_targets(octen_t h, float* T) {
  if (!h) return OCTEN_ERR_ARG;
  if (!T) return fail(h, OCTEN_ERR_ARG, "T is NULL");
  if (!h->ws_signs_ok) return fail(h, OCTEN_ERR_STATE, "features must be built first");
  HIPCHK(h, ws_columns(h->stream, h->F, h->lam, h->P, h->Q, h->R, h->ws_sk, h->ws_u, h->ws_D,
                       true, T, h->ws_signs, nullptr));
  return OCTEN_OK;
}

octen_status octen_get_state(octen_t h, int32_t what, void* dst, size_t bytes) {
  if (!h) return OCTEN_ERR_ARG;
  if (!dst) return fail(h, OCTEN_ERR_ARG, "dst is NULL");
  OKCHK(join_side(h));
  const int64_t P = h->P, Q = h->Q, R = h->R, M1 = h->M1;
  const void* src = nullptr;
  size_t n = 0;
  const size_t acc = h->acc_f64 ? 8 : 4;
  switch (what) {
    case OCTEN_STATE_Y: src = h->Y; n = P * Q * Q * Q * acc; break;
    case OCTEN_STATE_Z: src = h->Z; n = P * Q * Q * Q * acc; break;
    case OCTEN_STATE_FACTORS: src = h->F; n = P * 3 * Q * R * 8; break;
    case OCTEN_STATE_LAMBDA: src = h->lam; n = P * R * 8; break;
    case OCTEN_STATE_PERM: src = h->perm; n = P * R * 4; break;
    case OCTEN_STATE_ALIGNED: src = h->aligned; n = P * 3 * Q * R * 8; break;
    case OCTEN_STATE_RHS: src = h->rhs; n = 3 * M1 * R * 8; break;
    case OCTEN_STATE_H: src = h->H; n = M1 * R * 8; break;
    case OCTEN_STATE_TPERM: src = h->tperm; n = R * 4; break;
    case OCTEN_STATE_ITERS: src = h->iters; n = P * 4; break;
    case OCTEN_STATE_MARGIN: src = h->margin; n = P * 8; break;
    case OCTEN_STATE_FLAGS: src = h->flags; n = P * 4; break;
    case OCTEN_STATE_COO_SIZES:
    case OCTEN_STATE_COO_SEG_START:
    case OCTEN_STATE_COO_SEG_ROW:
    case OCTEN_STATE_COO_SLICE_SEG:
      if (h->coo_nseg < 0) return fail(h, OCTEN_ERR_STATE, "no sparse batch compressed yet");
      if (what == OCTEN_STATE_COO_SIZES) { src = h->coo_small + 1; n = 2 * 4; }
      if (what == OCTEN_STATE_COO_SEG_START) { src = h->seg_start; n = ((size_t)h->coo_nseg + 1) * 4; }
      if (what == OCTEN_STATE_COO_SEG_ROW) { src = h->seg_row; n = (size_t)h->coo_nseg * 4; }
      if (what == OCTEN_STATE_COO_SLICE_SEG) { src = h->slice_seg; n = ((size_t)h->coo_t + 1) * 4; }
      break;
    case OCTEN_STATE_WARM_KEEP:
    case OCTEN_STATE_WARM_FITS:
      if (!h->ws_keep) return fail(h, OCTEN_ERR_STATE, "no warm start set");
      if (what == OCTEN_STATE_WARM_KEEP) { src = h->ws_keep; n = P * 4; }
      else { src = h->ws_fits; n = P * 2 * 8; }
      break;
    default: return fail(h, OCTEN_ERR_ARG, "unknown state id");
  }
  if (bytes < n) return fail(h, OCTEN_ERR_ARG, "destination too small");
  HIPCHK(h, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, h->stream));
  return OCTEN_OK;
}

// ------------------------------------------------------------- autotuner ---

octen_status octen_compress_variant(octen_t h, int32_t variant) {
  if (!h) return OCTEN_ERR_ARG;
  OKCHK(join_side(h));
  if (!h->plan) return fail(h, OCTEN_ERR_UNSUPPORTED, "only MFMA compression has variants");
  if (variant < 0 || variant > 3) return fail(h, OCTEN_ERR_ARG, "variant must be in [0, 3]");
  if (variant == 3 && h->cfg.compress_dtype != OCTEN_BF16)
    return fail(h, OCTEN_ERR_UNSUPPORTED, "variant 3 is BF16 only");
  if (h->cfg.compress_dtype == OCTEN_BF16X2)
    return fail(h, OCTEN_ERR_UNSUPPORTED, "the two-term form has one kernel variant");
  mfma_plan_set_variant(h->plan, variant);
  return OCTEN_OK;
}

octen_status octen_autotune(octen_t h, const void* X, int64_t t, int32_t* choice_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (!h->plan) return fail(h, OCTEN_ERR_UNSUPPORTED, "only MFMA compression is tuned");
  if (!X || t < 1 || t > (1 << 24)) return fail(h, OCTEN_ERR_ARG, "X non-null and t >= 1 required");
  OKCHK(join_side(h));
  hipStream_t s = h->stream;
  const CompressShape sh{h->I, h->J, h->P, h->Q, h->S, h->M1};
  const int kind = mfma_kind(h->cfg.compress_dtype);
  const int gmax = mfma_plan_max_G(sh, kind);
  std::vector<int> gs{mfma_plan_G(h->plan)};
  if ((gmax + 1) / 2 != gs[0] && gmax > 1) gs.push_back((gmax + 1) / 2);
  const bool vec = (h->J % 4 == 0) && (((uintptr_t)X & 15) == 0);
  std::vector<int> variants = vec ? std::vector<int>{0, 1, 2} : std::vector<int>{2};
  if (vec && kind == 2) variants.push_back(3);   // half chunks, double-buffered fragments
  if (kind == 3) variants = {mfma_plan_variant(h->plan)};   // one kernel per load path
  std::vector<MfmaPlan*> plans{h->plan};
  for (size_t q = 1; q < gs.size(); ++q) {
    MfmaPlan* pl = nullptr;
    hipError_t e = mfma_plan_create(sh, kind, h->U, h->V, s, &pl, gs[q]);
    if (e != hipSuccess) break;
    plans.push_back(pl);
  }
  const size_t need = mfma_workspace_bytes(h->plan, t);
  if (need > h->mfma_work_bytes) {
    if (h->mfma_work) { hipStreamSynchronize(s); dfree(h, h->mfma_work); h->mfma_work = nullptr; }
    OKCHK(dalloc(h, (char**)&h->mfma_work, need));
    h->mfma_work_bytes = need;
  }
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  float best = 1e30f;
  size_t best_plan = 0;
  int best_var = mfma_plan_variant(h->plan);
  octen_status st = OCTEN_OK;
  for (size_t q = 0; q < plans.size() && st == OCTEN_OK; ++q) {
    for (int v : variants) {
      mfma_plan_set_variant(plans[q], v);
      hipError_t e = compress_mfma_main(s, plans[q], (const float*)X, t, nullptr, h->mfma_work);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r)
        e = compress_mfma_main(s, plans[q], (const float*)X, t, nullptr, h->mfma_work);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = fail(h, OCTEN_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
        break;
      }
      if (ms < best) { best = ms; best_plan = q; best_var = v; }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  for (size_t q = 0; q < plans.size(); ++q)
    if (q != best_plan && plans[q] != h->plan) mfma_plan_destroy(plans[q]);
  if (st != OCTEN_OK) {
    mfma_plan_set_variant(h->plan, 0);
    return st;
  }
  if (plans[best_plan] != h->plan) {
    mfma_plan_destroy(h->plan);
    h->plan = plans[best_plan];
  }
  mfma_plan_set_variant(h->plan, best_var);
  if (choice_host) *choice_host = 10 * mfma_plan_G(h->plan) + best_var;
  return OCTEN_OK;
}

octen_status octen_autotune_als(octen_t h, int32_t sweeps, int32_t* choice_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (sweeps < 1 || sweeps > 1000) return fail(h, OCTEN_ERR_ARG, "sweeps must be in [1, 1000]");
  if (!h->have_factors) return fail(h, OCTEN_ERR_STATE, "ALS must have run once (factors needed)");
  if (h->als_nw <= 0 || (h->cfg.flags & OCTEN_FLAG_ALS_ONE_WG))
    return fail(h, OCTEN_ERR_UNSUPPORTED, "no cooperative ALS on this handle");
  hipStream_t s = h->stream;
  const int P = h->P, Q = h->Q, R = h->R;
  const int per_xcd = (P + 7) / 8;
  int max_nw = 32 / per_xcd;
  if (max_nw > Q) max_nw = Q;
  const size_t cap = 160 * 1024;
  // candidates: (workgroups per replica, slab in global memory)
  std::vector<std::pair<int, bool>> cand;
  // every count that is the smallest one for its slab height ceil(Q / nw)
  for (int nw = 2; nw <= max_nw; ++nw) {
    if (balanced_nw(Q, nw) != nw) continue;
    if (als_coop_lds_bytes(Q, R, nw, h->acc_f64, false, h->als_split) <= cap) cand.push_back({nw, false});
    if (als_coop_lds_bytes(Q, R, nw, h->acc_f64, true, h->als_split) <= cap) cand.push_back({nw, true});
  }
  if (cand.empty()) return fail(h, OCTEN_ERR_UNSUPPORTED, "no cooperative configuration fits");
  // slots for the largest candidate; the current factors are kept aside
  int nw_big = 0;
  for (auto& c : cand) nw_big = c.first > nw_big ? c.first : nw_big;
  double* slots = nullptr;
  OKCHK(dalloc(h, &slots, (size_t)2 * P * nw_big * als_coop_slot_len(Q, R)));
  double *F0 = nullptr, *lam0 = nullptr;
  OKCHK(dalloc(h, &F0, (size_t)P * 3 * Q * R));
  OKCHK(dalloc(h, &lam0, (size_t)P * R));
  HIPCHK(h, hipMemcpyAsync(F0, h->F, (size_t)P * 3 * Q * R * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(lam0, h->lam, (size_t)P * R * 8, hipMemcpyDeviceToDevice, s));
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  // three rounds over the candidates (interleaved, so that a slow spell of
  // the device does not decide), the best time of each counts
  std::vector<float> best_ms(cand.size(), 1e30f);
  octen_status st = OCTEN_OK;
  for (int round = 0; round < 3; ++round) {
    for (size_t q = 0; q < cand.size(); ++q) {
      hipError_t e = als_coop(s, h->Y, h->acc_f64, P, Q, R, cand[q].first, cand[q].second, F0,
                              h->F, h->lam, h->iters, h->flags, slots, h->als_ctr, h->als_err, 1,
                              0.0, !(h->cfg.flags & OCTEN_FLAG_ALS_DEVICE_SYNC), h->als_split);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = als_coop(s, h->Y, h->acc_f64, P, Q, R, cand[q].first, cand[q].second, F0, h->F,
                     h->lam, h->iters, h->flags, slots, h->als_ctr, h->als_err, sweeps, 0.0,
                     !(h->cfg.flags & OCTEN_FLAG_ALS_DEVICE_SYNC), h->als_split);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      int err = 0;
      if (e == hipSuccess) e = hipMemcpy(&err, h->als_err, sizeof(int), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        continue;   // a configuration that cannot launch here is skipped
      }
      if (!err && ms < best_ms[q]) best_ms[q] = ms;
    }
  }
  int best_i = -1;
  for (size_t q = 0; q < cand.size(); ++q)
    if (best_ms[q] < 1e29f && (best_i < 0 || best_ms[q] < best_ms[best_i])) best_i = (int)q;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HIPCHK(h, hipMemcpyAsync(h->F, F0, (size_t)P * 3 * Q * R * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->lam, lam0, (size_t)P * R * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  dfree(h, F0);
  dfree(h, lam0);
  if (best_i < 0) {
    dfree(h, slots);
    return fail(h, OCTEN_ERR_HIP, "no cooperative ALS configuration ran");
  }
  dfree(h, h->als_slots);
  h->als_slots = slots;
  h->als_nw = cand[best_i].first;
  h->als_gx = cand[best_i].second;
  if (choice_host) *choice_host = 10 * h->als_nw + (h->als_gx ? 1 : 0);
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------- groups ---

struct octen_group {
  std::vector<octen_t> hs;
  hipStream_t user = nullptr;              // the handles' stream
  hipStream_t main = nullptr;              // capture origin
  std::vector<hipStream_t> branch;
  hipEvent_t fork = nullptr, done = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<octen_batch_desc> cap_desc;
  std::vector<int64_t> cap_tpend;
  std::vector<std::vector<const void*>> cap_bufs;
  int32_t cap_iters = 0;
  double cap_tol = 0.0;
  int32_t cap_init = 0;
  int32_t als_launches = 0;               // cooperative ALS launches per captured step
  std::string err;
};

namespace {

octen_status gfail(octen_group_t g, octen_status st, const std::string& m) {
  if (g) g->err = m;
  return st;
}

#define GHIP(g, expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return gfail((g), OCTEN_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// grow every buffer one step of depth t needs, so that a captured step
// allocates nothing
octen_status prepare_step(octen_t h, int64_t t) {
  const int64_t M1 = h->M1;
  OKCHK(dgrow(h, &h->Wz, &h->Wz_cap, t * M1));
  if (h->plan) {
    const size_t need = mfma_workspace_bytes(h->plan, t);
    if (need > h->mfma_work_bytes) {
      if (h->mfma_work) { hipStreamSynchronize(h->stream); dfree(h, h->mfma_work); h->mfma_work = nullptr; }
      OKCHK(dalloc(h, (char**)&h->mfma_work, need));
      h->mfma_work_bytes = need;
    }
  } else {
    int64_t rows_cap = ((int64_t)1 << 26) / M1;
    if (rows_cap < h->I) rows_cap = h->I;
    int64_t want = rows_cap < t * h->I ? rows_cap : t * h->I;
    want = (want / h->I) * h->I;
    OKCHK(dgrow(h, &h->T2, &h->T2_rows, want * M1));
    OKCHK(dgrow(h, &h->Mk, &h->Mk_cap, t * h->P * h->Q * h->Q));
  }
  if (h->t_pend + t > h->Wp_cap / M1) {
    double* nw = nullptr;
    const int64_t cap = (h->t_pend + t) * 2 * M1;
    OKCHK(dalloc(h, &nw, cap));
    if (h->t_pend > 0)
      HIPCHK(h, hipMemcpyAsync(nw, h->Wp, h->t_pend * M1 * 8, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    dfree(h, h->Wp);
    h->Wp = nw;
    h->Wp_cap = cap;
  }
  return OCTEN_OK;
}

struct HostState {
  bool z_ready, z_any, have_factors, factors_fresh;
  int64_t t_z, t_pend;
};
HostState save_state(octen_t h) {
  return {h->z_ready, h->z_any, h->have_factors, h->factors_fresh, h->t_z, h->t_pend};
}
void load_state(octen_t h, const HostState& s) {
  h->z_ready = s.z_ready; h->z_any = s.z_any; h->have_factors = s.have_factors;
  h->factors_fresh = s.factors_fresh; h->t_z = s.t_z; h->t_pend = s.t_pend;
}

// the buffers a captured step reads or writes besides the fixed ones
std::vector<const void*> step_buffers(octen_t h) {
  return {h->Wz, (const void*)h->Wz_cap, h->mfma_work, (const void*)h->mfma_work_bytes, h->T2,
          (const void*)h->T2_rows, h->Mk, (const void*)h->Mk_cap, h->Wp, (const void*)h->Wp_cap,
          h->plan, (const void*)(intptr_t)(h->plan ? mfma_plan_variant(h->plan) : -1)};
}

bool same_desc(const octen_batch_desc& a, const octen_batch_desc& b) {
  return a.X == b.X && a.t == b.t && a.W == b.W && a.slice_scale == b.slice_scale;
}

void drop_graph(octen_group_t g) {
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
}

}  // namespace

extern "C" {

octen_status octen_group_create(const octen_t* handles, int32_t n, octen_group_t* out) {
  if (!out) return OCTEN_ERR_ARG;
  *out = nullptr;
  if (!handles || n < 1 || n > 4096) return OCTEN_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!handles[i]) return OCTEN_ERR_ARG;
    if (handles[i]->stream != handles[0]->stream) return OCTEN_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (handles[j] == handles[i]) return OCTEN_ERR_ARG;
  }
  octen_group_t g = new octen_group();
  g->hs.assign(handles, handles + n);
  g->user = handles[0]->stream;
  bool ok = hipStreamCreateWithFlags(&g->main, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&g->done, hipEventDisableTiming) == hipSuccess;
  g->branch.assign(n, nullptr);
  g->join.assign(n, nullptr);
  for (int i = 0; ok && i < n; ++i)
    ok = hipStreamCreateWithFlags(&g->branch[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&g->join[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    octen_group_destroy(g);
    return OCTEN_ERR_HIP;
  }
  *out = g;
  return OCTEN_OK;
}

octen_status octen_group_destroy(octen_group_t g) {
  if (!g) return OCTEN_ERR_ARG;
  if (g->main) hipStreamSynchronize(g->main);
  drop_graph(g);
  for (auto b : g->branch)
    if (b) hipStreamDestroy(b);
  for (auto e : g->join)
    if (e) hipEventDestroy(e);
  if (g->fork) hipEventDestroy(g->fork);
  if (g->done) hipEventDestroy(g->done);
  if (g->main) hipStreamDestroy(g->main);
  delete g;
  return OCTEN_OK;
}

octen_status octen_group_recover(octen_group_t g, double* const* A, double* const* B,
                                 double* const* C, const int64_t* c_capacity) {
  if (!g) return OCTEN_ERR_ARG;
  if (!A || !B || !C || !c_capacity) return gfail(g, OCTEN_ERR_ARG, "null argument");
  const int n = (int)g->hs.size();
  GHIP(g, hipEventRecord(g->fork, g->user));
  octen_status st = OCTEN_OK;
  int used = 0;   // branches that hold work to join
  for (int i = 0; i < n && st == OCTEN_OK; ++i) {
    octen_t h = g->hs[i];
    if (h->stream != g->user) { st = gfail(g, OCTEN_ERR_STATE, "handle stream changed"); break; }
    const hipError_t e = hipStreamWaitEvent(g->branch[i], g->fork, 0);
    if (e != hipSuccess) { st = gfail(g, OCTEN_ERR_HIP, std::string("fork: ") + hipGetErrorString(e)); break; }
    used = i + 1;
    h->stream = g->branch[i];
    st = octen_recover_factors(h, A[i], B[i], C[i], c_capacity[i], nullptr);
    h->stream = g->user;
    if (st != OCTEN_OK) g->err = "handle " + std::to_string(i) + ": " + h->err;
  }
  // join every branch used, also after an error
  for (int i = 0; i < used; ++i) {
    hipError_t e = hipEventRecord(g->join[i], g->branch[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(g->user, g->join[i], 0);
    if (e != hipSuccess && st == OCTEN_OK)
      st = gfail(g, OCTEN_ERR_HIP, std::string("join: ") + hipGetErrorString(e));
  }
  return st;
}

octen_status octen_group_als_launches(octen_group_t g, int32_t* out_host) {
  if (!g || !out_host) return OCTEN_ERR_ARG;
  *out_host = g->exec ? g->als_launches : 0;
  return OCTEN_OK;
}

const char* octen_group_last_error(octen_group_t g) { return g ? g->err.c_str() : "null group"; }

octen_status octen_group_step(octen_group_t g, const octen_batch_desc* desc, int32_t max_iters,
                              double tol, int32_t init_mode, int32_t* replayed_host) {
  if (!g) return OCTEN_ERR_ARG;
  if (!desc || max_iters < 1 || !(tol >= 0.0)) return gfail(g, OCTEN_ERR_ARG, "bad arguments");
  if (init_mode != OCTEN_INIT_PREV && init_mode != OCTEN_INIT_LEARNED)
    return gfail(g, OCTEN_ERR_ARG, "init_mode must be OCTEN_INIT_PREV or OCTEN_INIT_LEARNED");
  const int n = (int)g->hs.size();
  for (int i = 0; i < n; ++i) {
    octen_t h = g->hs[i];
    if (!desc[i].X || !desc[i].W || desc[i].t < 1 || desc[i].t > (1 << 24))
      return gfail(g, OCTEN_ERR_ARG, "descriptor " + std::to_string(i) + " invalid");
    if (!h->have_factors)
      return gfail(g, OCTEN_ERR_STATE, "handle " + std::to_string(i) + " has no replica factors");
    if (h->z_ready)
      return gfail(g, OCTEN_ERR_STATE, "handle " + std::to_string(i) + " has a batch not yet added");
    if (h->stream != g->user) return gfail(g, OCTEN_ERR_STATE, "handle stream changed");
    if (init_mode == OCTEN_INIT_LEARNED && !h->ws_mlp)
      return gfail(g, OCTEN_ERR_STATE, "handle " + std::to_string(i) + " has no warm-start network");
  }
  bool replay = g->exec && g->cap_iters == max_iters && g->cap_tol == tol &&
                g->cap_init == init_mode;
  for (int i = 0; replay && i < n; ++i) {
    octen_t h = g->hs[i];
    replay = same_desc(desc[i], g->cap_desc[i]) && h->t_pend == g->cap_tpend[i] &&
             step_buffers(h) == g->cap_bufs[i];
  }
  // order after the user's stream
  GHIP(g, hipEventRecord(g->fork, g->user));
  GHIP(g, hipStreamWaitEvent(g->main, g->fork, 0));
  if (!replay) {
    drop_graph(g);
    std::vector<int64_t> tpend(n);
    std::vector<HostState> saved(n);
    int64_t replicas = 0;
    for (int i = 0; i < n; ++i) {
      OKCHK(prepare_step(g->hs[i], desc[i].t));
      if (init_mode == OCTEN_INIT_LEARNED) {
        const octen_status ms = octen_mlp_ensure_rows(g->hs[i]->ws_mlp, (int64_t)g->hs[i]->P * g->hs[i]->R);
        if (ms != OCTEN_OK) return gfail(g, ms, "warm-start network buffers");
      }
      tpend[i] = g->hs[i]->t_pend;
      saved[i] = save_state(g->hs[i]);
      replicas += g->hs[i]->P;
    }
    GHIP(g, hipStreamSynchronize(g->user));
    // A handle whose ALS is a cooperative grid runs it after the branches
    // join, one handle at a time, so that no cooperative grid ever shares the
    // GPU with other work of the step; the other handles run their ALS (one
    // workgroup per replica) inside their branch.
    (void)replicas;
    bool parallel_als = false;
    hipGraph_t graph = nullptr;
    octen_status st = OCTEN_OK;
    for (int attempt = 0; attempt < 2; ++attempt) {
      st = OCTEN_OK;
      graph = nullptr;
      GHIP(g, hipStreamBeginCapture(g->main, hipStreamCaptureModeThreadLocal));
      hipError_t he = hipEventRecord(g->fork, g->main);
      int done_i = 0;
      for (int i = 0; i < n && st == OCTEN_OK && he == hipSuccess; ++i) {
        octen_t h = g->hs[i];
        he = hipStreamWaitEvent(g->branch[i], g->fork, 0);
        if (he != hipSuccess) break;
        const bool timing = h->timing;
        h->timing = false;
        h->group_mode = true;
        h->stream = g->branch[i];
        st = octen_compress_batch(h, desc[i].X, desc[i].t, desc[i].W, desc[i].slice_scale);
        if (st == OCTEN_OK) st = octen_update_replicas(h);
        const bool coop = h->als_nw > 0 && !(h->cfg.flags & OCTEN_FLAG_ALS_ONE_WG);
        if (st == OCTEN_OK && (parallel_als || !coop))
          st = octen_cp_als_replicas(h, max_iters, tol, init_mode, nullptr, nullptr);
        h->stream = g->user;
        h->group_mode = false;
        h->timing = timing;
        if (st != OCTEN_OK) { g->err = "handle " + std::to_string(i) + ": " + h->err; break; }
        he = hipEventRecord(g->join[i], g->branch[i]);
        if (he == hipSuccess) he = hipStreamWaitEvent(g->main, g->join[i], 0);
        done_i = i + 1;
      }
      // after the join: every cooperative handle's starting point, then
      // their ALS in as few cooperative launches as fit, then the commits
      std::vector<AlsCoopItem> items;
      std::vector<int> who;
      for (int i = 0; !parallel_als && i < n && st == OCTEN_OK && he == hipSuccess && done_i == n;
           ++i) {
        octen_t h = g->hs[i];
        if (!(h->als_nw > 0 && !(h->cfg.flags & OCTEN_FLAG_ALS_ONE_WG))) continue;
        const bool timing = h->timing;
        AlsCoopItem it{};
        h->timing = false;
        h->stream = g->main;
        h->als_defer = &it;
        st = octen_cp_als_replicas(h, max_iters, tol, init_mode, nullptr, nullptr);
        h->als_defer = nullptr;
        h->stream = g->user;
        h->timing = timing;
        if (st != OCTEN_OK) g->err = "handle " + std::to_string(i) + ": " + h->err;
        if (st == OCTEN_OK && it.P > 0) {   // deferred (else run and committed in the call)
          items.push_back(it);
          who.push_back(i);
        }
      }
      if (st == OCTEN_OK && he == hipSuccess && !items.empty()) {
        int nl = 0;
        he = als_coop_group(g->main, items.data(), (int)items.size(), &nl);
        if (he == hipSuccess) g->als_launches = nl;
      }
      for (size_t k = 0; k < who.size() && st == OCTEN_OK && he == hipSuccess; ++k) {
        octen_t h = g->hs[who[k]];
        h->stream = g->main;
        st = als_finish(h);
        h->stream = g->user;
        if (st != OCTEN_OK) g->err = "handle " + std::to_string(who[k]) + ": " + h->err;
      }
      if (parallel_als) g->als_launches = 0;
      const hipError_t ee = hipStreamEndCapture(g->main, &graph);
      if (st == OCTEN_OK && he == hipSuccess && ee == hipSuccess && done_i == n) break;
      if (graph) hipGraphDestroy(graph);
      graph = nullptr;
      for (int i = 0; i < n; ++i) load_state(g->hs[i], saved[i]);
      (void)hipGetLastError();
      if (st == OCTEN_OK) {
        st = OCTEN_ERR_HIP;
        g->err = std::string("graph capture: ") + hipGetErrorString(he != hipSuccess ? he : ee);
      }
      if (parallel_als) return st;
      parallel_als = true;   // capture again with the ALS inside the branches
    }
    if (!graph) return st;
    g->graph = graph;
    GHIP(g, hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    g->cap_desc.assign(desc, desc + n);
    g->cap_tpend = tpend;
    g->cap_bufs.resize(n);
    for (int i = 0; i < n; ++i) g->cap_bufs[i] = step_buffers(g->hs[i]);
    g->cap_iters = max_iters;
    g->cap_tol = tol;
    g->cap_init = init_mode;
  } else {
    // the calls a capture records advance each handle's host state; a
    // replay applies the same transitions
    for (int i = 0; i < n; ++i) {
      octen_t h = g->hs[i];
      h->t_z = desc[i].t;
      h->z_any = true;
      h->t_pend += desc[i].t;
      h->z_ready = false;
      h->have_factors = true;
      h->factors_fresh = true;
    }
  }
  GHIP(g, hipGraphLaunch(g->exec, g->main));
  GHIP(g, hipEventRecord(g->done, g->main));
  GHIP(g, hipStreamWaitEvent(g->user, g->done, 0));
  if (replayed_host) *replayed_host = replay ? 1 : 0;
  return OCTEN_OK;
}

}  // extern "C"
