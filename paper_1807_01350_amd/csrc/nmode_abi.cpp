// C ABI of the N-mode extension (octen_nmode.h): handle state, argument
// validation and the launch sequence of each step for an N-mode tensor that
// grows in its last mode (supplement, "Extending to Higher-Order Tensors").
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/octen_nmode.h"
#include "octen_internal.h"

using namespace octen;

struct octen_nm_ctx {
  octen_nm_config cfg;
  int N = 0, nm = 0, R = 0, P = 0, Q = 0, S = 0, M1 = 0;
  int64_t dims[OCTEN_NM_MAX_MODES - 1] = {};
  int64_t QN = 0;                 // Q^N values per replica summary
  hipStream_t stream = nullptr;
  std::string err;

  // state machine (as in octen.h)
  bool z_ready = false;
  int64_t t_z = 0, t_pend = 0, K = 0;
  bool have_factors = false, factors_fresh = false, have_prev = false;

  // fixed operators, one per non-temporal mode
  double* U[OCTEN_NM_MAX_MODES - 1] = {};
  double* Op[OCTEN_NM_MAX_MODES - 1] = {};
  double *w = nullptr, *w2 = nullptr;       // [M1] row weights
  // summaries
  double *Y = nullptr, *Z = nullptr;        // [P][Q^N]
  // compression workspace
  double* Wz = nullptr;  int64_t Wz_cap = 0;
  double* Wp = nullptr;  int64_t Wp_cap = 0;
  double* T1 = nullptr;  int64_t T1_cap = 0;     // X times the last compression matrix
  double* Ta = nullptr;  int64_t Ta_cap = 0;     // per-replica partial contractions
  double* Tb = nullptr;  int64_t Tb_cap = 0;
  // ALS
  double *F = nullptr, *lam = nullptr, *F0 = nullptr, *lam0 = nullptr;
  int *flags = nullptr, *zbad = nullptr, *health = nullptr;
  double* als_work = nullptr;               // [P][nm_als_work_len] partial contractions
  unsigned* als_ctr = nullptr;              // [P] barrier counters of the ALS launch
  int* als_err = nullptr;                   // [1] a barrier of the ALS launch timed out
  // recovery
  double *aligned = nullptr, *margin = nullptr, *rhs = nullptr, *rhs_c = nullptr;
  int* perm = nullptr;
  double* Araw = nullptr;
  double* Ac[OCTEN_NM_MAX_MODES - 1] = {};
  double* Aprev[OCTEN_NM_MAX_MODES - 1] = {};
  double *kn = nullptr, *kprod = nullptr, *ones = nullptr, *kappa = nullptr;
  double *tsign = nullptr, *tmargin = nullptr;
  int* tperm = nullptr;
  double *cross = nullptr, *norms = nullptr;
  double *H = nullptr, *Hcur = nullptr;
  double *Chist = nullptr, *Ctmp = nullptr; int64_t C_cap = 0;
  double* Nt = nullptr; int64_t Nt_cap = 0;
  double* bt = nullptr; int64_t bt_cap = 0;
  int* info = nullptr;
  double *partials = nullptr, *fit_out = nullptr, *gj_work = nullptr, *rd_work = nullptr;
  static constexpr int64_t RD_WORK = 1 << 18;
  static constexpr int FIT_PARTS = 2048;

  std::vector<void*> allocs;
};

namespace {

octen_status fail(octen_nm_t h, octen_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

#define NMCHK(h, expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail((h), OCTEN_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define NMOK(expr)                       \
  do {                                   \
    octen_status s_ = (expr);            \
    if (s_ != OCTEN_OK) return s_;       \
  } while (0)

template <typename T>
octen_status dalloc(octen_nm_t h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(h, OCTEN_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = (T*)q;
  return OCTEN_OK;
}

void dfree(octen_nm_t h, void* p) {
  if (!p) return;
  for (auto& a : h->allocs)
    if (a == p) { hipFree(p); a = nullptr; return; }
}

// grow a device array to at least `count` elements (contents discarded)
template <typename T>
octen_status dgrow(octen_nm_t h, T** p, int64_t* cap, int64_t count) {
  if (*p && *cap >= count) return OCTEN_OK;
  if (*p) { hipStreamSynchronize(h->stream); dfree(h, *p); *p = nullptr; }
  const int64_t n = count < 1 ? 1 : count;
  octen_status st = dalloc(h, p, (size_t)n);
  if (st == OCTEN_OK) *cap = n;
  return st;
}

int64_t ipow(int64_t b, int e) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}

octen_status validate(const octen_nm_config* c, std::string* msg) {
  if (!c) { *msg = "config is NULL"; return OCTEN_ERR_ARG; }
  if (c->abi_version != OCTEN_ABI_VERSION) { *msg = "ABI version mismatch"; return OCTEN_ERR_ARG; }
  if (c->N < 3 || c->N > OCTEN_NM_MAX_MODES) { *msg = "N must be in [3, 6]"; return OCTEN_ERR_ARG; }
  if (c->R < 1 || c->R > 32) { *msg = "R must be in [1, 32]"; return OCTEN_ERR_ARG; }
  if (c->P < 1) { *msg = "P must be >= 1"; return OCTEN_ERR_ARG; }
  if (c->S < 1) { *msg = "S must be >= 1 (anchor rows are needed for matching)"; return OCTEN_ERR_ARG; }
  if (c->Q <= c->S) { *msg = "Q must be > S"; return OCTEN_ERR_ARG; }
  if (c->R > c->Q) { *msg = "R must be <= Q"; return OCTEN_ERR_ARG; }
  for (int n = 0; n < c->N - 1; ++n)
    if (c->dims[n] < 1 || c->dims[n] > (1LL << 30)) {
      *msg = "every dims[n] must be in [1, 2^30]";
      return OCTEN_ERR_ARG;
    }
  const int64_t M1 = (int64_t)c->S + (int64_t)c->P * (c->Q - c->S);
  if (M1 > (1 << 20)) { *msg = "too many compression columns"; return OCTEN_ERR_ARG; }
  // the replica ALS keeps one replica's factors and Grams in the LDS of one
  // workgroup
  if (c->Q > 32 || ipow(c->Q, c->N) > (1LL << 22) ||
      nm_als_lds_bytes(c->N, c->Q, c->R) > 160 * 1024 - 64) {
    *msg = "sizes outside the N-mode limits (Q <= 32, Q^N <= 2^22)";
    return OCTEN_ERR_UNSUPPORTED;
  }
  return OCTEN_OK;
}

// Least-squares operator of Eq. 7 for the fixed compression matrix Pt
// (n x M1) of one non-temporal mode: x = Op * rhs is the minimum-norm
// solution of the sqrt(P)-weighted deduplicated stack.
octen_status build_operator(octen_nm_t h, const double* Pt, int64_t n, double* Op) {
  hipStream_t s = h->stream;
  const int M1 = h->M1;
  double* Nm = nullptr;
  if (n <= M1) {
    NMOK(dalloc(h, &Nm, (size_t)(n * n)));
    NMCHK(h, gemm_f64(s, (int)n, (int)n, M1, 1, Pt, M1, 1, 0, Pt, 1, M1, 0, Nm, n, 1, 0, h->w2,
                      1.0, 0.0));
    NMCHK(h, spd_invert(s, Nm, (int)n, h->gj_work, h->info));
    NMCHK(h, gemm_f64(s, (int)n, M1, (int)n, 1, Nm, n, 1, 0, Pt, M1, 1, 0, Op, M1, 1, 0, nullptr,
                      1.0, 0.0));
    NMCHK(h, scale_cols(s, Op, n, M1, h->w2));
  } else {
    NMOK(dalloc(h, &Nm, (size_t)M1 * M1));
    NMCHK(h, gemm_f64(s, M1, M1, (int)n, 1, Pt, 1, M1, 0, Pt, M1, 1, 0, Nm, M1, 1, 0, nullptr, 1.0,
                      0.0));
    NMCHK(h, scale_rows_cols(s, Nm, M1, h->w));
    NMCHK(h, spd_invert(s, Nm, M1, h->gj_work, h->info));
    NMCHK(h, gemm_f64(s, (int)n, M1, M1, 1, Pt, M1, 1, 0, Nm, M1, 1, 0, Op, M1, 1, 0, h->w, 1.0,
                      0.0));
    NMCHK(h, scale_cols(s, Op, n, M1, h->w));
  }
  NMCHK(h, hipStreamSynchronize(s));
  dfree(h, Nm);
  return OCTEN_OK;
}

// Waits for the stream, reads and clears the health bits.
octen_status report_health(octen_nm_t h) {
  int v = 0;
  NMCHK(h, hipMemcpyAsync(&v, h->health, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  NMCHK(h, hipStreamSynchronize(h->stream));
  if (v == 0) return OCTEN_OK;
  NMCHK(h, fill_i32(h->stream, h->health, 1, 0));
  std::string what;
  if (v & OCTEN_HEALTH_NONFINITE_BATCH) what += "non-finite compressed batch (summaries not updated)";
  if (v & OCTEN_HEALTH_ALS_FAILED) {
    if (!what.empty()) what += "; ";
    what += "replica ALS failed (starting factors kept)";
  }
  return fail(h, OCTEN_ERR_NUMERIC, what);
}

}  // namespace

extern "C" {

octen_status octen_nm_init(const octen_nm_config* cfg, const double* const* U, void* stream,
                           octen_nm_t* out) {
  if (!out) return OCTEN_ERR_ARG;
  *out = nullptr;
  std::string msg;
  octen_status st = validate(cfg, &msg);
  if (st != OCTEN_OK) return st;
  if (!U) return OCTEN_ERR_ARG;
  for (int n = 0; n < cfg->N - 1; ++n)
    if (!U[n]) return OCTEN_ERR_ARG;
  octen_nm_t h = new octen_nm_ctx();
  h->cfg = *cfg;
  h->N = cfg->N; h->nm = cfg->N - 1;
  h->R = cfg->R; h->P = cfg->P; h->Q = cfg->Q; h->S = cfg->S;
  h->M1 = h->S + h->P * (h->Q - h->S);
  for (int n = 0; n < h->nm; ++n) h->dims[n] = cfg->dims[n];
  h->QN = ipow(h->Q, h->N);
  h->stream = (hipStream_t)stream;
  const int64_t P = h->P, Q = h->Q, R = h->R, M1 = h->M1, N = h->N, nm = h->nm;
  int64_t dmax = M1;
  for (int n = 0; n < nm; ++n) dmax = h->dims[n] > dmax ? h->dims[n] : dmax;
  auto bail = [&](octen_status s2) { octen_nm_destroy(h); return s2; };
#define IOK(expr)                        \
  do {                                   \
    octen_status s_ = (expr);            \
    if (s_ != OCTEN_OK) return bail(s_); \
  } while (0)
  for (int n = 0; n < nm; ++n) {
    IOK(dalloc(h, &h->U[n], h->dims[n] * M1));
    IOK(dalloc(h, &h->Op[n], h->dims[n] * M1));
    IOK(dalloc(h, &h->Ac[n], h->dims[n] * R));
    IOK(dalloc(h, &h->Aprev[n], h->dims[n] * R));
  }
  IOK(dalloc(h, &h->w, M1));
  IOK(dalloc(h, &h->w2, M1));
  IOK(dalloc(h, &h->Y, P * h->QN));
  IOK(dalloc(h, &h->Z, P * h->QN));
  IOK(dalloc(h, &h->F, P * N * Q * R));
  IOK(dalloc(h, &h->lam, P * R));
  IOK(dalloc(h, &h->F0, P * N * Q * R));
  IOK(dalloc(h, &h->lam0, P * R));
  IOK(dalloc(h, &h->als_work, P * nm_als_work_len((int)N, (int)Q, (int)R, (int)P)));
  IOK(dalloc(h, &h->als_ctr, P));
  IOK(dalloc(h, &h->als_err, 1));
  IOK(dalloc(h, &h->flags, P));
  IOK(dalloc(h, &h->zbad, P));
  IOK(dalloc(h, &h->health, 1));
  IOK(dalloc(h, &h->aligned, P * N * Q * R));
  IOK(dalloc(h, &h->margin, P));
  IOK(dalloc(h, &h->perm, P * R));
  IOK(dalloc(h, &h->rhs, N * M1 * R));
  IOK(dalloc(h, &h->rhs_c, M1 * R));
  IOK(dalloc(h, &h->Araw, dmax * R));
  IOK(dalloc(h, &h->kn, nm * R));
  IOK(dalloc(h, &h->kprod, R));
  IOK(dalloc(h, &h->ones, R));
  IOK(dalloc(h, &h->kappa, R));
  IOK(dalloc(h, &h->tsign, R));
  IOK(dalloc(h, &h->tmargin, 1));
  IOK(dalloc(h, &h->tperm, R));
  IOK(dalloc(h, &h->cross, nm * R * R));
  IOK(dalloc(h, &h->norms, nm * 2 * R));
  IOK(dalloc(h, &h->H, M1 * R));
  IOK(dalloc(h, &h->Hcur, M1 * R));
  IOK(dalloc(h, &h->info, 1));
  IOK(dalloc(h, &h->partials, 2 * octen_nm_ctx::FIT_PARTS));
  IOK(dalloc(h, &h->fit_out, 2));
  IOK(dalloc(h, &h->gj_work, 2 * dmax));
  IOK(dalloc(h, &h->rd_work, (size_t)octen_nm_ctx::RD_WORK));
  hipStream_t s = h->stream;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) { h->err = std::string(what) + ": " + hipGetErrorString(e); return false; }
    return true;
  };
  for (int n = 0; n < nm; ++n)
    if (!hip_ok(hipMemcpyAsync(h->U[n], U[n], h->dims[n] * M1 * 8, hipMemcpyDeviceToDevice, s),
                "copy U"))
      return bail(OCTEN_ERR_HIP);
  if (!hip_ok(fill_f64(s, h->Y, P * h->QN, 0.0), "zero Y") ||
      !hip_ok(fill_f64(s, h->Z, P * h->QN, 0.0), "zero Z") ||
      !hip_ok(fill_f64(s, h->H, M1 * R, 0.0), "zero H") ||
      !hip_ok(fill_f64(s, h->tsign, R, 1.0), "tsign") ||
      !hip_ok(fill_i32(s, h->info, 1, 0), "zero info") ||
      !hip_ok(fill_i32(s, h->flags, P, 0), "zero flags") ||
      !hip_ok(fill_i32(s, h->zbad, P, 0), "zero zbad") ||
      !hip_ok(fill_i32(s, h->health, 1, 0), "zero health") ||
      !hip_ok(rec_weights(s, (int)M1, h->S, (int)P, h->w, h->w2), "weights"))
    return bail(OCTEN_ERR_HIP);
  {
    std::vector<int> ident(R);
    for (int r = 0; r < R; ++r) ident[r] = r;
    if (!hip_ok(hipMemcpyAsync(h->tperm, ident.data(), R * sizeof(int), hipMemcpyHostToDevice, s),
                "tperm") ||
        !hip_ok(hipStreamSynchronize(s), "sync"))
      return bail(OCTEN_ERR_HIP);
  }
  for (int n = 0; n < nm; ++n) IOK(build_operator(h, h->U[n], h->dims[n], h->Op[n]));
  {
    int v = 0;
    if (!hip_ok(hipMemcpy(&v, h->info, sizeof(int), hipMemcpyDeviceToHost), "info"))
      return bail(OCTEN_ERR_HIP);
    if (v != 0) return bail(OCTEN_ERR_NUMERIC);   // a compression matrix without full rank
  }
#undef IOK
  *out = h;
  return OCTEN_OK;
}

octen_status octen_nm_destroy(octen_nm_t h) {
  if (!h) return OCTEN_ERR_ARG;
  hipStreamSynchronize(h->stream);
  for (void* p : h->allocs)
    if (p) hipFree(p);
  delete h;
  return OCTEN_OK;
}

const char* octen_nm_last_error(octen_nm_t h) { return h ? h->err.c_str() : "null handle"; }

// Supplement, compressed cubes: the last non-temporal mode against all M1
// compression columns at once (one GEMM, the shared columns computed once),
// the other non-temporal modes contracted from the last to the first on FP64
// matrix cores (the first of them reading each replica's columns of the GEMM
// output in place), the temporal mode with W_p last.
octen_status octen_nm_compress_batch(octen_nm_t h, const double* X, int64_t t, const double* W) {
  if (!h) return OCTEN_ERR_ARG;
  if (!X || !W || t < 1) return fail(h, OCTEN_ERR_ARG, "X, W must be non-null and t >= 1");
  if (t > (1 << 24)) return fail(h, OCTEN_ERR_ARG, "t too large");
  hipStream_t s = h->stream;
  const int nm = h->nm, P = h->P, Q = h->Q, S = h->S, M1 = h->M1;
  const int64_t Ilast = h->dims[nm - 1];
  int64_t rows = t;   // t * I_1 * ... * I_{N-2}
  for (int n = 0; n < nm - 1; ++n) rows *= h->dims[n];
  if (rows > 0x7fffffffLL) return fail(h, OCTEN_ERR_ARG, "batch too large (t * I_1 ... I_{N-2})");
  // workspace: the largest per-replica intermediate of the mode products
  // (after mode N-2: t I_1 ... I_{N-3} Q^2, then smaller)
  int64_t big = 0;
  {
    int64_t pre = rows, post = Q;
    for (int m = nm - 2; m >= 0; --m) {
      pre /= h->dims[m];
      big = pre * Q * post > big ? pre * Q * post : big;
      post *= Q;
    }
  }
  NMOK(dgrow(h, &h->Wz, &h->Wz_cap, t * M1));
  NMOK(dgrow(h, &h->T1, &h->T1_cap, rows * M1));
  NMOK(dgrow(h, &h->Ta, &h->Ta_cap, (int64_t)P * big));
  NMOK(dgrow(h, &h->Tb, &h->Tb_cap, (int64_t)P * big));
  NMCHK(h, hipMemcpyAsync(h->Wz, W, t * M1 * 8, hipMemcpyDeviceToDevice, s));
  NMCHK(h, fill_i32(s, h->zbad, P, 0));
  NMCHK(h, gemm_f64(s, (int)rows, M1, (int)Ilast, 1, X, Ilast, 1, 0, h->U[nm - 1], M1, 1, 0, h->T1,
                    M1, 1, 0, nullptr, 1.0, 0.0));
  // the remaining non-temporal modes, last to first; the first product reads
  // each replica's columns of T1 in place
  const double* cur = h->T1;
  double* nxt = h->Ta;
  int64_t pre = rows, post = Q;
  for (int m = nm - 2; m >= 0; --m) {
    const int64_t d = h->dims[m];
    pre /= d;
    const bool first = m == nm - 2;
    NMCHK(h, nm_ttm_mfma(s, cur, first ? 0 : pre * d * post, first, pre, (int)d, (int)post,
                         h->U[m], M1, P, Q, S, nxt, pre * Q * post));
    post *= Q;
    cur = nxt;
    nxt = nxt == h->Ta ? h->Tb : h->Ta;
  }
  // cur: [P][t][Q^{N-1}]
  NMCHK(h, nm_temporal(s, cur, t * post, t, post, h->Wz, M1, P, Q, S, h->Z, h->zbad));
  h->z_ready = true;
  h->t_z = t;
  return OCTEN_OK;
}

octen_status octen_nm_update_replicas(octen_nm_t h) {
  if (!h) return OCTEN_ERR_ARG;
  if (!h->z_ready) return fail(h, OCTEN_ERR_STATE, "update before compress");
  hipStream_t s = h->stream;
  NMCHK(h, update_masked(s, h->Y, h->Z, h->P, h->QN, true, h->zbad, h->health));
  const int64_t M1 = h->M1;
  if (h->t_pend + h->t_z > h->Wp_cap / M1) {
    double* nw = nullptr;
    const int64_t cap = (h->t_pend + h->t_z) * 2 * M1;
    NMOK(dalloc(h, &nw, cap));
    if (h->t_pend > 0)
      NMCHK(h, hipMemcpyAsync(nw, h->Wp, h->t_pend * M1 * 8, hipMemcpyDeviceToDevice, s));
    NMCHK(h, hipStreamSynchronize(s));
    dfree(h, h->Wp);
    h->Wp = nw;
    h->Wp_cap = cap;
  }
  NMCHK(h, hipMemcpyAsync(h->Wp + h->t_pend * M1, h->Wz, h->t_z * M1 * 8, hipMemcpyDeviceToDevice,
                          s));
  h->t_pend += h->t_z;
  h->z_ready = false;
  h->factors_fresh = false;
  return OCTEN_OK;
}

octen_status octen_nm_cp_als_replicas(octen_nm_t h, int32_t iters, int32_t init_mode,
                                      const double* init) {
  if (!h) return OCTEN_ERR_ARG;
  if (iters < 1) return fail(h, OCTEN_ERR_ARG, "iters must be >= 1");
  if (h->K + h->t_pend == 0) return fail(h, OCTEN_ERR_STATE, "no summaries yet");
  const double* src;
  if (init_mode == OCTEN_INIT_GIVEN) {
    if (!init) return fail(h, OCTEN_ERR_ARG, "init is NULL with OCTEN_INIT_GIVEN");
    src = init;
  } else if (init_mode == OCTEN_INIT_PREV) {
    if (!h->have_factors) return fail(h, OCTEN_ERR_STATE, "no previous factors");
    src = h->F;
  } else {
    return fail(h, OCTEN_ERR_ARG, "init_mode must be OCTEN_INIT_GIVEN or OCTEN_INIT_PREV");
  }
  hipStream_t s = h->stream;
  const int64_t per = (int64_t)h->N * h->Q * h->R;
  NMCHK(h, hipMemcpyAsync(h->F0, src, (size_t)h->P * per * 8, hipMemcpyDeviceToDevice, s));
  if (init_mode == OCTEN_INIT_GIVEN || !h->have_factors)
    NMCHK(h, fill_f64(s, h->lam0, (int64_t)h->P * h->R, 1.0));
  else
    NMCHK(h, hipMemcpyAsync(h->lam0, h->lam, (size_t)h->P * h->R * 8, hipMemcpyDeviceToDevice, s));
  NMCHK(h, fill_i32(s, h->flags, h->P, 0));
  NMCHK(h, nm_als(s, h->Y, h->P, h->N, h->Q, h->R, src, h->F, h->lam, h->flags, iters,
                  h->als_work, h->als_ctr, h->als_err));
  NMCHK(h, als_commit(s, h->P, (int)per, h->R, h->F, h->lam, h->F0, h->lam0, h->flags, h->health));
  h->have_factors = true;
  h->factors_fresh = true;
  return OCTEN_OK;
}

// Sec. 4.2 matching over N modes, Eq. 7 per non-temporal mode, canonical
// columns, the temporal rows with the carried history removed, the history
// update.
octen_status octen_nm_recover_factors(octen_nm_t h, double* const* A, double* C,
                                      int64_t c_capacity, int64_t* K_out_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (!A || !C) return fail(h, OCTEN_ERR_ARG, "A and C must be non-null");
  for (int n = 0; n < h->nm; ++n)
    if (!A[n]) return fail(h, OCTEN_ERR_ARG, "every A[n] must be non-null");
  if (!h->factors_fresh || h->t_pend == 0)
    return fail(h, OCTEN_ERR_STATE, "recover needs ALS after the latest update");
  const int64_t Knew = h->K + h->t_pend;
  if (c_capacity < Knew) return fail(h, OCTEN_ERR_ARG, "C capacity smaller than K");
  hipStream_t s = h->stream;
  const int P = h->P, Q = h->Q, R = h->R, S = h->S, M1 = h->M1, N = h->N, nm = h->nm;
  const int64_t t = h->t_pend;
  double* wk = h->rd_work;
  const int64_t wl = octen_nm_ctx::RD_WORK;
  NMCHK(h, nm_align(s, h->F, h->lam, P, N, Q, R, S, h->aligned, h->perm, h->margin));
  NMCHK(h, nm_stack(s, h->aligned, P, N, Q, R, S, h->rhs));
  for (int n = 0; n < nm; ++n) {
    const int64_t In = h->dims[n];
    NMCHK(h, rowdot(s, In, R, M1, h->Op[n], M1, 1, h->rhs + (int64_t)n * M1 * R, R, 1, nullptr,
                    1.0, 0.0, h->Araw, R, wk, wl));
    NMCHK(h, rec_canon(s, In, R, h->Araw, h->Ac[n], h->kn + (int64_t)n * R, wk, wl));
  }
  NMCHK(h, nm_kappa(s, h->kn, nm, R, h->kprod, h->ones));
  if (h->have_prev) {
    for (int n = 0; n < nm; ++n) {
      const int64_t In = h->dims[n];
      NMCHK(h, rowdot(s, R, R, In, h->Ac[n], 1, R, h->Aprev[n], R, 1, nullptr, 1.0, 0.0,
                      h->cross + (int64_t)n * R * R, R, wk, wl));
      NMCHK(h, rec_col_norms(s, In, R, h->Ac[n], h->norms + (int64_t)(2 * n) * R, wk, wl));
      NMCHK(h, rec_col_norms(s, In, R, h->Aprev[n], h->norms + (int64_t)(2 * n + 1) * R, wk, wl));
    }
    NMCHK(h, nm_tmatch(s, h->cross, h->norms, nm, R, h->tperm, h->tsign, h->tmargin));
  }
  const double* rhsT = h->rhs + (int64_t)(N - 1) * M1 * R;
  NMCHK(h, rec_temporal_prep(s, M1, R, h->H, h->tperm, h->tsign, h->kprod, h->ones, h->kappa,
                             h->Hcur, rhsT, h->rhs_c, h->have_prev ? 1 : 0));
  NMOK(dgrow(h, &h->bt, &h->bt_cap, (t > M1 ? t : (int64_t)M1) * R));
  if (t <= M1) {
    NMOK(dgrow(h, &h->Nt, &h->Nt_cap, t * t));
    NMCHK(h, rowdot(s, t, (int)t, M1, h->Wp, M1, 1, h->Wp, 1, M1, h->w2, 1.0, 0.0, h->Nt, t, wk, wl));
    NMCHK(h, rowdot(s, t, R, M1, h->Wp, M1, 1, h->rhs_c, R, 1, h->w2, 1.0, 0.0, h->bt, R, wk, wl));
    NMCHK(h, spd_solve_small(s, h->Nt, (int)t, h->bt, R, h->gj_work, h->info));
  } else {
    NMOK(dgrow(h, &h->Nt, &h->Nt_cap, (int64_t)M1 * M1 + (int64_t)M1 * R));
    double* y = h->Nt + (int64_t)M1 * M1;
    NMCHK(h, gemm_f64(s, M1, M1, (int)t, 1, h->Wp, 1, M1, 0, h->Wp, M1, 1, 0, h->Nt, M1, 1, 0,
                      nullptr, 1.0, 0.0));
    NMCHK(h, scale_rows_cols(s, h->Nt, M1, h->w));
    NMCHK(h, hipMemcpyAsync(y, h->rhs_c, (size_t)M1 * R * 8, hipMemcpyDeviceToDevice, s));
    NMCHK(h, scale_rows(s, y, M1, R, h->w));
    NMCHK(h, spd_solve_small(s, h->Nt, M1, y, R, h->gj_work, h->info));
    NMCHK(h, gemm_f64(s, (int)t, R, M1, 1, h->Wp, M1, 1, 0, y, R, 1, 0, h->bt, R, 1, 0, h->w, 1.0,
                      0.0));
  }
  if (h->C_cap < Knew * R) {
    const int64_t cap = Knew * R * 2;
    double *nc = nullptr, *nt = nullptr;
    NMOK(dalloc(h, &nc, cap));
    NMOK(dalloc(h, &nt, cap));
    if (h->K > 0)
      NMCHK(h, hipMemcpyAsync(nc, h->Chist, h->K * R * 8, hipMemcpyDeviceToDevice, s));
    NMCHK(h, hipStreamSynchronize(s));
    dfree(h, h->Chist);
    dfree(h, h->Ctmp);
    h->Chist = nc;
    h->Ctmp = nt;
    h->C_cap = cap;
  }
  NMCHK(h, rec_temporal_finish(s, R, h->K, t, h->kappa, h->tperm, h->tsign, h->bt, h->Chist,
                               h->Ctmp, h->have_prev ? 1 : 0));
  // H = Hcur + W^T C_new: the buffers trade places
  std::swap(h->H, h->Hcur);
  NMCHK(h, rowdot(s, M1, R, t, h->Wp, 1, M1, h->bt, R, 1, nullptr, 1.0, 1.0, h->H, R, wk, wl));
  for (int n = 0; n < nm; ++n)
    NMCHK(h, hipMemcpyAsync(A[n], h->Ac[n], h->dims[n] * R * 8, hipMemcpyDeviceToDevice, s));
  NMCHK(h, hipMemcpyAsync(C, h->Chist, Knew * R * 8, hipMemcpyDeviceToDevice, s));
  for (int n = 0; n < nm; ++n) std::swap(h->Ac[n], h->Aprev[n]);
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

octen_status octen_nm_fit(octen_nm_t h, const double* X, int64_t t, int64_t k0,
                          const double* const* A, const double* C, double* out_host) {
  if (!h) return OCTEN_ERR_ARG;
  if (!X || !A || !C || !out_host || t < 1 || k0 < 0)
    return fail(h, OCTEN_ERR_ARG, "bad fit arguments");
  for (int n = 0; n < h->nm; ++n)
    if (!A[n]) return fail(h, OCTEN_ERR_ARG, "every A[n] must be non-null");
  hipStream_t s = h->stream;
  NMCHK(h, nm_fit(s, X, t, h->dims, h->nm, A, C, h->R, k0, h->partials, octen_nm_ctx::FIT_PARTS,
                  h->fit_out));
  double o[2];
  NMCHK(h, hipMemcpyAsync(o, h->fit_out, sizeof(o), hipMemcpyDeviceToHost, s));
  NMCHK(h, hipStreamSynchronize(s));
  out_host[0] += o[0];
  out_host[1] += o[1];
  return OCTEN_OK;
}

octen_status octen_nm_get_state(octen_nm_t h, int32_t what, void* dst, size_t bytes) {
  if (!h) return OCTEN_ERR_ARG;
  if (!dst) return fail(h, OCTEN_ERR_ARG, "dst is NULL");
  const int64_t P = h->P, Q = h->Q, R = h->R, M1 = h->M1, N = h->N;
  const void* src = nullptr;
  size_t n = 0;
  switch (what) {
    case OCTEN_STATE_Y: src = h->Y; n = P * h->QN * 8; break;
    case OCTEN_STATE_Z: src = h->Z; n = P * h->QN * 8; break;
    case OCTEN_STATE_FACTORS: src = h->F; n = P * N * Q * R * 8; break;
    case OCTEN_STATE_LAMBDA: src = h->lam; n = P * R * 8; break;
    case OCTEN_STATE_PERM: src = h->perm; n = P * R * 4; break;
    case OCTEN_STATE_ALIGNED: src = h->aligned; n = P * N * Q * R * 8; break;
    case OCTEN_STATE_RHS: src = h->rhs; n = N * M1 * R * 8; break;
    case OCTEN_STATE_H: src = h->H; n = M1 * R * 8; break;
    case OCTEN_STATE_TPERM: src = h->tperm; n = R * 4; break;
    case OCTEN_STATE_MARGIN: src = h->margin; n = P * 8; break;
    case OCTEN_STATE_FLAGS: src = h->flags; n = P * 4; break;
    default: return fail(h, OCTEN_ERR_ARG, "unknown state id");
  }
  if (bytes < n) return fail(h, OCTEN_ERR_ARG, "destination too small");
  NMCHK(h, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, h->stream));
  return OCTEN_OK;
}

}  // extern "C"
