// C ABI of the warm-start network: creation from given parameters, forward,
// gradients, Adam and the fused training step.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/octen.h"
#include "mlp_ctx.h"
#include "octen_internal.h"

using namespace octen;

namespace {

constexpr int MSE_PARTS = 1024;

octen_status mfail(octen_mlp_t m, octen_status st, const std::string& msg) {
  if (m) m->err = msg;
  return st;
}

#define MHIP(m, expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return mfail((m), OCTEN_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
octen_status malloc_dev(octen_mlp_t m, T** p, int64_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)(count < 1 ? 1 : count) * sizeof(T));
  if (e != hipSuccess) return mfail(m, OCTEN_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  m->allocs.push_back(q);
  *p = (T*)q;
  return OCTEN_OK;
}

void free_dev(octen_mlp_t m, void* p) {
  for (auto& a : m->allocs)
    if (a == p) { hipFree(p); a = nullptr; }
}

// activation buffers for n rows
octen_status ensure_rows(octen_mlp_t m, int64_t n) {
  if (n <= m->cap) return OCTEN_OK;
  hipStreamSynchronize(m->stream);
  for (float* p : {m->H1, m->H2, m->Y, m->dY, m->dZ1, m->dZ2})
    if (p) free_dev(m, p);
  const int64_t nh = m->L.nh, nout = m->L.nout;
  octen_status st;
  if ((st = malloc_dev(m, &m->H1, n * nh)) != OCTEN_OK) return st;
  if ((st = malloc_dev(m, &m->H2, n * nh)) != OCTEN_OK) return st;
  if ((st = malloc_dev(m, &m->Y, n * nout)) != OCTEN_OK) return st;
  if ((st = malloc_dev(m, &m->dY, n * nout)) != OCTEN_OK) return st;
  if ((st = malloc_dev(m, &m->dZ1, n * nh)) != OCTEN_OK) return st;
  if ((st = malloc_dev(m, &m->dZ2, n * nh)) != OCTEN_OK) return st;
  m->cap = n;
  return OCTEN_OK;
}

octen_status check_rows(octen_mlp_t m, int64_t n) {
  if (n < 1 || n > (1 << 24)) return mfail(m, OCTEN_ERR_ARG, "row count must be in [1, 2^24]");
  return ensure_rows(m, n);
}

// forward, loss and backward into m->g; loss left on the device
octen_status grads_into(octen_mlp_t m, const float* X, const float* T, int64_t n) {
  octen_status st = check_rows(m, n);
  if (st != OCTEN_OK) return st;
  hipStream_t s = m->stream;
  MHIP(m, mlp_forward(s, m->L, m->w, X, n, m->H1, m->H2, m->Y));
  MHIP(m, mlp_mse(s, m->Y, T, n * m->L.nout, m->dY, m->partials, MSE_PARTS, m->loss));
  MHIP(m, mlp_backward(s, m->L, m->w, X, n, m->H1, m->H2, m->dY, m->dZ2, m->dZ1, m->g));
  return OCTEN_OK;
}

octen_status read_loss(octen_mlp_t m, double* loss_host) {
  if (!loss_host) return OCTEN_OK;
  MHIP(m, hipMemcpyAsync(loss_host, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->stream));
  MHIP(m, hipStreamSynchronize(m->stream));
  return OCTEN_OK;
}

}  // namespace

octen_status octen_mlp_ensure_rows(octen_mlp* m, int64_t n) { return ensure_rows(m, n); }

extern "C" {

int64_t octen_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out) {
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || n_out > n_in) return -1;
  return mlp_param_count(n_in, n_hidden, n_out);
}

octen_status octen_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, const float* params,
                              void* stream, octen_mlp_t* out) {
  if (!out) return OCTEN_ERR_ARG;
  *out = nullptr;
  if (!params || n_in < 1 || n_hidden < 1 || n_out < 1 || n_out > n_in || n_in > 8192 ||
      n_hidden > 8192)
    return OCTEN_ERR_ARG;
  octen_mlp_t m = new octen_mlp();
  m->L = mlp_layout(n_in, n_hidden, n_out);
  m->stream = (hipStream_t)stream;
  const int64_t np = m->L.total;
  octen_status st = OCTEN_OK;
  if ((st = malloc_dev(m, &m->w, np)) != OCTEN_OK || (st = malloc_dev(m, &m->g, np)) != OCTEN_OK ||
      (st = malloc_dev(m, &m->mo, np)) != OCTEN_OK || (st = malloc_dev(m, &m->vo, np)) != OCTEN_OK ||
      (st = malloc_dev(m, &m->partials, MSE_PARTS)) != OCTEN_OK ||
      (st = malloc_dev(m, &m->loss, 1)) != OCTEN_OK) {
    octen_mlp_destroy(m);
    return st;
  }
  if (hipMemcpyAsync(m->w, params, np * 4, hipMemcpyDeviceToDevice, m->stream) != hipSuccess ||
      hipMemsetAsync(m->mo, 0, np * 4, m->stream) != hipSuccess ||
      hipMemsetAsync(m->vo, 0, np * 4, m->stream) != hipSuccess) {
    octen_mlp_destroy(m);
    return OCTEN_ERR_HIP;
  }
  *out = m;
  return OCTEN_OK;
}

octen_status octen_mlp_destroy(octen_mlp_t m) {
  if (!m) return OCTEN_ERR_ARG;
  hipStreamSynchronize(m->stream);
  for (void* p : m->allocs)
    if (p) hipFree(p);
  delete m;
  return OCTEN_OK;
}

const char* octen_mlp_last_error(octen_mlp_t m) { return m ? m->err.c_str() : "null handle"; }

octen_status octen_mlp_forward(octen_mlp_t m, const float* X, int64_t n, float* Y) {
  if (!m) return OCTEN_ERR_ARG;
  if (!X || !Y) return mfail(m, OCTEN_ERR_ARG, "X and Y must be non-null");
  octen_status st = check_rows(m, n);
  if (st != OCTEN_OK) return st;
  MHIP(m, mlp_forward(m->stream, m->L, m->w, X, n, m->H1, m->H2, Y));
  return OCTEN_OK;
}

octen_status octen_mlp_gradients(octen_mlp_t m, const float* X, const float* T, int64_t n,
                                 float* grads, double* loss_host) {
  if (!m) return OCTEN_ERR_ARG;
  if (!X || !T || !grads) return mfail(m, OCTEN_ERR_ARG, "X, T and grads must be non-null");
  octen_status st = grads_into(m, X, T, n);
  if (st != OCTEN_OK) return st;
  MHIP(m, hipMemcpyAsync(grads, m->g, m->L.total * 4, hipMemcpyDeviceToDevice, m->stream));
  return read_loss(m, loss_host);
}

octen_status octen_mlp_adam(octen_mlp_t m, const float* grads, float lr) {
  if (!m) return OCTEN_ERR_ARG;
  if (!grads || !(lr > 0.f)) return mfail(m, OCTEN_ERR_ARG, "grads non-null and lr > 0 required");
  ++m->step;
  MHIP(m, mlp_adam(m->stream, m->w, grads, m->mo, m->vo, m->L.total, lr, 0.9f, 0.999f, 1e-8f,
                   m->step));
  return OCTEN_OK;
}

octen_status octen_mlp_train_step(octen_mlp_t m, const float* X, const float* T, int64_t n,
                                  float lr, double* loss_host) {
  if (!m) return OCTEN_ERR_ARG;
  if (!X || !T || !(lr > 0.f)) return mfail(m, OCTEN_ERR_ARG, "X, T non-null and lr > 0 required");
  octen_status st = grads_into(m, X, T, n);
  if (st != OCTEN_OK) return st;
  ++m->step;
  MHIP(m, mlp_adam(m->stream, m->w, m->g, m->mo, m->vo, m->L.total, lr, 0.9f, 0.999f, 1e-8f,
                   m->step));
  return read_loss(m, loss_host);
}

octen_status octen_mlp_last_activations(octen_mlp_t m, int64_t n, float* H1, float* H2) {
  if (!m) return OCTEN_ERR_ARG;
  if (!H1 || !H2 || n < 1 || n > m->cap)
    return mfail(m, OCTEN_ERR_ARG, "n must not exceed the rows of the last pass");
  const size_t bytes = (size_t)n * m->L.nh * 4;
  MHIP(m, hipMemcpyAsync(H1, m->H1, bytes, hipMemcpyDeviceToDevice, m->stream));
  MHIP(m, hipMemcpyAsync(H2, m->H2, bytes, hipMemcpyDeviceToDevice, m->stream));
  return OCTEN_OK;
}

octen_status octen_mlp_get_params(octen_mlp_t m, float* dst) {
  if (!m || !dst) return OCTEN_ERR_ARG;
  MHIP(m, hipMemcpyAsync(dst, m->w, m->L.total * 4, hipMemcpyDeviceToDevice, m->stream));
  return OCTEN_OK;
}

}  // extern "C"
