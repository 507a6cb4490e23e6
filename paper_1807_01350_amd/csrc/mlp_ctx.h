// Handle of the warm-start network (shared by the library's C++ sources).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/octen.h"
#include "octen_internal.h"

struct octen_mlp {
  octen::MlpLayout L{};
  hipStream_t stream = nullptr;
  float *w = nullptr, *g = nullptr;        // FP32 master parameters, gradients
  float *mo = nullptr, *vo = nullptr;      // Adam moments
  int64_t step = 0;                        // Adam steps taken
  float *H1 = nullptr, *H2 = nullptr, *Y = nullptr;
  float *dY = nullptr, *dZ1 = nullptr, *dZ2 = nullptr;
  int64_t cap = 0;                         // rows the activation buffers hold
  double *partials = nullptr, *loss = nullptr;
  std::string err;
  std::vector<void*> allocs;
};

// Grows the activation buffers of the network to n rows.
octen_status octen_mlp_ensure_rows(octen_mlp* m, int64_t n);
