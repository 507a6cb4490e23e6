// MFMA compression path (placeholder until the fused gfx950 kernel lands).
#include <hip/hip_runtime.h>

#include "octen_internal.h"

namespace octen {

struct MfmaPlan {
  int dummy;
};

hipError_t mfma_plan_create(const CompressShape&, int, const double*, const double*, hipStream_t,
                            MfmaPlan** out) {
  *out = nullptr;
  return hipErrorNotSupported;
}
void mfma_plan_destroy(MfmaPlan* p) { delete p; }
size_t mfma_workspace_bytes(const MfmaPlan*, int64_t) { return 0; }
hipError_t compress_mfma(hipStream_t, const MfmaPlan*, const float*, int64_t, const float*,
                         const double*, void*, float*) {
  return hipErrorNotSupported;
}

}  // namespace octen
