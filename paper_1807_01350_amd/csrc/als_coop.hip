// Cooperative launch of one handle's replica ALS (the kernel's statements are
// in als_coop_kernel_body.inc, its helpers in als_coop_body.h).
#include "als_coop_body.h"

namespace octen {
namespace {

#define OCTEN_ALS_INVERSE(...) spd_inverse<RMAX>(__VA_ARGS__)
template <typename T, int RMAX, bool GX, bool SPLIT>
__global__ __launch_bounds__(NT) void als_coop_kernel(CoopArgs g) {
  const unsigned bid = blockIdx.x;
#include "als_coop_kernel_body.inc"
}
#undef OCTEN_ALS_INVERSE

template <int RM>
const void* pick_single(bool split, bool gx, bool f64) {
  if (split)
    return gx ? (const void*)als_coop_kernel<float, RM, true, true>
              : (const void*)als_coop_kernel<float, RM, false, true>;
  if (gx)
    return f64 ? (const void*)als_coop_kernel<double, RM, true, false>
               : (const void*)als_coop_kernel<float, RM, true, false>;
  return f64 ? (const void*)als_coop_kernel<double, RM, false, false>
             : (const void*)als_coop_kernel<float, RM, false, false>;
}

const void* single_fn(const AlsCoopItem& it) {
  switch (rmax_class(it.R)) {
    case 6: return pick_single<6>(it.split, it.slab_global, it.y_f64);
    case 8: return pick_single<8>(it.split, it.slab_global, it.y_f64);
    case 10: return pick_single<10>(it.split, it.slab_global, it.y_f64);
    case 12: return pick_single<12>(it.split, it.slab_global, it.y_f64);
    case 16: return pick_single<16>(it.split, it.slab_global, it.y_f64);
    case 20: return pick_single<20>(it.split, it.slab_global, it.y_f64);
    case 24: return pick_single<24>(it.split, it.slab_global, it.y_f64);
    default: return pick_single<32>(it.split, it.slab_global, it.y_f64);
  }
}

hipError_t launch_single(hipStream_t s, const AlsCoopItem& it, const CoopArgs& a, size_t lds) {
  const void* fn = single_fn(it);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  CoopArgs arg = a;
  void* args[] = {&arg};
  return hipLaunchCooperativeKernel(fn, dim3(coop_grid(a)), dim3(NT), args, (unsigned)lds, s);
}

}  // namespace

size_t als_coop_lds_bytes(int Q, int R, int NW, bool x_f64, bool slab_global, bool split) {
  const int na_max = (Q + NW - 1) / NW;
  const size_t QR = (size_t)Q * R;
  const size_t QPAD = (size_t)((Q + 31) / 32) * 32;
  const size_t dbl = (size_t)pad_pairs(Q, NW) * R + 3 * QR + QPAD * R + (size_t)na_max * R +
                     5 * (size_t)R * R + 2 * MAXR + NT;
  // split: 16-byte alignment slack, then the fragments of C and (unless
  // they take T's place) W, in bf16
  const size_t RT = (size_t)(R + 15) / 16;
  const bool walias = (size_t)R >= 8 * RT;
  const size_t frag =
      split ? 16 + RT * (QPAD / 32 + (walias ? 0 : (size_t)pad_pairs(Q, NW) / 32)) * 2 * 512 * 2 : 0;
  return dbl * 8 + frag +
         (slab_global ? 0 : (size_t)pad_pairs(Q, NW) * (QPAD + 1) * (x_f64 ? 8 : 4));
}

hipError_t als_coop(hipStream_t s, const void* Y, bool y_f64, int P, int Q, int R, int NW,
                    bool slab_global, const double* init, double* F, double* lam, int* iters,
                    int* flags, double* slots, unsigned* counters, int* err, int max_iters,
                    double tol, bool allow_local, bool split, bool cleared) {
  AlsCoopItem it{Y, y_f64, P, Q, R, NW, slab_global, init, F, lam, iters, flags, slots,
                 counters, err, max_iters, tol, allow_local, split};
  CoopArgs a;
  size_t lds = 0;
  if (!coop_args(it, a, lds)) return hipErrorInvalidValue;
  if (!cleared) {
    hipError_t e = fill_i32(s, (int*)counters, 2 * P, 0);
    if (e != hipSuccess) return e;
    e = fill_i32(s, err, 1, 0);
    if (e != hipSuccess) return e;
  }
  return launch_single(s, it, a, lds);
}

}  // namespace octen
