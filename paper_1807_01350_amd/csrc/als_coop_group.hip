// Several handles' replica ALS in one cooperative launch (the kernel's
// statements are in als_coop_kernel_body.inc, its helpers in als_coop_body.h).
#include <algorithm>
#include <vector>

#include "als_coop_body.h"

namespace octen {
namespace {

// Several handles' ALS in one cooperative grid: member e owns workgroups
// start[e] .. start[e + 1] - 1 (each range a multiple of 8 long, so that a
// workgroup's XCD is the same as in a launch of its own).
constexpr int GROUP_MAX = 16;
struct CoopGroup {
  int n;
  int start[GROUP_MAX + 1];
  CoopArgs a[GROUP_MAX];
};

static_assert(sizeof(CoopGroup) <= 4096, "kernel argument block");

// The R x R inverse of rank class rc (wave-uniform): the same code as in a
// kernel instantiated for that class.
__device__ __forceinline__ void spd_inverse_class(int rc, const double* G, double* Ginv, int R,
                                                  int* bad) {
  switch (rc) {
    case 6: spd_inverse<6>(G, Ginv, R, bad); break;
    case 8: spd_inverse<8>(G, Ginv, R, bad); break;
    case 10: spd_inverse<10>(G, Ginv, R, bad); break;
    case 12: spd_inverse<12>(G, Ginv, R, bad); break;
    case 16: spd_inverse<16>(G, Ginv, R, bad); break;
    case 20: spd_inverse<20>(G, Ginv, R, bad); break;
    case 24: spd_inverse<24>(G, Ginv, R, bad); break;
    default: spd_inverse<32>(G, Ginv, R, bad); break;
  }
}

// Members of any rank class share a launch: each takes the inverse of its
// own class.
#define OCTEN_ALS_INVERSE(...) spd_inverse_class(rclass_, __VA_ARGS__)
template <typename T, bool GX, bool SPLIT>
__global__ __launch_bounds__(NT) void als_coop_group_kernel(CoopGroup grp_) {
  int m_ = 0;   // the member whose range holds this workgroup
  for (int i_ = 1; i_ < grp_.n; ++i_) m_ += (int)blockIdx.x >= grp_.start[i_] ? 1 : 0;
  m_ = __builtin_amdgcn_readfirstlane(m_);
  const CoopArgs& g = grp_.a[m_];
  const unsigned bid = blockIdx.x - (unsigned)grp_.start[m_];
  const int rclass_ = __builtin_amdgcn_readfirstlane(rmax_class(g.R));
#include "als_coop_kernel_body.inc"
}
#undef OCTEN_ALS_INVERSE

// The group kernel of an item: items of equal kernels may share a launch
// (summary precision, contraction form and slab placement; any rank class).
const void* group_fn(const AlsCoopItem& it) {
  if (it.split)
    return it.slab_global ? (const void*)als_coop_group_kernel<float, true, true>
                          : (const void*)als_coop_group_kernel<float, false, true>;
  if (it.slab_global)
    return it.y_f64 ? (const void*)als_coop_group_kernel<double, true, false>
                    : (const void*)als_coop_group_kernel<float, true, false>;
  return it.y_f64 ? (const void*)als_coop_group_kernel<double, false, false>
                  : (const void*)als_coop_group_kernel<float, false, false>;
}

// Workgroups of fn that fit on the device at once with lds bytes of LDS each.
hipError_t coop_capacity(const void* fn, size_t lds, int& cap) {
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, NT, lds);
  cap = per * cus;
  return e;
}

}  // namespace

hipError_t als_coop_group(hipStream_t s, const AlsCoopItem* items, int n, int* launches) {
  int nl = 0;
  std::vector<CoopArgs> args(n);
  std::vector<size_t> lds(n);
  std::vector<bool> done(n, false);
  for (int i = 0; i < n; ++i)
    if (!coop_args(items[i], args[i], lds[i])) return hipErrorInvalidValue;
  // A launch lasts as long as its slowest member: the handles in falling
  // order of the work of one workgroup per sweep (4 Q^3 R / NW flop, the
  // contractions), each pack opened by the costliest handle left and filled
  // first-fit with the next ones of the same kernel while their workgroups
  // fit on the device at once.
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) {
    return (double)items[i].Q * items[i].Q * items[i].Q * items[i].R / items[i].NW;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  for (int oi = 0; oi < n; ++oi) {
    const int i = order[oi];
    if (done[i]) continue;
    const void* gfn = group_fn(items[i]);
    std::vector<int> pack{i};
    done[i] = true;
    size_t plds = lds[i];
    int used = coop_grid(args[i]);
    for (int oj = oi + 1; gfn && oj < n && (int)pack.size() < GROUP_MAX; ++oj) {
      const int j = order[oj];
      if (done[j] || group_fn(items[j]) != gfn) continue;
      const size_t l2 = lds[j] > plds ? lds[j] : plds;
      int cap = 0;
      hipError_t e = coop_capacity(gfn, l2, cap);
      if (e != hipSuccess) return e;
      if (used + coop_grid(args[j]) > cap) continue;
      pack.push_back(j);
      done[j] = true;
      plds = l2;
      used += coop_grid(args[j]);
    }
    hipError_t e;
    if (pack.size() == 1) {
      const AlsCoopItem& it = items[i];
      e = als_coop(s, it.Y, it.y_f64, it.P, it.Q, it.R, it.NW, it.slab_global, it.init, it.F,
                   it.lam, it.iters, it.flags, it.slots, it.counters, it.err, it.max_iters, it.tol,
                   it.allow_local, it.split, true);
    } else {
      CoopGroup G;
      G.n = (int)pack.size();
      int off = 0;
      for (int k = 0; k < G.n; ++k) {
        G.start[k] = off;
        G.a[k] = args[pack[k]];
        off += coop_grid(args[pack[k]]);
      }
      for (int k = G.n; k <= GROUP_MAX; ++k) G.start[k] = off;
      e = hipFuncSetAttribute(gfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds);
      void* kargs[] = {&G};
      if (e == hipSuccess)
        e = hipLaunchCooperativeKernel(gfn, dim3(off), dim3(NT), kargs, (unsigned)plds, s);
    }
    if (e != hipSuccess) return e;
    ++nl;
  }
  if (launches) *launches = nl;
  return hipSuccess;
}

}  // namespace octen
