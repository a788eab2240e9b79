// Instantiations and dispatch of the sweep kernel in float.
#include "bte_sweep.hip"
#include "bte_launch.h"
#include "../../include/bte.h"

namespace bte {

// Largest dynamic LDS a launch of kernel k may request: the device's per-block
// limit minus the kernel's static LDS. The attribute is raised once per kernel;
// a refused request is cleared so that no sticky error is left in the runtime.
static int dyn_lds_limit(const void* k) {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, k) != hipSuccess) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  const int dyn = lim - (int)fa.sharedSizeBytes;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  return dyn;
}

template <int G, int NACC, int MODE, bool L3>
static hipError_t launch_one_f(const SweepArgs& a, int grid, int block, size_t lds, hipStream_t st) {
  auto k = sweep_kernel<float, G, NACC, MODE, L3>;
  static int lim = -1;
  if (lim < 0) lim = dyn_lds_limit(reinterpret_cast<const void*>(k));
  if ((long long)lds > lim) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <int G, int NACC, int MODE, bool L3>
static int occ_one_f(int block, size_t lds) {
  int n = 0;
  auto k = sweep_kernel<float, G, NACC, MODE, L3>;
  static int lim = -1;
  if (lim < 0) lim = dyn_lds_limit(reinterpret_cast<const void*>(k));
  if ((long long)lds > lim) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

#define BTE_DISPATCH(FN, ...)                                              \
  switch (G * 1000 + nacc * 100 + mode * 10 + (l3 ? 1 : 0)) {               \
    BTE_CASES_G(1, FN, __VA_ARGS__)                                        \
    BTE_CASES_G(2, FN, __VA_ARGS__)                                        \
    BTE_CASES_G(4, FN, __VA_ARGS__)                                        \
    default: break;                                                        \
  }
#define BTE_CASE(G_, N_, M_, L_, FN, ...) \
  case G_ * 1000 + N_ * 100 + M_ * 10 + L_: return FN<G_, N_, M_, (L_ != 0)>(__VA_ARGS__);
#define BTE_CASES_G(G_, FN, ...)               \
  BTE_CASE(G_, 1, 0, 1, FN, __VA_ARGS__)       \
  BTE_CASE(G_, 2, 0, 1, FN, __VA_ARGS__)       \
  BTE_CASE(G_, 4, 0, 1, FN, __VA_ARGS__)       \
  BTE_CASE(G_, 1, 1, 1, FN, __VA_ARGS__)       \
  BTE_CASE(G_, 2, 2, 1, FN, __VA_ARGS__)

hipError_t launch_sweep_f(bool l3, int G, int nacc, int mode, const SweepArgs& a, int grid,
                           int block, size_t lds, hipStream_t st) {
  BTE_DISPATCH(launch_one_f, a, grid, block, lds, st)
  return hipErrorInvalidValue;
}

int sweep_blocks_per_cu_f(bool l3, int G, int nacc, int mode, int block, size_t lds) {
  BTE_DISPATCH(occ_one_f, block, lds)
  return 0;
}

}  // namespace bte
