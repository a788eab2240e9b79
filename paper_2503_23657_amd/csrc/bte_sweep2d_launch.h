// Instantiation and dispatch of the 1D/2D sweep kernel for one precision
// (included once by bte_sweep2d_f.hip and once by bte_sweep2d_d.hip).
#pragma once
#include "bte_sweep2d.hip"
#include "bte_launch.h"

namespace bte {

// Largest dynamic LDS a launch of kernel k may request: the device's per-block
// limit minus the kernel's static LDS. The attribute is raised once per kernel;
// a refused request is cleared so that no sticky error is left in the runtime.
static inline int dyn_lds_limit_2d(const void* k) {
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

template <typename T, int G, int NR, int P, int NACC, int MODE, bool L3 = false>
static hipError_t launch2d_one(const SweepArgs& a, int grid, int block, size_t lds, hipStream_t st) {
  auto k = sweep2d_kernel<T, G, NR, P, NACC, MODE, L3>;
  static int lim = -1;
  if (lim < 0) lim = dyn_lds_limit_2d(reinterpret_cast<const void*>(k));
  if ((long long)lds > lim) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <typename T, int G, int NR, int P, int NACC, int MODE, bool L3 = false>
static int occ2d_one(int block, size_t lds) {
  int n = 0;
  auto k = sweep2d_kernel<T, G, NR, P, NACC, MODE, L3>;
  static int lim = -1;
  if (lim < 0) lim = dyn_lds_limit_2d(reinterpret_cast<const void*>(k));
  if ((long long)lds > lim) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

// compiled variants: NR in {1, 2, 4}, P in {1, 2, 4} and (NACC, mode) in
// {(1..3, plain), (1, store), (2, tau-gradient)}; each translation unit
// instantiates one (precision, G) pair
#define BTE2D_KEY(NR_, P_, N_, M_) ((NR_) * 1000 + (P_) * 100 + (N_) * 10 + (M_))
#define BTE2D_CASE(T_, G_, NR_, P_, N_, M_, FN, ...) \
  case BTE2D_KEY(NR_, P_, N_, M_): return FN<T_, G_, NR_, P_, N_, M_>(__VA_ARGS__);
#define BTE2D_CASES_P(T_, G_, NR_, P_, FN, ...)       \
  BTE2D_CASE(T_, G_, NR_, P_, 1, 0, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, P_, 2, 0, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, P_, 3, 0, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, P_, 1, 1, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, P_, 2, 2, FN, __VA_ARGS__)
#define BTE2D_CASES_NR(T_, G_, NR_, FN, ...)     \
  BTE2D_CASES_P(T_, G_, NR_, 1, FN, __VA_ARGS__) \
  BTE2D_CASES_P(T_, G_, NR_, 2, FN, __VA_ARGS__) \
  BTE2D_CASES_P(T_, G_, NR_, 4, FN, __VA_ARGS__)
#define BTE2D_DISPATCH(T_, G_, FN, ...)                 \
  switch (BTE2D_KEY(NR, P, nacc, mode)) {               \
    BTE2D_CASES_NR(T_, G_, 1, FN, __VA_ARGS__)          \
    BTE2D_CASES_NR(T_, G_, 2, FN, __VA_ARGS__)          \
    BTE2D_CASES_NR(T_, G_, 4, FN, __VA_ARGS__)          \
    default: break;                                     \
  }

// second-order sweeps (mode 3, temperature-only and flux iterations): one
// ordinate per lane only
#define BTE2D_CASES_SECOND_NR(T_, G_, NR_, FN, ...)   \
  BTE2D_CASE(T_, G_, NR_, 1, 1, 3, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, 1, 3, 3, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, 2, 1, 3, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, 2, 3, 3, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, 4, 1, 3, FN, __VA_ARGS__) \
  BTE2D_CASE(T_, G_, NR_, 4, 3, 3, FN, __VA_ARGS__)
#define BTE2D_DISPATCH_SECOND(T_, G_, FN, ...)          \
  switch (BTE2D_KEY(NR, P, nacc, mode)) {               \
    BTE2D_CASES_SECOND_NR(T_, G_, 1, FN, __VA_ARGS__)   \
    BTE2D_CASES_SECOND_NR(T_, G_, 2, FN, __VA_ARGS__)   \
    BTE2D_CASES_SECOND_NR(T_, G_, 4, FN, __VA_ARGS__)   \
    default: break;                                     \
  }

// one (precision, G) translation unit; SECOND: also the second-order variants
#define BTE2D_UNIT_IMPL(T_, G_, SUFFIX, SECOND_LAUNCH, SECOND_OCC)                                      \
  hipError_t launch_sweep2d_##SUFFIX(int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, \
                                     int block, size_t lds, hipStream_t st) {                         \
    BTE2D_DISPATCH(T_, G_, launch2d_one, a, grid, block, lds, st)                                     \
    SECOND_LAUNCH                                                                                     \
    return hipErrorInvalidValue;                                                                      \
  }                                                                                                   \
  int sweep2d_blocks_per_cu_##SUFFIX(int NR, int P, int nacc, int mode, int block, size_t lds) {      \
    BTE2D_DISPATCH(T_, G_, occ2d_one, block, lds)                                                     \
    SECOND_OCC                                                                                        \
    return 0;                                                                                         \
  }
#define BTE2D_UNIT(T_, G_, SUFFIX) BTE2D_UNIT_IMPL(T_, G_, SUFFIX, , )
#define BTE2D_UNIT_WITH_SECOND(T_, G_, SUFFIX)                                    \
  BTE2D_UNIT_IMPL(T_, G_, SUFFIX, BTE2D_DISPATCH_SECOND(T_, G_, launch2d_one, a, grid, block, lds, st), \
                  BTE2D_DISPATCH_SECOND(T_, G_, occ2d_one, block, lds))

// 3D rows-per-lane variants: one ordinate per lane, NR in {1, 2}, P in
// {1, 2, 4, 8}, (NACC, mode) in {(1, plain), (4, plain: flux iterations),
// (1, store), (2, tau-gradient), (1 and 4, second order)}
#define BTE3R_CASE(T_, NR_, P_, N_, M_, FN, ...) \
  case BTE2D_KEY(NR_, P_, N_, M_): return FN<T_, 1, NR_, P_, N_, M_, true>(__VA_ARGS__);
#define BTE3R_CASES_P(T_, NR_, P_, FN, ...)       \
  BTE3R_CASE(T_, NR_, P_, 1, 0, FN, __VA_ARGS__) \
  BTE3R_CASE(T_, NR_, P_, 4, 0, FN, __VA_ARGS__) \
  BTE3R_CASE(T_, NR_, P_, 1, 1, FN, __VA_ARGS__) \
  BTE3R_CASE(T_, NR_, P_, 2, 2, FN, __VA_ARGS__) \
  BTE3R_CASE(T_, NR_, P_, 1, 3, FN, __VA_ARGS__) \
  BTE3R_CASE(T_, NR_, P_, 4, 3, FN, __VA_ARGS__)
#define BTE3R_DISPATCH(T_, FN, ...)               \
  switch (BTE2D_KEY(NR, P, nacc, mode)) {         \
    BTE3R_CASES_P(T_, 1, 1, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 1, 2, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 1, 4, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 1, 8, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 2, 1, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 2, 2, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 2, 4, FN, __VA_ARGS__)      \
    BTE3R_CASES_P(T_, 2, 8, FN, __VA_ARGS__)      \
    default: break;                               \
  }
#define BTE3R_UNIT(T_, SUFFIX)                                                                          \
  hipError_t launch_sweep3r_##SUFFIX(int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, \
                                     int block, size_t lds, hipStream_t st) {                         \
    BTE3R_DISPATCH(T_, launch2d_one, a, grid, block, lds, st)                                         \
    return hipErrorInvalidValue;                                                                      \
  }                                                                                                   \
  int sweep3r_blocks_per_cu_##SUFFIX(int NR, int P, int nacc, int mode, int block, size_t lds) {      \
    BTE3R_DISPATCH(T_, occ2d_one, block, lds)                                                         \
    return 0;                                                                                         \
  }

}  // namespace bte
