// 1D/2D sweep kernel in double: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

hipError_t launch_sweep2d_d(int G, int NR, int nacc, int mode, const SweepArgs& a, int grid, int block,
                            size_t lds, hipStream_t st) {
  BTE2D_DISPATCH(double, launch2d_one, a, grid, block, lds, st)
  return hipErrorInvalidValue;
}

int sweep2d_blocks_per_cu_d(int G, int NR, int nacc, int mode, int block, size_t lds) {
  BTE2D_DISPATCH(double, occ2d_one, block, lds)
  return 0;
}

}  // namespace bte
