// Precision dispatch of the sweep launch helpers.
#include "bte_launch.h"
#include "../../include/bte.h"

namespace bte {

hipError_t launch_sweep_f(bool l3, int G, int nacc, int mode, const SweepArgs& a, int grid,
                          int block, size_t lds, hipStream_t st);
hipError_t launch_sweep_d(bool l3, int G, int nacc, int mode, const SweepArgs& a, int grid,
                          int block, size_t lds, hipStream_t st);
int sweep_blocks_per_cu_f(bool l3, int G, int nacc, int mode, int block, size_t lds);
int sweep_blocks_per_cu_d(bool l3, int G, int nacc, int mode, int block, size_t lds);

hipError_t launch_sweep2d_f(int G, int NR, int nacc, int mode, const SweepArgs& a, int grid, int block,
                            size_t lds, hipStream_t st);
hipError_t launch_sweep2d_d(int G, int NR, int nacc, int mode, const SweepArgs& a, int grid, int block,
                            size_t lds, hipStream_t st);
int sweep2d_blocks_per_cu_f(int G, int NR, int nacc, int mode, int block, size_t lds);
int sweep2d_blocks_per_cu_d(int G, int NR, int nacc, int mode, int block, size_t lds);

hipError_t launch_sweep2d(int prec, int G, int NR, int nacc, int mode, const SweepArgs& a, int grid, int block,
                          size_t lds, hipStream_t st) {
  return prec == BTE_PREC_FP32 ? launch_sweep2d_f(G, NR, nacc, mode, a, grid, block, lds, st)
                               : launch_sweep2d_d(G, NR, nacc, mode, a, grid, block, lds, st);
}

int sweep2d_blocks_per_cu(int prec, int G, int NR, int nacc, int mode, int block, size_t lds) {
  return prec == BTE_PREC_FP32 ? sweep2d_blocks_per_cu_f(G, NR, nacc, mode, block, lds)
                               : sweep2d_blocks_per_cu_d(G, NR, nacc, mode, block, lds);
}

hipError_t launch_sweep(int prec, bool l3, int G, int nacc, int mode, const SweepArgs& a,
                        int grid, int block, size_t lds, hipStream_t st) {
  return prec == BTE_PREC_FP32 ? launch_sweep_f(l3, G, nacc, mode, a, grid, block, lds, st)
                               : launch_sweep_d(l3, G, nacc, mode, a, grid, block, lds, st);
}

int sweep_blocks_per_cu(int prec, bool l3, int G, int nacc, int mode, int block, size_t lds) {
  return prec == BTE_PREC_FP32 ? sweep_blocks_per_cu_f(l3, G, nacc, mode, block, lds)
                               : sweep_blocks_per_cu_d(l3, G, nacc, mode, block, lds);
}

}  // namespace bte
