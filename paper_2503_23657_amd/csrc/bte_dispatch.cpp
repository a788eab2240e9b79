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

#define BTE2D_DECL(SUFFIX)                                                                            \
  hipError_t launch_sweep2d_##SUFFIX(int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, \
                                     int block, size_t lds, hipStream_t st);                          \
  int sweep2d_blocks_per_cu_##SUFFIX(int NR, int P, int nacc, int mode, int block, size_t lds);
hipError_t launch_sweep3r_f(int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, int block, size_t lds,
                           hipStream_t st);
hipError_t launch_sweep3r_d(int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, int block, size_t lds,
                           hipStream_t st);
int sweep3r_blocks_per_cu_f(int NR, int P, int nacc, int mode, int block, size_t lds);
int sweep3r_blocks_per_cu_d(int NR, int P, int nacc, int mode, int block, size_t lds);

hipError_t launch_sweep3r(int prec, int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, int block,
                          size_t lds, hipStream_t st) {
  return prec == BTE_PREC_FP32 ? launch_sweep3r_f(NR, P, nacc, mode, a, grid, block, lds, st)
                               : launch_sweep3r_d(NR, P, nacc, mode, a, grid, block, lds, st);
}

int sweep3r_blocks_per_cu(int prec, int NR, int P, int nacc, int mode, int block, size_t lds) {
  return prec == BTE_PREC_FP32 ? sweep3r_blocks_per_cu_f(NR, P, nacc, mode, block, lds)
                               : sweep3r_blocks_per_cu_d(NR, P, nacc, mode, block, lds);
}

BTE2D_DECL(f1)
BTE2D_DECL(f2)
BTE2D_DECL(d1)
BTE2D_DECL(d2)

hipError_t launch_sweep2d(int prec, int G, int NR, int P, int nacc, int mode, const SweepArgs& a, int grid,
                          int block, size_t lds, hipStream_t st) {
  if (prec == BTE_PREC_FP32)
    return G == 1 ? launch_sweep2d_f1(NR, P, nacc, mode, a, grid, block, lds, st)
                  : G == 2 ? launch_sweep2d_f2(NR, P, nacc, mode, a, grid, block, lds, st) : hipErrorInvalidValue;
  return G == 1 ? launch_sweep2d_d1(NR, P, nacc, mode, a, grid, block, lds, st)
                : G == 2 ? launch_sweep2d_d2(NR, P, nacc, mode, a, grid, block, lds, st) : hipErrorInvalidValue;
}

int sweep2d_blocks_per_cu(int prec, int G, int NR, int P, int nacc, int mode, int block, size_t lds) {
  if (prec == BTE_PREC_FP32)
    return G == 1 ? sweep2d_blocks_per_cu_f1(NR, P, nacc, mode, block, lds)
                  : G == 2 ? sweep2d_blocks_per_cu_f2(NR, P, nacc, mode, block, lds) : 0;
  return G == 1 ? sweep2d_blocks_per_cu_d1(NR, P, nacc, mode, block, lds)
                : G == 2 ? sweep2d_blocks_per_cu_d2(NR, P, nacc, mode, block, lds) : 0;
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
