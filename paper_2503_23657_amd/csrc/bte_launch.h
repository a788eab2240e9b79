// Launch helpers exported by the kernel translation units to the host runtime.
#pragma once
#include <hip/hip_runtime.h>

#include "bte_device.h"

namespace bte {


// Sweep modes.
enum { SWEEP_PLAIN = 0, SWEEP_STORE = 1, SWEEP_TAUGRAD = 2, SWEEP_SECOND = 3 };

// One sweep launch. prec: BTE_PREC_*; l3: 3D layout; returns hipErrorInvalidValue
// for a (G, nacc, mode) combination that is not compiled.
hipError_t launch_sweep(int prec, bool l3, int G, int nacc, int mode, const SweepArgs& a,
                        int grid, int block, size_t lds, hipStream_t st);

// Workgroups of the sweep kernel that fit on one CU at once (0 on error).
int sweep_blocks_per_cu(int prec, bool l3, int G, int nacc, int mode, int block, size_t lds);

// One launch of the 1D/2D rows-per-lane sweep (bte_sweep2d.hip); returns
// hipErrorInvalidValue for a (G, NR, P, nacc, mode) combination that is not compiled.
hipError_t launch_sweep2d(int prec, int G, int NR, int P, int nacc, int mode, const SweepArgs& a, int grid,
                          int block, size_t lds, hipStream_t st);
int sweep2d_blocks_per_cu(int prec, int G, int NR, int P, int nacc, int mode, int block, size_t lds);

// One launch of the 3D rows-per-lane sweep (the 1D/2D kernel with a plane
// axis; one ordinate per lane, NR in {1, 2}).
hipError_t launch_sweep3r(int prec, int NR, int P, int nacc, int mode, const SweepArgs& a, int grid, int block,
                          size_t lds, hipStream_t st);
int sweep3r_blocks_per_cu(int prec, int NR, int P, int nacc, int mode, int block, size_t lds);

hipError_t launch_finalize(int prec, const FinArgs& a, const FinInst* fi, hipStream_t st);
hipError_t launch_wall_update(int prec, const WallArgs& a, int n_oct, hipStream_t st);
hipError_t launch_spec_update(int prec, const SpecArgs& a, hipStream_t st);
hipError_t launch_init_state(int prec, const InitArgs& a, int ncell, hipStream_t st);
hipError_t launch_output(const double* X, const unsigned char* active, int n, double T_ref,
                         double add_ref, double* out, hipStream_t st);
hipError_t launch_status_reset(StatusDev* stt, double n_active, hipStream_t st);
hipError_t launch_ubf_init(int prec, const UbfInitArgs& a, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// second-order faces: the correction of every group from the stored field,
// and the stored field set to the initial temperature deviation X
hipError_t launch_corr(int prec, const CorrArgs& a, long long n_pos, hipStream_t st);

}  // namespace bte
