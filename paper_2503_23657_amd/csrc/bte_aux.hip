// Per-iteration kernels around the sweep: finalize (new temperature, heat flux,
// residuals and the convergence flag), lagged diffuse-wall update, state set-up
// and output.
#include <hip/hip_runtime.h>

#include "bte_device.h"
#include "bte_launch.h"
#include "../../include/bte.h"

namespace bte {

// Sum over the jobs j = js, js + kFinSlices, ... of one partial-sum plane for
// cell c, in FP64 with four loads in flight; the association is fixed, so the
// result does not depend on timing.
template <typename T>
__device__ __forceinline__ double job_sum(const T* pl, int n_jobs, int ncell, int c, int js) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = js;
  for (; j + 3 * kFinSlices < n_jobs; j += 4 * kFinSlices) {
    s0 += (double)pl[(size_t)j * ncell + c];
    s1 += (double)pl[(size_t)(j + kFinSlices) * ncell + c];
    s2 += (double)pl[(size_t)(j + 2 * kFinSlices) * ncell + c];
    s3 += (double)pl[(size_t)(j + 3 * kFinSlices) * ncell + c];
  }
  for (; j < n_jobs; j += kFinSlices) s0 += (double)pl[(size_t)j * ncell + c];
  return (s0 + s1) + (s2 + s3);
}

// Sum of the kFinSlices job slices of one cell, pairwise in a fixed order.
__device__ __forceinline__ double slice_sum(const double (*sl)[kFinCells], int cl) {
  double v[kFinSlices];
#pragma unroll
  for (int i = 0; i < kFinSlices; ++i) v[i] = sl[i][cl];
#pragma unroll
  for (int w = 1; w < kFinSlices; w *= 2)
#pragma unroll
    for (int i = 0; i + w < kFinSlices; i += 2 * w) v[i] += v[i + w];
  return v[0];
}

// Block-wide reduction of (sum, max, sum, max) over the block's threads;
// every thread calls it; the result is valid in thread 0.
__device__ __forceinline__ void block_reduce4(double (*red)[kFinThreads], double v[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) red[i][t] = v[i];
  __syncthreads();
  for (int s = kFinThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] = fmax(red[1][t], red[1][t + s]);
      red[2][t] += red[2][t + s];
      red[3][t] = fmax(red[3][t], red[3][t + s]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = red[i][0];
}

// New state (Eq. updatee0_t: Delta T, or the adjoint lambda), heat flux (Eq. 4)
// or dJ/dQ, and the residuals of Eq. 22. A block covers kFinCells cells with
// kFinSlices threads per cell, each adding a slice of the jobs' partial sums.
template <typename T>
__global__ void __launch_bounds__(kFinThreads) finalize_kernel(FinArgs A, const FinInst* FI) {
  __shared__ double red[4][kFinThreads];
  __shared__ double slc[4][kFinSlices][kFinCells];
  __shared__ int s_last;
  const int2 bi = A.blocks[blockIdx.x];
  const InstDev& I = A.inst[bi.x];
  const FinInst& F = FI[bi.x];
  StatusDev* st = reinterpret_cast<StatusDev*>(I.status);
  if (st->done) return;
  const int iter = st->iter;
  const int cur = iter & 1, nxt = cur ^ 1;
  const int cl = threadIdx.x % kFinCells, js = threadIdx.x / kFinCells;
  const int c = bi.y * kFinCells + cl;
  const size_t plane = (size_t)I.n_jobs * I.ncell;
  const T* part = reinterpret_cast<const T*>(I.part);
  const bool adj = (A.flags & FIN_ADJ) != 0, withq = (A.flags & FIN_Q) != 0;
  const int nq = withq ? (adj ? 1 : I.dim) : 0;
  const bool act = c < I.ncell && F.active[c];
  // ---- the job slices of every needed plane
  if (act) {
    slc[0][js][cl] = job_sum(part, I.n_jobs, I.ncell, c, js);
    for (int d = 0; d < nq; ++d) slc[1 + d][js][cl] = job_sum(part + (size_t)(1 + d) * plane, I.n_jobs, I.ncell, c, js);
  }
  __syncthreads();
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // sum dT^2, max |x|, sum d|q|^2, max |q| (+inf: non-finite)
  if (js == 0 && c < I.ncell) {
    if (act) {
      double x = adj ? F.g[c] : 0.0;
      x += slice_sum(slc[0], cl);
      const double old = F.X[cur][c];
      F.X[nxt][c] = x;
      // scatter into the skewed layouts of every octant
      T* xq = reinterpret_cast<T*>(I.xq[nxt]);
      for (int o = 0; o < I.n_oct; ++o) {
        const int ps = I.pos[(size_t)o * I.ncell + c];
        xq[2 * ((size_t)o * I.pos_per_oct + ps)] = (T)x;
      }
      bool bad = !isfinite(x);
      const double d = x - old;
      v[0] = d * d;
      v[1] = fabs(x);
      if (withq) {
        if (adj) {
          F.q[c] = slice_sum(slc[1], cl);
        } else {
          double m2 = 0.0;
          for (int d2 = 0; d2 < I.dim; ++d2) {
            const double qv = slice_sum(slc[1 + d2], cl);
            F.q[(size_t)c * I.dim + d2] = qv;
            m2 += qv * qv;
            bad = bad || !isfinite(qv);
          }
          const double qm = sqrt(m2);
          if (A.flags & FIN_QPREV) {
            const double dq = qm - F.qmag_prev[c];
            v[2] = dq * dq;
          }
          v[3] = qm;
          F.qmag_prev[c] = qm;
        }
      }
      if (bad) v[3] = INFINITY;
    } else {
      F.X[nxt][c] = 0.0;
      if (withq) {
        if (adj) F.q[c] = 0.0;
        else
          for (int d2 = 0; d2 < I.dim; ++d2) F.q[(size_t)c * I.dim + d2] = 0.0;
      }
    }
  }
  if (!(A.flags & FIN_CHECK)) {
    // no residual needed: only the iteration counter moves (last block);
    // non-finite values are caught at the next check
    if (threadIdx.x == 0) {
      __threadfence();
      const int t = atomicAdd(&st->ticket, 1);
      if (t == A.n_blocks_inst[bi.x] - 1) {
        st->ticket = 0;
        st->iter = iter + 1;
        __threadfence();
      }
    }
    return;
  }
  block_reduce4(red, v);
  const int nb = A.n_blocks_inst[bi.x];
  if (threadIdx.x == 0) {
    double* bp = F.blockpart + (size_t)bi.y * 4;
    bp[0] = v[0];
    bp[1] = v[1];
    bp[2] = v[2];
    bp[3] = v[3];
    __threadfence();
    s_last = atomicAdd(&st->ticket, 1) == nb - 1;
  }
  __syncthreads();
  if (!s_last) return;
  // the last block of the instance reduces the block partials (fixed order per
  // thread, fixed tree across threads)
  __threadfence();
  double w[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kFinThreads) {
    const volatile double* q = F.blockpart + (size_t)b * 4;
    w[0] += q[0];
    w[1] = fmax(w[1], q[1]);
    w[2] += q[2];
    w[3] = fmax(w[3], q[3]);
  }
  block_reduce4(red, w);
  if (threadIdx.x == 0) {
    const double a0 = w[0], a1 = w[1], a2 = w[2], a3 = w[3];
    // active cell count is stored by the host in red[0] of the status block
    const double nact = st->red[0];
    const double rT = sqrt(a0 / nact), rq = sqrt(a2 / nact);
    const double eT = a1 > 0.0 ? rT / a1 : (rT == 0.0 ? 0.0 : INFINITY);
    double eq = a3 > 0.0 ? rq / a3 : (rq == 0.0 ? 0.0 : INFINITY);
    if (!withq || adj) eq = 0.0;
    const bool nonfin = !isfinite(a1) || !isfinite(a3) || !isfinite(a0);
    st->iter = iter + 1;
    st->eps_T = eT;
    st->eps_q = eq;
    st->checked = iter + 1;
    if (A.tol_T > 0.0 && A.tol_q > 0.0 && eT < A.tol_T && eq < A.tol_q) st->done = 1;
    if (nonfin) {
      st->nonfinite = 1;
      st->done = 1;
    }
    st->ticket = 0;
    __threadfence();
  }
}

template <typename T>
__global__ void __launch_bounds__(256) wall_update_kernel(WallArgs A) {
  const InstDev& I = A.inst[A.inst_id];
  const StatusDev* st = reinterpret_cast<const StatusDev*>(I.status);
  if (st->done) return;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= A.n_dface * A.B) return;
  const int b = t / A.n_dface, df = t - b * A.n_dface;
  const int slot = A.dface_slot[df];
  const T* outv = reinterpret_cast<const T*>(I.outv);
  double s = 0.0;
  for (int o = 0; o < I.n_oct; ++o) {
    const int k = A.ofk[(size_t)o * I.n_bface + slot];
    if (k < 0) continue;
    const int2 gr = A.grp_ob[o * A.B + b];
    for (int g = 0; g < gr.y; ++g) s += (double)outv[(size_t)(gr.x + g) * I.n_out_stride + k];
  }
  T* ubf = const_cast<T*>(reinterpret_cast<const T*>(I.ubf));
  ubf[(size_t)b * I.n_bface + slot] = (T)(s * A.inv_half[df]);
}

template <typename T>
__global__ void __launch_bounds__(256) init_state_kernel(InitArgs A) {
  const InstDev& I = A.inst[A.inst_id];
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= I.ncell) return;
  double x = 0.0, q = 0.0;
  if (A.active[c]) {
    if (A.X0) x = A.adjoint ? A.X0[c] : (A.X0[c] - A.T_ref);
    if (A.Q) q = A.Q[c];
  }
  A.X[0][c] = x;
  A.X[1][c] = x;
  if (!A.active[c]) return;
  for (int b = 0; b < 2; ++b) {
    T* xq = reinterpret_cast<T*>(I.xq[b]);
    for (int o = 0; o < I.n_oct; ++o) {
      const int ps = I.pos[(size_t)o * I.ncell + c];
      xq[2 * ((size_t)o * I.pos_per_oct + ps)] = (T)x;
      xq[2 * ((size_t)o * I.pos_per_oct + ps) + 1] = (T)q;
    }
  }
}

// Output: absolute temperature T = T_ref + Delta T (0 on inactive cells).
__global__ void __launch_bounds__(256) output_kernel(const double* X, const unsigned char* active, int n,
                                                     double T_ref, double add_ref, double* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  out[c] = active[c] ? X[c] + add_ref * T_ref : 0.0;
}

// Status reset for a new solve (n_active is kept for the residual means).
__global__ void status_reset_kernel(StatusDev* st, double n_active) {
  st->iter = 0;
  st->done = 0;
  st->nonfinite = 0;
  st->ticket = 0;
  st->checked = 0;
  st->eps_T = INFINITY;
  st->eps_q = INFINITY;
  st->lam_dT = 0.0;
  st->red[0] = n_active;
}

// Copy of the current state's (X, Q) skewed buffer (used as the forward state
// by the tau-gradient pass).
__global__ void copy_kernel(const double4* src, double4* dst, long long n4) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}


// Boundary inflow table at the start of a solve: isothermal faces hold
// T_w - T_ref; diffuse faces start from the adjacent cell's initial deviation
// (the reflection of an isotropic distribution is itself); every band alike.
template <typename T>
__global__ void __launch_bounds__(256) ubf_init_kernel(UbfInitArgs A) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)A.n_bface * A.B) return;
  const int f = (int)(t % A.n_bface);
  double u = 0.0;
  if (!A.zero) {
    const int bc = A.bf_bc[f];
    if (A.bc_kind[bc] == 0) u = A.bc_T[bc] - A.T_ref;
    else u = A.T_init ? A.T_init[A.bf_cell[f]] - A.T_ref : 0.0;
  }
  reinterpret_cast<T*>(A.ubf)[t] = (T)u;
}

__global__ void zero_kernel(unsigned* p, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template __global__ void finalize_kernel<float>(FinArgs, const FinInst*);
template __global__ void finalize_kernel<double>(FinArgs, const FinInst*);
template __global__ void wall_update_kernel<float>(WallArgs);
template __global__ void wall_update_kernel<double>(WallArgs);
template __global__ void init_state_kernel<float>(InitArgs);
template __global__ void init_state_kernel<double>(InitArgs);


// ---------------------------------------------------------------- launchers
static inline int nblk(long long n) { return (int)((n + 255) / 256); }

hipError_t launch_finalize(int prec, const FinArgs& a, const FinInst* fi, hipStream_t st) {
  if (a.n_blocks_total <= 0) return hipSuccess;
  if (prec == BTE_PREC_FP32)
    hipLaunchKernelGGL(finalize_kernel<float>, dim3(a.n_blocks_total), dim3(kFinThreads), 0, st, a, fi);
  else
    hipLaunchKernelGGL(finalize_kernel<double>, dim3(a.n_blocks_total), dim3(kFinThreads), 0, st, a, fi);
  return hipGetLastError();
}

hipError_t launch_wall_update(int prec, const WallArgs& a, hipStream_t st) {
  const long long n = (long long)a.n_dface * a.B;
  if (n == 0) return hipSuccess;
  if (prec == BTE_PREC_FP32)
    hipLaunchKernelGGL(wall_update_kernel<float>, dim3(nblk(n)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(wall_update_kernel<double>, dim3(nblk(n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_init_state(int prec, const InitArgs& a, int ncell, hipStream_t st) {
  if (prec == BTE_PREC_FP32)
    hipLaunchKernelGGL(init_state_kernel<float>, dim3(nblk(ncell)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(init_state_kernel<double>, dim3(nblk(ncell)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_output(const double* X, const unsigned char* active, int n, double T_ref,
                         double add_ref, double* out, hipStream_t st) {
  hipLaunchKernelGGL(output_kernel, dim3(nblk(n)), dim3(256), 0, st, X, active, n, T_ref, add_ref, out);
  return hipGetLastError();
}

hipError_t launch_status_reset(StatusDev* stt, double n_active, hipStream_t st) {
  hipLaunchKernelGGL(status_reset_kernel, dim3(1), dim3(1), 0, st, stt, n_active);
  return hipGetLastError();
}

hipError_t launch_ubf_init(int prec, const UbfInitArgs& a, hipStream_t st) {
  const long long n = (long long)a.n_bface * a.B;
  if (n == 0) return hipSuccess;
  if (prec == BTE_PREC_FP32)
    hipLaunchKernelGGL(ubf_init_kernel<float>, dim3(nblk(n)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(ubf_init_kernel<double>, dim3(nblk(n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  // a fill kernel rather than a memset node, so that the call can be captured
  const long long n4 = (long long)(bytes / 4);
  if (n4 > 0) hipLaunchKernelGGL(zero_kernel, dim3(nblk(n4)), dim3(256), 0, st, (unsigned*)p, n4);
  return hipGetLastError();
}

}  // namespace bte
