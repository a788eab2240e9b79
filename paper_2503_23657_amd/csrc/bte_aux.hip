// Per-iteration kernels around the sweep: finalize (new temperature, heat flux,
// residuals and the convergence flag), lagged diffuse-wall update, state set-up
// and output.
#include <hip/hip_runtime.h>

#include "bte_device.h"
#include "bte_launch.h"
#include "../../include/bte.h"

namespace bte {

// The finalize gathers the jobs' partial sums of kFinCells cells with
// 16-byte loads: a thread holds VW = 16 / sizeof(T) neighbouring cells and a
// slice of the jobs (j = js, js + S, ...), kFinLoads loads in flight; the S
// slices of a cell are then added in LDS, pairwise in a fixed order.
constexpr int kFinLoads = 8;
template <typename T>
struct FinShape {
  static constexpr int VW = 16 / (int)sizeof(T);       // cells per load
  static constexpr int NG = kFinCells / VW;             // cell groups per block
  static constexpr int S = kFinThreads / NG;            // job slices
  static_assert(NG * S == kFinThreads && kPartBlk % VW == 0, "finalize shape");
};

// pl: the block's cell block of job 0 (a job group's blocks follow at
// kPartBlk strides, the next group's 2^jg * part_ld elements on), c0: the
// thread's first cell within it
template <typename T>
__device__ __forceinline__ void job_sum_vec(const T* pl, int n_jobs, int jg, int part_ld, int c0, int js,
                                            double* acc) {
  using Sh = FinShape<T>;
  typedef T V __attribute__((ext_vector_type(Sh::VW)));
  auto at = [&](int j) { return pl + part_job(j, jg, part_ld) + c0; };
#pragma unroll
  for (int e = 0; e < Sh::VW; ++e) acc[e] = 0.0;
  int j = js;
  for (; j + (kFinLoads - 1) * Sh::S < n_jobs; j += kFinLoads * Sh::S) {
    V v[kFinLoads];
#pragma unroll
    for (int u = 0; u < kFinLoads; ++u) v[u] = *reinterpret_cast<const V*>(at(j + u * Sh::S));
#pragma unroll
    for (int u = 0; u < kFinLoads; ++u)
#pragma unroll
      for (int e = 0; e < Sh::VW; ++e) acc[e] += (double)v[u][e];
  }
  for (; j < n_jobs; j += Sh::S) {
    const V v = *reinterpret_cast<const V*>(at(j));
#pragma unroll
    for (int e = 0; e < Sh::VW; ++e) acc[e] += (double)v[e];
  }
}

// One plane's per-cell totals: every thread gathers its slice, the slices meet
// in LDS, and thread cl < kFinCells returns cell cl's total (pairwise over the
// slices in a fixed order); the others return 0.
template <typename T>
__device__ __forceinline__ double plane_total(const T* pl, int n_jobs, int jg, int part_ld, int ncell, int cbase,
                                              double (*slc)[kFinCells]) {
  using Sh = FinShape<T>;
  const int t = threadIdx.x;
  const int gi = t % Sh::NG, js = t / Sh::NG;
  const int c0 = cbase + gi * Sh::VW;
  double acc[Sh::VW];
  if (c0 < ncell) {
    job_sum_vec(pl + ((size_t)cbase << jg), n_jobs, jg, part_ld, gi * Sh::VW, js, acc);
  } else {
#pragma unroll
    for (int e = 0; e < Sh::VW; ++e) acc[e] = 0.0;
  }
#pragma unroll
  for (int e = 0; e < Sh::VW; ++e) slc[js][gi * Sh::VW + e] = acc[e];
  __syncthreads();
  double r = 0.0;
  if (t < kFinCells) {
    double v[Sh::S];
#pragma unroll
    for (int i = 0; i < Sh::S; ++i) v[i] = slc[i][t];
#pragma unroll
    for (int w = 1; w < Sh::S; w *= 2)
#pragma unroll
      for (int i = 0; i + w < Sh::S; i += 2 * w) v[i] += v[i + w];
    r = v[0];
  }
  __syncthreads();  // the next plane reuses slc
  return r;
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
// or dJ/dQ, and the residuals of Eq. 22. A block covers kFinCells cells; its
// threads first gather the jobs' partial sums (plane_total), then thread
// cl < kFinCells finishes cell cl.
template <typename T>
__global__ void __launch_bounds__(kFinThreads) finalize_kernel(FinArgs A, const FinInst* FI) {
  __shared__ double red[4][kFinThreads];
  __shared__ double slc[FinShape<T>::S][kFinCells];
  __shared__ int s_last, s_iter;
  const int2 bi = A.blocks[blockIdx.x];
  const InstDev& I = A.inst[bi.x];
  const FinInst& F = FI[bi.x];
  StatusDev* st = reinterpret_cast<StatusDev*>(I.status);
  if (st->done) return;
  // thread 0 reads the counter for the block: its read has returned before it
  // takes the block's ticket below, so the last block's increment can never
  // reach a block that has not read it yet
  if (threadIdx.x == 0) s_iter = st->iter;
  __syncthreads();
  const int iter = s_iter;
  const int cur = iter & 1, nxt = cur ^ 1;
  const int cl = threadIdx.x;  // the cell of threads < kFinCells
  const int cbase = bi.y * kFinCells;
  const int c = cbase + cl;
  const size_t plane = (size_t)part_plane_len(I.n_jobs, I.part_jg, I.part_ld);
  const T* part = reinterpret_cast<const T*>(I.part);
  const bool adj = (A.flags & FIN_ADJ) != 0, withq = (A.flags & FIN_Q) != 0;
  const int nq = withq ? (adj ? 1 : I.dim) : 0;
  // ---- per-cell totals of every needed plane (inactive cells' entries are
  //      gathered with their neighbours and dropped below)
  double tot[4];
  tot[0] = plane_total(part, I.n_jobs, I.part_jg, I.part_ld, I.ncell, cbase, slc);
  for (int d = 0; d < nq; ++d)
    tot[1 + d] = plane_total(part + (size_t)(1 + d) * plane, I.n_jobs, I.part_jg, I.part_ld, I.ncell, cbase, slc);
  const bool in_blk = cl < kFinCells && c < I.ncell;
  const bool act = in_blk && F.active[c];
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // sum dT^2, max |x|, sum d|q|^2, max |q| (+inf: non-finite)
  if (in_blk) {
    if (act) {
      double x = adj ? F.g[c] : 0.0;
      x += tot[0];
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
          F.q[c] = tot[1];
        } else {
          double m2 = 0.0;
          for (int d2 = 0; d2 < I.dim; ++d2) {
            const double qv = tot[1 + d2];
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
    // non-finite values are caught at the next check. No block reads another
    // block's results here, and each block read the counter before taking its
    // ticket, so no fence is needed: the kernel's end publishes the writes.
    if (threadIdx.x == 0) {
      const int t = atomicAdd(&st->ticket, 1);
      if (t == A.n_blocks_inst[bi.x] - 1) {
        st->ticket = 0;
        st->iter = iter + 1;
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

// Lagged diffuse walls, in two passes so that every read of the out-stream is
// coalesced. First one thread per (octant, band, out-stream entry of that
// octant's schedule): the sum over the octant's groups of that band of the
// entry's value, kept per (octant, band, diffuse face). Then one thread per
// (band, diffuse face): the octants' sums in octant order, scaled into the
// face's inflow value.
template <typename T>
__global__ void __launch_bounds__(256) wall_sum_kernel(WallArgs A) {
  const InstDev& I = A.inst[A.inst_id];
  const StatusDev* st = reinterpret_cast<const StatusDev*>(I.status);
  if (st->done) return;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)I.n_oct * A.B * A.n_out) return;
  const int k = (int)(t % A.n_out);
  const int ob = (int)(t / A.n_out);
  const int b = ob % A.B, o = ob / A.B;
  const int df = A.ent_df[(size_t)o * A.n_out + k];
  if (df < 0) return;
  // o: the octant whose schedule emitted the entries; its groups belong to
  // octant o ^ oct_xor (the transposed sweeps run the flipped schedule)
  const int2 gr = A.grp_ob[(o ^ A.oct_xor) * A.B + b];
  const T* outv = reinterpret_cast<const T*>(I.outv);
  double s = 0.0;
  // (unrolled so that the loads are in flight together; the sum keeps group order)
#pragma unroll 8
  for (int g = 0; g < gr.y; ++g) s += (double)outv[(size_t)(gr.x + g) * A.n_out + k];
  A.wsum[((size_t)o * A.B + b) * A.n_dface + df] = s;
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
  double s = 0.0;
  for (int o = 0; o < I.n_oct; ++o)
    if (A.ofk[(size_t)o * I.n_bface + slot] >= 0) s += A.wsum[((size_t)o * A.B + b) * A.n_dface + df];
  T* ubf = const_cast<T*>(reinterpret_cast<const T*>(I.ubf));
  // a diffuse wall's inflow is the same for every ordinate of the band
  const double sc = A.scale ? A.scale[b * 3 + A.dface_axis[df]] : 1.0;
  const T u = (T)(s * A.inv_half[df] * sc);
  for (int r = 0; r < A.rows; ++r) ubf[((size_t)b * A.rows + r) * I.n_bface + slot] = u;
}

// Lagged specular walls (Eq. 7): one thread per (ordinate, specular face), over
// all bands; ordinates that leave through the face keep their (unused) entries.
template <typename T>
__global__ void __launch_bounds__(256) spec_update_kernel(SpecArgs A) {
  const InstDev& I = A.inst[A.inst_id];
  const StatusDev* st = reinterpret_cast<const StatusDev*>(I.status);
  if (st->done) return;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)A.n_sface * A.M) return;
  const int i = (int)(t % A.n_sface);
  const int a = (int)(t / A.n_sface);
  const int fd = A.sface_dir[i];
  const int2 src = A.src[fd * A.M + a];
  if (src.x < 0) return;
  const int slot = A.sface_slot[i];
  // the mirror's group sweeps the schedule of octant src.x ^ oct_xor
  const int k = A.ofk[(size_t)(src.x ^ A.oct_xor) * I.n_bface + slot];
  const double iwq = A.inv_wq[fd * A.M + a];
  const T* outv = reinterpret_cast<const T*>(I.outv);
  T* ubf = const_cast<T*>(reinterpret_cast<const T*>(I.ubf));
  for (int b = 0; b < A.B; ++b) {
    const int g = A.grp_ob[src.x * A.B + b].x + src.y;
    const double v = (double)outv[(size_t)g * I.n_out_stride + k];
    const double sc = A.scale ? A.scale[b * 3 + fd / 2] : 1.0;
    ubf[((size_t)b * A.M + a) * I.n_bface + slot] = (T)(v * iwq * sc);
  }
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

// ---------------------------------------------- second-order faces
// The deferred correction of Eq. rhs_b for every position of each group's
// octant layout (positions of no cell get 0): the Green-Gauss gradient
// difference between the cell and its upwind neighbour along each grid axis,
// from the field the last sweep stored in the same layout. The neighbours come
// from the octant's stencil table (positions, or boundary codes), so that
// every read but the stencil's field values is in position order. A thread
// takes one position for kCorrGrp consecutive groups (groups are
// octant-major).
constexpr int kCorrGrp = 16;

// Workgroups go to the chip's 8 XCDs in turn. The correction kernel remaps
// its dispatch order so that each XCD takes a contiguous range of (group
// chunk, position) blocks: the neighbour values a wave gathers, a step or a
// plane period away, were then loaded into the same XCD's L2 by the blocks
// beside it.
__device__ __forceinline__ void xcd_blocks(int& bx, int& by) {
  const int nx = gridDim.x, total = nx * gridDim.y;
  const int lin = blockIdx.x + blockIdx.y * nx;
  const int per = total / 8;
  const int l = lin < per * 8 ? (lin % 8) * per + lin / 8 : lin;
  bx = l % nx;
  by = l / nx;
}

template <typename T>
__global__ void __launch_bounds__(256) corr_kernel(CorrArgs A) {
  const InstDev& I = A.inst[A.inst_id];
  const StatusDev* st = reinterpret_cast<const StatusDev*>(I.status);
  if (st->done) return;
  int bx, by;
  xcd_blocks(bx, by);
  const long long ppo = I.pos_per_oct;
  const long long p = (long long)bx * 256 + threadIdx.x;
  if (p >= ppo) return;
  const int dim = I.dim;
  const int n_bface = I.n_bface;
  const int* __restrict__ stencil = A.stencil;
  const T* __restrict__ ufld = reinterpret_cast<const T*>(I.store_u);
  const T* __restrict__ ubf0 = reinterpret_cast<const T*>(I.ubf);
  T* __restrict__ corr0 = reinterpret_cast<T*>(I.corr);
  T ih[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ih[d] = T(1) / (T)A.h[d];
  const int g0 = by * kCorrGrp, g1 = min(g0 + kCorrGrp, A.n_grp);
  // the correction of group g from its field values: the cell, and per axis
  // its downwind and upwind neighbours and the upwind one's upwind neighbour
  auto corr_of = [&](int g, int o, const int* en, const int* eu, const int* euu, T uc, const T* un, const T* uu,
                     const T* uuu) -> T {
    const T* ubf = ubf0 + (size_t)A.grp[g].w * n_bface;
    const T h5 = T(0.5), t15 = T(1.5);
    T corr = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d >= dim) break;
      // face values of the cell: downwind (never an inflow face: the mean
      // with the neighbour, else the extrapolation from the upwind side) and
      // upwind (the mean, the isothermal wall value, else the extrapolation
      // from the downwind side); the cell's own value when the opposite face
      // is a boundary too
      const T fd = en[d] >= 0 ? h5 * (uc + un[d]) : (eu[d] >= 0 ? t15 * uc - h5 * uu[d] : uc);
      const T fu = eu[d] >= 0 ? h5 * (uc + uu[d])
                              : (eu[d] <= -2 ? ubf[-eu[d] - 2] : (en[d] >= 0 ? t15 * uc - h5 * un[d] : uc));
      // the upwind cell: its downwind face is shared with this cell
      T du = T(0);
      if (eu[d] >= 0) {
        const T fuu = euu[d] >= 0 ? h5 * (uu[d] + uuu[d])
                                  : (euu[d] <= -2 ? ubf[-euu[d] - 2] : t15 * uu[d] - h5 * uc);
        du = h5 * (uu[d] + uc) - fuu;
      }
      // (fd - fu) - du is the gradient difference along the ordinate's
      // direction times h; along +d it changes sign in odd octants
      const T dd = ((o >> d) & 1) ? du - (fd - fu) : (fd - fu) - du;
      corr += (T)A.coef[(size_t)g * 3 + d] * ih[d] * dd;
    }
    return corr;
  };
  // groups in batches of kCorrBatch of one octant: every field value of a
  // batch is loaded before any is used, so the gathers overlap
  constexpr int kCorrBatch = 4;
  for (int gb = g0; gb < g1; gb += kCorrBatch) {
    const int nb = min(kCorrBatch, g1 - gb);
    const int o = A.grp[gb].y;
    bool same = true;
    for (int i = 1; i < nb; ++i) same = same && A.grp[gb + i].y == o;
    const int* e = stencil + ((size_t)o * ppo + p) * (3 * dim);
    const bool cell = e[0] != kNoCell;
    int en[3] = {-1, -1, -1}, eu[3] = {-1, -1, -1}, euu[3] = {-1, -1, -1};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d < dim) {
        en[d] = e[3 * d];
        eu[d] = e[3 * d + 1];
        euu[d] = e[3 * d + 2];
      }
    if (same && nb == kCorrBatch) {
      T uc[kCorrBatch], un[kCorrBatch][3], uu[kCorrBatch][3], uuu[kCorrBatch][3];
#pragma unroll
      for (int i = 0; i < kCorrBatch; ++i) {
        const T* u = ufld + (size_t)(gb + i) * ppo;
        uc[i] = cell ? u[p] : T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          un[i][d] = cell && en[d] >= 0 ? u[en[d]] : T(0);
          uu[i][d] = cell && eu[d] >= 0 ? u[eu[d]] : T(0);
          uuu[i][d] = cell && eu[d] >= 0 && euu[d] >= 0 ? u[euu[d]] : T(0);
        }
      }
#pragma unroll
      for (int i = 0; i < kCorrBatch; ++i)
        corr0[(size_t)(gb + i) * ppo + p] = cell ? corr_of(gb + i, o, en, eu, euu, uc[i], un[i], uu[i], uuu[i]) : T(0);
    } else {
      for (int g = gb; g < gb + nb; ++g) {
        const int og = A.grp[g].y;
        const int* eg = stencil + ((size_t)og * ppo + p) * (3 * dim);
        const bool cg = eg[0] != kNoCell;
        int gn[3] = {-1, -1, -1}, gu[3] = {-1, -1, -1}, guu[3] = {-1, -1, -1};
        T un[3] = {}, uu[3] = {}, uuu[3] = {};
        const T* u = ufld + (size_t)g * ppo;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (d < dim) {
            gn[d] = eg[3 * d];
            gu[d] = eg[3 * d + 1];
            guu[d] = eg[3 * d + 2];
            if (cg) {
              un[d] = gn[d] >= 0 ? u[gn[d]] : T(0);
              uu[d] = gu[d] >= 0 ? u[gu[d]] : T(0);
              uuu[d] = gu[d] >= 0 && guu[d] >= 0 ? u[guu[d]] : T(0);
            }
          }
        corr0[(size_t)g * ppo + p] = cg ? corr_of(g, og, gn, gu, guu, u[p], un, uu, uuu) : T(0);
      }
    }
  }
}

// The field before the first sweep: X0 at every position of each group's
// octant layout (0 at positions of no cell).
template <typename T>
__global__ void __launch_bounds__(256) corr_fill_kernel(CorrArgs A) {
  const InstDev& I = A.inst[A.inst_id];
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= I.pos_per_oct) return;
  const int g0 = blockIdx.y * kCorrGrp, g1 = min(g0 + kCorrGrp, A.n_grp);
  // the position's cell: the lane-step record of its octant, row p mod nr
  const int nr = I.nr;
  const int k = (int)(p % nr);
  const int rb = I.dim == 3 ? F3_ROW_BITS : F2_ROW_BITS;
  int o = -1;
  T v = T(0);
  for (int g = g0; g < g1; ++g) {
    const int og = A.grp[g].y;
    if (og != o) {
      o = og;
      const int2 rec = I.sched[(size_t)o * (I.pos_per_oct / nr) + p / nr];
      const bool on = rec.x >= 0 && ((rec.y >> (rb * k)) & 1);
      const int dy = I.dim == 3 ? I.dyo[o] : ((o & 2) ? -I.nx : I.nx);
      v = on ? (T)A.X0[(rec.x >> 5) + k * dy] : T(0);
    }
    reinterpret_cast<T*>(I.store_u)[(size_t)g * I.pos_per_oct + p] = v;
  }
}

template __global__ void finalize_kernel<float>(FinArgs, const FinInst*);
template __global__ void finalize_kernel<double>(FinArgs, const FinInst*);
template __global__ void wall_sum_kernel<float>(WallArgs);
template __global__ void wall_sum_kernel<double>(WallArgs);
template __global__ void wall_update_kernel<float>(WallArgs);
template __global__ void wall_update_kernel<double>(WallArgs);
template __global__ void spec_update_kernel<float>(SpecArgs);
template __global__ void spec_update_kernel<double>(SpecArgs);
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

hipError_t launch_wall_update(int prec, const WallArgs& a, int n_oct, hipStream_t st) {
  const long long n = (long long)a.n_dface * a.B;
  if (n == 0) return hipSuccess;
  const long long ns = (long long)n_oct * a.B * a.n_out;
  if (prec == BTE_PREC_FP32) {
    hipLaunchKernelGGL(wall_sum_kernel<float>, dim3(nblk(ns)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(wall_update_kernel<float>, dim3(nblk(n)), dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL(wall_sum_kernel<double>, dim3(nblk(ns)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(wall_update_kernel<double>, dim3(nblk(n)), dim3(256), 0, st, a);
  }
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

hipError_t launch_spec_update(int prec, const SpecArgs& a, hipStream_t st) {
  const long long n = (long long)a.n_sface * a.M;
  if (n == 0) return hipSuccess;
  if (prec == BTE_PREC_FP32)
    hipLaunchKernelGGL(spec_update_kernel<float>, dim3(nblk(n)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(spec_update_kernel<double>, dim3(nblk(n)), dim3(256), 0, st, a);
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

hipError_t launch_corr(int prec, const CorrArgs& a, long long n_pos, hipStream_t st) {
  if (a.n_grp <= 0 || n_pos <= 0) return hipSuccess;
  const dim3 grid(nblk(n_pos), (a.n_grp + kCorrGrp - 1) / kCorrGrp);
  if (a.X0) {
    if (prec == BTE_PREC_FP32) hipLaunchKernelGGL(corr_fill_kernel<float>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(corr_fill_kernel<double>, grid, dim3(256), 0, st, a);
  }
  if (prec == BTE_PREC_FP32) hipLaunchKernelGGL(corr_kernel<float>, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(corr_kernel<double>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  // a fill kernel rather than a memset node, so that the call can be captured
  const long long n4 = (long long)(bytes / 4);
  if (n4 > 0) hipLaunchKernelGGL(zero_kernel, dim3(nblk(n4)), dim3(256), 0, st, (unsigned*)p, n4);
  return hipGetLastError();
}

}  // namespace bte
