// 1D/2D transport sweep kernel for gfx950 (MI355X), rows-per-lane layout.
//
// One launch performs one source-iteration sweep (paper Methods, "Iterative
// matrix formulation and solution scheme", step 2): for every (band,
// direction) pair the first-order upwind system A e = b (Eqs. Axb, A_matrix with
// first-order faces) is solved exactly by one pass in upwind order, and in the
// same pass the band/direction sums of Eq. updatee0_t (new lattice temperature)
// and Eq. 4 (heat flux) are accumulated, plus the outgoing values at the
// reflecting walls (diffuse, Eq. 6, and specular, Eq. 7).
//
// Work decomposition:
//   * lane l of a wave owns NR consecutive rows (64*NR rows per strip) and
//     sweeps them along x with a skew of one step per lane: at step t it
//     updates column t - l of its rows, bottom row first, so the upwind y value
//     of row k is row k-1 of the same step and, for row 0, the top row of lane
//     l-1 from the previous step, moved with one DPP wave shift;
//   * lane 0's upwind row (the previous strip, or the bottom wall) comes from a
//     column-indexed LDS ring; the ring values of a whole chunk of kC2 steps are
//     read once per chunk into one register (lane m holds step m) and taken
//     with readlane, so no step waits on LDS;
//   * the per-step inputs, a record {cell of row 0, flags} and the (X, Q) pairs
//     of the lane's rows, are stored in the skewed order and prefetched a whole
//     chunk ahead (half a chunk when the ring would not fit in ~96 registers)
//     without any conditional, the schedule being padded; no load inside the
//     chunk loop depends on another one, and no global access in it sits
//     behind a branch (masked lanes get an offset past the buffer), so every
//     wait is for data loaded a chunk earlier;
//   * boundary inflows are an ordered stream whose chunk values sit in LDS
//     (gathered two chunks ahead from a padded per-chunk table); a lane finds
//     its entries from the offset stored in its record;
//   * the P waves of a workgroup sweep P ordinate groups of one octant in
//     lockstep; per step each wave stages its per-row sums over its G ordinates
//     in LDS, and the P partials of every cell are added in a fixed order and
//     written as contiguous row segments: for the temperature-only sweep
//     (double-buffered staging, one barrier per chunk) during the next chunk's
//     steps, otherwise after the chunk;
//   * chunks run in runs of one kind (no boundary entries / x- and row-0
//     y-inflows / any inflow), each kind in a loop of its own, so that the
//     registers of the prefetch ring stay in place from chunk to chunk;
//   * the R wave slots of a workgroup pipeline successive strips (slot r owns
//     strips r, r+R, ...), the top rows reaching the next slot through its ring.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bte_device.h"
#include "bte_kutil.h"
#include "bte_strips.h"

namespace bte {
namespace s2d {

// the kernel's lambdas are inlined whatever their size: the chunk steps index
// register arrays with the step number, which must fold to a constant
#define BTE_INL __attribute__((always_inline))

template <typename T, int N>
struct Vec {
  typedef T type __attribute__((ext_vector_type(N)));
};

// DPP wave_shr:1 (GFX9 encoding 0x138): lane i takes lane i-1, lane 0 keeps `old`.
__device__ __forceinline__ float shr1(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double shr1(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Workgroup barrier for LDS traffic only: wait for this wave's LDS operations,
// then meet the other waves. Outstanding global loads (the prefetch) keep
// flying across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt unchanged
  __builtin_amdgcn_s_barrier();
}

constexpr int min_c(int a, int b) { return a < b ? a : b; }
// largest power of two <= x (1 for x < 1)
constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// the flag bits `bits` repeated for rows 0..nr-1 (rb flag bits per row)
constexpr unsigned rowmask(unsigned bits, int nr, int rb = F2_ROW_BITS) {
  unsigned m = 0;
  for (int k = 0; k < nr; ++k) m |= bits << (rb * k);
  return m;
}

}  // namespace s2d

// M2_SECOND: second-order faces by deferred correction (Methods, "Spatial
// discretization"; Eq. rhs_b): each cell's source gains the group's correction
// term computed from the previous iterate (read per step from the group's
// skewed correction array), and the new angular field is stored for the next
// correction in the same skewed layout (one vector store per lane-step)
enum { M2_PLAIN = 0, M2_STORE = 1, M2_TAUGRAD = 2, M2_SECOND = 3 };

// L3: the 3D rows-per-lane layout (see bte_device.h): the same kernel with
// lanes along the grid's lane axis and the step axis cut into blocks of kC2
// columns, streamed block by block and in a block plane by plane, so that a
// chunk of kC2 steps is one plane period of every lane. The plane-axis upwind
// value is the lane's own value of the same chunk step one chunk earlier,
// kept in registers; the step-axis upwind value of a block's first column is
// the previous block's last column in the same plane, kept per plane in a
// buffer of the wave (one load and one store per lane and chunk, the first
// block's wall values prefilled); lane 0's lane-axis upwind value comes from
// the wall table gpre.
template <typename T, int G, int NR, int P, int NACC, int MODE, bool L3 = false>
__global__ void __launch_bounds__(L3 ? 512 : 256) sweep2d_kernel(SweepArgs A) {
  using namespace s2d;
  static_assert(!L3 || (NR <= 2 && G == 1), "3D rows-per-lane: NR <= 2, one ordinate per lane");
  static_assert(MODE != M2_SECOND || G == 1, "second-order faces: one ordinate per lane");
  constexpr int RB = L3 ? F3_ROW_BITS : F2_ROW_BITS;  // flag bits per row
  constexpr unsigned B_ACT = L3 ? F3_ACT : F2_ACT;
  constexpr unsigned B_INX = L3 ? F3_INX : F2_INX;
  constexpr unsigned B_INY = L3 ? F3_INY : F2_INY;
  constexpr unsigned B_INZ = L3 ? F3_INZ : 0u;
  constexpr unsigned B_OUTX = L3 ? F3_OUTX : F2_OUTX;
  constexpr int ND = L3 ? 3 : 2;  // kernel axes with outflow entries
  constexpr int NV = 2 * NR;                  // (X, Q) values of one lane-step
  // prefetch distance in steps (divides kC2): a whole chunk while the ring of
  // prefetched records and values fits in ~96 registers (G ordinates' worth
  // of other state scales with it), half a chunk above that; a chunk and half
  // a chunk time the same on the bench shapes, so registers decide. The 3D
  // flux and second-order sweeps (eight-wave workgroups; four accumulators,
  // or the correction ring) take half a chunk: a whole one spilled to scratch
  // (a quarter chunk for the second-order flux sweep, which has both)
  constexpr int kRingRegs = 2 + NV * (int)sizeof(T) / 4 * (MODE == M2_TAUGRAD ? 2 : 1) +
                            (MODE == M2_SECOND ? NR * (int)sizeof(T) / 4 : 0);
  constexpr int KD = (L3 && NACC > 2 && MODE == M2_SECOND) ? kC2 / 4
                     : (kRingRegs * kC2 * G <= 96 && !(L3 && (NACC > 2 || MODE == M2_SECOND))) ? kC2
                                                                                              : kC2 / 2;
  using VX = typename Vec<T, NV>::type;
  using VR = typename Vec<T, NR>::type;
  constexpr int GS = grp_stride(G);
  // staged row stride (elements) and record row stride (ints): 8 dwords of
  // padding put the (step, lane) pairs a write-out read takes in one LDS pass
  // on distinct banks
  constexpr int RS = 64 * NR + 32 / (int)sizeof(T);
  constexpr int CS = 64 + 8;
  constexpr int kEPL = 4;                     // inflow entries per lane per chunk (<= 256)
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_job;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = L3 ? 1 : A.R;  // (3D rows plans have one wave slot per ordinate group)
  const int r = wave % R;
  const int p = wave / R;
  const int rprev = (r + R - 1) % R;
  const int W_max = A.W_max;
  const int E = A.e_max;  // LDS inflow buffer entries per chunk (multiple of 64)

  T* ring = reinterpret_cast<T*>(lds + A.lds_zring);    // [P][R][W_max + 1][G] (+1: dummy slot)
  int* scid = reinterpret_cast<int*>(lds + A.lds_cid);  // [2][R][kC2][CS]
  T* inb = reinterpret_cast<T*>(lds + A.lds_in);        // [P*R][2][E]
  T* outb = reinterpret_cast<T*>(lds + A.lds_out);      // [P*R][o_max]
  T* stage = reinterpret_cast<T*>(lds + A.lds_stage);   // [planes][P*R][kC2][RS]
  const int plane_sz = P * R * kC2 * RS;
  const int RW = (W_max + 1) * G;  // ring slot stride
  T* my_ring = ring + (size_t)(p * R + r) * RW;
  const T* prev_ring = ring + (size_t)(p * R + rprev) * RW;
  T* my_inb = inb + (size_t)(p * R + r) * 2 * E;
  T* my_outb = outb + (size_t)(p * R + r) * A.o_max;

  for (;;) {
    __syncthreads();
    if (tid == 0) s_job = atomicAdd(&A.counters[0], 1);
    __syncthreads();
    const int job = __builtin_amdgcn_readfirstlane(s_job);
    if (job >= A.n_jobs) break;
    const JobDev jd = cp(A.jobs)[job];
    const CAS InstDev& I = cp(A.inst)[jd.inst];
    const CAS StatusDev* st = cp(reinterpret_cast<const StatusDev*>(I.status));
    if (!A.force && st->done) continue;
    const int iter = st->iter;

    // ---- this wave's group: band constants and per-ordinate coefficients
    const int g_glob = __builtin_amdgcn_readfirstlane(jd.grp + p);
    const int4 gi = cp(A.grp_i)[g_glob];
    const int ubf_row = gi.w;  // row of the inflow table: the band, or (band, ordinate) with specular walls
    const int g_loc = gi.z;
    const CAS T* gt = cp(reinterpret_cast<const T*>(A.grp_t)) + (size_t)g_glob * GS;
    T kS = gt[0], cQ = gt[1];
    T a0[G], a1[G], a2[G], den[G], inv[G], wo0[G], wo1[G], wo2[G];
    T wacc[NACC][G];
    // grid axes of the kernel's step, lane and plane axes (1D/2D: x, y)
    const int ax0 = L3 ? I.ax[0] : 0, ax1 = L3 ? I.ax[1] : 1, ax2 = L3 ? I.ax[2] : 2;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      a0[g] = gt[go_a(G, ax0) + g];
      a1[g] = gt[go_a(G, ax1) + g];
      a2[g] = L3 ? gt[go_a(G, ax2) + g] : T(0);
      den[g] = gt[go_den(G) + g];
      inv[g] = gt[go_inv(G) + g];
      wo0[g] = gt[go_wo(G, ax0) + g];
      wo1[g] = gt[go_wo(G, ax1) + g];
      wo2[g] = L3 ? gt[go_wo(G, ax2) + g] : T(0);
#pragma unroll
      for (int a = 0; a < NACC; ++a) wacc[a][g] = gt[go_wacc(G, a) + g];
    }
    // one ordinate per lane: the lane carries w0 * f, w0 the ordinate's weight
    // in the temperature sum (the recurrence is linear), so that sum needs no
    // multiply; what enters f is scaled by w0 and what is read from it by
    // 1 / w0 (a padding ordinate has w0 = 0: its lanes carry 0)
    constexpr bool PS = G == 1;
    double tg_scale = 1.0;
    if constexpr (PS) {
      const T w0 = wacc[0][0];
      const T iw = w0 > T(0) ? T(1) / w0 : T(0);
      kS *= w0;
      cQ *= w0;
      den[0] *= w0;
      inv[0] *= iw;
      wo0[0] *= iw;
      wo1[0] *= iw;
      wo2[0] *= iw;
#pragma unroll
      for (int a = 1; a < NACC; ++a) wacc[a][0] *= iw;
      tg_scale = (double)iw;
    }

    const int o = jd.oct;
    const int T_steps = I.T;
    const int Tp = T_steps + kPad2;
    const int nch = T_steps / kC2;
    const int nx = I.nx, ny = I.ny;
    const int du = I.du, n_strip = I.n_strip;
    const bool ring_w = !L3 && n_strip > 1;  // some strip has a successor (1D/2D lane-axis link)
    const int H = 64 * NR;
    const int dy = L3 ? I.dyo[o] : ((o & 2) ? -nx : nx);  // cell-index step from row k to row k+1
    const long long slot = (long long)o * R + r;
    // uniform bases; lanes add 32-bit offsets
    const GAS int2* REC = gp(I.sched + slot * Tp * 64);
    const GAS VX* XQ = gp(reinterpret_cast<const VX*>(I.xq[iter & 1]) + slot * Tp * 64);
    const GAS VX* XF = MODE == M2_TAUGRAD ? gp(reinterpret_cast<const VX*>(I.xf) + slot * Tp * 64) : nullptr;
    // second-order correction of this group: [n_grp][pos_per_oct] in the
    // octant's skewed layout, a VR of the lane's rows per step
    const GAS VR* XC = MODE == M2_SECOND
                           ? gp(reinterpret_cast<const VR*>(reinterpret_cast<const T*>(I.corr) +
                                                            (size_t)g_loc * I.pos_per_oct) +
                                (long long)r * Tp * 64)
                           : nullptr;
    const int lo_xc = lane * (int)sizeof(VR);
    // the group's stored field, in the same layout
    GAS VR* XS = MODE == M2_SECOND ? gp(reinterpret_cast<VR*>(reinterpret_cast<T*>(I.store_u) +
                                                               (size_t)g_loc * I.pos_per_oct) +
                                         (long long)r * Tp * 64)
                                   : nullptr;
    const GAS T* UBF = gp(reinterpret_cast<const T*>(I.ubf) + (size_t)ubf_row * I.n_bface);
    const int Ei = I.in_E;  // this instance's entries per chunk row of in_tab (<= E)
    const GAS int* ITAB = gp(I.in_tab + slot * (nch + 2) * Ei);
    GAS T* OUTV = gp(reinterpret_cast<T*>(I.outv) + (size_t)g_loc * I.n_out_stride + cp(I.out_base)[slot]);
    const size_t part_plane = (size_t)part_plane_len(I.n_jobs, I.part_jg, I.part_ld);
    // (a view spans the job's group; a cell outside the grid lands past its
    // end or in the job's own padding)
    GAS T* PARTJ = gp(reinterpret_cast<T*>(I.part) + part_job(jd.jl, I.part_jg, I.part_ld));
    const unsigned pgrp = (unsigned)(((size_t)I.part_ld << I.part_jg) - (size_t)(jd.jl & ((1 << I.part_jg) - 1)) * kPartBlk);
    // buffer views of the chunk loop's global data (sizes in bytes)
    const int out_b = cp(I.out_base)[slot];
    const rsrc_t UBR = mkrsrc(UBF, (unsigned)I.n_bface * (unsigned)sizeof(T));
    const rsrc_t ITR = mkrsrc(ITAB, (unsigned)((nch + 2) * Ei) * 4u);
    const rsrc_t OUR = mkrsrc(OUTV, (unsigned)(I.n_out_stride - out_b) * (unsigned)sizeof(T));
    rsrc_t PRS[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) PRS[a] = mkrsrc(PARTJ + a * part_plane, pgrp * (unsigned)sizeof(T));
    const int pgap = part_gap(I.part_jg);  // cell c at c + (c >> 8) * pgap (part_off)
    // 3D: this wave's step-axis buffer (a VR per plane and lane)
    const int n_pl = L3 ? I.n_pl : 1;
    const int zrow = 64 * NR * (int)sizeof(T);  // bytes per plane
    GAS T* ZR = L3 ? gp(reinterpret_cast<T*>(A.zg) + ((long long)blockIdx.x * P + p) * A.zg_stride) : nullptr;
    const rsrc_t ZRR = mkrsrc(ZR, L3 ? (unsigned)(n_pl * zrow) : 0u);
    const int lo_z = lane * NR * (int)sizeof(T);

    // ---- clear the ring; prefill the ring read by strip 0 (slot R-1's) with
    //      the bottom-wall inflow of every column
    if constexpr (!L3)
      for (int e = lane; e < RW; e += 64) my_ring[e] = T(0);
    __syncthreads();
    if constexpr (L3) {
      // the first block's step-axis wall values, one per plane
      const GAS int* xp = gp(I.xpre + (size_t)o * n_pl * H);
      for (int pl = 0; pl < n_pl; ++pl) {
        VR zv;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          const int sl = xp[(size_t)pl * H + lane * NR + k];
          zv[k] = sl >= 0 ? UBF[sl] * den[0] : T(0);
        }
        stv(zv, ZRR, lo_z, pl * zrow);
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the buffer is written before it is read
    } else if (r == 0) {
      T* zr = ring + (size_t)(p * R + (R - 1)) * RW;
      const GAS int* pre = gp(I.pre_slot + (size_t)o * I.W);
      for (int c = lane; c < I.W; c += 64) {
        const int sl = pre[c];
        const T u = sl >= 0 ? UBF[sl] : T(0);
#pragma unroll
        for (int g = 0; g < G; ++g) zr[c * G + g] = u * den[g];
      }
    }

    // ---- inflow stream: the values of chunk k sit in LDS buffer (k & 1); the
    //      values of chunk k+1 and the face slots of chunk k+2 wait in registers
    const int NE = Ei >> 6;
    int slot_n[kEPL];
    T inval[kEPL];
#pragma unroll
    for (int m = 0; m < kEPL; ++m) {
      if (m < NE) {
        const int s0 = ITAB[m * 64 + lane];
        my_inb[m * 64 + lane] = s0 >= 0 ? UBF[s0] * (L3 ? den[0] : T(1)) : T(0);
        const int s1 = ITAB[Ei + m * 64 + lane];
        inval[m] = s1 >= 0 ? UBF[s1] : T(0);
        slot_n[m] = ITAB[2 * Ei + m * 64 + lane];
      } else {
        inval[m] = T(0);
        slot_n[m] = -1;
      }
    }
    __syncthreads();

    // ---- per-lane state
    T f[G][NR];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < NR; ++k) f[g][k] = T(0);
    double tg0 = 0.0, tg1 = 0.0;
    int out_tot = 0;

    // ---- per-step inputs, prefetched KD steps ahead into a register ring
    //      (the schedule is padded by kPad2 >= KD steps)
    const int lo_rec = lane * 8, lo_xq = lane * (int)sizeof(VX);
    // one buffer view per array over the slot's steps; a chunk adds its first
    // prefetched step as a uniform offset
    const unsigned nposs = (unsigned)Tp * 64u;
    const rsrc_t RRB = mkrsrc(REC, nposs * 8u);
    const rsrc_t RXB = mkrsrc(XQ, nposs * (unsigned)sizeof(VX));
    const rsrc_t RFB = MODE == M2_TAUGRAD ? mkrsrc(XF, nposs * (unsigned)sizeof(VX)) : RXB;
    const rsrc_t RCB = MODE == M2_SECOND ? mkrsrc(XC, nposs * (unsigned)sizeof(VR)) : RXB;
    const rsrc_t RSB = MODE == M2_SECOND ? mkrsrc(XS, nposs * (unsigned)sizeof(VR)) : RXB;
    int2 RR[KD];
    VX RX[KD];
    VX RXF[KD];
    VR RC[KD];
    {
#pragma unroll
      for (int u = 0; u < KD; ++u) {
        RR[u] = ldrec_b(RRB, lo_rec, u * 64 * 8);
        RX[u] = ldv<VX>(RXB, lo_xq, u * 64 * (int)sizeof(VX));
        if (MODE == M2_TAUGRAD) RXF[u] = ldv<VX>(RFB, lo_xq, u * 64 * (int)sizeof(VX));
        if (MODE == M2_SECOND) RC[u] = ldv<VR>(RCB, lo_xc, u * 64 * (int)sizeof(VR));
      }
    }

    // 3D plane link and block link. Lane l's chunk-step u is column
    // (u - l) mod kC2 of its block: column 0 at u = l mod kC2 (plane period
    // q = ch - l/kC2 of chunk ch), the last column at u = l - 1 mod kC2
    // (period ch - (l + kC2 - 1)/kC2). zreg[u]: the value of chunk-step u one
    // chunk earlier (the same column one plane back); xl: the step-axis value
    // of this chunk's column-0 step, xn: the next chunk's (in flight). The
    // last-column value is read back from the chunk's staged sums (the lane's
    // own values) and stored at the end of the chunk to the period's plane.
    // The plane of a period comes from the period table (plane + 1, 0: no
    // period), read a chunk before it is needed.
    VR zreg[L3 ? kC2 : 1], xl, xn;
    // 3D inflow chunks: the next step's stream values of the lane's rows
    // (step, lane, plane axis), read from LDS one step ahead
    T pin[L3 ? NR : 1][3];
    int qL = 0, qS = 0, pL1 = 0, pS1 = 0;  // period and plane + 1 of the next load / store
    const rsrc_t GPR = mkrsrc(L3 ? gp(I.gpre) + (size_t)o * (T_steps + I.n_per) : nullptr,
                              L3 ? (unsigned)(T_steps + I.n_per) * 4u : 0u);
    auto ptab = [&](int q) BTE_INL { return bld<int>(GPR, q >= 0 && q < I.n_per ? (T_steps + q) * 4 : kOOB); };
    auto xoff = [&](int p1) BTE_INL { return p1 > 0 ? (p1 - 1) * zrow + lo_z : kOOB; };
    if constexpr (L3) {
#pragma unroll
      for (int u = 0; u < kC2; ++u)
#pragma unroll
        for (int k = 0; k < NR; ++k) zreg[u][k] = T(0);
      qL = -(lane / kC2);
      xl = ldv_glc<VR>(ZRR, xoff(ptab(qL)), 0);
      ++qL;
      xn = ldv_glc<VR>(ZRR, xoff(ptab(qL)), 0);
      ++qL;
      pL1 = ptab(qL);
      qS = -((lane + kC2 - 1) / kC2);
      pS1 = ptab(qS);
    }

    // ghost values (lane 0's upwind row) and ring-write offsets (lane 63's top
    // row; the dummy slot W_max when there is nothing to write) of a chunk:
    // lane m < kC2 holds step m's
    StripTrack gt_, wt_;  // lane 0 at clock chunk*kC2 + m, lane 63 at that clock - 63
    gt_.init(lane, r, R, du, n_strip);
    wt_.init(lane - 63, r, R, du, n_strip);
    T ghv[G];
    int wcv;
    // 3D: lane 0's lane-axis wall values, pipelined so that no chunk waits on
    // a gather: ghv holds chunk c's values (lane m: step m), ghn the raw
    // gathered values of chunk c+1, gsl the wall slots (+1, 0: none) of chunk c+2
    T ghn = T(0);
    int gsl = 0, gch = 0;  // gch: chunk of the slots to load next
    auto gslot = [&]() BTE_INL {
      const int t = gch * kC2 + lane;
      ++gch;
      return bld<int>(GPR, lane < kC2 && t < T_steps ? t * 4 : kOOB);
    };
    auto ggather = [&](int g1) BTE_INL { return bld<T>(UBR, g1 > 0 ? (g1 - 1) * (int)sizeof(T) : kOOB); };
    if constexpr (L3) {
      ghv[0] = ggather(gslot()) * den[0];
      ghn = ggather(gslot());
      gsl = gslot();
    }
    auto chunk_cols = [&]() BTE_INL {
      const bool gok = lane < kC2 && gt_.valid(n_strip, nx);
      if constexpr (L3) {
        // the gather issued a chunk ago, then the next one and the slots after
        ghv[0] = ghn * den[0];
        ghn = ggather(gsl);
        gsl = gslot();
        wcv = W_max * G;
        (void)gok;
      } else {
#pragma unroll
        for (int g = 0; g < G; ++g) ghv[g] = gok ? prev_ring[gt_.v * G + g] : T(0);
        const bool wok = lane < kC2 && wt_.valid(n_strip, nx) && wt_.s * H + H - 1 < ny;
        wcv = (wok ? wt_.v : W_max) * G;
      }
      gt_.advance(kC2, R);
      wt_.advance(kC2, R);
    };
    if constexpr (!L3) chunk_cols();
    // per-chunk flags (CF2_*), uniform: scalar loads from read-only memory
    const CAS int* CFL = cp(I.chunk_fl) + slot * (nch + 1);
    int cfl = CFL[0];
    int cfl_next = CFL[nch > 0 ? 1 : 0];
    // let the loads above land before the chunk loop: the loop's waits are
    // counted for its steady state (a whole chunk of loads after each slot's),
    // which a partly drained prologue would otherwise cut to its own shorter
    // tail for every chunk
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt unchanged

    // ---- write-out of the staged sums: the P waves of slot r add their
    //      partials in a fixed order and write contiguous row segments. A
    //      thread takes whole (lane, step) pairs: pair e -> lane e/8, step e%8,
    //      so 8 neighbouring threads write 8 consecutive cells of each of the
    //      lane's rows; the NR rows of a pair are one vector read per wave.
    //      Temperature-only sweeps (NACC == 1, double-buffered staging) write a
    //      chunk out during the next chunk's steps, a batch of pairs read at
    //      an even step and stored at the odd step after it, so no step waits
    //      on LDS and the stores need no wait at all.
    constexpr bool PIPE = NACC == 1;
    constexpr int PAIRS = kC2 / P;
    constexpr int NB = PIPE ? (PAIRS < kC2 / 2 ? PAIRS : kC2 / 2) : 1;
    // pairs per batch: the pipelined write-out splits the pairs over NB
    // batches; the chunk-end write-out takes a power of two (so it divides
    // PAIRS) that keeps a batch's reads within ~32 registers
    constexpr int MB = PIPE ? PAIRS / NB
                            : pow2_floor(min_c(PAIRS, 32 / (NACC * NR * (int)(sizeof(T) / 4))));
    static_assert(MB >= 1 && PAIRS % MB == 0 && (!PIPE || MB * NB == PAIRS),
                  "write-out batches must tile the pairs exactly");
    const int t_wo = p * 64 + lane;
    int wvv[MB];
    // the pipelined write-out holds every wave's partial until the store step
    // (its adds then wait on nothing); the chunk-end one adds as it reads
    constexpr int PQ = PIPE ? P : 1;
    VR wraw[NACC][MB][PQ];
    // read a batch of pairs of chunk chw (its records and every wave's sums)
    auto wo_read = [&](int b, int chw) BTE_INL {
      const int bw = chw & 1;
      const int* scr = scid + (bw * R + r) * kC2 * CS;
#pragma unroll
      for (int mi = 0; mi < MB; ++mi) {
        const int e = (b * MB + mi) * (P * 64) + t_wo;
        const int ln = e >> 3, cc = e & 7;
        wvv[mi] = scr[cc * CS + ln];
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
          const T* sp = stage + (size_t)(NACC == 1 ? bw : a) * plane_sz + (size_t)r * kC2 * RS + cc * RS + ln * NR;
          if constexpr (PIPE) {
#pragma unroll
            for (int q = 0; q < P; ++q) wraw[a][mi][q] = *reinterpret_cast<const VR*>(sp + (size_t)q * R * kC2 * RS);
          } else {
            wraw[a][mi][0] = *reinterpret_cast<const VR*>(sp);
#pragma unroll
            for (int q = 1; q < P; ++q) wraw[a][mi][0] += *reinterpret_cast<const VR*>(sp + (size_t)q * R * kC2 * RS);
          }
        }
      }
    };
    // add the batch's partials and store the lane's rows (inactive cells'
    // entries are ignored by the finalize); `on` false: nothing
    auto wo_store = [&](bool on) BTE_INL {
#pragma unroll
      for (int mi = 0; mi < MB; ++mi) {
        const int v = on ? wvv[mi] : -1;
        const int cid0 = v >> 5;
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
          VR sm = wraw[a][mi][0];
#pragma unroll
          for (int q = 1; q < PQ; ++q) sm += wraw[a][mi][q];
          if constexpr (!L3) {
            // 1D/2D planes keep one job per group: the cell index itself. The
            // lane axis is the grid's slowest, so a row of the lane outside
            // the grid has a cell index past either end of the plane (or in
            // the job's padding) and the buffer's range check drops it
#pragma unroll
            for (int k = 0; k < NR; ++k) bst(sm[k], PRS[a], v >= 0 ? (cid0 + k * dy) * (int)sizeof(T) : kOOB);
          } else {
            // 3D: the lane axis may be a faster grid axis, where the index of
            // a row past the grid's end is a cell of the next line: rows
            // outside the grid (record bit k clear) are not stored
#pragma unroll
            for (int k = 0; k < NR; ++k) {
              const int c = cid0 + k * dy;
              int off = (v >= 0 && ((v >> k) & 1)) ? (c + __mul24(c >> 8, pgap)) * (int)sizeof(T) : kOOB;
              // (opaque, so that the store stays one instruction rather than
              // being split into a branch per case of the select)
              asm volatile("" : "+v"(off));
              bst(sm[k], PRS[a], off);
            }
          }
        }
      }
    };

    // ---- 3D: a chunk's reflecting-wall outflows, read back from its staged
    //      values (one ordinate per lane: the staged temperature partial of
    //      the wave is the lane's own value) and written to the out-stream
    //      after the chunk; oe holds the entries of chunk `c`, och its stream
    //      offset, and the entries of the chunk after are loaded behind them
    constexpr int kOPL = 4;  // entries per lane per chunk (<= 256 per chunk)
    int oe[kOPL];
    int och = 0;
    const int NOE = L3 ? I.out_E >> 6 : 0;
    const rsrc_t OTR = mkrsrc(L3 ? gp(I.out_tab) + (size_t)o * (nch + 2) * I.out_E : nullptr,
                              L3 ? (unsigned)((nch + 2) * I.out_E) * 4u : 0u);
    const CAS int* OCH = L3 ? cp(I.out_chunk) + (size_t)o * (nch + 1) : nullptr;
    auto out_load = [&](int c) BTE_INL {
      // entry m of the lane at (c * out_E + m * 64 + lane) * 4; an entry
      // past the row (m >= NOE) gets an offset past the buffer (uniform, so
      // no per-lane mask is kept)
      const int lo = (c * I.out_E + lane) * 4;
#pragma unroll
      for (int m = 0; m < kOPL; ++m) oe[m] = bld<int>(OTR, lo + (m < NOE ? m * 256 : kOOB));
    };
    if constexpr (L3) {
      out_load(0);
      och = OCH[0];
    }
    auto emit = [&](int c) BTE_INL {
      const T* sb = stage + (size_t)(NACC == 1 ? (c & 1) : 0) * plane_sz + (size_t)(p * R + r) * kC2 * RS;
      // the axis weight of an entry by arithmetic (a select between the
      // three would be turned into an indexed read of a stack copy)
      const T wA = wo0[0], wB = wo1[0] - wo0[0], wC = wo2[0] - wo1[0];
#pragma unroll
      for (int m = 0; m < kOPL; ++m) {
        const int e = oe[m] - 1;  // stored + 1 (0: no entry, also what a read past the table gives)
        const int idx = e >> 2, d = e & 3;
        const T v = sb[(e >= 0 ? idx / (64 * NR) : 0) * RS + (idx & (64 * NR - 1))];
        const T w = fma(T(d >= 2), wC, fma(T(d >= 1), wB, wA));
        bst(w * v, OUR, e >= 0 ? (och + m * 64 + lane) * (int)sizeof(T) : kOOB);
      }
      out_load(c + 1);
      och = OCH[min(c + 1, nch)];
    };

    // ---- one chunk of kC2 steps; IN: 0 no flagged inflow entries in the
    //      chunk, 1 x-inflows and row-0 y-inflows only (folded into the chain
    //      inputs), 2 any inflow (its own chain with selects); OUT: reflecting-wall
    //      outflow entries present; XS: lanes entering their strip at the x wall
    //      (F2_XSTART), whose x-inflows are read from LDS a step ahead
    auto chunk = [&](auto in_tag, auto out_tag, auto xs_tag, const int ch) BTE_INL {
      constexpr int IN = decltype(in_tag)::value;
      constexpr bool OUT = decltype(out_tag)::value && !L3;  // 3D: outflows leave after the chunk
      constexpr bool XS = decltype(xs_tag)::value && !L3;  // 3D: every inflow goes through the stream
      const int bufi = ch & 1;
      const T* inbuf = my_inb + bufi * E;
      T* stg0 = stage + (size_t)(NACC == 1 ? bufi : 0) * plane_sz + (size_t)(p * R + r) * kC2 * RS;
      int* scw = scid + (bufi * R + r) * kC2 * CS;
      int out_cnt = 0;
      // the chunk's prefetch: 3D through the fixed views with a uniform offset
      // (fewer scalar registers live), 1D/2D through views based at the first
      // position prefetched in the chunk (immediate offsets per step)
      const int s0 = (ch * kC2 + KD) * 64;
      auto cview = [&](auto base, int esz, rsrc_t fixed) BTE_INL {
        return L3 ? fixed : mkrsrc((const char*)base + (size_t)s0 * esz, 0xFFFFFFFFu);
      };
      const rsrc_t rr = cview(REC, 8, RRB), rx = cview(XQ, (int)sizeof(VX), RXB);
      const rsrc_t rf = MODE == M2_TAUGRAD ? cview(XF, (int)sizeof(VX), RFB) : rx;
      const rsrc_t rc = MODE == M2_SECOND ? cview(XC, (int)sizeof(VR), RCB) : rx;
      const int sb = L3 ? s0 : 0;  // offset of the chunk's first prefetched position in its view
      // strip-entry x-inflows of the step about to run (read one step ahead;
      // the chunk's first step reads its own after the chunk barrier)
      // (two register sets by step parity, so no value is copied)
      T xv[2][NR];
      auto read_xv = [&](const int2 rnext, T* dst) BTE_INL {
        // a lane-step's entries end inside the chunk's stream: clamping the
        // offset keeps the reads of the other lanes in bounds
        const int e0 = min((int)(((unsigned)rnext.y >> F2_INOFF_SHIFT) & F2_INOFF_MASK), E - NR);
        const T* ip = inbuf + e0;
#pragma unroll
        for (int k = 0; k < NR; ++k) dst[k] = ip[k];
      };
      if constexpr (XS) read_xv(RR[0], xv[0]);
      // 3D: a lane's stream entries (rows ascending, then the step, lane and
      // plane axes, from its offset), for the step of record rn. The offset
      // of an axis without an inflow may point up to six entries past the
      // chunk's buffer, still inside the workgroup's LDS (the next buffer or
      // the staging area); that value is never selected
      auto in_read = [&](const int2 rn) BTE_INL {
        const unsigned fr = (unsigned)rn.y;
        const int e0 = (int)((fr >> F2_INOFF_SHIFT) & F2_INOFF_MASK);
        constexpr unsigned kAll = rowmask(B_INX | B_INY | B_INZ, NR, RB);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          const unsigned b = fr >> (RB * k);
          const int ex = e0 + __builtin_popcount(fr & kAll & ((1u << (RB * k)) - 1u));
          const int ey = ex + ((b & B_INX) ? 1 : 0);
          const int ez = ey + ((b & B_INY) ? 1 : 0);
          pin[k][0] = inbuf[ex];
          pin[k][1] = inbuf[ey];
          pin[k][2] = inbuf[ez];
        }
      };
      if constexpr (L3 && IN == 2) in_read(RR[0]);

      auto step = [&](const int u) BTE_INL {
        const int sl = u % KD;
        const int2 rec = RR[sl];
        // both halves of the record stay live until here, whatever the body
        // uses: a half the body ignores would otherwise free its register
        // while the load is in flight, and reusing it waits for that load
        asm volatile("" ::"v"(rec.x), "v"(rec.y));
        const VX xq = RX[sl];
        VX xf;
        if (MODE == M2_TAUGRAD) xf = RXF[sl];
        // 3D: the plane-axis upwind values (chunk-step u one chunk back) and
        // the step-axis ones (the previous column, or for the block's first
        // column the buffer value)
        // (3D: the previous step's values are zreg[um], so the lane's own
        // state is the delay line alone)
        const int um = (u + kC2 - 1) % kC2;
        VR zr;
        T xin[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) xin[k] = f[0][k];
        if constexpr (L3) {
          zr = zreg[u];
          const bool c0 = (lane & (kC2 - 1)) == u;
#pragma unroll
          for (int k = 0; k < NR; ++k) xin[k] = c0 ? xl[k] : zreg[um][k];
        }
        const unsigned fl = (unsigned)rec.y;
        T S[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) S[k] = kS * xq[2 * k] + cQ * xq[2 * k + 1];
        if constexpr (MODE == M2_SECOND) {
          const VR xc = RC[sl];
#pragma unroll
          for (int k = 0; k < NR; ++k) S[k] += xc[k];
        }

        // upwind value of row 0: the lane below's top row of the previous step;
        // lane 0 takes the ring value of this step
        T zc[G];
        if constexpr (L3) {
          zc[0] = shr1(rdlane(ghv[0], u), zreg[um][NR - 1]);
        } else {
#pragma unroll
          for (int g = 0; g < G; ++g) zc[g] = shr1(rdlane(ghv[g], u), f[g][NR - 1]);
        }

        // a lane entering its strip at the x wall takes its x-inflows as the
        // rows' x-upwind values (after the lane below has had the old top row)
        if constexpr (XS) {
          const bool xs = (fl & F2_XSTART) != 0;
#pragma unroll
          for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int g = 0; g < G; ++g) f[g][k] = xs ? xv[u & 1][k] * den[g] : f[g][k];
          if (u + 1 < kC2) read_xv(RR[(u + 1) % KD], xv[(u + 1) & 1]);
        }

        constexpr unsigned kInAll = rowmask(B_INX | B_INY | B_INZ, NR, RB);
        if (!L3 && IN == 1 && __ballot(fl & kInAll) != 0ull) {
          // x-inflows replace the rows' x-upwind values and a row-0 y-inflow
          // the lane-below value before the common chain (the lane's entries:
          // rows ascending, x before y, from its offset)
          const int e0 = (int)((fl >> F2_INOFF_SHIFT) & F2_INOFF_MASK);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const unsigned b = fl >> (F2_ROW_BITS * k);
            const int ex = e0 + __builtin_popcount(fl & kInAll & ((1u << (F2_ROW_BITS * k)) - 1u));
            const T vx = inbuf[min(ex, E - 1)];
#pragma unroll
            for (int g = 0; g < G; ++g) f[g][k] = (b & F2_INX) ? vx * den[g] : f[g][k];
            if (k == 0) {
              const T vy = inbuf[min(ex + ((b & F2_INX) ? 1 : 0), E - 1)];
#pragma unroll
              for (int g = 0; g < G; ++g) zc[g] = (b & F2_INY) ? vy * den[g] : zc[g];
            }
          }
        }
        if constexpr (L3 && IN == 2) {
          // 3D inflow chunks: every step takes the selects, with the values
          // read a step ahead (no LDS wait in the chain); then the next
          // step's values
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const unsigned b = fl >> (RB * k);
            const T xu = (b & B_INX) ? pin[k][0] : xin[k];
            const T zu = (b & B_INY) ? pin[k][1] : zc[0];
            const T pu = (b & B_INZ) ? pin[k][2] : zr[k];
            const T fn = fma(a1[0], zu, fma(a0[0], xu, fma(a2[0], pu, S[k])));
            f[0][k] = fn;
            zc[0] = fn;
          }
          if (u + 1 < kC2) in_read(RR[(u + 1) % KD]);
        } else if (IN == 2 && __ballot(fl & kInAll) != 0ull) {
          // entries of this lane: rows ascending, then the step, lane and
          // plane axes, from its offset
          const int e0 = (int)((fl >> F2_INOFF_SHIFT) & F2_INOFF_MASK);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const unsigned b = fl >> (RB * k);
            const unsigned below = fl & kInAll & ((1u << (RB * k)) - 1u);
            const int ex = e0 + __builtin_popcount(below);
            const int ey = ex + ((b & B_INX) ? 1 : 0);
            const T vx = inbuf[min(ex, E - 1)];
            const T vy = inbuf[min(ey, E - 1)];
            T vz = T(0);
            if constexpr (L3) vz = inbuf[min(ey + ((b & B_INY) ? 1 : 0), E - 1)];
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const T xu = (b & B_INX) ? vx * den[g] : (L3 ? xin[k] : f[g][k]);
              const T zu = (b & B_INY) ? vy * den[g] : zc[g];
              T fn = fma(a1[g], zu, fma(a0[g], xu, S[k]));
              if constexpr (L3) fn = fma(a2[g], (b & B_INZ) ? vz * den[g] : zr[k], fn);
              f[g][k] = fn;
              zc[g] = fn;
            }
          }
        } else {
          // the common chain
#pragma unroll
          for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int g = 0; g < G; ++g) {
              // the lane-axis value (the step's critical chain) enters last
              T fn;
              if constexpr (L3)  // accumulated in the plane-link value's register
                fn = fma(a1[g], zc[g],
                         fma(a0[g], xin[k],
                             fma(kS, xq[2 * k],
                                 fma(cQ, xq[2 * k + 1],
                                     MODE == M2_SECOND ? fma(a2[g], zr[k], RC[sl][k]) : a2[g] * zr[k]))));
              else
                fn = fma(a1[g], zc[g], fma(a0[g], f[g][k], S[k]));
              f[g][k] = fn;
              zc[g] = fn;
            }
        }
        if constexpr (L3) {
          // the plane link of the next chunk
#pragma unroll
          for (int k = 0; k < NR; ++k) zreg[u][k] = f[0][k];
        }

        // ---- fused band/direction sums of the rows, staged for the workgroup
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
          VR acc;
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            T sm = T(0);
#pragma unroll
            for (int g = 0; g < G; ++g) sm = (PS && a == 0) ? f[g][k] : fma(wacc[a][g], f[g][k], sm);
            acc[k] = sm;
          }
          *reinterpret_cast<VR*>(stg0 + (size_t)(NACC == 1 ? 0 : a) * plane_sz + u * RS + lane * NR) = acc;
        }
        scw[u * CS + lane] = rec.x;  // every wave of the slot writes the same records

        // ---- the strip's top row for the next slot (lane 63), when a strip
        //      follows at all
        if (ring_w) {
          const int wc = rdlane(wcv, u);
          if (lane == 63) {
#pragma unroll
            for (int g = 0; g < G; ++g) my_ring[wc + g] = f[g][NR - 1];
          }
        }

        // ---- reflecting-wall outflow stream: rows, then axes, then lanes
        constexpr unsigned kOutAll = rowmask(B_OUTX | (B_OUTX << 1) | (L3 ? B_OUTX << 2 : 0u), NR, RB);
        if (OUT && __ballot(fl & kOutAll) != 0ull) {
#pragma unroll
          for (int k = 0; k < NR; ++k) {
#pragma unroll
            for (int d = 0; d < ND; ++d) {
              const unsigned bit = (B_OUTX << d) << (RB * k);
              const unsigned long long m = __ballot(fl & bit);
              if (m != 0ull) {
                if (fl & bit) {
                  T v = T(0);
#pragma unroll
                  for (int g = 0; g < G; ++g) v = fma(d == 0 ? wo0[g] : (d == 1 ? wo1[g] : wo2[g]), f[g][k], v);
                  my_outb[out_cnt + lanes_below(m)] = v;
                }
                out_cnt += __popcll(m);
              }
            }
          }
        }

        // ---- stored angular field / tau-gradient sums
        if constexpr (MODE == M2_SECOND) {
          VR v;
#pragma unroll
          for (int k = 0; k < NR; ++k) v[k] = f[0][k] * inv[0];
          stv<VR>(v, RSB, lo_xc, (ch * kC2 + u) * 64 * (int)sizeof(VR));
        }
        if (MODE == M2_STORE && rec.x >= 0) {
#pragma unroll
          for (int k = 0; k < NR; ++k)
            if ((fl >> (RB * k)) & B_ACT) {
              GAS T* su =
                  gp(reinterpret_cast<T*>(I.store_u) + ((size_t)g_loc * I.ncell + (rec.x >> 5) + k * dy) * G);
#pragma unroll
              for (int g = 0; g < G; ++g) su[g] = f[g][k] * inv[g];
            }
        }
        if (MODE == M2_TAUGRAD && rec.x >= 0) {
          const CAS T* wt0 = gt + go_wt(G, 0);
          const CAS T* wt1 = gt + go_wt(G, 1);
#pragma unroll
          for (int k = 0; k < NR; ++k)
            if ((fl >> (RB * k)) & B_ACT) {
              const GAS T* su =
                  gp(reinterpret_cast<const T*>(I.store_u) + ((size_t)g_loc * I.ncell + (rec.x >> 5) + k * dy) * G);
              double s0 = 0.0, s1 = 0.0;
#pragma unroll
              for (int g = 0; g < G; ++g) {
                const double uf = (double)su[g];
                s0 += (double)wt0[g] * tg_scale * (double)f[g][k] * (uf - (double)xf[2 * k]);
                s1 += (double)wt1[g] * uf;
              }
              tg0 += s0;
              tg1 += (double)xq[2 * k] * s1;
            }
        }

        // ---- the previous chunk's write-out (temperature-only sweeps)
        if constexpr (PIPE) {
          if (u % 2 == 0 && u / 2 < NB) wo_read(u / 2, ch - 1);
          if (u % 2 == 1 && u / 2 < NB) wo_store(ch > 0);
          // and its outflows
          if (L3 && u == kC2 - 3 && ch > 0) emit(ch - 1);
        }
        // ---- inflow pipeline, one stream row per step at the chunk's end,
        //      rows in descending order: values of chunk ch+1 to LDS (a row
        //      past the stream writes row 0, which row 0's own write then
        //      replaces: no branch); gather chunk ch+2's values (a slot of -1
        //      reads 0); load the face slots of chunk ch+3
        if (u >= kC2 - kEPL) {
          const int m = kC2 - 1 - u;
          // (3D: stored scaled into the lane's variable, read once per use)
          my_inb[((ch + 1) & 1) * E + (m < NE ? m : 0) * 64 + lane] = L3 ? inval[m] * den[0] : inval[m];
          inval[m] = bld<T>(UBR, slot_n[m] * (int)sizeof(T));
          slot_n[m] = bld<int>(ITR, m < NE && ch + 3 < nch + 2 ? ((ch + 3) * Ei + m * 64 + lane) * 4 : kOOB);
        }

        // ---- prefetch step ch*kC2 + u + KD into the slot just consumed; the
        //      fence keeps the loads after the last use of the old values, so
        //      every slot is reloaded in place
        __builtin_amdgcn_sched_barrier(0);
        RR[sl] = ldrec_b(rr, lo_rec, (sb + u * 64) * 8);
        RX[sl] = ldv<VX>(rx, lo_xq, (sb + u * 64) * (int)sizeof(VX));
        if (MODE == M2_TAUGRAD) RXF[sl] = ldv<VX>(rf, lo_xq, (sb + u * 64) * (int)sizeof(VX));
        if (MODE == M2_SECOND) RC[sl] = ldv<VR>(rc, lo_xc, (sb + u * 64) * (int)sizeof(VR));
      };
#pragma unroll
      for (int u = 0; u < kC2; ++u) step(u);

      // ---- end of chunk: the staged sums, the ring and the outflow entries
      //      of every wave are complete
      lds_barrier();
      if constexpr (L3) {
        // the block's last column of this chunk's period to its plane; the
        // column-0 value of the chunk after the next one (its plane was
        // written at least a chunk ago: four or more planes)
        // (the lane's last column is chunk step u = l - 1 mod kC2)
        const VR xs = *reinterpret_cast<const VR*>(stg0 + ((lane + kC2 - 1) & (kC2 - 1)) * RS + lane * NR);
        stv(xs, ZRR, xoff(pS1), 0);
        pS1 = ptab(++qS);
        xl = xn;
        xn = ldv_glc<VR>(ZRR, xoff(pL1), 0);
        pL1 = ptab(++qL);
      }
      // flags of the next chunk were read a chunk ago; read the one after
      cfl = cfl_next;
      cfl_next = CFL[min(ch + 2, nch)];
      chunk_cols();
      if (OUT) {
        // flush this chunk's outflow entries (at most 256)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int e = lane + 64 * m;
          const T v = my_outb[min(e, A.o_max - 1)];
          bst(v, OUR, e < out_cnt ? (out_tot + e) * (int)sizeof(T) : kOOB);
        }
        out_tot += out_cnt;
      }
      if constexpr (!PIPE) {
        // single-buffered staging: write the chunk (and its outflows) out
        // now, then wait for every reader before the next chunk stages again
        if constexpr (L3) emit(ch);
#pragma unroll
        for (int b = 0; b < PAIRS / MB; ++b) {
          wo_read(b, ch);
          wo_store(true);
        }
        lds_barrier();
      }
      __builtin_amdgcn_wave_barrier();
    };

    // runs of chunks of one kind, each in a loop of its own: the registers of
    // the prefetch ring stay in place within a run (a join of differently
    // compiled bodies would copy them, waiting for every load in flight);
    // most chunks have no boundary entries at all, and on a rectangle the rest
    // only have lanes entering their strip at the x wall (kind 3)
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using B0 = std::integral_constant<bool, false>;
    using B1 = std::integral_constant<bool, true>;
    auto kind = [](int fl) {
      return fl == 0 ? 0 : (fl == CF2_XST ? 3 : ((fl & CF2_INY_UP) ? 2 : 1));
    };
    // a run's entry copies the ring between the runs' registers; draining
    // there keeps those copies' loads out of the waits inside the run. Each
    // run's drain is a distinct instruction (vmcnt(0) with a different, unused
    // export count) so that none is merged into a common block the compiler
    // could route around.
    auto drain0 = []() { __builtin_amdgcn_s_waitcnt(0x0F70); };  // vmcnt(0) expcnt(7)
    auto drain1 = []() { __builtin_amdgcn_s_waitcnt(0x0F60); };  // vmcnt(0) expcnt(6)
    auto drain2 = []() { __builtin_amdgcn_s_waitcnt(0x0F50); };  // vmcnt(0) expcnt(5)
    auto drain3 = []() { __builtin_amdgcn_s_waitcnt(0x0F40); };  // vmcnt(0) expcnt(4)
    int ch = 0;
    while (ch < nch) {
      const int kd = kind(cfl);
      if (kd == 0) {
        drain0();
        do {
          chunk(I0(), B0(), B0(), ch);
          ++ch;
        } while (ch < nch && kind(cfl) == 0);
      } else if (kd == 3) {
        drain3();
        do {
          chunk(I0(), B0(), B1(), ch);
          ++ch;
        } while (ch < nch && kind(cfl) == 3);
      } else if (kd == 1) {
        drain1();
        do {
          chunk(I1(), B1(), B1(), ch);
          ++ch;
        } while (ch < nch && kind(cfl) == 1);
      } else {
        drain2();
        do {
          chunk(I2(), B1(), B1(), ch);
          ++ch;
        } while (ch < nch && kind(cfl) == 2);
      }
    }
    if constexpr (PIPE) {
      // the last chunk's write-out (its staging is complete: the chunk ended
      // with a barrier)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        wo_read(b, nch - 1);
        wo_store(nch > 0);
      }
      if (L3 && nch > 0) emit(nch - 1);
    }

    if (MODE == M2_TAUGRAD) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        tg0 += __shfl_xor(tg0, off);
        tg1 += __shfl_xor(tg1, off);
      }
      // the R slots share the group: add them in slot order
      GAS double* tgp = gp(I.tgrad + (size_t)g_loc * 2);
      for (int rr = 0; rr < R; ++rr) {
        if (r == rr && lane == 0) {
          tgp[0] += tg0;
          tgp[1] += tg1;
        }
        __syncthreads();
      }
    }
  }
  // the last workgroup out resets the queue counters for the next launch
  if (tid == 0) {
    const int e = atomicAdd(&A.counters[1], 1);
    if (e == (int)gridDim.x - 1) {
      atomicExch(&A.counters[0], 0);
      atomicExch(&A.counters[1], 0);
    }
  }
}

}  // namespace bte
