// Transport sweep kernel for gfx950 (MI355X).
//
// One launch performs one source-iteration sweep (paper Methods, "Iterative
// matrix formulation and solution scheme", step 2): for every (band,
// direction) pair the first-order upwind system A e = b (Eqs. Axb, A_matrix with
// first-order faces) is solved exactly by one pass in upwind order, and in the
// same pass the band/direction sums of Eq. updatee0_t (new lattice temperature)
// and Eq. 4 (heat flux) are accumulated, plus the outgoing values at the
// reflecting walls (diffuse, Eq. 6, and specular, Eq. 7).
//
// Work decomposition, 3D problems (1D/2D ones have their own rows-per-lane
// kernel; see bte_device.h for the terms):
//   * the 64 lanes of a wave own an 8 x 8 block of the (j, k) cross-section and
//     sweep it along i, skewed by j + k; a lane's G register slots hold G
//     ordinates of one band and one octant;
//   * the upwind neighbour in i is the lane's own previous value; the one in j
//     is lane - 1 of its 8-lane group, moved with DPP row_shr:1; the one in k is
//     lane - 8, through a per-wave LDS exchange block;
//   * one wave streams all pencil blocks; the j-link between blocks goes
//     through an LDS ring, the k-link between strips through a global ring whose
//     values are prefetched D steps ahead;
//   * every per-step input comes from the precomputed skewed schedule, so each
//     wave reads 64 contiguous entries per step, prefetched D steps ahead;
//   * boundary inflows are consumed as an ordered stream per wave, staged into
//     LDS one chunk ahead, so no lane waits on a dependent load; no step has a
//     lane-divergent branch (unowned entries are read in range and discarded,
//     unowned writes go to dummy entries or past the buffer view);
//   * per-cell partial sums of the P waves of a workgroup are staged in LDS,
//     added, and written back as contiguous row segments.
#include <hip/hip_runtime.h>

#include "bte_device.h"
#include "bte_kutil.h"

namespace bte {

template <typename T>
struct V2;
template <>
struct V2<float> {
  using t = float2;
};
template <>
struct V2<double> {
  using t = double2;
};

// DPP controls (GFX9 encoding): wave_shr:1 = 0x138, row_shr:1 = 0x111.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ unsigned long long ballot64(bool p) { return __ballot(p); }

// HIP's vector types cannot bind address-space references: load pairs through
// clang vector types
typedef int iv2_t __attribute__((ext_vector_type(2)));
typedef float fv2_t __attribute__((ext_vector_type(2)));
typedef double dv2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int2 ld2(const GAS int2* p) {
  const iv2_t v = *(const GAS iv2_t*)p;
  return make_int2(v.x, v.y);
}
__device__ __forceinline__ float2 ld2(const GAS float2* p) {
  const fv2_t v = *(const GAS fv2_t*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld2(const GAS double2* p) {
  const dv2_t v = *(const GAS dv2_t*)p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

enum { M_PLAIN = 0, M_STORE = 1, M_TAUGRAD = 2 };

constexpr int kD = 8;    // prefetch distance (steps) of the per-step inputs
static_assert(kD <= kPad2, "the schedule padding must cover the prefetch distance");
constexpr int kEPL = 4;  // in-stream entries per lane per chunk (e_max <= 256)

// ============================================================================
// 3D layout (LJ = 8, LK = 8, j = y, k = z), R = 1; 1D/2D problems have a
// kernel of their own (bte_sweep2d.hip). L3 is always true.
// ============================================================================
template <typename T, int G, int NACC, int MODE, bool L3>
__global__ void __launch_bounds__(512) sweep_kernel(SweepArgs A) {
  static_assert(L3, "the pencil-block kernel sweeps 3D problems only");
  using T2 = typename V2<T>::t;
  constexpr int LJ = 8;
  constexpr int LK = 8;
  constexpr int GS = grp_stride(G);
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_job;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = A.R, P = A.P, C = A.C;
  const int r = wave % R;
  const int p = wave / R;
  const int jl = lane & 7;
  const int kl = lane >> 3;

  // LDS carve-up (byte offsets computed on the host)
  T* yring = reinterpret_cast<T*>(lds + A.lds_yring);  // 3D: [P][LK * W_max + 64][G] (64 dummy entries)
  T* xb = reinterpret_cast<T*>(lds + A.lds_xb);        // 3D: [P][72][G] (entries 8.. hold lane - 8's value)
  T* stage = reinterpret_cast<T*>(lds + A.lds_stage);  // [P*R][NACC][C][65]
  int* scid = reinterpret_cast<int*>(lds + A.lds_cid); // [R][C][65]
  T* inb = reinterpret_cast<T*>(lds + A.lds_in);       // [P*R][2][e_max]
  T* outb = reinterpret_cast<T*>(lds + A.lds_out);     // [P*R][o_max + 64] (64 dummy entries)
  const int W_max = A.W_max;
  T* my_yring = yring + (size_t)p * (LK * W_max + 64) * G;
  T* my_xb = xb + (size_t)p * 72 * G;
  T* my_stage = stage + (size_t)(p * R + r) * NACC * C * 65;
  int* my_scid = scid + (size_t)r * C * 65;
  T* my_inb = inb + (size_t)(p * R + r) * 2 * A.e_max;
  T* my_outb = outb + (size_t)(p * R + r) * (A.o_max + 64);
  GAS T* my_zg = gp(reinterpret_cast<T*>(A.zg) + ((size_t)blockIdx.x * P + p) * A.zg_stride);

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
    const T kS = gt[0], cQ = gt[1];
    T a0[G], a1[G], a2[G], den[G], inv[G];
    T wacc[NACC][G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      a0[g] = gt[go_a(G, 0) + g];
      a1[g] = gt[go_a(G, 1) + g];
      a2[g] = gt[go_a(G, 2) + g];
      den[g] = gt[go_den(G) + g];
      inv[g] = gt[go_inv(G) + g];
#pragma unroll
      for (int a = 0; a < NACC; ++a) wacc[a][g] = gt[go_wacc(G, a) + g];
    }

    const int o = jd.oct;
    const int T_steps = I.T;
    const int nch = T_steps / C;
    // per-slot schedule rows are padded (pos_per_oct = R * (T + kPad2) * 64),
    // so the prefetch of step tau + kD needs no condition
    const long long Tp = I.pos_per_oct / ((long long)R * 64);
    const long long slot_base = (long long)o * I.pos_per_oct + (long long)r * Tp * 64;
    const GAS int2* SCH = gp(I.sched + slot_base);
    const GAS T2* XQ = gp(reinterpret_cast<const T2*>(I.xq[iter & 1]) + slot_base);
    const GAS T2* XF = MODE == M_TAUGRAD ? gp(reinterpret_cast<const T2*>(I.xf) + slot_base) : nullptr;
    const GAS T* UBF = gp(reinterpret_cast<const T*>(I.ubf) + (size_t)ubf_row * I.n_bface);
    const GAS int* ISLOT = gp(I.in_slot);
    const CAS int* ich = cp(I.in_chunk) + (size_t)(o * R + r) * (nch + 1);
    // buffer views of the chunk loop's global data (sizes in bytes): masked
    // lanes get an offset past the end instead of a branch
    const rsrc_t UBR = mkrsrc(UBF, (unsigned)I.n_bface * (unsigned)sizeof(T));
    const rsrc_t ISR = mkrsrc(ISLOT, (unsigned)ich[nch] * 4u);
    GAS T* OUTV = gp(reinterpret_cast<T*>(I.outv) + (size_t)g_loc * I.n_out_stride + cp(I.out_base)[o * R + r]);
    const size_t part_plane = (size_t)part_plane_len(I.n_jobs, I.part_jg, I.part_ld);
    // (a view spans the job's group; a cell outside the grid lands past its
    // end or in the job's own padding)
    GAS T* PARTJ = gp(reinterpret_cast<T*>(I.part) + part_job(jd.jl, I.part_jg, I.part_ld));
    const unsigned pgrp = (unsigned)(((size_t)I.part_ld << I.part_jg) - (size_t)(jd.jl & ((1 << I.part_jg) - 1)) * kPartBlk);
    rsrc_t PRS[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) PRS[a] = mkrsrc(PARTJ + a * part_plane, pgrp * (unsigned)sizeof(T));
    const int pgap = part_gap(I.part_jg);  // cell c at c + (c >> 8) * pgap (part_off)
    const int zmask = I.ring - 1;
    const int zlag = I.lag;
    // buffer view of this wave's global z ring (I.ring steps x 8 lanes x G)
    const rsrc_t ZGR = mkrsrc(my_zg, (unsigned)(I.ring * LJ * G) * (unsigned)sizeof(T));

    // ---- clear the exchange buffers
    for (int e = lane; e < LK * W_max * G; e += 64) my_yring[e] = T(0);
    for (int e = lane; e < 72 * G; e += 64) my_xb[e] = T(0);
    __syncthreads();

    // ---- inflow stream pipeline: slots of chunk k+1 wait in registers, the
    //      values of chunk k sit in LDS buffer (k & 1)
    int slot_n[kEPL];
    {
      const int b0 = ich[0], e0 = ich[1];
#pragma unroll
      for (int m = 0; m < kEPL; ++m) {
        const int idx = b0 + lane + 64 * m;
        const T v = idx < e0 ? UBF[ISLOT[idx]] : T(0);
        if (lane + 64 * m < A.e_max) my_inb[lane + 64 * m] = v;
      }
      const int b1 = nch > 1 ? ich[1] : 0, e1 = nch > 1 ? ich[2] : 0;
#pragma unroll
      for (int m = 0; m < kEPL; ++m) {
        const int idx = b1 + lane + 64 * m;
        slot_n[m] = idx < e1 ? ISLOT[idx] : -1;
      }
    }
    __syncthreads();

    // ---- per-lane state
    T f[G];
#pragma unroll
    for (int g = 0; g < G; ++g) f[g] = T(0);
    int out_cur = 0;
    double tg0 = 0.0, tg1 = 0.0;

    // prefetch ring of the per-step inputs
    int2 rcf[kD];
    T2 rxq[kD];
    T2 rxf[kD];
    T rzg[kD][G];
#pragma unroll
    for (int u = 0; u < kD; ++u) {
      rcf[u] = ld2(SCH + u * 64 + lane);
      rxq[u] = ld2(XQ + u * 64 + lane);
      if (MODE == M_TAUGRAD) rxf[u] = ld2(XF + u * 64 + lane);
#pragma unroll
      for (int g = 0; g < G; ++g) rzg[u][g] = T(0);
      if (kl == 0 && u >= zlag) {
#pragma unroll
        for (int g = 0; g < G; ++g) rzg[u][g] = my_zg[(size_t)(((u - zlag) & zmask) * LJ + jl) * G + g];
      }
    }

    for (int ch = 0; ch < nch; ++ch) {
      // gather the next chunk's inflow values now; they are written to LDS at
      // the end of the chunk
      T inval[kEPL];
#pragma unroll
      for (int m = 0; m < kEPL; ++m) inval[m] = bld<T>(UBR, slot_n[m] * (int)sizeof(T));  // slot -1: 0
      {
        const bool more = ch + 2 < nch;
        const int b2 = more ? ich[min(ch + 2, nch)] : 0;
        const int e2 = more ? ich[min(ch + 3, nch)] : 0;
#pragma unroll
        for (int m = 0; m < kEPL; ++m) {
          const int idx = b2 + lane + 64 * m;
          const int sv = bld<int>(ISR, idx < e2 ? idx * 4 : kOOB);
          slot_n[m] = idx < e2 ? sv : -1;
        }
      }
      const T* inbuf = my_inb + (ch & 1) * A.e_max;
      int in_cur = 0;
      const int out_chunk0 = out_cur;

      for (int cc0 = 0; cc0 < C; cc0 += kD) {
#pragma unroll
        for (int u = 0; u < kD; ++u) {
          const int cc = cc0 + u;
          const int tau = ch * C + cc;
          const int2 cf = rcf[u];
          const T2 xq = rxq[u];
          T2 xf;
          if (MODE == M_TAUGRAD) xf = rxf[u];
          T zg[G];
#pragma unroll
          for (int g = 0; g < G; ++g) zg[g] = rzg[u][g];
          {
            const int tn = tau + kD;
            rcf[u] = ld2(SCH + tn * 64 + lane);
            rxq[u] = ld2(XQ + tn * 64 + lane);
            if (MODE == M_TAUGRAD) rxf[u] = ld2(XF + tn * 64 + lane);
            // every lane loads (the ring index wraps in bounds); the z-entry
            // lanes keep the value once the ring holds data
            const bool zk = kl == 0 && tn >= zlag;
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const T zv = my_zg[(size_t)(((tn - zlag) & zmask) * LJ + jl) * G + g];
              rzg[u][g] = zk ? zv : T(0);
            }
          }
          const int cid = cf.x;
          const unsigned fl = (unsigned)cf.y;
          const int col = (int)((fl >> F_COL_SHIFT) & F_COL_MASK);
          const T S = kS * xq.x + cQ * xq.y;

          // lanes exchange values through LDS: keep this step's reads after the
          // previous step's writes (the compiler cannot see the cross-lane use)
          __builtin_amdgcn_wave_barrier();

          // ---- upwind values
          T xu[G], yu[G], zu[G];
#pragma unroll
          for (int g = 0; g < G; ++g) xu[g] = f[g];
          {
            // j-neighbour (y): lane - 1 inside each 8-lane group; jl == 0 takes
            // the previous J-block's value from the y-ring. The other lanes read
            // their own dummy entry instead: the columns of a step repeat along
            // the block's anti-diagonals, so their ring reads would fall on few
            // LDS banks
            const int yr = jl == 0 ? kl * W_max + col : LK * W_max + lane;
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const T gv = my_yring[yr * G + g];
              const T d = dpp_move<0x111>(T(0), f[g]);
              yu[g] = jl == 0 ? gv : d;
            }
            // k-neighbour (z): lane - 8 through the exchange block; the entry
            // row (kl == 0) takes the previous strip's value from its own
            // prefetched ring register
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const T xv = my_xb[lane * G + g];
              zu[g] = kl == 0 ? zg[g] : xv;
            }
          }

          // ---- boundary inflows from the stream
          if (ballot64(fl & (F_IN_X | F_IN_Y | F_IN_Z)) != 0ull) {
            const bool bx = fl & F_IN_X, by = fl & F_IN_Y, bz = fl & F_IN_Z;
            const unsigned long long mx = ballot64(bx), my = ballot64(by), mz = ballot64(bz);
            // a lane's entries are consecutive (x, y, z); every lane reads three
            // in-range entries and keeps those it owns
            const int kx = in_cur + lanes_below(mx) + lanes_below(my) + lanes_below(mz);
            const int ky = kx + (bx ? 1 : 0), kz = ky + (by ? 1 : 0);
            const int kmax = A.e_max - 1;
            const T ux = inbuf[min(kx, kmax)], uy = inbuf[min(ky, kmax)], uz = inbuf[min(kz, kmax)];
#pragma unroll
            for (int g = 0; g < G; ++g) {
              xu[g] = bx ? ux * den[g] : xu[g];
              yu[g] = by ? uy * den[g] : yu[g];
              zu[g] = bz ? uz * den[g] : zu[g];
            }
            in_cur += __popcll(mx) + __popcll(my) + __popcll(mz);
          }

          // ---- the transport update and the fused band/direction sums
          T acc[NACC];
#pragma unroll
          for (int a = 0; a < NACC; ++a) acc[a] = T(0);
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const T fn = fma(a2[g], zu[g], fma(a1[g], yu[g], fma(a0[g], xu[g], S)));
            f[g] = fn;
#pragma unroll
            for (int a = 0; a < NACC; ++a) acc[a] = fma(wacc[a][g], fn, acc[a]);
          }

          // ---- exchange writes for the downstream neighbours
          __builtin_amdgcn_wave_barrier();
          {
#pragma unroll
            for (int g = 0; g < G; ++g) my_xb[(lane + 8) * G + g] = f[g];
            {
              // the last lane of each 8-lane group publishes its value to the
              // y-ring; the others write a dummy entry of their own
              const int ye = (jl == LJ - 1 && cid >= 0) ? kl * W_max + col : LK * W_max + lane;
#pragma unroll
              for (int g = 0; g < G; ++g) my_yring[ye * G + g] = f[g];
            }
            {
              // the top row of the block publishes to the global z ring; the
              // other lanes' stores fall outside the buffer view
              const int zo = kl == LK - 1 ? (((tau & zmask) * LJ + jl) * G) * (int)sizeof(T) : (int)kOOB;
#pragma unroll
              for (int g = 0; g < G; ++g) bst(f[g], ZGR, kl == LK - 1 ? zo + g * (int)sizeof(T) : (int)kOOB);
            }
          }

          // ---- reflecting-wall outflow stream
          if (ballot64(fl & (F_OUT_X | F_OUT_Y | F_OUT_Z)) != 0ull) {
            const bool ox = fl & F_OUT_X, oy = fl & F_OUT_Y, oz = fl & F_OUT_Z;
            const unsigned long long mx = ballot64(ox), my = ballot64(oy), mz = ballot64(oz);
            const int kx = out_cur - out_chunk0 + lanes_below(mx) + lanes_below(my) + lanes_below(mz);
            const int ky = kx + (ox ? 1 : 0), kz = ky + (oy ? 1 : 0);
            const CAS T* wo = gt + go_wo(G, 0);
            T vx = T(0), vy = T(0), vz = T(0);
#pragma unroll
            for (int g = 0; g < G; ++g) {
              vx = fma(wo[g], f[g], vx);
              vy = fma(wo[G + g], f[g], vy);
              vz = fma(wo[2 * G + g], f[g], vz);
            }
            // entries a lane does not own go to its dummy slot
            const int dmy = A.o_max + lane;
            my_outb[ox ? kx : dmy] = vx;
            my_outb[oy ? ky : dmy] = vy;
            my_outb[oz ? kz : dmy] = vz;
            out_cur += __popcll(mx) + __popcll(my) + __popcll(mz);
          }

          // ---- stored angular field / tau-gradient sums
          if (MODE == M_STORE && cid >= 0 && (fl & F_ACTIVE)) {
            GAS T* su = gp(reinterpret_cast<T*>(I.store_u) + ((size_t)g_loc * I.ncell + cid) * G);
#pragma unroll
            for (int g = 0; g < G; ++g) su[g] = f[g] * inv[g];
          }
          if (MODE == M_TAUGRAD && cid >= 0 && (fl & F_ACTIVE)) {
            const GAS T* su = gp(reinterpret_cast<const T*>(I.store_u) + ((size_t)g_loc * I.ncell + cid) * G);
            const CAS T* wt0 = gt + go_wt(G, 0);
            const CAS T* wt1 = gt + go_wt(G, 1);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const double uf = (double)su[g];
              s0 += (double)wt0[g] * (double)f[g] * (uf - (double)xf.x);
              s1 += (double)wt1[g] * uf;
            }
            tg0 += s0;
            tg1 += (double)xq.x * s1;
          }

          // ---- stage the partial sums of this step
#pragma unroll
          for (int a = 0; a < NACC; ++a) my_stage[(a * C + cc) * 65 + lane] = acc[a];
          if (p == 0) my_scid[cc * 65 + lane] = (fl & F_ACTIVE) ? cid : -1;
        }
      }

      // ---- end of chunk: publish ring values, then write the partial sums
      __syncthreads();
      {
        // the P waves of slot r add their partials; P*64 threads share C*64 entries
        const int t = p * 64 + lane;
        const int per = C / P;
        for (int m = 0; m < per; ++m) {
          const int e = m * (P * 64) + t;
          const int lp = e / C, cc = e - lp * C;
          const int cid = my_scid[cc * 65 + lp];
#pragma unroll
          for (int a = 0; a < NACC; ++a) {
            T v = T(0);
            for (int q = 0; q < P; ++q) v += stage[((size_t)(q * R + r) * NACC * C + a * C + cc) * 65 + lp];
            bst(v, PRS[a], cid >= 0 ? (cid + __mul24(cid >> 8, pgap)) * (int)sizeof(T) : kOOB);
          }
        }
      }
      // flush this chunk's outflow entries
      for (int e = lane; e < out_cur - out_chunk0; e += 64) OUTV[out_chunk0 + e] = my_outb[e];
      // the gathered inflow values of the next chunk
#pragma unroll
      for (int m = 0; m < kEPL; ++m)
        if (lane + 64 * m < A.e_max) my_inb[((ch + 1) & 1) * A.e_max + lane + 64 * m] = inval[m];
      __syncthreads();
    }

    if (MODE == M_TAUGRAD) {
      // wave reduction of the tau-gradient sums of this group
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        tg0 += __shfl_xor(tg0, off);
        tg1 += __shfl_xor(tg1, off);
      }
      // the R waves of a slot column share the group: add them in slot order
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
