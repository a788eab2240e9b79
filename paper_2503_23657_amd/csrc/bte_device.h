// Structures shared by the host runtime and the HIP kernels of the sweep library.
//
// Terminology used throughout the sources:
//   octant    sign pattern of a direction along the grid axes (2^dim of them);
//             every ordinate of an octant sweeps the grid in the same upwind order.
//   group     G ordinates of one band and one octant, swept together by one wave
//             (one ordinate per register slot of every lane).
//   bundle    P groups of one octant swept in lockstep by the P waves of a
//             workgroup; their band/direction partial sums are added per cell
//             before they leave the workgroup.
//   job       (instance, bundle): the unit of work a workgroup takes from the
//             persistent queue.
//   kernel axes (i, j, k): i is swept inside a lane (x); lanes form an LJ x LK
//             block over (j, k) (2D/1D: LJ = 1, LK = 64 with k = y; 3D: LJ = 8,
//             LK = 8 with j = y, k = z). A strip is a row of LK cells in k. In
//             2D the R waves of a workgroup pipeline successive strips through an
//             LDS ring; in 3D one wave streams every strip, its J-blocks of LJ
//             cells in j and, inside a block, the cells in i ("virtual column"
//             v = J*W + i), the link between strips going through a global ring.
//   schedule  for each octant and each of the R wave slots, which cell lane l
//             processes at clock step t (the "skewed" layout): position
//             p = (slot*T + t)*64 + l. Every per-step input of the sweep is
//             stored in this layout, so a wave's loads for one step are one
//             contiguous 64-element read.
//   variables the sweep works in temperature units: u = 4 pi e~ / C_b (K), with
//             e~ the deviational energy, and in time units of t0. The swept
//             quantity is f = u / inv with inv = 1/(t0/tau_b + sum_d t0 v_b |s_d|/h_d);
//             f = S + sum_d a_d f_upwind,d, a_d = t0 v_b |s_d| / h_d * inv, and the
//             source S = kS * X + cQ * Q (X = Delta T forward, lambda adjoint).
#pragma once
#include <stdint.h>

namespace bte {

constexpr int kWave = 64;
constexpr int kMaxG = 8;
constexpr int kNAcc = 4;  // partial-sum planes: [0] temperature, [1..dim] heat flux (or [1] dJ/dQ)

// per-position flag bits of the schedule
constexpr uint32_t F_ACTIVE = 1u << 0;
constexpr uint32_t F_IN_X = 1u << 1;   // upwind face on axis x is a boundary: consume one inflow entry
constexpr uint32_t F_IN_Y = 1u << 2;
constexpr uint32_t F_IN_Z = 1u << 3;
constexpr uint32_t F_OUT_X = 1u << 4;  // downwind face on axis x is a diffuse or specular wall: emit one outflow entry
constexpr uint32_t F_OUT_Y = 1u << 5;
constexpr uint32_t F_OUT_Z = 1u << 6;
// bits 7..22 of the flags: i index of the position's cell in sweep orientation
constexpr int F_COL_SHIFT = 7;
constexpr uint32_t F_COL_MASK = 0xFFFFu;

// 1D/2D sweep (rows-per-lane layout): a lane owns NR consecutive rows of a
// strip of 64*NR rows; the per-(step, lane) record is int2 {cid0 << 5 | full
// << 4 | gm, flags} where cid0 is the cell of the lane's first row, bit k of gm
// says that row k lies inside the grid and full that all NR rows do (-1: no
// cell), and flags holds 5 bits per row k at bit 5k (active, inflow x/y,
// outflow x/y) and, at bit 20, the chunk-relative offset of the lane's first
// inflow entry.
constexpr int kC2 = 8;                 // steps per chunk
constexpr int kPad2 = 8;               // schedule padding steps (prefetch runs ahead)
constexpr uint32_t F2_ACT = 1u << 0;
constexpr uint32_t F2_INX = 1u << 1;
constexpr uint32_t F2_INY = 1u << 2;
constexpr uint32_t F2_OUTX = 1u << 3;
constexpr uint32_t F2_OUTY = 1u << 4;
constexpr int F2_ROW_BITS = 5;
constexpr int F2_INOFF_SHIFT = 20;
constexpr uint32_t F2_INOFF_MASK = 0xFFu;
// the lane enters its strip at the x wall in this step: its NR x-inflows are the
// stream entries from its offset on (rows ascending, -1 for a row without one)
// and replace the rows' x-upwind values; no other inflow in the lane-step
constexpr uint32_t F2_XSTART = 1u << 28;
// per-chunk flags of the 1D/2D schedule
constexpr int CF2_IN = 1;       // some inflow entry in the chunk
constexpr int CF2_INY_UP = 2;   // some y-inflow on a row k >= 1 of a lane
constexpr int CF2_OUT = 4;      // some outflow entry in the chunk
constexpr int CF2_XST = 8;      // some lane-step with F2_XSTART in the chunk

// 3D rows-per-lane sweep: the 1D/2D kernel with a third (plane) axis. Kernel
// axes: steps along grid axis ax[0], cut into blocks of kC2 columns, lanes (NR
// <= 2 rows each) along ax[1], planes along ax[2]; a lane streams block after
// block, in a block plane after plane, in a plane the block's columns. 8 flag
// bits per row (k at bit 8k): active, inflow along the step / lane / plane
// axis, outflow (reflecting wall) along them (the outflows themselves are
// listed per chunk in out_tab). The inflow offset sits at F2_INOFF_SHIFT as in
// 1D/2D.
constexpr uint32_t F3_ACT = 1u << 0;
constexpr uint32_t F3_INX = 1u << 1;
constexpr uint32_t F3_INY = 1u << 2;
constexpr uint32_t F3_INZ = 1u << 3;
constexpr uint32_t F3_OUTX = 1u << 4;
constexpr uint32_t F3_OUTY = 1u << 5;
constexpr uint32_t F3_OUTZ = 1u << 6;
constexpr int F3_ROW_BITS = 8;

// group coefficient record: GS(G) values of the sweep type, in this order
//   kS, cQ, a[3][G], den[G], wacc[kNAcc][G], wo[3][G], wt[2][G], inv[G]
__host__ __device__ constexpr int grp_stride(int G) { return 2 + G * (3 + 1 + kNAcc + 3 + 2 + 1); }
__host__ __device__ constexpr int go_a(int G, int d) { return 2 + d * G; }
__host__ __device__ constexpr int go_den(int G) { return 2 + 3 * G; }
__host__ __device__ constexpr int go_wacc(int G, int a) { return 2 + 4 * G + a * G; }
__host__ __device__ constexpr int go_wo(int G, int d) { return 2 + (4 + kNAcc) * G + d * G; }
__host__ __device__ constexpr int go_wt(int G, int t) { return 2 + (7 + kNAcc) * G + t * G; }
__host__ __device__ constexpr int go_inv(int G) { return 2 + (9 + kNAcc) * G; }

// Per-instance descriptor (device memory). Pointers are device pointers.
struct InstDev {
  int dim, nx, ny, nz;
  int ncell;        // bounding-box cells
  int n_bface;      // boundary faces
  int n_jobs;       // jobs of this instance
  int n_grp;        // groups of this instance
  int T;            // schedule clock steps (multiple of C)
  int n_oct;        // 2^dim
  int W;            // 2D: cells per strip row (nx); 3D: max pencil length
  int e_max;        // max inflow entries of one wave slot in one chunk (all axes)
  int o_max;        // max outflow entries of one wave slot in one chunk (all axes)
  int band_dummy;   // unused padding
  long long pos_per_oct;  // positions of one octant's layout: R*(T + kPad2)*64*nr (rows per lane),
                          //   R*(T + kPad2)*64 (3D pencil blocks)
  // schedule (per octant, R slots): cell index (-1 idle/inactive) and flags
  const int2* sched;        // [n_oct][R][T + kPad2][64] (cell, flags)
  const int* pos;           // [n_oct][ncell] position of cell c in octant o's layout (-1 inactive)
  // inflow stream: boundary-face slots in consumption order, per (octant, slot)
  const int* in_slot;       // concatenated
  const int* in_chunk;      // [n_oct][R][nchunks+1] start offset of each chunk (absolute into in_slot)
  const int* out_base;      // [n_oct][R] start offset of the outflow stream (absolute)
  const int* pre_slot;      // 2D: [n_oct][W] face slot of the strip-0 lane-0 upwind y face per column (-1)
  // state in the skewed layout: (X, Q) pairs per position, sweep precision, ping-pong
  void* xq[2];              // [n_oct][R*T*64] T2
  const void* xf;           // tau-gradient pass: forward (Delta T, Q) pairs per position
  const void* ubf;          // [B][n_bface] inflow u of every boundary face (K); zeros for the adjoint
  void* outv;               // [n_grp][n_out_entries_of_octant] outflow stream values
  void* part;               // [kNAcc] planes of partial sums (sweep precision), each in groups of
                            //   2^part_jg jobs, cell-block major inside a group:
                            //   [n_jobs / 2^part_jg][part_ld / kPartBlk][2^part_jg][kPartBlk]
  int part_ld;              // cells per job in a plane: ncell rounded up to a multiple of kPartBlk
  int part_jg;              // log2 of the jobs per group (a group's part of a plane < 2 GiB)
  void* store_u;            // [n_grp][ncell][G] angular field u (forward, when stored for the
                            //   adjoint); second-order faces: [n_grp][pos_per_oct] in the octant's
                            //   skewed layout
  double* tgrad;            // [n_grp][2] tau-gradient partial sums
  int* status;              // StatusDev
  int lag;                  // 3D: clock lag between a z-front write and its read
  int ring;                 // 3D: global z-ring length in steps (power of two)
  int n_out_stride;         // stride of one group's row of outv
  // 1D/2D rows-per-lane schedule
  int nr;                   // rows per lane
  int du;                   // clock distance between the starts of consecutive strips
  int n_strip;              // strips of 64*nr rows
  int in_E;                 // entries per chunk row of in_tab (multiple of 64, <= 256)
  const int* in_tab;        // [n_oct][R][T/kC2 + 2][in_E] inflow face slot of each stream entry (-1 pad)
  const int* chunk_fl;      // [n_oct][R][T/kC2 + 1] CF2_* flags of each chunk (0 pad)
  // second-order faces (rows-per-lane layouts, one ordinate per group): the
  // deferred correction of each group's source, in its octant's skewed layout
  void* corr;               // [n_grp][pos_per_oct] sweep precision
  // 3D rows-per-lane layout
  int ax[3];                // grid axis of the step, lane and plane axes
  int dyo[8];               // cell-index step from row k to row k + 1, per octant
  int n_pl;                 // planes
  int n_per;                // plane periods of kC2 steps (the most of any octant)
  const int* xpre;          // [n_oct][n_pl][64*nr] step-axis wall face of the first column's cells (-1)
  const int* gpre;          // [n_oct][T + n_per] lane-axis wall face + 1 of lane 0's row 0 at each step
                            //   (0: none), then the plane + 1 of each plane period (0: none)
  const int* out_tab;       // [n_oct][T/kC2 + 2][out_E] outflow entries of each chunk, read from the staging
                            //   ((((u*64 + l)*nr + k) << 2 | kernel axis) + 1, 0 pad)
  const int* out_chunk;     // [n_oct][T/kC2 + 1] stream offset of each chunk's first outflow entry
  int out_E;                // entries per chunk row of out_tab (multiple of 64, <= 256)
};

// Job: instance, first group of the bundle (global index), instance-local job
// index (row of the partial-sum buffer) and octant.
struct JobDev {
  int inst;
  int grp;
  int jl;
  int oct;
};

// Per-instance status (device).
struct StatusDev {
  int iter;         // completed iterations
  int done;         // 1: converged or stopped; kernels skip the instance
  int nonfinite;    // 1: a non-finite value appeared
  int ticket;       // block ticket for the finalize reduction
  int checked;      // iteration index of the last residual check
  int pad[3];
  double eps_T, eps_q;
  double lam_dT;    // sum_c lambda_c * DeltaT_c (adjoint)
  double red[4];    // scratch
};

struct SweepArgs {
  const InstDev* inst;
  const JobDev* jobs;
  int n_jobs;
  int* counters;        // [2]: job ticket, exit ticket (self-resetting)
  const int4* grp_i;    // [n_grp_total] (band, octant, instance-local group, inflow-table row)
  const void* grp_t;    // [n_grp_total][grp_stride(G)]
  int B;
  int R, P, C;
  int lds_zring;        // byte offsets into dynamic LDS
  int lds_yring;
  int lds_xb;
  int lds_stage;
  int lds_cid;
  int lds_in;
  int lds_out;
  int lds_total;
  int zring_len;        // entries per slot of the z-ring (2D: W_max columns; 3D: ring length)
  int W_max;
  int e_max, o_max;
  int force;            // 1: sweep even instances marked done (timing / store passes)
  void* zg;             // 3D: pencil layout: global z-rings; rows layout: step-axis buffers
                        //     of the planes; one per (workgroup, wave p)
  long long zg_stride;  // elements per (workgroup, wave p)
};


// ---------------------------------------------------------------- aux kernels
enum { FIN_Q = 1, FIN_CHECK = 2, FIN_ADJ = 4, FIN_QPREV = 8 };
constexpr int kFinCells = 256;    // cells per finalize block
constexpr int kFinThreads = 512;  // threads per finalize block: cell groups x job slices
constexpr int kPartBlk = 256;     // cells per block of the partial-sum planes (= kFinCells)
static_assert(kPartBlk == kFinCells, "a finalize block reads one cell block of every job");

// offset (elements) of cell c from a job's first element in a partial-sum
// plane with 2^jg jobs per group (a negative c gives a negative offset, which
// buffer views drop), and of a job's first element from the plane's start
__host__ __device__ constexpr int part_off(int c, int jg) {
  return ((c >> 8) << (jg + 8)) + (c & (kPartBlk - 1));
}
// the same as c + (c / kPartBlk) * part_gap(jg), one multiply-add
__host__ __device__ constexpr int part_gap(int jg) { return ((1 << jg) - 1) * kPartBlk; }
__host__ __device__ constexpr long long part_job(int j, int jg, int part_ld) {
  return ((long long)(j >> jg) * part_ld << jg) + (long long)(j & ((1 << jg) - 1)) * kPartBlk;
}
// elements of one partial-sum plane (whole groups)
__host__ __device__ constexpr long long part_plane_len(int n_jobs, int jg, int part_ld) {
  return ((long long)((n_jobs + (1 << jg) - 1) >> jg) << jg) * part_ld;
}

struct FinArgs {
  const InstDev* inst;
  const int2* blocks;        // [n_blocks_total] (instance, block index within the instance)
  int n_blocks_total;
  const int* n_blocks_inst;  // [n_inst]
  int flags;                 // FIN_*
  double tol_T, tol_q;
};

// Per-instance finalize pointers (device memory).
struct FinInst {
  double* X[2];              // master state (Delta T or lambda), [ncell], ping-pong
  const double* g;           // adjoint right-hand side dJ/dT [ncell] (FIN_ADJ)
  double* q;                 // [ncell*dim] heat flux output (forward) or dJ/dQ [ncell] (adjoint)
  double* qmag_prev;         // [ncell] |q| of the previous flux iteration
  double* blockpart;         // [n_blocks_inst][4]
  const unsigned char* active;  // [ncell]
};

struct WallArgs {
  const InstDev* inst;
  int inst_id;
  int n_dface;
  const int* dface_slot;     // [n_dface] boundary-face slot of each diffuse face
  const double* inv_half;    // [n_dface] 1 / sum_{in} w |s.n|
  const int* ofk;            // [n_oct][n_bface] index of the face in octant o's out-stream, or -1
  const int2* grp_ob;        // [n_oct][B] (first instance-local group, count)
  int B;
  int rows;                  // inflow-table rows per band (1, or the ordinate count with specular walls)
  const int* dface_axis;     // [n_dface] grid axis of each diffuse face
  int oct_xor;               // 0: forward; n_oct - 1: transposed sweeps (groups sweep the flipped octant)
  const double* scale;       // [B][3] factor per band and face axis (transposed sweeps), or NULL
  const int* ent_df;         // [n_oct][n_out] diffuse face of each out-stream entry, or -1
  double* wsum;              // [n_oct][B][n_dface] per-octant sums
  int n_out;                 // out-stream entries per octant (the stride of outv's rows)
};

// Lagged specular-wall values (Eq. 7): the inflow of ordinate a at a specular
// face is the outgoing value of its mirror ordinate a' at the same cell, read
// from the sweep's out-stream (w_a' |s_a'.n| u for one ordinate per group).
// The transposed sweeps use the same kernel with the roles of incoming and
// outgoing ordinates exchanged (the src table of the other side).
struct SpecArgs {
  const InstDev* inst;
  int inst_id;
  int n_sface;
  const int* sface_slot;     // [n_sface] boundary-face slot of each specular face
  const int* sface_dir;      // [n_sface] face direction 0..5 (-x, +x, -y, +y, -z, +z)
  const int2* src;           // [6][M] (octant, member index) of the mirror of a, or (-1, -1) when a
                             //        does not enter through that face direction
  const double* inv_wq;      // [6][M] 1 / (w_a' |s_a'.n|)
  const int* ofk;            // [n_oct][n_bface] index of the face in octant o's out-stream, or -1
  const int2* grp_ob;        // [n_oct][B] (first instance-local group, count)
  int B, M;
  int oct_xor;               // 0: forward; n_oct - 1: transposed sweeps
  const double* scale;       // [B][3] factor per band and face axis (transposed sweeps), or NULL
};

// Deferred correction of the second-order faces (Methods, "Spatial
// discretization"; Eq. rhs_b): for every group (one ordinate) and active cell,
// from the stored angular field u of the last sweep,
//   corr = sum_d coef_d (grad_d u(c) - grad_d u(up_d(c))),
// grad by Green-Gauss (face value: the mean of two cells, the wall value at an
// isothermal face the ordinate enters through, else the linear extrapolation
// from the cell and its neighbour across the opposite face); the upwind cell's
// term is absent when the upwind side is a wall. Written to the group's
// skewed layout, in the sweep's variable.
struct CorrArgs {
  const InstDev* inst;
  int inst_id;
  int n_grp;                 // groups of the instance
  const int4* grp;           // [n_grp] (band, octant, local group, inflow-table row)
  const double* coef;        // [n_grp][3] -t0 w0 v_b s_d / 2 per grid axis (0: padding group)
  const int* stencil;        // [n_oct][pos_per_oct][3*dim] neighbour positions or boundary codes
                             //   (downwind, upwind, upwind's upwind per axis; -1 boundary,
                             //   -(2 + slot) isothermal inflow wall, kNoCell first: no cell)
  double h[3];
  const double* X0;          // [ncell] equilibrium field of every ordinate, filled in first (before the
                             //   first sweep), or NULL: the field the last sweep stored
};
constexpr int kNoCell = (int)0x80000000;  // stencil code of a position of no cell

struct InitArgs {
  const InstDev* inst;
  int inst_id;
  const double* X0;          // [ncell] initial absolute temperature (forward) / dJ/dT (adjoint) / NULL
  double T_ref;
  const double* Q;           // [ncell] source (forward) or NULL
  const unsigned char* active;
  double* X[2];
  int adjoint;
};

struct UbfInitArgs {
  void* ubf;                 // [B][rows][n_bface]
  int n_bface, B;            // B: bands x rows
  const int* bf_bc;          // [n_bface]
  const int* bf_cell;        // [n_bface]
  const int* bc_kind;        // [n_bc]
  const double* bc_T;        // [n_bc]
  const double* T_init;      // [ncell] or NULL
  double T_ref;
  int zero;                  // 1: all zeros (adjoint)
};

}  // namespace bte
