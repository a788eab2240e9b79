// Host-side problem set-up shared by the C ABI implementation: validation,
// ordinate folding, ordinate groups and their coefficients, boundary-face
// tables and the sweep schedule. Plain C++ (no HIP calls).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bte.h"
#include "bte_device.h"

namespace bte {

struct Ordinate {
  double s[3];  // direction
  double w;     // weight (sum of the folded members)
  int oct;      // bit d set: negative direction along grid axis d
};

struct Plan {
  int G = 4, R = 4, P = 1, C = 16;
  int NR = 1;  // 1D/2D: rows per lane (1, 2 or 4)
};

// One problem instance on the host.
struct HostInst {
  int dim = 0;
  int n[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int ncell = 0, n_active = 0;
  std::vector<uint8_t> active;       // [ncell]
  // boundary faces: active cells ascending, faces ascending
  std::vector<int> bf_cell, bf_face, bf_bc;
  std::vector<int> bslot;            // [ncell*6] -> boundary-face slot or -1
  std::vector<int> bc_kind;          // copy of the bc table
  std::vector<double> bc_T;
  std::vector<int> dface;            // slots of diffuse faces
  std::vector<int> sface;            // slots of specular faces
  bool has_iso = false;
};

// Ordinate groups of an instance (same for every instance of a batch, but the
// coefficients depend on the cell size).
struct GroupSet {
  int G = 0, P = 0;
  std::vector<int> band;             // [n_grp]
  std::vector<int> oct;              // [n_grp]
  std::vector<int> ords;             // [n_grp*G] ordinate index or -1 (dummy slot)
  std::vector<int> bundle_first;     // [n_bundle] first group of each bundle
  std::vector<int> bundle_oct;       // [n_bundle]
  std::vector<int> ob_first, ob_count;  // [n_oct*B] groups of (octant, band): contiguous run
};

// Schedule of an instance for one plan (see bte_device.h).
//   3D: sched[n_oct][R][T][64] (cell, flags F_*), positions (slot*T + t)*64 + l;
//   1D/2D: sched[n_oct][R][T + kPad2][64] (cid0, flags F2_*), positions
//          ((slot*(T + kPad2) + t)*64 + l)*NR + k, and the per-chunk inflow table.
struct Schedule {
  int T = 0, n_oct = 0, R = 1, C = 16, W = 0, lag = 0, ring = 0;
  int NR = 1, du = 0, nS = 0;
  int e_max = 0, o_max = 0;
  long long pos_per_oct = 0;
  std::vector<int2> sched;           // [n_oct][R][T][64] (cell, flags)
  std::vector<int> pos;              // [n_oct][ncell]
  std::vector<int> in_slot;          // concatenated inflow slots
  std::vector<int> in_chunk;         // [n_oct][R][nch+1] absolute offsets
  std::vector<int> out_base;         // [n_oct][R]
  std::vector<int> ofk;              // [n_oct][n_bface]
  std::vector<int> pre_slot;         // 2D: [n_oct][W]
  std::vector<int> in_tab;           // 1D/2D: [n_oct][R][T/C + 2][in_E]
  std::vector<int> chunk_fl;         // 1D/2D: [n_oct][R][T/C + 1] CF2_* flags
  int in_E = 64;
  int n_out_stride = 1;              // max out-stream length over octants
  // 3D rows-per-lane layout (the 1D/2D kernel with a plane axis): the step
  // axis is cut into blocks of kC2 columns; a lane streams block by block, in
  // each block plane by plane, in each plane the block's columns
  bool l3r = false;
  int ax[3] = {0, 1, 2};             // grid axis of the kernel's step, lane and plane axes
  int n_pl = 0;                      // planes (cells along the plane axis)
  int n_per = 0;                     // plane periods of kC2 steps (the most of any octant)
  std::vector<int> xpre;             // [n_oct][n_pl][64*NR] step-axis wall face of the first column's cells (-1)
  std::vector<int> gpre;             // [n_oct][T + n_per] lane-axis wall face + 1 of lane 0's row 0 at each
                                     // step (0: none), then the plane + 1 of each plane period
  // reflecting-wall outflows, emitted per chunk from the staged values: entry
  // (((u*64 + l)*NR + k) << 2 | axis) + 1 of each outflow of chunk step u,
  // lane l, row k, in stream order (0 pad), and the stream offset of each chunk
  int out_E = 64;
  std::vector<int> out_tab;          // [n_oct][T/C + 2][out_E]
  std::vector<int> out_chunk;        // [n_oct][T/C + 1]
};

// Validation of the public structures; returns "" when valid.
std::string validate_problem(const bte_geometry* g, const bte_bands* b, const bte_quadrature* q);

// Build the host instance from a validated geometry.
void build_instance(const bte_geometry* g, HostInst& out);

// Fold ordinates with identical projections on the grid axes (2D: +-z mirror
// pairs), summing their weights.
std::vector<Ordinate> fold_ordinates(const bte_quadrature* q, int dim);

// Groups of G ordinates of one band and one octant, bundles of P groups of one
// octant (padded with zero-weight dummies).
GroupSet build_groups(const std::vector<Ordinate>& ords, int B, int dim, int G, int P);

// Coefficient records (grp_stride(G) doubles per group) of every group.
// adjoint = false: forward sweep; true: transposed sweep (octant flipped).
void group_coefficients(const GroupSet& gs, const std::vector<Ordinate>& ords, const HostInst& hi,
                        const std::vector<double>& v, const std::vector<double>& tau,
                        const std::vector<double>& C, double t0, bool adjoint,
                        std::vector<double>& out);

// Sweep schedule of an instance. For 3D problems plan.NR = 0 selects the
// pencil-block layout; NR >= 1 the rows-per-lane layout when the problem fits
// it (a lane axis of at most 128 cells, at most 256 stream entries per chunk),
// else the pencil-block layout.
bool build_schedule(const HostInst& hi, const Plan& plan, Schedule& s, std::string& err);

// 3D rows-per-lane schedule (false, with err, when the problem does not fit).
bool build_schedule_3r(const HostInst& hi, const Plan& plan, Schedule& s, std::string& err);

// Second-order faces: the Green-Gauss stencil of every position of each
// octant's layout, [n_oct][pos_per_oct][3*dim] codes, three per grid axis d:
// the cell's downwind neighbour along d, its upwind neighbour, and the upwind
// neighbour's own upwind neighbour. A code >= 0 is the neighbour's position in
// the same octant's layout; -1 a boundary face (domain edge or inactive
// neighbour) that is not an isothermal inflow; -(2 + slot) an isothermal wall
// the ordinate enters through (its boundary-face slot). A position of no cell
// has kNoCell as its first code.
std::vector<int> corr_stencil(const HostInst& hi, const Schedule& s);

// sum over incoming directions of w |s . n| for a face normal to axis d.
double half_range(const std::vector<Ordinate>& ords, int d);

}  // namespace bte
