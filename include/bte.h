/*
 * bte.h -- C ABI of the MI355X phonon-BTE source-iteration library.
 *
 * Inputs and outputs follow the paper's problem statement (Methods, "Forward
 * and inverse modeling workflow"): a geometry (here a Cartesian voxel mask with
 * per-face boundary conditions), the phonon band properties, the angular
 * quadrature and the heat source go in; the lattice temperature and the heat
 * flux come out, and for inverse problems the gradients of an objective with
 * respect to the relaxation times and the heat source.
 *
 * The library solves the steady, nongray phonon Boltzmann transport equation in
 * the relaxation-time approximation (paper Methods, "Phonon BTE", Eq. 1 with the
 * relaxation sign of Eq. eq:bte-2), discretized by spectral bands (Eqs. 8-13)
 * times discrete ordinates (Eq. 14) and first-order upwind finite volumes on a
 * Cartesian voxel mask (Eq. eq:fvm-1 with upwind face values), by source
 * iteration: every iteration sweeps every (band, direction) pair exactly (the
 * first-order upwind matrix A of Eq. A_matrix is triangular in upwind order)
 * and updates the lattice temperature from the weighted band/direction sum
 * (Eq. updatee0_t), until the residuals of Eq. 22 fall below the targets
 * (Methods, "Iterative matrix formulation and solution scheme").
 *
 * Conventions for every entry point:
 *   - Every call returns a bte_status; bte_last_error() describes the most
 *     recent failure on the calling thread (static, thread-local storage).
 *   - Cells are indexed c = i + n0*(j + n1*k) (x fastest). Cell arrays cover
 *     the whole bounding box; inactive cells are ignored on input and written
 *     as 0 on output.
 *   - Faces of a cell are numbered 0..5 = -x, +x, -y, +y, -z, +z.
 *   - Pointers named h_* are host pointers; d_* are device pointers on the
 *     device that was current when the handle was created. The caller owns all
 *     memory it passes; the library never frees it and never retains it beyond
 *     the call, except a workspace bound with bte_bind_workspace, which it uses
 *     until the handle is destroyed or another workspace is bound.
 *   - Device memory: bte_create allocates none. With a workspace bound
 *     (bte_workspace_bytes, bte_bind_workspace) every device array of the
 *     handle lives in it and the library allocates no device memory. A handle
 *     used without one makes its own arrays at the first call that needs the
 *     device and frees them in bte_destroy.
 *   - hip_stream is a hipStream_t (NULL = the null stream). Work is enqueued on
 *     it; calls that report convergence synchronise with it before returning.
 *   - Handles are not thread-safe; use one handle from one thread at a time.
 *   - Temperatures are absolute (K). The library works internally with
 *     deviations from T_ref, which is exact because the equations are linear in
 *     (e, T) when C does not depend on T.
 */
#ifndef BTE_H
#define BTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BTE_OK = 0,
  BTE_ERR_INVALID = 1,        /* bad argument; outputs untouched */
  BTE_ERR_HIP = 2,            /* HIP runtime error (message in bte_last_error) */
  BTE_ERR_NOT_CONVERGED = 3,  /* max_iters reached; outputs hold the last iterate */
  BTE_ERR_NONFINITE = 4,      /* a non-finite temperature or flux appeared */
  BTE_ERR_STATE = 5,          /* call order violated (e.g. adjoint before solve) */
  BTE_ERR_WORKSPACE = 6       /* the bound workspace is too small for the request */
} bte_status;

/* Boundary-condition kinds (paper Methods, "Boundary conditions"). */
enum {
  BTE_BC_ISOTHERMAL = 0, /* thermalizing wall at bc_T (Eq. 5) */
  BTE_BC_DIFFUSE = 1,    /* diffusely reflecting adiabatic wall (Eq. 6) */
  BTE_BC_SPECULAR = 2    /* specularly reflecting adiabatic wall (Eq. 7): an incoming
                            ordinate takes the outgoing value of its mirror direction
                            at the same cell, lagged one iteration like the diffuse
                            walls. Needs plans with G = 1. */
};

/* Arithmetic of the sweeps. FP64: everything in double. FP32: the transport
   sweep in float, band/direction partial sums promoted to double across
   ordinate groups, temperatures and residuals in double. */
enum { BTE_PREC_FP64 = 0, BTE_PREC_FP32 = 1 };

/* Geometry of one problem: the voxel form of the paper's mesh (Methods,
   "Spatial discretization": uniform Cartesian cells, V_i = h0 h1 h2 and
   S_ij / V_i = 1 / h_d for a face normal to axis d) and its boundary conditions
   (Methods, "Boundary conditions", Eqs. 5-7). */
typedef struct {
  int dim;                  /* 1, 2 or 3 */
  int n[3];                 /* cells per axis; unused axes must be 1 */
  double h[3];              /* cell size per axis (m); unused axes ignored */
  const uint8_t* h_mask;    /* [ncell] 1 = active; NULL = all active */
  const uint8_t* h_face_bc; /* [ncell*6] bc id of face f of cell c when that face
                               is a boundary (domain edge or inactive neighbour);
                               other entries ignored; NULL = every boundary face bc 0 */
  int n_bc;                 /* number of boundary conditions (1..255) */
  const int* h_bc_kind;     /* [n_bc] BTE_BC_* */
  const double* h_bc_T;     /* [n_bc] wall temperature (K), isothermal walls */
} bte_geometry;

/* Spectral bands (Methods, "Band discretization", Eqs. 8-13): per band the group
   velocity, relaxation time and heat capacity; C does not depend on T. */
typedef struct {
  int n_bands;              /* B >= 1 */
  const double* h_v;        /* [B] group velocity (m/s), > 0 */
  const double* h_tau;      /* [B] relaxation time (s), > 0 */
  const double* h_C;        /* [B] volumetric heat capacity (J m^-3 K^-1), > 0 */
} bte_bands;

/* Discrete ordinates (Methods, "Angle discretization", Eq. 14). */
typedef struct {
  int n_dirs;               /* M >= 1 */
  const double* h_s;        /* [M*3] unit directions (x, y, z) */
  const double* h_w;        /* [M] weights, > 0, summing to 4*pi */
} bte_quadrature;

/* Kernel shape of the sweep (chosen by bte_autotune, or set by hand).
   G: ordinates per register slot of a lane (1D/2D: 1 or 2; 3D rows-per-lane:
      1; 3D pencil blocks: 1, 2 or 4; 1 whenever a specular wall is present).
   R: 1D/2D only, waves per workgroup that pipeline successive strips of
      64*NR rows (R*P <= 4); 3D: always 1.
   P: waves per workgroup that sweep different ordinate groups of one octant
      in lockstep and add their partial sums per cell before writing them
      (1D/2D: 1, 2 or 4 with R*P <= 4; 3D rows-per-lane: 1, 2, 4 or 8; 3D
      pencil blocks: 1..8).
   C: 3D pencil blocks only, steps between workgroup barriers (multiple of 8
      in 8..64 and of P); the other layouts use chunks of 8 steps.
   NR: 1D/2D, rows owned by each lane of a strip (1, 2 or 4). 3D: a negative
      value selects the pencil-block layout (reported as 0), 1 or 2 the
      rows-per-lane layout (lanes along one grid axis of at most 128 cells,
      each lane NR cells of it; the step axis cut into blocks of 8 columns
      streamed block by block, plane by plane along the third axis; the axes
      are assigned for the fewest boundary entries; taken when the problem
      fits, with the NR the grid needs), reported back as the rows per lane
      used.
   Zero fields mean "keep the current value". A shape whose LDS need exceeds
   the per-workgroup limit is rejected with BTE_ERR_INVALID. */
typedef struct { int G, R, P, C, NR; } bte_plan;

/* Options of a solve or adjoint (Methods, "Iterative matrix formulation and
   solution scheme": the iteration and its stop test, Eq. 22). */
typedef struct {
  double tol_T;        /* target eps_T (Eq. 22, normalised by max |T - T_ref|); <= 0: run max_iters */
  double tol_q;        /* target eps_q (Eq. 22); <= 0: run max_iters */
  int max_iters;       /* >= 1 */
  int check_every;     /* iterations between convergence checks (>= 1); 0 = default (8) */
  double T_ref;        /* reference temperature (K) of the deviational variables; <= 0 selects the
                          mean wall temperature over the instance's isothermal boundary faces.
                          Exact for any value (the equations are linear in (e, T)); the FP32
                          sweeps keep more digits of T - T_ref when it is near the solution. */
  int use_graph;       /* 1 = replay a captured hipGraph of check_every iterations */
  int store_angular;   /* solves: keep what bte_adjoint needs (the angular field) */
  const char* autotune_cache; /* NULL, or the path of a plan-cache text file: a solve applies the
                          plan stored for its problem and device, or runs bte_autotune (30
                          iterations per candidate) and appends the result; lines read
                          "<key> plan G R P C NR" */
} bte_opts;

typedef struct {
  int iters;           /* iterations performed */
  double eps_T, eps_q; /* residuals at the last check */
  double seconds;      /* wall time of the iteration loop */
  int status;          /* bte_status of this solve */
} bte_report;

typedef struct bte_ctx* bte_handle;

/* Library version string (static storage). */
const char* bte_version(void);

/* Description of the most recent failure on this thread (static storage). */
const char* bte_last_error(void);

/* Host-only validation of a problem (no device call). Returns BTE_OK or
   BTE_ERR_INVALID for: dim not in 1..3; n < 1 or h <= 0 on a used axis, or
   n != 1 on an unused axis; no active cell; n_bc out of range, a bc kind other
   than isothermal/diffuse/specular, a face_bc entry >= n_bc on a boundary face;
   no isothermal boundary face (no unique steady state: the T_L update
   conserves energy, so heat can leave only through isothermal walls);
   B < 1, any v, tau or C <= 0 or non-finite; M < 1, |s| != 1 (1e-12),
   w <= 0, |sum w - 4 pi| > 1e-10 * 4 pi, or a quadrature not closed under the
   reflection of each grid axis. */
bte_status bte_validate(const bte_geometry* geom, const bte_bands* bands,
                        const bte_quadrature* quad);

/* Gauss-Legendre quadrature in mu = cos(theta) for a 1D slab: s_a = (mu_a,
   sqrt(1 - mu_a^2), 0), w_a = 2 pi g_a. h_s: [n_mu*3], h_w: [n_mu]. */
bte_status bte_quadrature_gl_mu(int n_mu, double* h_s, double* h_w);

/* Octant-product Gauss-Legendre quadrature (paper Eq. 14): per octant an
   n_theta x n_phi product of Gauss-Legendre rules in theta and phi on (0, pi/2)
   with weights beta_theta * beta_phi * sin(theta), rescaled so they sum to 4 pi.
   polar_axis 0 gives s = (cos t, sin t cos p, sin t sin p) as in the paper; 2
   puts the polar axis on z. h_s: [8*n_theta*n_phi*3], h_w: [8*n_theta*n_phi]. */
bte_status bte_quadrature_octant_gl(int n_theta, int n_phi, int polar_axis, double* h_s,
                                    double* h_w);

/* Create a solver for one problem on the current device (the per-band,
   per-ordinate equations of Eq. eq:bte-2 discretized by Eq. eq:fvm-1 with
   first-order upwind faces; Methods, "Spatial discretization"). Validates as
   bte_validate, derives the per-band and per-ordinate constants (the diagonal
   and upwind couplings of Eq. A_matrix), the boundary-face tables and the sweep
   schedule. Allocates no device memory (see bte_bind_workspace).
   precision: BTE_PREC_*. *out: the new handle (NULL on failure). */
bte_status bte_create(const bte_geometry* geom, const bte_bands* bands,
                      const bte_quadrature* quad, int precision, bte_handle* out);

/* Device bytes the handle needs for its current plan: *bytes. with_adjoint = 1
   adds the angular field that a solve with store_angular keeps for
   bte_adjoint. A later bte_set_plan or bte_autotune may change the figure. */
bte_status bte_workspace_bytes(bte_handle h, int with_adjoint, size_t* bytes);

/* Bind caller-owned device memory (e.g. torch.empty(bytes, dtype=torch.uint8)
   on the handle's device; 256-byte aligned) as the handle's workspace: every
   device array of the handle is carved from it and the library allocates no
   device memory from then on. The caller keeps the memory alive and unchanged
   until the handle is destroyed or rebound; the library never frees it.
   BTE_ERR_WORKSPACE when bytes is below bte_workspace_bytes(h, 0); with fewer
   than bte_workspace_bytes(h, 1) bytes a solve with store_angular returns
   BTE_ERR_WORKSPACE, and so does a plan change that would not fit. d_ws = NULL
   unbinds (the handle makes its own memory at the next call that needs it).
   Binding or unbinding drops any solver state (solve again). */
bte_status bte_bind_workspace(bte_handle h, void* d_ws, size_t bytes);

/* Replace the relaxation times tau_b (Eq. eq:bte-2; e.g. between optimisation
   steps of an inverse problem, Methods, "Forward and inverse modeling
   workflow"). h_tau: [B], finite and > 0. A state kept for bte_adjoint is
   dropped when tau changes. */
bte_status bte_set_tau(bte_handle h, const double* h_tau);

/* Face reconstruction of the finite volumes (Methods, "Spatial
   discretization"): order 1, first-order upwind faces (the default); order 2,
   the paper's second-order face value e_ij = e' + grad e' . d' of the upwind
   cell with Green-Gauss gradients, taken by deferred correction: each sweep
   keeps the first-order A of Eq. A_matrix and adds to the source the
   difference of the second-order and first-order face fluxes of the previous
   iterate (the b^n of Eq. rhs_b), so the fixed point is that of the
   second-order scheme. Green-Gauss face values: the mean of the two cells at
   an interior face, the wall value at an isothermal face the ordinate enters
   through, the linear extrapolation from the cell and its neighbour across
   the opposite face at any other boundary face. Order 2 forces plans with
   G = 1 and, in 3D, the rows-per-lane layout (a pencil plan moves to it;
   bte_set_plan with a pencil plan then returns BTE_ERR_INVALID); it keeps the
   angular field and a correction per ordinate, and a stencil table per
   octant, in device memory (bte_workspace_bytes counts them), and has no
   adjoint (bte_adjoint returns BTE_ERR_STATE). Drops any solver state. */
bte_status bte_set_order(bte_handle h, int order);

/* Set / get the sweep kernel shape. */
bte_status bte_set_plan(bte_handle h, const bte_plan* plan);
bte_status bte_get_plan(bte_handle h, bte_plan* plan);

/* Time candidate kernel shapes on this problem and keep the fastest; writes it
   to *best (may be NULL). Each candidate runs n_iters whole source iterations
   (sweep, finalize, diffuse-wall update) after one warm-up iteration, from a
   fresh state; the current shape is kept unless another is at least 3% faster.
   The solver state afterwards is that of a fresh start (solve again).
   d_Q: [ncell] heat source used for the timing runs (NULL = zero); a batch
   handle takes NULL only (BTE_ERR_STATE otherwise: one array cannot serve
   instances of different sizes). With a bound workspace, shapes that do not
   fit in it are skipped. */
bte_status bte_autotune(bte_handle h, const double* d_Q, int n_iters, void* hip_stream,
                        bte_plan* best);

/* Solve by source iteration (Methods, "Iterative matrix formulation and
   solution scheme": step 1 from the initial temperature, step 2 the exact
   solve of Eq. Axb for every (band, direction), step 3 the T_L update of
   Eq. updatee0_t and the lagged wall values of Eqs. 6-7, step 4 the test of
   Eq. 22). h_tau: [B] relaxation times for this solve, or NULL to keep the
   current ones (as bte_set_tau). d_Q: [ncell] heat source (W/m^3) or NULL;
   d_T_init: [ncell] initial temperature (K) or NULL for T_ref everywhere (a
   previous result resumes the iteration: warm start); d_T: [ncell] output
   temperature T_L (K); d_q: [ncell*dim] output heat flux (Eq. 4, W/m^2, grid
   axes) or NULL. Returns BTE_OK when converged, BTE_ERR_NOT_CONVERGED after
   max_iters (outputs hold the last iterate), BTE_ERR_NONFINITE on a non-finite
   iterate, BTE_ERR_INVALID (outputs untouched) for bad arguments. */
bte_status bte_solve(bte_handle h, const double* h_tau, const double* d_Q, const double* d_T_init,
                     double* d_T, double* d_q, const bte_opts* opts, void* hip_stream,
                     bte_report* h_rep);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): bte_solve
   with every device array of the handle in a workspace the library holds as a
   static device array of 64 MiB per device (part of its code object, held
   until the process ends). Makes no hipMalloc or hipFree and no other
   allocating call: the handle is (re)bound to that array when another handle
   used it last (its tables are rebuilt there), the iteration runs without a
   hipGraph and without the autotune cache. Same arguments, results and
   statuses as bte_solve; a stored angular field (store_angular) must fit in
   the array too. BTE_ERR_WORKSPACE when the problem needs more than 64 MiB
   (bte_workspace_bytes); BTE_ERR_STATE for a handle that holds device memory
   of its own (a previous bte_solve made it: use a fresh handle). Every call on
   a device shares that device's array: a handle that used it before loses its
   arrays and state to the next call of another handle, and calls that overlap
   on one device race. */
bte_status bte_solve_noalloc(bte_handle h, const double* h_tau, const double* d_Q,
                             const double* d_T_init, double* d_T, double* d_q,
                             const bte_opts* opts, void* hip_stream, bte_report* h_rep);

/* Adjoint of the converged source-iteration fixed point (the gradient
   workflow of Methods, "Forward and inverse modeling workflow": a discrete
   adjoint of the implicit solves). Needs a previous bte_solve on h with
   opts->store_angular = 1 and unchanged tau.
   Given d_dJdT = dJ/dT [ncell], iterates lambda = dJ/dT + sum_b k_b sum_a psi
   with psi = transpose sweeps (direction -s_a) of lambda. Isothermal walls give
   the transposed sweeps zero inflow; diffuse and specular walls give them the
   adjoint of the lagged reflection (Eqs. 6, 7), iterated with lambda. Then
   writes h_dJdtau [B] (host) and d_dJdQ [ncell] (device); either may be NULL. */
bte_status bte_adjoint(bte_handle h, const double* d_dJdT, double* h_dJdtau, double* d_dJdQ,
                       const bte_opts* opts, void* hip_stream, bte_report* h_rep);

/* Derivative of the adjoint's objective with respect to a common factor s on
   every cell size h_d (s = 1: the geometry as created), i.e. L dJ/dL when all
   lengths scale with L (Results, "1D inverse problem for system size": the
   film-thickness gradient). Every beta_d = v|s_d|/h_d scales as 1/s, so by the forward
   equation dJ/ds = -sum_b (1/tau_b) sum_{a,c} psi (u - dT) + sum_c Q_c dJ/dQ_c
   with the adjoint field psi of the last bte_adjoint / bte_batch_adjoint on h.
   h_dJds: [n_inst] host output. BTE_ERR_STATE when no adjoint has run since the
   last solve. */
bte_status bte_adjoint_dscale(bte_handle h, double* h_dJds);

/* Average device time (ms) of one launch of the forward sweep kernel on the
   current state, measured with HIP events around n_launches back-to-back
   launches on hip_stream; also returns the number of cell x ordinate x band
   updates one launch performs. Requires a previous bte_solve. */
bte_status bte_time_sweep(bte_handle h, int n_launches, void* hip_stream, double* h_ms,
                          double* h_updates);

/* Batched solver: n_inst problems of the same dimension, band table and
   quadrature (the "parallel forward simulations" of the paper's
   Introduction), swept by one persistent launch per iteration with
   per-instance convergence and retirement. geoms: [n_inst]. Allocates no
   device memory (as bte_create). */
bte_status bte_batch_create(int n_inst, const bte_geometry* geoms, const bte_bands* bands,
                            const bte_quadrature* quad, int precision, bte_handle* out);

/* Solve every instance as bte_solve does (same iteration and stop test, per
   instance; opts->T_ref <= 0 takes each instance's own default).
   d_Q[i], d_T[i], d_q[i]: device arrays of instance i (d_q may be NULL or hold
   NULL entries). h_reps: [n_inst] or NULL. Returns BTE_OK when every instance
   converged, else the worst status. */
bte_status bte_batch_solve(bte_handle h, const double* const* d_Q, double* const* d_T,
                           double* const* d_q, const bte_opts* opts, void* hip_stream,
                           bte_report* h_reps);

/* Batched adjoint, per instance as bte_adjoint (after bte_batch_solve with
   store_angular). h_dJdtau: [n_inst*B]. */
bte_status bte_batch_adjoint(bte_handle h, const double* const* d_dJdT, double* h_dJdtau,
                             double* const* d_dJdQ, const bte_opts* opts, void* hip_stream,
                             bte_report* h_reps);

/* Free the handle and its device memory. NULL is allowed. */
bte_status bte_destroy(bte_handle h);

#ifdef __cplusplus
}
#endif
#endif /* BTE_H */
