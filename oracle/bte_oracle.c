/*
 * FP64 CPU oracle for the steady, nongray phonon BTE solved by source iteration.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the independent reference that the HIP
 * library is checked against. Only the test suite, the smoke entry and the
 * bench's CPU-baseline leg may load it; the library never calls it and shares
 * no code with it.
 *
 * What it computes follows the paper's Methods section, in the paper's own
 * variables (absolute phonon energy e and lattice temperature T_L) and order:
 *
 *   Model      v_l . grad e_{a,l} = -(e_{a,l} - e0_l)/tau_l + Q_l/(4 pi)
 *              (Methods, "Spatial discretization", Eq. eq:bte-2; relaxation
 *              sign as in eq:bte-2; per-ordinate source Q_l/(4 pi) with
 *              Q_l = C_l Q / sum C (Eq. 11) so that div q = Q).
 *   Equilibrium e0_l = C_l T_L/(4 pi),
 *              T_L = sum_l sum_a w_a e_{a,l}/tau_l / sum_l C_l/tau_l
 *              (Eq. updatee0_t; the weight there is the angular weight w_a).
 *   Walls      isothermal: incoming e = C T_w/(4 pi)                (Eq. 5)
 *              diffuse: incoming e = sum_{out} w (s.n) e / sum_{in} w |s.n|
 *              (Eq. 6 with the discrete half-range normalisation), lagged one
 *              iteration.
 *              specular: incoming e along s equals the outgoing e along the
 *              mirror direction s' = s - 2 n (s.n) at the same boundary cell
 *              (Eq. 7); s' must be one of the quadrature's directions. Lagged
 *              one iteration like the diffuse walls, and starting, like them,
 *              from the adjacent cell's equilibrium.
 *   FVM        upwind face values, uniform Cartesian cells: S_ij/V_i = 1/h_d
 *              for a face normal to axis d. order = 1: first-order faces (the
 *              face gradient term of the paper's reconstruction dropped);
 *              order = 2: the paper's second-order face value
 *              e_ij = e' + grad e' . d' of the upwind cell (Methods, "Spatial
 *              discretization"), grad e' by Green-Gauss, entering the
 *              right-hand side b^n of Eq. rhs_b only (A of Eq. A_matrix stays
 *              first order: a deferred correction). Green-Gauss face values:
 *              the mean of the two cells at an interior face; at an
 *              isothermal face the ordinate enters through, the wall value;
 *              at any other boundary face the linear extrapolation from the
 *              cell and its neighbour across the opposite face. A wall face's
 *              entering value is the wall value with no gradient term.
 *   Iteration  (Methods, "Iterative matrix formulation and solution scheme")
 *              1. e = e0 from the initial temperature;
 *              2. for every (band, direction) solve A Delta e = b^n (Eqs. Axb,
 *                 A_matrix, rhs_b; b^n evaluated from e^n by face fluxes, A
 *                 solved exactly by forward substitution in upwind order, which
 *                 is exact because first-order upwind A is triangular in that
 *                 order), then e += Delta e;
 *              3. update T_L and e0 (Eq. updatee0_t), and the lagged diffuse
 *                 and specular wall values;
 *              4. repeat until eps_T and eps_q (Eq. 22) fall below the targets.
 *   Heat flux  q = sum_l sum_a w_a v_l s_a e_{a,l}   (Eq. 4, grid axes only)
 *   Residuals  eps_T = RMS_i(T^{n+1} - T^n) / max_i |T^{n+1} - T_ref|,
 *              eps_q = RMS_i(|q|^{n+1} - |q|^n) / max_i |q^{n+1}|
 *              (Eq. 22, normalised by the deviation from T_ref rather than by
 *              the absolute maximum temperature; 0/0 counts as 0).
 *
 * Parallelism: the (band, direction) solves of one iteration are independent
 * (OpenMP over them); the band/direction sums are done per cell in a fixed
 * order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_INVALID 1
#define OR_NOT_CONVERGED 3
#define OR_NONFINITE 4

#define BC_ISOTHERMAL 0
#define BC_DIFFUSE 1
#define BC_SPECULAR 2
#define NO_BC 255

static const double PI = 3.14159265358979323846;

typedef struct {
  int dim;
  int n[3];
  double h[3];
  long ncell;
  const uint8_t* mask;
  const uint8_t* face_bc;
} grid_t;

static int active(const grid_t* g, long c) { return g->mask ? g->mask[c] != 0 : 1; }

/* neighbour of cell c across face f (0..5 = -x,+x,-y,+y,-z,+z); -1 if the face
   is a boundary (domain edge or inactive neighbour). */
static long neighbour(const grid_t* g, long c, int f) {
  int d = f / 2, side = f % 2;
  long idx[3];
  idx[0] = c % g->n[0];
  idx[1] = (c / g->n[0]) % g->n[1];
  idx[2] = c / ((long)g->n[0] * g->n[1]);
  idx[d] += side ? 1 : -1;
  if (idx[d] < 0 || idx[d] >= g->n[d]) return -1;
  long nb = idx[0] + (long)g->n[0] * (idx[1] + (long)g->n[1] * idx[2]);
  return active(g, nb) ? nb : -1;
}

/* Boundary faces, enumerated once: cell, face direction, bc id. */
typedef struct {
  long n;
  long* cell;
  int* face;
  int* bc;
  long* slot; /* [ncell*6] -> boundary face index or -1 */
} bfaces_t;

static void build_bfaces(const grid_t* g, bfaces_t* bf) {
  long cnt = 0;
  bf->slot = (long*)malloc(sizeof(long) * g->ncell * 6);
  for (long c = 0; c < g->ncell * 6; ++c) bf->slot[c] = -1;
  for (long c = 0; c < g->ncell; ++c) {
    if (!active(g, c)) continue;
    for (int f = 0; f < 2 * g->dim; ++f)
      if (neighbour(g, c, f) < 0) ++cnt;
  }
  bf->n = cnt;
  bf->cell = (long*)malloc(sizeof(long) * (cnt ? cnt : 1));
  bf->face = (int*)malloc(sizeof(int) * (cnt ? cnt : 1));
  bf->bc = (int*)malloc(sizeof(int) * (cnt ? cnt : 1));
  cnt = 0;
  for (long c = 0; c < g->ncell; ++c) {
    if (!active(g, c)) continue;
    for (int f = 0; f < 2 * g->dim; ++f) {
      if (neighbour(g, c, f) >= 0) continue;
      bf->cell[cnt] = c;
      bf->face[cnt] = f;
      bf->bc[cnt] = g->face_bc ? g->face_bc[c * 6 + f] : 0;
      bf->slot[c * 6 + f] = cnt;
      ++cnt;
    }
  }
}

static void free_bfaces(bfaces_t* bf) {
  free(bf->cell);
  free(bf->face);
  free(bf->bc);
  free(bf->slot);
}

/* outward normal component of direction s on face f */
static double s_dot_n(const double* s, int f) {
  int d = f / 2;
  return (f % 2) ? s[d] : -s[d];
}

/* wall value of this ordinate at boundary face slot k */
static double wall_value(const bfaces_t* bf, const int* bc_kind, long k, const double* eb_l, const double* es_la) {
  return bc_kind[bf->bc[k]] == BC_SPECULAR ? es_la[k] : eb_l[k];
}

/*
 * Green-Gauss gradient of one ordinate's energy in every active cell:
 * grad_d(c) = (sum over the two faces of c normal to axis d of e_f n_d S_f)/V
 * = (e_f+ - e_f-)/h_d, with e_f the mean of the two cells' values at an
 * interior face, the wall value at an isothermal face the ordinate enters
 * through, and at any other boundary face the value extrapolated linearly
 * from the cell and the neighbour across its opposite face.
 */
static void green_gauss(const grid_t* g, const bfaces_t* bf, const int* bc_kind, const double* s,
                        const double* eb_l, const double* es_la, const double* e_la, double* grad) {
  for (long c = 0; c < g->ncell; ++c) {
    if (!active(g, c)) continue;
    for (int d = 0; d < g->dim; ++d) {
      double ef[2];
      for (int side = 0; side < 2; ++side) {
        int f = 2 * d + side;
        long nb = neighbour(g, c, f);
        if (nb >= 0) {
          ef[side] = 0.5 * (e_la[c] + e_la[nb]);
        } else if (s_dot_n(s, f) < 0.0 && bc_kind[bf->bc[bf->slot[c * 6 + f]]] == BC_ISOTHERMAL) {
          ef[side] = wall_value(bf, bc_kind, bf->slot[c * 6 + f], eb_l, es_la);
        } else {
          /* leaving through a wall, or entering from a reflecting wall (whose
             value is itself lagged): extrapolated linearly from the cell and
             its neighbour across the opposite face (the cell's value alone
             when that face is a boundary too) */
          long ob = neighbour(g, c, f ^ 1);
          ef[side] = ob >= 0 ? 1.5 * e_la[c] - 0.5 * e_la[ob] : e_la[c];
        }
      }
      grad[c * g->dim + d] = (ef[1] - ef[0]) / g->h[d];
    }
  }
}

/*
 * One (band l, direction a) solve of A Delta e = b^n followed by e += Delta e.
 * e_la: this ordinate's energies (updated in place); eb: boundary face values
 * of band l (absolute energy on incoming faces); T: current T_L. grad: scratch
 * [ncell*dim] for the second-order faces (order 2), else unused.
 */
static void solve_ordinate(const grid_t* g, const bfaces_t* bf, const int* bc_kind, double v,
                           double tau, double C, double Csum, const double* s, const double* Q,
                           const double* T, const double* eb_l, const double* es_la, double* e_la,
                           double* rhs, double* de, int order, double* grad) {
  const long ncell = g->ncell;
  if (order == 2) green_gauss(g, bf, bc_kind, s, eb_l, es_la, e_la, grad);
  /* b^n (Eq. rhs_b with first-order faces): minus the net upwind face flux of
     e^n, minus (e^n - e0^n)/tau, plus the band's source share. */
  for (long c = 0; c < ncell; ++c) {
    if (!active(g, c)) continue;
    double flux = 0.0;
    for (int f = 0; f < 2 * g->dim; ++f) {
      int d = f / 2;
      double vn = v * s_dot_n(s, f);       /* v . n_ij */
      if (vn == 0.0) continue;
      /* vector from the upwind cell's centre to the face centre, along axis d */
      double half = 0.5 * g->h[d];
      double e_face;
      if (vn > 0.0) {
        e_face = e_la[c];                  /* upwind cell is the cell itself */
        if (order == 2) e_face += grad[c * g->dim + d] * ((f % 2) ? half : -half);
      } else {
        long nb = neighbour(g, c, f);
        if (nb >= 0) {
          e_face = e_la[nb];
          if (order == 2) e_face += grad[nb * g->dim + d] * ((f % 2) ? -half : half);
        } else {
          e_face = wall_value(bf, bc_kind, bf->slot[c * 6 + f], eb_l, es_la);
        }
      }
      flux += vn / g->h[d] * e_face;       /* (1/V) v.n S e_face */
    }
    double e0 = C * T[c] / (4.0 * PI);
    double Qs = (Q ? Q[c] : 0.0) * C / Csum / (4.0 * PI);
    rhs[c] = -flux - (e_la[c] - e0) / tau + Qs;
  }
  /* A: diagonal 1/tau + sum of outflow v.n/h, off-diagonal -v|s_d|/h_d to the
     upwind neighbour (Eq. A_matrix). Forward substitution in upwind raster
     order: along each axis, ascending index when s_d >= 0, else descending. */
  double diag = 1.0 / tau;
  for (int d = 0; d < g->dim; ++d) diag += v * fabs(s[d]) / g->h[d];
  int n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
  for (int kk = 0; kk < n2; ++kk) {
    int k = (g->dim >= 3 && s[2] < 0) ? n2 - 1 - kk : kk;
    for (int jj = 0; jj < n1; ++jj) {
      int j = (g->dim >= 2 && s[1] < 0) ? n1 - 1 - jj : jj;
      for (int ii = 0; ii < n0; ++ii) {
        int i = (s[0] < 0) ? n0 - 1 - ii : ii;
        long c = i + (long)n0 * (j + (long)n1 * k);
        if (!active(g, c)) continue;
        double r = rhs[c];
        for (int d = 0; d < g->dim; ++d) {
          if (s[d] == 0.0) continue;
          int f = 2 * d + (s[d] > 0 ? 0 : 1); /* the inflow face on axis d */
          long nb = neighbour(g, c, f);
          if (nb >= 0) r += v * fabs(s[d]) / g->h[d] * de[nb];
        }
        de[c] = r / diag;
      }
    }
  }
  for (long c = 0; c < ncell; ++c)
    if (active(g, c)) e_la[c] += de[c];
}

static int finite_all(const double* x, long n) {
  for (long i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

/*
 * oracle_solve: see the file header. Arrays:
 *   n[3], h[3]; mask[ncell] (NULL = all active); face_bc[ncell*6] (NULL = bc 0);
 *   bc_kind[n_bc], bc_T[n_bc]; v,tau,C[B]; s[M*3], w[M]; Q[ncell] (W/m^3, NULL = 0);
 *   T_init[ncell] (NULL = T_ref); order 1 or 2 (face reconstruction, see the header).
 * Outputs: T_out[ncell] (absolute, 0 on inactive cells), q_out[ncell*dim],
 *   e_out[B*M*ncell] (absolute angular energy of the last iterate, optional),
 *   eb_out[B*n_bfaces] (boundary face values used by the last sweep, optional),
 *   info[4] = {iterations, eps_T, eps_q, n_boundary_faces}.
 * max_iters >= 1. tol_T, tol_q <= 0 run exactly max_iters iterations.
 * Returns 0 converged, 3 not converged, 1 invalid input, 4 non-finite.
 */
int oracle_solve(int dim, const int* n, const double* h, const uint8_t* mask,
                 const uint8_t* face_bc, int n_bc, const int* bc_kind, const double* bc_T,
                 int B, const double* v, const double* tau, const double* C, int M,
                 const double* s, const double* w, const double* Q, const double* T_init,
                 double T_ref, int max_iters, double tol_T, double tol_q, int nthreads,
                 double* T_out, double* q_out, double* e_out, double* eb_out, double* info, int order) {
  if (dim < 1 || dim > 3 || B < 1 || M < 1 || max_iters < 1 || order < 1 || order > 2) return OR_INVALID;
  grid_t g;
  g.dim = dim;
  g.ncell = 1;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = n[d];
    g.h[d] = h[d];
    if (g.n[d] < 1) return OR_INVALID;
    g.ncell *= g.n[d];
  }
  g.mask = mask;
  g.face_bc = face_bc;
  const long ncell = g.ncell;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif

  bfaces_t bf;
  build_bfaces(&g, &bf);
  for (long f = 0; f < bf.n; ++f)
    if (bf.bc[f] < 0 || bf.bc[f] >= n_bc) { free_bfaces(&bf); return OR_INVALID; }

  /* mirror directions for specular faces (Eq. 7): for a face normal to grid
     axis d, s' = s with its d component negated; it must be a quadrature
     direction. mir[d*M + a] = index of s', or -1. */
  int has_spec = 0;
  for (long f = 0; f < bf.n; ++f)
    if (bc_kind[bf.bc[f]] == BC_SPECULAR) has_spec = 1;
  int* mir = (int*)malloc(sizeof(int) * 3 * M);
  if (!mir) { free_bfaces(&bf); return OR_INVALID; }
  for (int d = 0; d < 3; ++d)
    for (int a = 0; a < M; ++a) {
      mir[d * M + a] = -1;
      for (int m = 0; m < M; ++m) {
        int same = 1;
        for (int k = 0; k < 3; ++k) {
          double want = (k == d) ? -s[3 * a + k] : s[3 * a + k];
          if (fabs(s[3 * m + k] - want) > 1e-12) same = 0;
        }
        if (same) { mir[d * M + a] = m; break; }
      }
    }
  for (long f = 0; f < bf.n; ++f) {
    if (bc_kind[bf.bc[f]] != BC_SPECULAR) continue;
    for (int a = 0; a < M; ++a)
      if (mir[(bf.face[f] / 2) * M + a] < 0) { free(mir); free_bfaces(&bf); return OR_INVALID; }
  }

  double Csum = 0.0, D = 0.0;
  for (int l = 0; l < B; ++l) { Csum += C[l]; D += C[l] / tau[l]; }

  double* T = (double*)calloc(ncell, sizeof(double));
  double* Tn = (double*)calloc(ncell, sizeof(double));
  double* q = (double*)calloc(ncell * dim, sizeof(double));
  double* qn = (double*)calloc(ncell * dim, sizeof(double));
  double* e = (double*)malloc(sizeof(double) * (size_t)B * M * ncell);
  double* eb = (double*)calloc((size_t)B * (bf.n ? bf.n : 1), sizeof(double));
  double* inv_half = (double*)calloc(bf.n ? bf.n : 1, sizeof(double));
  /* specular wall values per (band, direction, face) */
  double* es = has_spec ? (double*)calloc((size_t)B * M * bf.n, sizeof(double)) : NULL;
  if (!T || !Tn || !q || !qn || !e || !eb || !inv_half || (has_spec && !es)) {
    free(T); free(Tn); free(q); free(qn); free(e); free(eb); free(inv_half); free(es); free(mir);
    free_bfaces(&bf);
    return OR_INVALID;
  }

  /* step 1: initial temperature, e = e0 */
  for (long c = 0; c < ncell; ++c) T[c] = active(&g, c) ? (T_init ? T_init[c] : T_ref) : 0.0;
  for (int l = 0; l < B; ++l)
    for (int a = 0; a < M; ++a)
      for (long c = 0; c < ncell; ++c) e[((size_t)l * M + a) * ncell + c] = C[l] * T[c] / (4.0 * PI);
  /* wall values: isothermal fixed; diffuse starts at the adjacent cell's
     equilibrium (the reflection of an isotropic distribution is itself). */
  for (long f = 0; f < bf.n; ++f) {
    int kind = bc_kind[bf.bc[f]];
    double half = 0.0;
    for (int a = 0; a < M; ++a) {
      double sn = s_dot_n(&s[3 * a], bf.face[f]);
      if (sn < 0.0) half += w[a] * (-sn);
    }
    inv_half[f] = half > 0.0 ? 1.0 / half : 0.0;
    for (int l = 0; l < B; ++l) {
      double Tw = (kind == BC_ISOTHERMAL) ? bc_T[bf.bc[f]] : T[bf.cell[f]];
      eb[(size_t)l * bf.n + f] = C[l] * Tw / (4.0 * PI);
      if (kind == BC_SPECULAR)
        for (int a = 0; a < M; ++a) es[((size_t)l * M + a) * bf.n + f] = C[l] * Tw / (4.0 * PI);
    }
  }

  int it = 0, status = OR_NOT_CONVERGED;
  double epsT = INFINITY, epsq = INFINITY;
  const double* Qp = Q;
  while (it < max_iters) {
    /* step 2: every (band, direction) */
#pragma omp parallel
    {
      double* rhs = (double*)malloc(sizeof(double) * ncell);
      double* de = (double*)malloc(sizeof(double) * ncell);
      double* grad = order == 2 ? (double*)malloc(sizeof(double) * ncell * dim) : NULL;
#pragma omp for schedule(dynamic, 1)
      for (int la = 0; la < B * M; ++la) {
        int l = la / M, a = la % M;
        solve_ordinate(&g, &bf, bc_kind, v[l], tau[l], C[l], Csum, &s[3 * a], Qp, T,
                       &eb[(size_t)l * bf.n], es ? &es[(size_t)la * bf.n] : NULL,
                       &e[(size_t)la * ncell], rhs, de, order, grad);
      }
      free(rhs);
      free(de);
      free(grad);
    }
    /* step 3: T_L (Eq. updatee0_t) and q (Eq. 4), per cell in a fixed order */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; ++c) {
      if (!active(&g, c)) { Tn[c] = 0.0; for (int d = 0; d < dim; ++d) qn[c * dim + d] = 0.0; continue; }
      double num = 0.0, qq[3] = {0.0, 0.0, 0.0};
      for (int l = 0; l < B; ++l) {
        double sl = 0.0, sq[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < M; ++a) {
          double ev = e[((size_t)l * M + a) * ncell + c];
          sl += w[a] * ev;
          for (int d = 0; d < dim; ++d) sq[d] += w[a] * s[3 * a + d] * ev;
        }
        num += sl / tau[l];
        for (int d = 0; d < dim; ++d) qq[d] += v[l] * sq[d];
      }
      Tn[c] = num / D;
      for (int d = 0; d < dim; ++d) qn[c * dim + d] = qq[d];
    }
    /* lagged diffuse wall values from the new outgoing energies (Eq. 6) */
#pragma omp parallel for schedule(static)
    for (long f = 0; f < bf.n; ++f) {
      if (bc_kind[bf.bc[f]] != BC_DIFFUSE) continue;
      long c = bf.cell[f];
      for (int l = 0; l < B; ++l) {
        double out = 0.0;
        for (int a = 0; a < M; ++a) {
          double sn = s_dot_n(&s[3 * a], bf.face[f]);
          if (sn > 0.0) out += w[a] * sn * e[((size_t)l * M + a) * ncell + c];
        }
        eb[(size_t)l * bf.n + f] = out * inv_half[f];
      }
    }
    /* lagged specular wall values: the new outgoing energy along the mirror
       direction at the same cell (Eq. 7) */
    if (has_spec) {
#pragma omp parallel for schedule(static)
      for (long f = 0; f < bf.n; ++f) {
        if (bc_kind[bf.bc[f]] != BC_SPECULAR) continue;
        long c = bf.cell[f];
        int d = bf.face[f] / 2;
        for (int l = 0; l < B; ++l)
          for (int a = 0; a < M; ++a)
            if (s_dot_n(&s[3 * a], bf.face[f]) < 0.0)
              es[((size_t)l * M + a) * bf.n + f] = e[((size_t)l * M + mir[d * M + a]) * ncell + c];
      }
    }
    ++it;
    /* step 4: residuals (Eq. 22) */
    double sT = 0.0, mT = 0.0, sq2 = 0.0, mq = 0.0;
    long nact = 0;
    for (long c = 0; c < ncell; ++c) {
      if (!active(&g, c)) continue;
      ++nact;
      double dT = Tn[c] - T[c];
      sT += dT * dT;
      double aT = fabs(Tn[c] - T_ref);
      if (aT > mT) mT = aT;
      double qa = 0.0, qb = 0.0;
      for (int d = 0; d < dim; ++d) {
        qa += qn[c * dim + d] * qn[c * dim + d];
        qb += q[c * dim + d] * q[c * dim + d];
      }
      qa = sqrt(qa);
      qb = sqrt(qb);
      sq2 += (qa - qb) * (qa - qb);
      if (qa > mq) mq = qa;
    }
    double rT = sqrt(sT / (double)nact), rq = sqrt(sq2 / (double)nact);
    epsT = (mT > 0.0) ? rT / mT : (rT == 0.0 ? 0.0 : INFINITY);
    epsq = (mq > 0.0) ? rq / mq : (rq == 0.0 ? 0.0 : INFINITY);
    memcpy(T, Tn, sizeof(double) * ncell);
    memcpy(q, qn, sizeof(double) * ncell * dim);
    if (!finite_all(T, ncell) || !finite_all(q, ncell * dim)) { status = OR_NONFINITE; break; }
    if (tol_T > 0.0 && tol_q > 0.0 && epsT < tol_T && epsq < tol_q) { status = OR_OK; break; }
  }

  for (long c = 0; c < ncell; ++c) T_out[c] = T[c];
  if (q_out) memcpy(q_out, q, sizeof(double) * ncell * dim);
  if (e_out) memcpy(e_out, e, sizeof(double) * (size_t)B * M * ncell);
  if (eb_out) memcpy(eb_out, eb, sizeof(double) * (size_t)B * bf.n);
  if (info) {
    info[0] = it;
    info[1] = epsT;
    info[2] = epsq;
    info[3] = (double)bf.n;
  }
  free(T); free(Tn); free(q); free(qn); free(e); free(eb); free(inv_half); free(es); free(mir);
  free_bfaces(&bf);
  return status;
}

/* Number of boundary faces of a geometry (for sizing eb_out). */
long oracle_count_bfaces(int dim, const int* n, const uint8_t* mask) {
  grid_t g;
  g.dim = dim;
  g.ncell = 1;
  for (int d = 0; d < 3; ++d) { g.n[d] = n[d]; g.h[d] = 1.0; g.ncell *= n[d]; }
  g.mask = mask;
  g.face_bc = NULL;
  bfaces_t bf;
  build_bfaces(&g, &bf);
  long r = bf.n;
  free_bfaces(&bf);
  return r;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
