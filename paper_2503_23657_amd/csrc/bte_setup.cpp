// Host-side problem set-up: validation, boundary tables, ordinate folding and
// grouping, group coefficients and the sweep schedule.
#include "bte_setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>

namespace bte {

static const double kPi = 3.14159265358979323846;

static std::string fmt(const char* f, double a = 0, double b = 0) {
  char buf[256];
  snprintf(buf, sizeof(buf), f, a, b);
  return buf;
}

std::string validate_problem(const bte_geometry* g, const bte_bands* b, const bte_quadrature* q) {
  if (!g || !b || !q) return "null geometry, bands or quadrature";
  if (g->dim < 1 || g->dim > 3) return fmt("dim must be 1, 2 or 3 (got %g)", g->dim);
  long long ncell = 1;
  for (int d = 0; d < 3; ++d) {
    if (g->n[d] < 1) return fmt("n[%g] must be >= 1", d);
    if (d >= g->dim && g->n[d] != 1) return fmt("n[%g] must be 1 for an unused axis", d);
    if (d < g->dim && !(g->h[d] > 0.0 && std::isfinite(g->h[d]))) return fmt("h[%g] must be > 0", d);
    ncell *= g->n[d];
  }
  if (ncell > (1ll << 30)) return "grid too large";
  if (g->n[0] > 65535) return "n[0] must be <= 65535";
  if (g->n_bc < 1 || g->n_bc > 255) return "n_bc must be in 1..255";
  if (!g->h_bc_kind || !g->h_bc_T) return "bc tables missing";
  for (int k = 0; k < g->n_bc; ++k) {
    if (g->h_bc_kind[k] != BTE_BC_ISOTHERMAL && g->h_bc_kind[k] != BTE_BC_DIFFUSE &&
        g->h_bc_kind[k] != BTE_BC_SPECULAR)
      return fmt("unknown bc kind %g", g->h_bc_kind[k]);
    if (!std::isfinite(g->h_bc_T[k])) return "non-finite wall temperature";
  }
  if (b->n_bands < 1 || !b->h_v || !b->h_tau || !b->h_C) return "band table missing";
  for (int i = 0; i < b->n_bands; ++i) {
    if (!(b->h_v[i] > 0 && std::isfinite(b->h_v[i]))) return fmt("v[%g] must be > 0", i);
    if (!(b->h_tau[i] > 0 && std::isfinite(b->h_tau[i]))) return fmt("tau[%g] must be > 0", i);
    if (!(b->h_C[i] > 0 && std::isfinite(b->h_C[i]))) return fmt("C[%g] must be > 0", i);
  }
  if (q->n_dirs < 1 || !q->h_s || !q->h_w) return "quadrature missing";
  double ws = 0.0;
  for (int a = 0; a < q->n_dirs; ++a) {
    const double* s = q->h_s + 3 * a;
    const double nn = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (!(std::fabs(nn - 1.0) <= 1e-12)) return fmt("direction %g is not a unit vector", a);
    if (!(q->h_w[a] > 0 && std::isfinite(q->h_w[a]))) return fmt("weight %g must be > 0", a);
    ws += q->h_w[a];
  }
  if (std::fabs(ws - 4.0 * kPi) > 1e-10 * 4.0 * kPi) return fmt("weights sum to %g, not 4 pi", ws);
  // closed under the reflection of each grid axis (same weight)
  for (int d = 0; d < g->dim; ++d) {
    for (int a = 0; a < q->n_dirs; ++a) {
      double r[3] = {q->h_s[3 * a], q->h_s[3 * a + 1], q->h_s[3 * a + 2]};
      r[d] = -r[d];
      bool found = false;
      for (int c = 0; c < q->n_dirs && !found; ++c) {
        const double* s = q->h_s + 3 * c;
        if (std::fabs(s[0] - r[0]) < 1e-12 && std::fabs(s[1] - r[1]) < 1e-12 &&
            std::fabs(s[2] - r[2]) < 1e-12 && std::fabs(q->h_w[c] - q->h_w[a]) <= 1e-12 * q->h_w[a])
          found = true;
      }
      if (!found) return fmt("quadrature not closed under reflection of axis %g", d);
    }
  }
  // geometry: active cells and boundary ids
  long long nact = 0;
  bool iso = false;
  const int n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
  for (long long c = 0; c < ncell; ++c) {
    if (g->h_mask && !g->h_mask[c]) continue;
    ++nact;
    const int i = (int)(c % n0), j = (int)((c / n0) % n1), k = (int)(c / ((long long)n0 * n1));
    for (int f = 0; f < 2 * g->dim; ++f) {
      int idx[3] = {i, j, k};
      const int d = f / 2;
      idx[d] += (f & 1) ? 1 : -1;
      bool bnd = idx[d] < 0 || idx[d] >= g->n[d];
      if (!bnd && g->h_mask) {
        const long long nb = idx[0] + (long long)n0 * (idx[1] + (long long)n1 * idx[2]);
        bnd = !g->h_mask[nb];
      }
      if (!bnd) continue;
      const int bc = g->h_face_bc ? g->h_face_bc[c * 6 + f] : 0;
      if (bc >= g->n_bc) return fmt("face_bc of cell %g face %g out of range", (double)c, f);
      if (g->h_bc_kind[bc] == BTE_BC_ISOTHERMAL) iso = true;
    }
  }
  if (nact == 0) return "no active cell";
  if (!iso) return "no isothermal boundary face: the steady state is not unique";
  return "";
}

void build_instance(const bte_geometry* g, HostInst& hi) {
  hi.dim = g->dim;
  for (int d = 0; d < 3; ++d) {
    hi.n[d] = g->n[d];
    hi.h[d] = d < g->dim ? g->h[d] : 1.0;
  }
  hi.ncell = g->n[0] * g->n[1] * g->n[2];
  hi.active.assign(hi.ncell, 1);
  if (g->h_mask)
    for (int c = 0; c < hi.ncell; ++c) hi.active[c] = g->h_mask[c] ? 1 : 0;
  hi.n_active = 0;
  for (int c = 0; c < hi.ncell; ++c) hi.n_active += hi.active[c];
  hi.bc_kind.assign(g->h_bc_kind, g->h_bc_kind + g->n_bc);
  hi.bc_T.assign(g->h_bc_T, g->h_bc_T + g->n_bc);
  hi.bslot.assign((size_t)hi.ncell * 6, -1);
  hi.bf_cell.clear();
  hi.bf_face.clear();
  hi.bf_bc.clear();
  hi.dface.clear();
  hi.sface.clear();
  hi.has_iso = false;
  const int n0 = hi.n[0], n1 = hi.n[1];
  for (int c = 0; c < hi.ncell; ++c) {
    if (!hi.active[c]) continue;
    const int i = c % n0, j = (c / n0) % n1, k = c / (n0 * n1);
    for (int f = 0; f < 2 * hi.dim; ++f) {
      int idx[3] = {i, j, k};
      const int d = f / 2;
      idx[d] += (f & 1) ? 1 : -1;
      bool bnd = idx[d] < 0 || idx[d] >= hi.n[d];
      if (!bnd) bnd = !hi.active[idx[0] + n0 * (idx[1] + n1 * idx[2])];
      if (!bnd) continue;
      const int bc = g->h_face_bc ? g->h_face_bc[(size_t)c * 6 + f] : 0;
      const int slot = (int)hi.bf_cell.size();
      hi.bslot[(size_t)c * 6 + f] = slot;
      hi.bf_cell.push_back(c);
      hi.bf_face.push_back(f);
      hi.bf_bc.push_back(bc);
      if (hi.bc_kind[bc] == BTE_BC_DIFFUSE) hi.dface.push_back(slot);
      else if (hi.bc_kind[bc] == BTE_BC_SPECULAR) hi.sface.push_back(slot);
      else hi.has_iso = true;
    }
  }
}

std::vector<Ordinate> fold_ordinates(const bte_quadrature* q, int dim) {
  std::vector<Ordinate> out;
  for (int a = 0; a < q->n_dirs; ++a) {
    const double* s = q->h_s + 3 * a;
    bool merged = false;
    if (dim < 3) {
      for (auto& o : out) {
        bool same = true;
        for (int d = 0; d < dim; ++d) same = same && std::fabs(o.s[d] - s[d]) < 1e-12;
        if (same) {
          o.w += q->h_w[a];
          merged = true;
          break;
        }
      }
    }
    if (merged) continue;
    Ordinate o;
    o.s[0] = s[0];
    o.s[1] = s[1];
    o.s[2] = s[2];
    for (int d = dim; d < 3; ++d) o.s[d] = 0.0;  // off-grid components do not transport
    o.w = q->h_w[a];
    o.oct = 0;
    for (int d = 0; d < dim; ++d)
      if (s[d] < 0.0) o.oct |= 1 << d;
    out.push_back(o);
  }
  return out;
}

GroupSet build_groups(const std::vector<Ordinate>& ords, int B, int dim, int G, int P) {
  GroupSet gs;
  gs.G = G;
  gs.P = P;
  const int n_oct = 1 << dim;
  gs.ob_first.assign(n_oct * B, 0);
  gs.ob_count.assign(n_oct * B, 0);
  for (int o = 0; o < n_oct; ++o) {
    std::vector<int> members;
    for (int a = 0; a < (int)ords.size(); ++a)
      if (ords[a].oct == o) members.push_back(a);
    if (members.empty()) continue;
    const int first_grp = (int)gs.band.size();
    for (int b = 0; b < B; ++b) {
      gs.ob_first[o * B + b] = (int)gs.band.size();
      for (size_t m = 0; m < members.size(); m += G) {
        gs.band.push_back(b);
        gs.oct.push_back(o);
        for (int g = 0; g < G; ++g)
          gs.ords.push_back(m + g < members.size() ? members[m + g] : -1);
        gs.ob_count[o * B + b]++;
      }
    }
    // bundles of P groups of this octant; pad with all-dummy groups
    int ng = (int)gs.band.size() - first_grp;
    while (ng % P) {
      gs.band.push_back(0);
      gs.oct.push_back(o);
      for (int g = 0; g < G; ++g) gs.ords.push_back(-1);
      ++ng;
    }
    for (int k = 0; k < ng; k += P) {
      gs.bundle_first.push_back(first_grp + k);
      gs.bundle_oct.push_back(o);
    }
  }
  return gs;
}

double half_range(const std::vector<Ordinate>& ords, int d) {
  double h = 0.0;
  for (const auto& o : ords)
    if (o.s[d] > 0.0) h += o.w * o.s[d];
  return h;
}

void group_coefficients(const GroupSet& gs, const std::vector<Ordinate>& ords, const HostInst& hi,
                        const std::vector<double>& v, const std::vector<double>& tau,
                        const std::vector<double>& Cb, double t0, bool adjoint,
                        std::vector<double>& out) {
  const int G = gs.G;
  const int GS = grp_stride(G);
  const int ngrp = (int)gs.band.size();
  out.assign((size_t)ngrp * GS, 0.0);
  double Csum = 0.0, D = 0.0;
  for (size_t b = 0; b < v.size(); ++b) {
    Csum += Cb[b];
    D += Cb[b] / tau[b];
  }
  const double gamma = t0 / Csum;
  for (int k = 0; k < ngrp; ++k) {
    double* r = out.data() + (size_t)k * GS;
    const int b = gs.band[k];
    const double rho = t0 / tau[b];
    // an ordinate that gives the dummy slots valid transport coefficients
    int ref = -1;
    for (int g = 0; g < G && ref < 0; ++g) ref = gs.ords[(size_t)k * G + g];
    if (ref < 0) {
      for (int a = 0; a < (int)ords.size(); ++a)
        if (ords[a].oct == gs.oct[k]) { ref = a; break; }
    }
    r[0] = adjoint ? 1.0 : rho;
    r[1] = adjoint ? 0.0 : gamma;
    for (int g = 0; g < G; ++g) {
      const int a = gs.ords[(size_t)k * G + g];
      const Ordinate& o = ords[a >= 0 ? a : ref];
      const double w = a >= 0 ? o.w : 0.0;
      double beta[3] = {0, 0, 0};
      double den = rho;
      for (int d = 0; d < hi.dim; ++d) {
        beta[d] = t0 * v[b] * std::fabs(o.s[d]) / hi.h[d];
        den += beta[d];
      }
      const double inv = 1.0 / den;
      for (int d = 0; d < 3; ++d) r[go_a(G, d) + g] = beta[d] * inv;
      r[go_den(G) + g] = den;
      r[go_inv(G) + g] = inv;
      // omega = w C_b / (4 pi tau_b D): weight of u in the new temperature
      const double omega = w * Cb[b] / (4.0 * kPi * tau[b] * D);
      if (!adjoint) {
        r[go_wacc(G, 0) + g] = omega * inv;
        for (int d = 0; d < hi.dim; ++d)
          r[go_wacc(G, 1 + d) + g] = v[b] * w * o.s[d] * Cb[b] * inv / (4.0 * kPi);
        for (int d = 0; d < hi.dim; ++d) r[go_wo(G, d) + g] = w * std::fabs(o.s[d]) * inv;
      } else {
        r[go_wacc(G, 0) + g] = rho * omega * inv;
        r[go_wacc(G, 1) + g] = gamma * omega * inv;
        r[go_wt(G, 0) + g] = omega * inv;
        r[go_wt(G, 1) + g] = omega;
        // outflow entries of the transposed sweep at reflecting walls: the
        // wall-value adjoint beta_d psi with psi = omega * inv * (sweep value)
        for (int d = 0; d < hi.dim; ++d) r[go_wo(G, d) + g] = beta[d] * omega * inv;
      }
    }
  }
}

// walls whose inflow is computed from the sweep's outflow (Eqs. 6 and 7)
static bool reflecting(int kind) { return kind == BTE_BC_DIFFUSE || kind == BTE_BC_SPECULAR; }

static int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// 1D/2D schedule of the rows-per-lane sweep. Lane l of wave slot r owns rows
// 64*NR*s + NR*l + k (k < NR) of strip s and processes column i of it at clock
// step t = s*du + l + i (strips r, r+R, ... belong to slot r). Positions of
// the (X, Q) layout: ((r*Tp + t)*64 + l)*NR + k with Tp = T + kPad2.
// Inflow entries: per step, lanes in order, rows k ascending, x before y.
// Outflow entries: per step, rows k ascending, axis x before y, lanes in order.
static bool build_schedule_2d(const HostInst& hi, const Plan& plan, Schedule& s, std::string& err) {
  const int NR = plan.NR, R = plan.R, C = kC2;
  if (NR != 1 && NR != 2 && NR != 4) {
    err = "plan NR must be 1, 2 or 4";
    return false;
  }
  const int dim = hi.dim;
  const int nx = hi.n[0], ny = dim >= 2 ? hi.n[1] : 1;
  const int H = 64 * NR;
  const int nS = (ny + H - 1) / H;
  const int V = nx;
  // strips start du steps apart: at least 63 + C (the previous strip's top
  // row reaches the ring a chunk before it is read) and, when a slot owns
  // several strips, long enough for its strips not to overlap (R*du >= V)
  const int du = nS > R ? std::max(63 + C, (V + R - 1) / R) : 63 + C;
  int T = (nS - 1) * du + V + 63;
  T = (T + C - 1) / C * C;
  const int Tp = T + kPad2;
  s.T = T;
  s.R = R;
  s.C = C;
  s.W = nx;
  s.NR = NR;
  s.du = du;
  s.nS = nS;
  s.lag = 0;
  s.ring = 0;
  s.n_oct = 1 << dim;
  s.pos_per_oct = (long long)R * Tp * 64 * NR;
  if (s.pos_per_oct * s.n_oct > (1ll << 31) - 1) {
    err = "schedule too large";
    return false;
  }
  const int n_oct = s.n_oct;
  const int nch = T / C;
  const int nbf = (int)hi.bf_cell.size();
  s.sched.assign((size_t)n_oct * R * Tp * 64, make_int2(-1, 0));
  s.pos.assign((size_t)n_oct * hi.ncell, -1);
  s.in_slot.clear();
  s.in_chunk.assign((size_t)n_oct * R * (nch + 1), 0);
  s.out_base.assign((size_t)n_oct * R, 0);
  s.ofk.assign((size_t)n_oct * std::max(nbf, 1), -1);
  s.pre_slot.assign((size_t)n_oct * nx, -1);
  s.e_max = 1;
  s.o_max = 1;
  int n_out_max = 1;
  // strip and column of slot r at lane-relative clock q; false when idle.
  // Slot r owns strips r, r+R, ...; strip s starts at s*du, so consecutive
  // strips of a slot start SP = R*du apart (SP unbounded when a slot owns one
  // strip at most)
  const long long SP = nS > R ? (long long)R * du : (1ll << 40);
  auto strip_at = [&](int r, int q, int& sidx, int& v) {
    const long long a = (long long)q - (long long)r * du;
    const long long m = a >= 0 ? a / SP : -((-a + SP - 1) / SP);
    sidx = (int)(r + m * R);
    if (sidx < 0) return false;
    v = q - sidx * du;
    return sidx < nS && v >= 0 && v < V;
  };
  std::vector<int> out_face(64 * NR * 2);
  for (int o = 0; o < n_oct; ++o) {
    const bool fx = o & 1, fy = (o >> 1) & 1;
    const int up[2] = {fx ? 1 : 0, fy ? 3 : 2};
    const int dn[2] = {fx ? 0 : 1, fy ? 2 : 3};
    int out_count = 0;
    for (int r = 0; r < R; ++r) {
      s.out_base[o * R + r] = out_count;
      int* chk = &s.in_chunk[((size_t)o * R + r) * (nch + 1)];
      int out_k = 0;
      for (int tau = 0; tau < T; ++tau) {
        if (tau % C == 0) chk[tau / C] = (int)s.in_slot.size();
        int sidx, v;
        std::fill(out_face.begin(), out_face.end(), -1);
        for (int l = 0; l < 64; ++l) {
          if (!strip_at(r, tau - l, sidx, v)) continue;
          const int ip = v;
          const int ix = fx ? nx - 1 - ip : ip;
          unsigned fl = 0;
          int cid0 = -1;
          const int in_first = (int)s.in_slot.size() - chk[tau / C];
          bool any_in = false;
          // a lane entering its strip at the x wall with no other inflow takes
          // its x-inflows as NR consecutive entries (F2_XSTART) instead of
          // per-row flags
          bool xstart = ip == 0;
          for (int k = 0; k < NR && xstart; ++k) {
            const int kp = sidx * H + l * NR + k;
            if (kp >= ny) break;
            const int iy = dim >= 2 ? (fy ? ny - 1 - kp : kp) : 0;
            const int cell = ix + nx * iy;
            if (!hi.active[cell]) continue;
            if (dim >= 2 && kp > 0 && hi.bslot[(size_t)cell * 6 + up[1]] >= 0) xstart = false;
          }
          if (xstart) {
            fl |= F2_XSTART;
            for (int k = 0; k < NR; ++k) {
              const int kp = sidx * H + l * NR + k;
              int su = -1;
              if (kp < ny) {
                const int iy = dim >= 2 ? (fy ? ny - 1 - kp : kp) : 0;
                const int cell = ix + nx * iy;
                if (hi.active[cell]) su = hi.bslot[(size_t)cell * 6 + up[0]];
              }
              s.in_slot.push_back(su);
            }
            any_in = true;
          }
          for (int k = 0; k < NR; ++k) {
            const int kp = sidx * H + l * NR + k;
            if (kp >= ny) break;
            const int iy = dim >= 2 ? (fy ? ny - 1 - kp : kp) : 0;
            const int cell = ix + nx * iy;
            if (k == 0) cid0 = cell;
            if (!hi.active[cell]) continue;
            const int sh = F2_ROW_BITS * k;
            fl |= F2_ACT << sh;
            s.pos[(size_t)o * hi.ncell + cell] = (int)((((long long)r * Tp + tau) * 64 + l) * NR + k);
            for (int d = 0; d < dim; ++d) {
              const int su = hi.bslot[(size_t)cell * 6 + up[d]];
              if (su < 0) continue;
              if (d == 0 && xstart) continue;  // taken as an F2_XSTART entry
              if (d == 1 && kp == 0) {
                // strip 0, lane 0, row 0: the lane-0 ghost is prefilled with this face
                s.pre_slot[(size_t)o * nx + ip] = su;
              } else {
                fl |= (F2_INX << d) << sh;
                s.in_slot.push_back(su);
                any_in = true;
              }
            }
            for (int d = 0; d < dim; ++d) {
              const int sd = hi.bslot[(size_t)cell * 6 + dn[d]];
              if (sd >= 0 && reflecting(hi.bc_kind[hi.bf_bc[sd]])) {
                fl |= (F2_OUTX << d) << sh;
                out_face[(k * 2 + d) * 64 + l] = sd;
              }
            }
          }
          if (any_in) {
            if (in_first > (int)F2_INOFF_MASK) {
              err = "too many boundary inflows per chunk";
              return false;
            }
            fl |= (unsigned)in_first << F2_INOFF_SHIFT;
          }
          // rows of the lane inside the grid (their partial sums are written;
          // inactive cells' entries are ignored downstream)
          int gm = 0;
          for (int k = 0; k < NR; ++k)
            if (sidx * H + l * NR + k < ny) gm |= 1 << k;
          const int full = gm == (1 << NR) - 1 ? 16 : 0;
          s.sched[(((size_t)o * R + r) * Tp + tau) * 64 + l] = make_int2(cid0 >= 0 ? (cid0 << 5) | full | gm : -1, (int)fl);
        }
        for (int kd = 0; kd < NR * 2; ++kd)
          for (int l = 0; l < 64; ++l) {
            const int sd = out_face[kd * 64 + l];
            if (sd < 0) continue;
            s.ofk[(size_t)o * nbf + sd] = out_count + out_k;
            ++out_k;
          }
      }
      chk[nch] = (int)s.in_slot.size();
      for (int ch = 0; ch < nch; ++ch) s.e_max = std::max(s.e_max, chk[ch + 1] - chk[ch]);
      out_count += out_k;
    }
    n_out_max = std::max(n_out_max, out_count);
  }
  for (int o = 0; o < n_oct; ++o)
    for (int r = 0; r < R; ++r)
      for (int ch = 0; ch < nch; ++ch) {
        int cnt = 0;
        for (int tau = ch * C; tau < (ch + 1) * C; ++tau)
          for (int l = 0; l < 64; ++l) {
            const unsigned fl = (unsigned)s.sched[(((size_t)o * R + r) * Tp + tau) * 64 + l].y;
            for (int k = 0; k < NR; ++k) {
              const unsigned b = fl >> (F2_ROW_BITS * k);
              cnt += ((b & F2_OUTX) != 0) + ((b & F2_OUTY) != 0);
            }
          }
        s.o_max = std::max(s.o_max, cnt);
      }
  s.n_out_stride = n_out_max;
  if (s.e_max > 256) {
    err = "too many boundary inflows per chunk";
    return false;
  }
  if (s.o_max > 256) {
    err = "too many diffuse-wall outflows per chunk";
    return false;
  }
  // per-chunk flags (one padding row: the kernel reads a chunk ahead)
  s.chunk_fl.assign((size_t)n_oct * R * (nch + 1), 0);
  {
    const unsigned in_up = [&] {
      unsigned m = 0;
      for (int k = 1; k < NR; ++k) m |= F2_INY << (F2_ROW_BITS * k);
      return m;
    }();
    unsigned in_all = 0, out_all = 0;
    for (int k = 0; k < NR; ++k) {
      in_all |= (F2_INX | F2_INY) << (F2_ROW_BITS * k);
      out_all |= (F2_OUTX | F2_OUTY) << (F2_ROW_BITS * k);
    }
    for (int o = 0; o < n_oct; ++o)
      for (int r = 0; r < R; ++r)
        for (int ch = 0; ch < nch; ++ch) {
          int cf = 0;
          for (int tau = ch * C; tau < (ch + 1) * C; ++tau)
            for (int l = 0; l < 64; ++l) {
              const unsigned fl = (unsigned)s.sched[(((size_t)o * R + r) * Tp + tau) * 64 + l].y;
              if (fl & in_all) cf |= CF2_IN;
              if (fl & in_up) cf |= CF2_INY_UP;
              if (fl & out_all) cf |= CF2_OUT;
              if (fl & F2_XSTART) cf |= CF2_XST;
            }
          s.chunk_fl[((size_t)o * R + r) * (nch + 1) + ch] = cf;
        }
  }
  // per-chunk inflow table, two padding chunk rows at the end of every slot
  s.in_E = std::max(64, (s.e_max + 63) / 64 * 64);
  s.in_tab.assign((size_t)n_oct * R * (nch + 2) * s.in_E, -1);
  for (int o = 0; o < n_oct; ++o)
    for (int r = 0; r < R; ++r) {
      const int* chk = &s.in_chunk[((size_t)o * R + r) * (nch + 1)];
      for (int ch = 0; ch < nch; ++ch)
        for (int e = chk[ch]; e < chk[ch + 1]; ++e)
          s.in_tab[(((size_t)o * R + r) * (nch + 2) + ch) * s.in_E + (e - chk[ch])] = s.in_slot[e];
    }
  if ((long long)hi.ncell >= (1ll << 26)) {
    err = "too many cells for the 1D/2D sweep (limit 2^26)";
    return false;
  }
  for (int o = 0; o < n_oct; ++o)
    for (int c = 0; c < hi.ncell; ++c)
      if (hi.active[c] && s.pos[(size_t)o * hi.ncell + c] < 0) {
        err = "internal: cell missing from the schedule";
        return false;
      }
  return true;
}

// 3D rows-per-lane schedule for one choice of the lane and plane axes (the
// step axis is x, so that consecutive steps of a lane are consecutive cells).
// The step axis is cut into blocks of C = kC2 columns. Every lane runs
// through the same sequence of positions: block after block, in a block the
// planes from the first to the last that hold an active cell of the block (in
// sweep order), in a plane the block's C columns; lane l takes position
// s = t - l at clock step t (s = q*C + c: plane period q, column c; the period
// table ptab gives the plane of each period). So lane l works on the cell lane
// l-1 had one step before (the lane-axis link), its plane-axis upwind cell is
// its own position s - C (the value it computed C steps earlier, kept in
// registers; at a block's first plane that cell is inactive or outside, and
// the inflow is a stream entry) and, inside a block, its step-axis upwind
// cell is position s - 1. The first column of a block takes the step-axis
// value of the previous block's last column in the same plane, which every
// lane keeps per plane in a buffer of its own (a plane the previous block
// skipped left no value there: its cells are inactive, so the inflow is a
// stream entry); for the first block that buffer is prefilled with the wall
// faces of xpre. Lane 0's row 0 takes
// the lane-axis wall face of gpre at each step (stored as slot + 1, 0: none).
// Every other boundary value (the first plane's walls included) is an entry
// of the inflow stream, in order per step: lanes, rows ascending, step / lane
// / plane axis. Outflow entries, per step: rows, axes, lanes; the kernel
// emits a chunk's entries after the chunk from its staged values, as listed in
// out_tab. Positions: (t*64 + l)*NR + k.
static bool build_3r_axes(const HostInst& hi, int A0, int A1, int A2, const Plan& plan, Schedule& s,
                          std::string& err) {
  const int C = kC2;
  const int n0 = hi.n[A0], n1 = hi.n[A1], n2 = hi.n[A2];
  const int NR = std::max(std::min(plan.NR, 2), n1 <= 64 ? 1 : 2);
  if (n1 > 128) {
    err = "lane axis longer than 128 cells";
    return false;
  }
  if (n2 < 4) {
    // the step-axis buffer of a plane is written back at least three plane
    // periods before it is read again
    err = "fewer than 4 planes";
    return false;
  }
  const int nb = (n0 + C - 1) / C;
  const int stride[3] = {1, hi.n[0], hi.n[0] * hi.n[1]};
  const int ax[3] = {A0, A1, A2};
  // per octant and block (sweep orientation): the planes it streams
  std::vector<int> blo((size_t)8 * nb), bhi((size_t)8 * nb);
  int n_per = 0;
  for (int o = 0; o < 8; ++o) {
    const bool f0 = (o >> A0) & 1, f2 = (o >> A2) & 1;
    int np = 0;
    for (int b = 0; b < nb; ++b) {
      int lo = n2, hi_ = -1;
      for (int v = b * C; v < std::min(n0, b * C + C); ++v)
        for (int p = 0; p < n2; ++p)
          for (int j = 0; j < n1; ++j) {
            const int g0 = f0 ? n0 - 1 - v : v;
            if (!hi.active[(size_t)g0 * stride[A0] + (size_t)j * stride[A1] + (size_t)p * stride[A2]]) continue;
            const int ps = f2 ? n2 - 1 - p : p;
            lo = std::min(lo, ps);
            hi_ = std::max(hi_, ps);
          }
      blo[(size_t)o * nb + b] = lo;
      bhi[(size_t)o * nb + b] = hi_;
    }
    // a plane two consecutive blocks share is stored by the first (at the end
    // of its period's chunk) at least 3 periods before the second loads it
    // (a chunk ahead): widen ranges that overlap by fewer planes
    for (int b = 0; b + 1 < nb; ++b) {
      int& h0 = bhi[(size_t)o * nb + b];
      int& l1 = blo[(size_t)o * nb + b + 1];
      if (h0 < 0 || l1 >= n2) continue;
      while (h0 - l1 + 1 >= 1 && h0 - l1 + 1 < 3) {
        if (h0 < n2 - 1)
          ++h0;
        else
          --l1;
      }
    }
    for (int b = 0; b < nb; ++b) {
      const int lo = blo[(size_t)o * nb + b], hi_ = bhi[(size_t)o * nb + b];
      np += hi_ >= lo ? hi_ - lo + 1 : 0;
    }
    n_per = std::max(n_per, np);
  }
  const int T = n_per * C + 64;  // the last lane ends 63 steps after lane 0 (rounded to whole chunks)
  const int Tp = T + kPad2;
  s = Schedule();
  s.l3r = true;
  s.ax[0] = A0;
  s.ax[1] = A1;
  s.ax[2] = A2;
  s.T = T;
  s.R = 1;
  s.C = C;
  s.W = nb * C;
  s.NR = NR;
  s.du = 0;
  s.nS = 1;
  s.lag = 0;
  s.ring = 0;
  s.n_pl = n2;
  s.n_per = n_per;
  s.n_oct = 8;
  s.pos_per_oct = (long long)Tp * 64 * NR;
  if (s.pos_per_oct * s.n_oct > (1ll << 31) - 1) {
    err = "schedule too large";
    return false;
  }
  if ((long long)hi.ncell >= (1ll << 26)) {
    err = "too many cells for the rows-per-lane sweep (limit 2^26)";
    return false;
  }
  const int n_oct = 8, nch = T / C, nbf = (int)hi.bf_cell.size();
  const int H = 64 * NR;
  s.sched.assign((size_t)n_oct * Tp * 64, make_int2(-1, 0));
  s.pos.assign((size_t)n_oct * hi.ncell, -1);
  s.in_slot.clear();
  s.in_chunk.assign((size_t)n_oct * (nch + 1), 0);
  s.out_base.assign(n_oct, 0);
  s.ofk.assign((size_t)n_oct * std::max(nbf, 1), -1);
  s.xpre.assign((size_t)n_oct * n2 * H, -1);
  s.gpre.assign((size_t)n_oct * (T + n_per), 0);
  s.e_max = 1;
  s.o_max = 1;
  // period -> (block, plane) of each octant; the plane + 1 also goes to the
  // period table after the octant's gpre row
  std::vector<int> per_b((size_t)n_oct * n_per, -1), per_p((size_t)n_oct * n_per, -1);
  for (int o = 0; o < n_oct; ++o) {
    int q = 0;
    for (int b = 0; b < nb; ++b)
      for (int p = blo[(size_t)o * nb + b]; p <= bhi[(size_t)o * nb + b]; ++p, ++q) {
        per_b[(size_t)o * n_per + q] = b;
        per_p[(size_t)o * n_per + q] = p;
        s.gpre[(size_t)o * (T + n_per) + T + q] = p + 1;
      }
  }
  std::vector<int> out_face((size_t)NR * 3 * 64);
  std::vector<int> out_count(n_oct, 0);
  std::vector<std::vector<int>> out_ent(n_oct);
  s.out_chunk.assign((size_t)n_oct * (nch + 1), 0);
  for (int o = 0; o < n_oct; ++o) {
    int* chk = &s.in_chunk[(size_t)o * (nch + 1)];
    int* och = &s.out_chunk[(size_t)o * (nch + 1)];
    bool flip[3];
    int up[3], dn[3];
    for (int e = 0; e < 3; ++e) {
      flip[e] = (o >> ax[e]) & 1;
      up[e] = 2 * ax[e] + (flip[e] ? 1 : 0);
      dn[e] = 2 * ax[e] + (flip[e] ? 0 : 1);
    }
    int out_k = 0;
    for (int t = 0; t < T; ++t) {
      if (t % C == 0) chk[t / C] = (int)s.in_slot.size();
      std::fill(out_face.begin(), out_face.end(), -1);
      for (int l = 0; l < 64; ++l) {
        const int q = t - l;
        if (q < 0 || q >= n_per * C) continue;
        const int per = q / C, c = q % C;
        const int bk = per_b[(size_t)o * n_per + per], pl = per_p[(size_t)o * n_per + per];
        if (bk < 0) continue;  // past this octant's periods
        const int v = bk * C + c;
        if (v >= n0) continue;
        const int in_first = (int)s.in_slot.size() - chk[t / C];
        bool any_in = false;
        unsigned fl = 0;
        int cid0 = -1, gm = 0;
        for (int k = 0; k < NR; ++k) {
          const int jp = l * NR + k;
          if (jp >= n1) break;
          gm |= 1 << k;
          int co[3];
          co[0] = flip[0] ? n0 - 1 - v : v;
          co[1] = flip[1] ? n1 - 1 - jp : jp;
          co[2] = flip[2] ? n2 - 1 - pl : pl;
          int cell = 0;
          for (int e = 0; e < 3; ++e) cell += co[e] * stride[ax[e]];
          if (k == 0) cid0 = cell;
          if (!hi.active[cell]) continue;
          const int sh = F3_ROW_BITS * k;
          fl |= F3_ACT << sh;
          s.pos[(size_t)o * hi.ncell + cell] = (int)(((long long)t * 64 + l) * NR + k);
          for (int e = 0; e < 3; ++e) {
            const int su = hi.bslot[(size_t)cell * 6 + up[e]];
            if (su < 0) continue;
            if (e == 0 && v == 0) {
              s.xpre[((size_t)o * n2 + pl) * H + jp] = su;
            } else if (e == 1 && jp == 0) {
              s.gpre[(size_t)o * (T + n_per) + t] = su + 1;
            } else {
              fl |= (F3_INX << e) << sh;
              s.in_slot.push_back(su);
              any_in = true;
            }
          }
          for (int e = 0; e < 3; ++e) {
            const int sd = hi.bslot[(size_t)cell * 6 + dn[e]];
            if (sd < 0 || !reflecting(hi.bc_kind[hi.bf_bc[sd]])) continue;
            fl |= (F3_OUTX << e) << sh;
            out_face[((size_t)k * 3 + e) * 64 + l] = sd;
          }
        }
        if (any_in) {
          if (in_first > (int)F2_INOFF_MASK) {
            err = "too many boundary inflows per chunk";
            return false;
          }
          fl |= (unsigned)in_first << F2_INOFF_SHIFT;
        }
        const int full = gm == (1 << NR) - 1 ? 16 : 0;
        s.sched[((size_t)o * Tp + t) * 64 + l] = make_int2(cid0 >= 0 ? (cid0 << 5) | full | gm : -1, (int)fl);
      }
      if (t % C == 0) och[t / C] = out_k;
      for (int kd = 0; kd < NR * 3; ++kd)
        for (int l = 0; l < 64; ++l) {
          const int sd = out_face[(size_t)kd * 64 + l];
          if (sd < 0) continue;
          s.ofk[(size_t)o * nbf + sd] = out_k++;
          const int k = kd / 3, e = kd % 3;
          out_ent[o].push_back((((((t % C) * 64 + l) * NR + k) << 2) | e) + 1);
        }
    }
    och[nch] = out_k;
    chk[nch] = (int)s.in_slot.size();
    for (int ch = 0; ch < nch; ++ch) s.e_max = std::max(s.e_max, chk[ch + 1] - chk[ch]);
    out_count[o] = out_k;
  }
  int n_stream = 1;
  for (int o = 0; o < n_oct; ++o) n_stream = std::max(n_stream, out_count[o]);
  s.n_out_stride = n_stream;
  // per-chunk flags (inflow entries only: the outflows leave after the chunk)
  s.chunk_fl.assign((size_t)n_oct * (nch + 1), 0);
  unsigned in_all = 0;
  for (int k = 0; k < NR; ++k) in_all |= (F3_INX | F3_INY | F3_INZ) << (F3_ROW_BITS * k);
  for (int o = 0; o < n_oct; ++o)
    for (int ch = 0; ch < nch; ++ch) {
      int cf = 0;
      for (int t = ch * C; t < (ch + 1) * C; ++t)
        for (int l = 0; l < 64; ++l) {
          const unsigned fl = (unsigned)s.sched[((size_t)o * Tp + t) * 64 + l].y;
          if (fl & in_all) cf |= CF2_IN | CF2_INY_UP;
        }
      const int* och = &s.out_chunk[(size_t)o * (nch + 1)];
      s.o_max = std::max(s.o_max, och[ch + 1] - och[ch]);
      s.chunk_fl[(size_t)o * (nch + 1) + ch] = cf;
    }
  if (s.e_max > 256) {
    err = "too many boundary inflows per chunk";
    return false;
  }
  if (s.o_max > 256) {
    err = "too many reflecting-wall outflows per chunk";
    return false;
  }
  s.in_E = std::max(64, (s.e_max + 63) / 64 * 64);
  s.in_tab.assign((size_t)n_oct * (nch + 2) * s.in_E, -1);
  for (int o = 0; o < n_oct; ++o) {
    const int* chk = &s.in_chunk[(size_t)o * (nch + 1)];
    for (int ch = 0; ch < nch; ++ch)
      for (int e = chk[ch]; e < chk[ch + 1]; ++e)
        s.in_tab[((size_t)o * (nch + 2) + ch) * s.in_E + (e - chk[ch])] = s.in_slot[e];
  }
  s.out_E = std::max(64, (s.o_max + 63) / 64 * 64);
  s.out_tab.assign((size_t)n_oct * (nch + 2) * s.out_E, 0);
  for (int o = 0; o < n_oct; ++o) {
    const int* och = &s.out_chunk[(size_t)o * (nch + 1)];
    for (int ch = 0; ch < nch; ++ch)
      for (int e = och[ch]; e < och[ch + 1]; ++e)
        s.out_tab[((size_t)o * (nch + 2) + ch) * s.out_E + (e - och[ch])] = out_ent[o][e];
  }
  for (int o = 0; o < n_oct; ++o)
    for (int c = 0; c < hi.ncell; ++c)
      if (hi.active[c] && s.pos[(size_t)o * hi.ncell + c] < 0) {
        err = "internal: cell missing from the schedule";
        return false;
      }
  return true;
}

// relative cost of a 3D rows-per-lane schedule: its chunks, a chunk with
// inflow entries (they run the slow path) counting twice
static double cost_3r(const Schedule& s) {
  const int nch = s.T / s.C;
  double c = 0.0;
  for (int o = 0; o < s.n_oct; ++o)
    for (int ch = 0; ch < nch; ++ch) c += (s.chunk_fl[(size_t)o * (nch + 1) + ch] & CF2_IN) ? 2.0 : 1.0;
  return c;
}

bool build_schedule_3r(const HostInst& hi, const Plan& plan, Schedule& s, std::string& err) {
  if (hi.dim != 3) {
    err = "the rows-per-lane 3D layout needs a 3D problem";
    return false;
  }
  // every assignment of the grid axes to the step, lane and plane axes whose
  // lane axis fits 128 cells; the cheapest schedule wins
  static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  double best = -1.0;
  std::string e1;
  for (const auto& pm : perm) {
    if (hi.n[pm[1]] > 128) continue;
    Schedule cand;
    std::string e;
    if (!build_3r_axes(hi, pm[0], pm[1], pm[2], plan, cand, e)) {
      if (e1.empty()) e1 = e;
      continue;
    }
    const double c = cost_3r(cand);
    if (best < 0.0 || c < best) {
      best = c;
      s = std::move(cand);
    }
  }
  if (best >= 0.0) return true;
  err = e1.empty() ? "no lane axis of at most 128 cells" : e1;
  return false;
}

bool build_schedule(const HostInst& hi, const Plan& plan, Schedule& s, std::string& err) {
  if (hi.dim < 3) return build_schedule_2d(hi, plan, s, err);
  if (plan.NR >= 1) {
    std::string e3;
    if (build_schedule_3r(hi, plan, s, e3)) return true;
  }
  s = Schedule();
  const bool L3 = hi.dim == 3;
  const int LJ = L3 ? 8 : 1, LK = L3 ? 8 : 64;
  const int R = L3 ? 1 : plan.R;
  const int C = plan.C;
  const int nx = hi.n[0];
  const int nJc = L3 ? hi.n[1] : 1;            // cells along kernel j
  const int nKc = L3 ? hi.n[2] : hi.n[1];      // cells along kernel k
  const int W = L3 ? std::max(nx, 8) : nx;
  const int nJB = (nJc + LJ - 1) / LJ;
  const int nS = (nKc + LK - 1) / LK;
  const int V = nJB * W;
  int du;
  if (R == 1) du = std::max(V, LK);
  else du = std::max(LK - 1 + C, (V + R - 1) / R);
  int T = (nS - 1) * du + V + (LJ - 1) + (LK - 1) + 1;
  T = (T + C - 1) / C * C;
  s.T = T;
  s.R = R;
  s.C = C;
  s.W = W;
  s.n_oct = 1 << hi.dim;
  s.lag = L3 ? du - (LK - 1) : 0;
  s.ring = L3 ? next_pow2(s.lag + C + 16 + 8) : 0;
  // padded by kPad2 steps so that the kernel's prefetch needs no condition
  const int Tp = T + kPad2;
  s.pos_per_oct = (long long)R * Tp * 64;
  const long long npos = s.pos_per_oct * s.n_oct;
  if (npos > (1ll << 31) - 1) {
    err = "schedule too large";
    return false;
  }
  s.sched.assign(npos, make_int2(-1, 0));
  s.pos.assign((size_t)s.n_oct * hi.ncell, -1);
  s.in_slot.clear();
  const int nch = T / C;
  s.in_chunk.assign((size_t)s.n_oct * R * (nch + 1), 0);
  s.out_base.assign((size_t)s.n_oct * R, 0);
  const int nbf = (int)hi.bf_cell.size();
  s.ofk.assign((size_t)s.n_oct * std::max(nbf, 1), -1);
  s.pre_slot.assign((size_t)s.n_oct * (L3 ? 1 : W), -1);
  s.e_max = 1;
  s.o_max = 1;
  int n_out_max = 1;
  const int n0 = hi.n[0], n1 = hi.n[1];
  for (int o = 0; o < s.n_oct; ++o) {
    const bool fx = o & 1, fy = (o >> 1) & 1, fz = (o >> 2) & 1;
    // upwind / downwind physical faces per axis for this octant
    const int up[3] = {fx ? 1 : 0, fy ? 3 : 2, fz ? 5 : 4};
    const int dn[3] = {fx ? 0 : 1, fy ? 2 : 3, fz ? 4 : 5};
    int out_count = 0;
    for (int r = 0; r < R; ++r) {
      s.out_base[o * R + r] = out_count;
      int* chk = &s.in_chunk[((size_t)o * R + r) * (nch + 1)];
      int out_k = 0;
      for (int tau = 0; tau < T; ++tau) {
        if (tau % C == 0) chk[tau / C] = (int)s.in_slot.size();
        int chunk_in = 0, chunk_out = 0;
        (void)chunk_in;
        (void)chunk_out;
        for (int l = 0; l < 64; ++l) {
          const int jl = L3 ? (l & 7) : 0, kl = L3 ? (l >> 3) : l;
          // which strip / virtual column does lane l of slot r process at tau?
          int sidx = -1, v = -1;
          if (R == 1) {
            const int q = tau - jl - kl;
            if (q >= 0) {
              sidx = q / du;
              v = q - sidx * du;
            }
          } else {
            // strips r, r+R, ... start at s*du
            const int q = tau - jl - kl;
            if (q >= 0) {
              int m = q / du;  // candidate strip index
              // the strip of slot r with start <= q: s = largest s = r mod R with s*du <= q
              int sc = m - ((m - r) % R + R) % R;
              if (sc >= 0) {
                sidx = sc;
                v = q - sc * du;
              }
            }
          }
          if (sidx < 0 || sidx >= nS || v < 0 || v >= V) continue;
          const int J = v / W, ip = v - J * W;
          if (ip >= nx) continue;
          const int jp = J * LJ + jl, kp = sidx * LK + kl;
          if (jp >= nJc || kp >= nKc) continue;
          // physical cell
          int ix = fx ? nx - 1 - ip : ip;
          int iy, iz;
          if (L3) {
            iy = fy ? hi.n[1] - 1 - jp : jp;
            iz = fz ? hi.n[2] - 1 - kp : kp;
          } else {
            iy = fy ? hi.n[1] - 1 - kp : kp;
            iz = 0;
          }
          const int cell = ix + n0 * (iy + n1 * iz);
          const long long pidx = ((long long)o * R + r) * Tp * 64 + (long long)tau * 64 + l;
          unsigned fl = (unsigned)ip << F_COL_SHIFT;
          if (hi.active[cell]) {
            fl |= F_ACTIVE;
            s.pos[(size_t)o * hi.ncell + cell] = (int)(((long long)r * Tp + tau) * 64 + l);
            for (int d = 0; d < hi.dim; ++d) {
              const int su = hi.bslot[(size_t)cell * 6 + up[d]];
              if (su >= 0) {
                // 2D: the first strip's lane-0 k-ghost is prefilled from pre_slot
                if (!L3 && d == 1 && kp == 0) {
                  s.pre_slot[(size_t)o * W + ip] = su;
                } else {
                  fl |= F_IN_X << d;
                  s.in_slot.push_back(su);
                }
              }
            }
            for (int d = 0; d < hi.dim; ++d) {
              const int sd = hi.bslot[(size_t)cell * 6 + dn[d]];
              if (sd >= 0 && reflecting(hi.bc_kind[hi.bf_bc[sd]])) {
                fl |= F_OUT_X << d;
                s.ofk[(size_t)o * nbf + sd] = out_count + out_k;
                ++out_k;
              }
            }
          }
          s.sched[pidx] = make_int2(cell, (int)fl);
        }
      }
      chk[nch] = (int)s.in_slot.size();
      for (int ch = 0; ch < nch; ++ch) s.e_max = std::max(s.e_max, chk[ch + 1] - chk[ch]);
      out_count += out_k;
    }
    n_out_max = std::max(n_out_max, out_count);
  }
  // maximum outflow entries of one slot in one chunk
  for (int o = 0; o < s.n_oct; ++o)
    for (int r = 0; r < R; ++r)
      for (int ch = 0; ch < nch; ++ch) {
        int cnt = 0;
        for (int tau = ch * C; tau < (ch + 1) * C; ++tau)
          for (int l = 0; l < 64; ++l) {
            const unsigned fl = (unsigned)s.sched[((long long)o * R + r) * Tp * 64 + (long long)tau * 64 + l].y;
            cnt += ((fl & F_OUT_X) != 0) + ((fl & F_OUT_Y) != 0) + ((fl & F_OUT_Z) != 0);
          }
        s.o_max = std::max(s.o_max, cnt);
      }
  s.n_out_stride = n_out_max;
  if (s.e_max > 256) {
    err = "too many boundary inflows per chunk: use a smaller C";
    return false;
  }
  // every active cell must be scheduled exactly once per octant
  for (int o = 0; o < s.n_oct; ++o)
    for (int c = 0; c < hi.ncell; ++c)
      if (hi.active[c] && s.pos[(size_t)o * hi.ncell + c] < 0) {
        err = "internal: cell missing from the schedule";
        return false;
      }
  return true;
}

std::vector<int> corr_stencil(const HostInst& hi, const Schedule& s) {
  const int dim = hi.dim, W = 3 * dim;
  const long long ppo = s.pos_per_oct;
  std::vector<int> out((size_t)s.n_oct * ppo * W, kNoCell);
  const int st[3] = {1, hi.n[0], hi.n[0] * hi.n[1]};
  for (int o = 0; o < s.n_oct; ++o) {
    const int* pos = s.pos.data() + (size_t)o * hi.ncell;
    for (int c = 0; c < hi.ncell; ++c) {
      if (!hi.active[c] || pos[c] < 0) continue;
      const int q[3] = {c % hi.n[0], (c / hi.n[0]) % hi.n[1], c / (hi.n[0] * hi.n[1])};
      int* e = out.data() + ((size_t)o * ppo + pos[c]) * W;
      for (int d = 0; d < dim; ++d) {
        const int sg = ((o >> d) & 1) ? -1 : 1;  // the ordinate's direction along d
        // cell x's neighbour at distance k*sg along d (x's coordinate along d
        // is qd), as a position, or the face code when that face is a boundary
        auto code = [&](int x, int qd, int k) {
          const int y = qd + k * sg;
          const int f = 2 * d + ((k * sg) > 0 ? 1 : 0);
          if (y >= 0 && y < hi.n[d] && hi.active[x + k * sg * st[d]]) return pos[x + k * sg * st[d]];
          const int slot = hi.bslot[(size_t)x * 6 + f];
          // only an upwind face is an inflow face
          if (k < 0 && slot >= 0 && hi.bc_kind[hi.bf_bc[slot]] == BTE_BC_ISOTHERMAL) return -(2 + slot);
          return -1;
        };
        e[3 * d] = code(c, q[d], 1);
        e[3 * d + 1] = code(c, q[d], -1);
        e[3 * d + 2] = e[3 * d + 1] >= 0 ? code(c - sg * st[d], q[d] - sg, -1) : -1;
      }
    }
  }
  return out;
}

}  // namespace bte
