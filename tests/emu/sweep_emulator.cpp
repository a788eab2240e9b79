// CPU emulation of the sweep kernels' data flow (1D/2D and 3D layouts) driven by
// the library's own host-side schedule builder, inflow/outflow stream ordering
// and group coefficient tables (bte_setup.cpp), in FP64. Used by the CPU test
// suite to check that host logic against the oracle without a GPU: it mirrors
// what each lane reads (own previous value, the lane below, the previous strip's
// ring, the boundary stream) at each clock step of the schedule.
// Usage: sweep_emulator problem.bin [dJdT.bin | --order2]
//   prints T after n iterations, or, with dJ/dT, the adjoint gradients;
//   --order2: second-order faces (deferred correction, rows layouts, G = 1).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../paper_2503_23657_amd/csrc/bte_setup.h"
#include "../../paper_2503_23657_amd/csrc/bte_strips.h"

using namespace bte;

int main(int argc, char** argv) {
  FILE* fp = fopen(argv[1], "rb");
  int hdr[8];
  fread(hdr, 4, 8, fp);
  int dim = hdr[0], n0 = hdr[1], n1 = hdr[2], n2 = hdr[3], B = hdr[4], M = hdr[5], nbc = hdr[6], iters = hdr[7];
  double h[3];
  fread(h, 8, 3, fp);
  int G = 2, R = 2, P = 1, Cc = 16, NR = 1;
  int pl[5];
  fread(pl, 4, 5, fp);
  G = pl[0]; R = pl[1]; P = pl[2]; Cc = pl[3]; NR = pl[4];
  int ncell = n0 * n1 * n2;
  std::vector<uint8_t> mask(ncell), fbc(ncell * 6);
  fread(mask.data(), 1, ncell, fp);
  fread(fbc.data(), 1, ncell * 6, fp);
  std::vector<int> bck(nbc);
  std::vector<double> bcT(nbc), v(B), tau(B), C(B), s(3 * M), w(M), Q(ncell);
  fread(bck.data(), 4, nbc, fp);
  fread(bcT.data(), 8, nbc, fp);
  fread(v.data(), 8, B, fp);
  fread(tau.data(), 8, B, fp);
  fread(C.data(), 8, B, fp);
  fread(s.data(), 8, 3 * M, fp);
  fread(w.data(), 8, M, fp);
  fread(Q.data(), 8, ncell, fp);
  double Tref;
  fread(&Tref, 8, 1, fp);
  fclose(fp);
  bte_geometry g{};
  g.dim = dim; g.n[0] = n0; g.n[1] = n1; g.n[2] = n2; g.h[0] = h[0]; g.h[1] = h[1]; g.h[2] = h[2];
  g.h_mask = mask.data(); g.h_face_bc = fbc.data(); g.n_bc = nbc; g.h_bc_kind = bck.data(); g.h_bc_T = bcT.data();
  bte_bands bb{B, v.data(), tau.data(), C.data()};
  bte_quadrature qq{M, s.data(), w.data()};
  std::string e = validate_problem(&g, &bb, &qq);
  if (!e.empty()) { printf("invalid %s\n", e.c_str()); return 1; }
  HostInst hi;
  build_instance(&g, hi);
  auto ords = fold_ordinates(&qq, dim);
  Plan plan{G, R, P, Cc, NR};
  if (dim == 3) plan.R = 1;
  if (dim == 3 && NR == 0) plan.C = Cc;
  if (dim < 3) plan.C = Cc = kC2;
  Schedule S;
  std::string err;
  if (!build_schedule(hi, plan, S, err)) { printf("sched %s\n", err.c_str()); return 1; }
  GroupSet gs = build_groups(ords, B, dim, G, P);
  double t0 = tau[0];
  for (double t : tau) t0 = std::min(t0, t);
  std::vector<double> coef;
  group_coefficients(gs, ords, hi, v, tau, C, t0, false, coef);
  const int GS = grp_stride(G);
  const bool L3 = dim == 3;
  const int LJ = L3 ? 8 : 1, LK = L3 ? 8 : 64;
  const int nbf = (int)hi.bf_cell.size();
  // state
  std::vector<double> X(ncell, 0.0);
  // inflow table: one row per band, or per (band, ordinate) with specular walls
  const bool has_spec = !hi.sface.empty();
  const int Mf = (int)ords.size();
  const int rows = has_spec ? Mf : 1;
  if (has_spec && G != 1) { printf("specular walls need G = 1\n"); return 1; }
  std::vector<double> ubf((size_t)B * rows * std::max(nbf, 1), 0.0);
  for (int f = 0; f < nbf; ++f) {
    const int bc = hi.bf_bc[f];
    for (int br = 0; br < B * rows; ++br) ubf[(size_t)br * nbf + f] = hi.bc_kind[bc] == 0 ? hi.bc_T[bc] - Tref : 0.0;
  }
  // position of each ordinate among the members of its octant
  std::vector<int> member(Mf, 0);
  {
    std::vector<int> cnt(8, 0);
    for (int a = 0; a < Mf; ++a) member[a] = cnt[ords[a].oct]++;
  }
  const int n_oct = S.n_oct, T = S.T, W = S.W;
  const int nch = T / Cc;
  std::vector<double> outv((size_t)gs.band.size() * S.n_out_stride, 0.0);
  // second-order faces (argv[2] = "--order2"; rows-per-lane layouts, G = 1):
  // each group's correction and stored field in its octant's position layout
  // (position ((r*(T + kPad2) + t)*64 + l)*NR + k), as the kernels keep them
  const bool second = argc > 2 && std::string(argv[2]) == "--order2";
  if (second && (G != 1 || (dim == 3 && !S.l3r))) { printf("second order needs G = 1 and a rows layout\n"); return 1; }
  const long long ppo = S.pos_per_oct;
  std::vector<double> so_corr, so_fld;
  if (second) {
    so_corr.assign((size_t)gs.band.size() * ppo, 0.0);
    so_fld.assign((size_t)gs.band.size() * ppo, 0.0);
  }
  // one sweep: returns per-cell sums of wacc[0] and wacc[1] terms; optionally
  // stores u (forward) or accumulates the tau-gradient sums (adjoint)
  auto sweep = [&](const std::vector<double>& Xs, const std::vector<double>& Qs, const std::vector<double>& cf,
                   bool adj, const std::vector<double>& ub, std::vector<double>& acc0, std::vector<double>& acc1,
                   std::vector<double>* store, const std::vector<double>* stored, const std::vector<double>* dTf,
                   std::vector<double>* tg) {
    acc0.assign(ncell, 0.0);
    acc1.assign(ncell, 0.0);
    for (size_t bu = 0; bu < gs.bundle_first.size(); ++bu) {
      const int o = adj ? (gs.bundle_oct[bu] ^ (n_oct - 1)) : gs.bundle_oct[bu];
      for (int p = 0; p < P; ++p) {
        const int grp = gs.bundle_first[bu] + p;
        const double* gt = cf.data() + (size_t)grp * GS;
        const int band = gs.band[grp];
        const int urow = has_spec ? band * Mf + std::max(0, gs.ords[(size_t)grp * G]) : band;
        const double kS = gt[0], cQ = gt[1];
        std::vector<std::vector<double>> f(R, std::vector<double>(64 * G, 0.0));
        std::vector<std::vector<double>> zring(R, std::vector<double>((size_t)W * G, 0.0));
        std::vector<double> yring((size_t)LK * W * G, 0.0);
        std::vector<double> zg((size_t)std::max(S.ring, 1) * 8 * G, 0.0);
        std::vector<int> in_cur(R, 0), out_cur(R, 0);
        if (!L3)
          for (int c = 0; c < W; ++c) {
            const int sl = S.pre_slot[(size_t)o * W + c];
            const double u = sl >= 0 ? ub[(size_t)urow * nbf + sl] : 0.0;
            for (int gg = 0; gg < G; ++gg) zring[R - 1][c * G + gg] = u * gt[go_den(G) + gg];
          }
        for (int tau_ = 0; tau_ < T; ++tau_) {
          for (int r = 0; r < R; ++r) {
            const int rprev = (r + R - 1) % R;
            const int* ich = &S.in_chunk[((size_t)o * R + r) * (nch + 1)];
            const int ch = tau_ / Cc;
            if (tau_ % Cc == 0) in_cur[r] = 0;
            std::vector<double> fold = f[r], fnew(64 * G), xu(64 * G), yu(64 * G), zu(64 * G);
            std::vector<int2> ent(64);
            const size_t Tp3 = (size_t)(S.pos_per_oct / (64 * R));  // padded steps per slot
            for (int l = 0; l < 64; ++l) ent[l] = S.sched[((size_t)o * R + r) * Tp3 * 64 + (size_t)tau_ * 64 + l];
            for (int l = 0; l < 64; ++l) {
              const int jl = L3 ? (l & 7) : 0, kl = L3 ? (l >> 3) : l;
              const unsigned fl = (unsigned)ent[l].y;
              const int col = (fl >> F_COL_SHIFT) & F_COL_MASK;
              for (int gg = 0; gg < G; ++gg) {
                xu[l * G + gg] = fold[l * G + gg];
                if (!L3) {
                  zu[l * G + gg] = l == 0 ? zring[rprev][col * G + gg] : fold[(l - 1) * G + gg];
                  yu[l * G + gg] = 0.0;
                } else {
                  yu[l * G + gg] = jl == 0 ? yring[(kl * W + col) * G + gg] : fold[(l - 1) * G + gg];
                  if (kl == 0) {
                    const int tt = tau_ - S.lag;
                    zu[l * G + gg] = tt >= 0 ? zg[((size_t)(tt & (S.ring - 1)) * 8 + jl) * G + gg] : 0.0;
                  } else zu[l * G + gg] = fold[(l - 8) * G + gg];
                }
              }
            }
            int k = ich[ch] + in_cur[r];
            for (int l = 0; l < 64; ++l) {
              const unsigned fl = (unsigned)ent[l].y;
              for (int d = 0; d < 3; ++d)
                if (fl & (F_IN_X << d)) {
                  const double u = ub[(size_t)urow * nbf + S.in_slot[k++]];
                  in_cur[r]++;
                  for (int gg = 0; gg < G; ++gg) {
                    const double val = u * gt[go_den(G) + gg];
                    if (d == 0) xu[l * G + gg] = val;
                    else if (d == 1) { if (L3) yu[l * G + gg] = val; else zu[l * G + gg] = val; }
                    else zu[l * G + gg] = val;
                  }
                }
            }
            for (int l = 0; l < 64; ++l) {
              const int cid = ent[l].x;
              const unsigned fl = (unsigned)ent[l].y;
              const bool act = cid >= 0 && (fl & F_ACTIVE);
              double a0 = 0.0, a1 = 0.0;
              for (int gg = 0; gg < G; ++gg) {
                const double S_ = kS * (cid >= 0 ? Xs[cid] : 0.0) + cQ * (act ? Qs[cid] : 0.0);
                double fn;
                if (L3) fn = gt[go_a(G, 2) + gg] * zu[l * G + gg] + gt[go_a(G, 1) + gg] * yu[l * G + gg] + gt[go_a(G, 0) + gg] * xu[l * G + gg] + S_;
                else fn = gt[go_a(G, 1) + gg] * zu[l * G + gg] + gt[go_a(G, 0) + gg] * xu[l * G + gg] + S_;
                fnew[l * G + gg] = fn;
                a0 += gt[go_wacc(G, 0) + gg] * fn;
                a1 += gt[go_wacc(G, 1) + gg] * fn;
                if (act && store) (*store)[((size_t)grp * ncell + cid) * G + gg] = fn * gt[go_inv(G) + gg];
                if (act && tg) {
                  const double uf = (*stored)[((size_t)grp * ncell + cid) * G + gg];
                  (*tg)[2 * grp] += gt[go_wt(G, 0) + gg] * fn * (uf - (*dTf)[cid]);
                  (*tg)[2 * grp + 1] += Xs[cid] * gt[go_wt(G, 1) + gg] * uf;
                }
              }
              if (act) { acc0[cid] += a0; acc1[cid] += a1; }
              for (int d = 0; d < 3; ++d)
                if (fl & (F_OUT_X << d)) {
                  double vv = 0.0;
                  for (int gg = 0; gg < G; ++gg) vv += gt[go_wo(G, d) + gg] * fnew[l * G + gg];
                  outv[(size_t)grp * S.n_out_stride + S.out_base[o * R + r] + out_cur[r]++] = vv;
                }
            }
            for (int l = 0; l < 64; ++l) {
              const int jl = L3 ? (l & 7) : 0, kl = L3 ? (l >> 3) : l;
              const int cid = ent[l].x;
              const unsigned fl = (unsigned)ent[l].y;
              const int col = (fl >> F_COL_SHIFT) & F_COL_MASK;
              for (int gg = 0; gg < G; ++gg) {
                if (!L3 && l == 63 && cid >= 0) zring[r][col * G + gg] = fnew[l * G + gg];
                if (L3 && jl == 7 && cid >= 0) yring[(kl * W + col) * G + gg] = fnew[l * G + gg];
                if (L3 && kl == 7) zg[((size_t)(tau_ & (S.ring - 1)) * 8 + jl) * G + gg] = fnew[l * G + gg];
              }
            }
            f[r] = fnew;
          }
        }
      }
    }
  };
  // 1D/2D rows-per-lane kernel: lane l of slot r owns rows NR*l + k of its
  // strip; per chunk of kC2 steps the ghost values of lane 0 and the ring-write
  // columns of lane 63 are taken at the chunk start; inflows come from the
  // per-chunk table at the offset stored in each record
  auto sweep2d = [&](const std::vector<double>& Xs, const std::vector<double>& Qs, const std::vector<double>& cf,
                     bool adj, const std::vector<double>& ub, std::vector<double>& acc0, std::vector<double>& acc1,
                     std::vector<double>* store, const std::vector<double>* stored, const std::vector<double>* dTf,
                     std::vector<double>* tg) {
    acc0.assign(ncell, 0.0);
    acc1.assign(ncell, 0.0);
    const int Tp = T + kPad2, H = 64 * NR, nx = n0, ny = dim >= 2 ? n1 : 1;
    const int nchk = T / kC2;
    const unsigned kInAll = [&] { unsigned m = 0; for (int k = 0; k < NR; ++k) m |= (F2_INX | F2_INY) << (F2_ROW_BITS * k); return m; }();
    const long long SPe = S.nS > R ? (long long)R * S.du : (1ll << 40);
    auto strip_at = [&](int q, int r, int& sidx, int& v) {
      const long long a = (long long)q - (long long)r * S.du;
      const long long m = a >= 0 ? a / SPe : -((-a + SPe - 1) / SPe);
      sidx = (int)(r + m * R);
      if (sidx < 0) return false;
      v = q - sidx * S.du;
      return sidx < S.nS && v >= 0 && v < nx;
    };
    for (size_t bu = 0; bu < gs.bundle_first.size(); ++bu) {
      const int o = adj ? (gs.bundle_oct[bu] ^ (n_oct - 1)) : gs.bundle_oct[bu];
      const int dyc = (o & 2) ? -nx : nx;
      for (int p = 0; p < P; ++p) {
        const int grp = gs.bundle_first[bu] + p;
        const double* gt = cf.data() + (size_t)grp * GS;
        const int band = gs.band[grp];
        const int urow = has_spec ? band * Mf + std::max(0, gs.ords[(size_t)grp * G]) : band;
        const double kS = gt[0], cQ = gt[1];
        std::vector<std::vector<double>> f(R, std::vector<double>((size_t)64 * NR * G, 0.0));
        std::vector<std::vector<double>> ring(R, std::vector<double>((size_t)(W + 1) * G, 0.0));
        for (int c = 0; c < W; ++c) {
          const int sl = S.pre_slot[(size_t)o * W + c];
          const double u = sl >= 0 ? ub[(size_t)urow * nbf + sl] : 0.0;
          for (int gg = 0; gg < G; ++gg) ring[R - 1][c * G + gg] = u * gt[go_den(G) + gg];
        }
        std::vector<int> out_cnt(R, 0);
        std::vector<std::vector<double>> gh(R, std::vector<double>((size_t)kC2 * G));
        std::vector<std::vector<int>> wc(R, std::vector<int>(kC2));
        // the kernel's incremental strip tracking, one tracker per chunk lane m
        std::vector<std::vector<StripTrack>> gtr(R, std::vector<StripTrack>(kC2)), wtr = gtr;
        for (int r = 0; r < R; ++r)
          for (int m = 0; m < kC2; ++m) {
            gtr[r][m].init(m, r, R, S.du, S.nS);
            wtr[r][m].init(m - 63, r, R, S.du, S.nS);
          }
        for (int tau_ = 0; tau_ < T; ++tau_) {
          const int ch = tau_ / kC2, u = tau_ % kC2;
          if (u == 0)
            for (int r = 0; r < R; ++r) {
              const int rprev = (r + R - 1) % R;
              for (int m = 0; m < kC2; ++m) {
                int sidx, v;
                const int q = ch * kC2 + m;
                // the tracker must agree with the schedule's own strip mapping
                const bool gref = strip_at(q, r, sidx, v);
                if (gref != gtr[r][m].valid(S.nS, nx) || (gref && (v != gtr[r][m].v || sidx != gtr[r][m].s))) {
                  printf("strip tracker mismatch (lane 0)\n");
                  exit(2);
                }
                const bool wref = strip_at(q - 63, r, sidx, v);
                if (wref != wtr[r][m].valid(S.nS, nx) || (wref && (v != wtr[r][m].v || sidx != wtr[r][m].s))) {
                  printf("strip tracker mismatch (lane 63)\n");
                  exit(2);
                }
                const int gc = gtr[r][m].valid(S.nS, nx) ? gtr[r][m].v : -1;
                for (int gg = 0; gg < G; ++gg) gh[r][m * G + gg] = gc >= 0 ? ring[rprev][gc * G + gg] : 0.0;
                wc[r][m] = (wtr[r][m].valid(S.nS, nx) && wtr[r][m].s * H + H - 1 < ny) ? wtr[r][m].v : W;
                gtr[r][m].advance(kC2, R);
                wtr[r][m].advance(kC2, R);
              }
            }
          for (int r = 0; r < R; ++r) {
            const long long slot = (long long)o * R + r;
            const int* itab = &S.in_tab[(size_t)slot * (nchk + 2) * S.in_E + (size_t)ch * S.in_E];
            std::vector<double> fold = f[r], fnew = f[r];
            std::vector<int2> ent(64);
            for (int l = 0; l < 64; ++l) ent[l] = S.sched[((size_t)slot * Tp + tau_) * 64 + l];
            for (int l = 0; l < 64; ++l) {
              const unsigned fl = (unsigned)ent[l].y;
              const int cid0 = ent[l].x >= 0 ? (ent[l].x >> 5) : -1;
              const int e0 = (int)((fl >> F2_INOFF_SHIFT) & F2_INOFF_MASK);
              std::vector<double> zc(G);
              for (int gg = 0; gg < G; ++gg)
                zc[gg] = l == 0 ? gh[r][u * G + gg] : fold[((size_t)(l - 1) * NR + NR - 1) * G + gg];
              // the kernel's write-out decodes rows from the record: every active
              // row must be marked inside the grid, and "full" must mean all rows
              if (ent[l].x >= 0) {
                const int gm = ent[l].x & 15, full = (ent[l].x >> 4) & 1;
                if (full != (gm == (1 << NR) - 1 ? 1 : 0)) { printf("bad full bit\n"); exit(2); }
                for (int k = 0; k < NR; ++k)
                  if (((fl >> (F2_ROW_BITS * k)) & F2_ACT) && !((gm >> k) & 1)) { printf("bad grid mask\n"); exit(2); }
              }
              // a lane entering its strip at the x wall: its NR x-inflows are the
              // entries from its offset on (slot -1: zero), replacing the rows'
              // x-upwind values
              std::vector<double> xst;
              if (fl & F2_XSTART) {
                if (fl & kInAll) { printf("F2_XSTART with other inflows\n"); exit(2); }
                xst.resize((size_t)NR * G);
                for (int k = 0; k < NR; ++k)
                  for (int gg = 0; gg < G; ++gg) {
                    const int sl = itab[e0 + k];
                    xst[(size_t)k * G + gg] = (sl >= 0 ? ub[(size_t)urow * nbf + sl] : 0.0) * gt[go_den(G) + gg];
                  }
              }
              for (int k = 0; k < NR; ++k) {
                const unsigned b = fl >> (F2_ROW_BITS * k);
                const bool act = (b & F2_ACT) != 0;
                const int cell = act ? cid0 + k * dyc : -1;
                const long long pos = (((long long)r * Tp + tau_) * 64 + l) * NR + k;
                const double S_ = (act ? kS * Xs[cell] + cQ * Qs[cell] : 0.0) +
                                  (second && !adj ? so_corr[(size_t)grp * ppo + pos] : 0.0);
                const unsigned below = fl & kInAll & ((1u << (F2_ROW_BITS * k)) - 1u);
                const int ex = e0 + __builtin_popcount(below);
                const int ey = ex + ((b & F2_INX) ? 1 : 0);
                double a0s = 0.0, a1s = 0.0;
                for (int gg = 0; gg < G; ++gg) {
                  const double den = gt[go_den(G) + gg];
                  const double xu = (b & F2_INX) ? ub[(size_t)urow * nbf + itab[ex]] * den
                                    : !xst.empty() ? xst[(size_t)k * G + gg]
                                                   : fold[((size_t)l * NR + k) * G + gg];
                  const double zu = (b & F2_INY) ? ub[(size_t)urow * nbf + itab[ey]] * den : zc[gg];
                  const double fn = gt[go_a(G, 1) + gg] * zu + gt[go_a(G, 0) + gg] * xu + S_;
                  fnew[((size_t)l * NR + k) * G + gg] = fn;
                  zc[gg] = fn;
                  if (second && !adj) so_fld[(size_t)grp * ppo + pos] = fn * gt[go_inv(G)];
                  a0s += gt[go_wacc(G, 0) + gg] * fn;
                  a1s += gt[go_wacc(G, 1) + gg] * fn;
                  if (act && store) (*store)[((size_t)grp * ncell + cell) * G + gg] = fn * gt[go_inv(G) + gg];
                  if (act && tg) {
                    const double uf = (*stored)[((size_t)grp * ncell + cell) * G + gg];
                    (*tg)[2 * grp] += gt[go_wt(G, 0) + gg] * fn * (uf - (*dTf)[cell]);
                    (*tg)[2 * grp + 1] += Xs[cell] * gt[go_wt(G, 1) + gg] * uf;
                  }
                }
                if (act) { acc0[cell] += a0s; acc1[cell] += a1s; }
              }
            }
            // outflow entries: rows, then axes, then lanes
            for (int k = 0; k < NR; ++k)
              for (int d = 0; d < 2; ++d)
                for (int l = 0; l < 64; ++l) {
                  const unsigned fl = (unsigned)ent[l].y;
                  if (!((fl >> (F2_ROW_BITS * k)) & (F2_OUTX << d))) continue;
                  double vv = 0.0;
                  for (int gg = 0; gg < G; ++gg) vv += gt[go_wo(G, d) + gg] * fnew[((size_t)l * NR + k) * G + gg];
                  outv[(size_t)grp * S.n_out_stride + S.out_base[slot] + out_cnt[r]++] = vv;
                }
            // lane 63's top row to the ring
            for (int gg = 0; gg < G; ++gg) ring[r][wc[r][u] * G + gg] = fnew[((size_t)63 * NR + NR - 1) * G + gg];
            f[r] = fnew;
          }
        }
      }
    }
  };
  // 3D rows-per-lane kernel: lane l owns rows NR*l + k along the lane axis;
  // the step axis is cut into blocks of kC2 columns and every lane runs
  // through block b, plane p, column c at position s = q*kC2 + c (plane
  // period q; the schedule's period table gives its plane), taking position s
  // at clock t = s + l. Its plane-axis upwind value is its
  // own value of chunk step t mod kC2 one chunk earlier (zreg), its step-axis
  // upwind value the previous step's, except in a block's first column: there
  // the value its per-plane buffer held when it was loaded, at the end of the
  // chunk two chunks back (the buffer takes each chunk's last-column values at
  // the chunk's end, and is prefilled with the first block's wall values).
  // Lane 0's lane-axis upwind value is the wall value of gpre; other wall
  // values come from the inflow stream.
  auto sweep3r = [&](const std::vector<double>& Xs, const std::vector<double>& Qs, const std::vector<double>& cf,
                     bool adj, const std::vector<double>& ub, std::vector<double>& acc0, std::vector<double>& acc1,
                     std::vector<double>* store, const std::vector<double>* stored, const std::vector<double>* dTf,
                     std::vector<double>* tg) {
    acc0.assign(ncell, 0.0);
    acc1.assign(ncell, 0.0);
    const int NR = S.NR;
    const int Tp = T + kPad2, H = 64 * NR, nchk = T / kC2, npl = S.n_pl, nper = S.n_per;
    const int stride[3] = {1, n0, n0 * n1};
    const int FB = F3_ROW_BITS;
    unsigned kInAll = 0;
    for (int k = 0; k < NR; ++k) kInAll |= (F3_INX | F3_INY | F3_INZ) << (FB * k);
    const int TP = T + nper;  // gpre row: wall slots per step, then the period table
    // plane + 1 of period q of octant o (0: none)
    auto ptab = [&](int o, int q) { return q >= 0 && q < nper ? S.gpre[(size_t)o * TP + T + q] : 0; };
    // the job's partial-sum planes as the kernel writes them: every row of a
    // lane-step inside the grid (grid bit k of the record) at cell index
    // cid0 + k * dy, active or not; rows outside the grid are not written
    // (their index would be a cell of the next line when the lane axis is x
    // or y); the finalize then reads the active cells
    std::vector<double> jp0(ncell), jp1(ncell);
    for (size_t bu = 0; bu < gs.bundle_first.size(); ++bu) {
      const int o = adj ? (gs.bundle_oct[bu] ^ (n_oct - 1)) : gs.bundle_oct[bu];
      const int dyc = (((o >> S.ax[1]) & 1) ? -1 : 1) * stride[S.ax[1]];
      std::fill(jp0.begin(), jp0.end(), 0.0);
      std::fill(jp1.begin(), jp1.end(), 0.0);
      for (int p = 0; p < P; ++p) {
        const int grp = gs.bundle_first[bu] + p;
        const double* gt = cf.data() + (size_t)grp * GS;
        const int band = gs.band[grp];
        const int urow = has_spec ? band * Mf + std::max(0, gs.ords[(size_t)grp * G]) : band;
        const double kS = gt[0], cQ = gt[1], den = gt[go_den(G)];
        if (G != 1) { printf("3D rows layout with G > 1\n"); exit(2); }
        std::vector<double> f(H, 0.0), zreg((size_t)kC2 * H, 0.0), xb((size_t)npl * H, 0.0);
        std::vector<double> xl(H, 0.0), xn(H, 0.0), xs(H, 0.0);
        // the first block's step-axis wall values
        for (int pl = 0; pl < npl; ++pl)
          for (int j = 0; j < H; ++j) {
            const int sl = S.xpre[((size_t)o * npl + pl) * H + j];
            xb[(size_t)pl * H + j] = sl >= 0 ? ub[(size_t)urow * nbf + sl] * den : 0.0;
          }
        std::vector<int> qL(64), qS(64);
        auto xload = [&](int l, std::vector<double>& dst) {
          const int p1 = ptab(o, qL[l]);
          for (int k = 0; k < NR; ++k) dst[(size_t)l * NR + k] = p1 > 0 ? xb[(size_t)(p1 - 1) * H + l * NR + k] : 0.0;
          ++qL[l];
        };
        for (int l = 0; l < 64; ++l) {
          qL[l] = -(l / kC2);
          qS[l] = -((l + kC2 - 1) / kC2);
          xload(l, xl);
          xload(l, xn);
        }
        int out_cnt = 0;
        for (int t = 0; t < T; ++t) {
          const int ch = t / kC2, u = t % kC2;
          const int* itab = &S.in_tab[((size_t)o * (nchk + 2) + ch) * S.in_E];
          const int sg = S.gpre[(size_t)o * TP + t];  // face slot + 1
          const double gh = sg > 0 ? ub[(size_t)urow * nbf + sg - 1] * den : 0.0;
          std::vector<double> fold = f, fnew = f;
          std::vector<int2> ent(64);
          for (int l = 0; l < 64; ++l) ent[l] = S.sched[((size_t)o * Tp + t) * 64 + l];
          for (int l = 0; l < 64; ++l) {
            if (ent[l].x < 0) continue;
            const unsigned fl = (unsigned)ent[l].y;
            const int cid0 = ent[l].x >> 5;
            const int gm = ent[l].x & 15;
            const int e0 = (int)((fl >> F2_INOFF_SHIFT) & F2_INOFF_MASK);
            const bool c0 = (l % kC2) == u;
            double zc = l == 0 ? gh : fold[(size_t)(l - 1) * NR + NR - 1];
            for (int k = 0; k < NR; ++k) {
              const unsigned b = fl >> (FB * k);
              if ((b & F3_ACT) && !((gm >> k) & 1)) { printf("bad grid mask\n"); exit(2); }
              const bool act = (b & F3_ACT) != 0;
              const int cell = act ? cid0 + k * dyc : -1;
              const long long pos = ((long long)t * 64 + l) * NR + k;
              const double S_ = (act ? kS * Xs[cell] + cQ * Qs[cell] : 0.0) +
                                (second && !adj ? so_corr[(size_t)grp * ppo + pos] : 0.0);
              const unsigned below = fl & kInAll & ((1u << (FB * k)) - 1u);
              const int ex = e0 + __builtin_popcount(below);
              const int ey = ex + ((b & F3_INX) ? 1 : 0);
              const int ez = ey + ((b & F3_INY) ? 1 : 0);
              const double xin = c0 ? xl[(size_t)l * NR + k] : fold[(size_t)l * NR + k];
              const double xu = (b & F3_INX) ? ub[(size_t)urow * nbf + itab[ex]] * den : xin;
              const double yu = (b & F3_INY) ? ub[(size_t)urow * nbf + itab[ey]] * den : zc;
              const double zr = zreg[(size_t)u * H + l * NR + k];
              const double zu = (b & F3_INZ) ? ub[(size_t)urow * nbf + itab[ez]] * den : zr;
              const double fn = gt[go_a(G, S.ax[2])] * zu + gt[go_a(G, S.ax[1])] * yu + gt[go_a(G, S.ax[0])] * xu + S_;
              fnew[(size_t)l * NR + k] = fn;
              zc = fn;
              if (second && !adj) so_fld[(size_t)grp * ppo + pos] = fn * gt[go_inv(G)];
              if ((gm >> k) & 1) {
                const int idx = cid0 + k * dyc;
                if (idx < 0 || idx >= ncell) { printf("partial-sum row outside the plane\n"); exit(2); }
                jp0[idx] += gt[go_wacc(G, 0)] * fn;
                jp1[idx] += gt[go_wacc(G, 1)] * fn;
              }
              if (act) {
                if (store) (*store)[(size_t)grp * ncell + cell] = fn * gt[go_inv(G)];
                if (tg) {
                  const double uf = (*stored)[(size_t)grp * ncell + cell];
                  (*tg)[2 * grp] += gt[go_wt(G, 0)] * fn * (uf - (*dTf)[cell]);
                  (*tg)[2 * grp + 1] += Xs[cell] * gt[go_wt(G, 1)] * uf;
                }
              }
            }
          }
          // outflow stream: rows, then axes, then lanes
          for (int k = 0; k < NR; ++k)
            for (int e = 0; e < 3; ++e)
              for (int l = 0; l < 64; ++l) {
                const unsigned fl = (unsigned)ent[l].y;
                if (ent[l].x < 0 || !((fl >> (FB * k)) & (F3_OUTX << e))) continue;
                outv[(size_t)grp * S.n_out_stride + out_cnt++] = gt[go_wo(G, S.ax[e])] * fnew[(size_t)l * NR + k];
              }
          // the plane link and the last-column capture (idle lanes keep
          // their values: nothing active reads them)
          for (int l = 0; l < 64; ++l) {
            if (ent[l].x < 0) continue;
            const bool c7 = (l % kC2) == (u + 1) % kC2;
            for (int k = 0; k < NR; ++k) {
              zreg[(size_t)u * H + l * NR + k] = fnew[(size_t)l * NR + k];
              if (c7) xs[(size_t)l * NR + k] = fnew[(size_t)l * NR + k];
            }
          }
          f = fnew;
          if (u == kC2 - 1) {
            // end of chunk: last-column values to their planes, then the loads
            for (int l = 0; l < 64; ++l) {
              const int p1 = ptab(o, qS[l]);
              if (p1 > 0)
                for (int k = 0; k < NR; ++k) xb[(size_t)(p1 - 1) * H + l * NR + k] = xs[(size_t)l * NR + k];
              ++qS[l];
            }
            for (int l = 0; l < 64; ++l) {
              for (int k = 0; k < NR; ++k) xl[(size_t)l * NR + k] = xn[(size_t)l * NR + k];
              xload(l, xn);
            }
          }
        }
      }
      for (int c = 0; c < ncell; ++c)
        if (hi.active[c]) {
          acc0[c] += jp0[c];
          acc1[c] += jp1[c];
        }
    }
  };
  auto run_sweep = [&](const std::vector<double>& Xs, const std::vector<double>& Qs, const std::vector<double>& cf,
                       bool adj, const std::vector<double>& ub, std::vector<double>& a0v, std::vector<double>& a1v,
                       std::vector<double>* store, const std::vector<double>* stored, const std::vector<double>* dTf,
                       std::vector<double>* tg) {
    if (dim < 3) sweep2d(Xs, Qs, cf, adj, ub, a0v, a1v, store, stored, dTf, tg);
    else if (S.l3r) sweep3r(Xs, Qs, cf, adj, ub, a0v, a1v, store, stored, dTf, tg);
    else sweep(Xs, Qs, cf, adj, ub, a0v, a1v, store, stored, dTf, tg);
  };
  // lagged wall values from the last sweep's outflow entries. Forward: the
  // diffuse and specular inflows. Transposed sweeps (adj): the wall-value
  // adjoint, read from the entries of the flipped schedules and scaled by
  // 4 pi tau_b D h_d / (C_b t0 v_b).
  double Dsum = 0.0;
  for (int b = 0; b < B; ++b) Dsum += C[b] / tau[b];
  auto wall_scale = [&](bool adj, int b, int d) {
    return adj ? 4.0 * M_PI * tau[b] * Dsum * hi.h[d] / (C[b] * t0 * v[b]) : 1.0;
  };
  auto update_walls = [&](bool adj, std::vector<double>& tab) {
    const int ox = adj ? n_oct - 1 : 0;
    for (int df : hi.dface) {
      for (int b = 0; b < B; ++b) {
        double sacc = 0.0;
        for (int o = 0; o < n_oct; ++o) {
          const int k = S.ofk[(size_t)o * nbf + df];
          if (k < 0) continue;
          const int og = o ^ ox;
          for (int gg = 0; gg < gs.ob_count[og * B + b]; ++gg)
            sacc += outv[(size_t)(gs.ob_first[og * B + b] + gg) * S.n_out_stride + k];
        }
        const double val = sacc / half_range(ords, hi.bf_face[df] / 2) * wall_scale(adj, b, hi.bf_face[df] / 2);
        for (int r = 0; r < rows; ++r) tab[((size_t)b * rows + r) * nbf + df] = val;
      }
    }
    // specular faces: forward, an incoming ordinate takes its mirror's entry;
    // transposed, an outgoing one does
    for (int sf : hi.sface) {
      const int fd = hi.bf_face[sf], d = fd / 2;
      for (int a = 0; a < Mf; ++a) {
        const double sn = (fd & 1) ? ords[a].s[d] : -ords[a].s[d];
        if (adj ? !(sn > 0.0) : !(sn < 0.0)) continue;
        int m = -1;
        for (int c = 0; c < Mf && m < 0; ++c) {
          bool same = true;
          for (int e2 = 0; e2 < dim; ++e2)
            same = same && std::fabs(ords[c].s[e2] - (e2 == d ? -ords[a].s[e2] : ords[a].s[e2])) < 1e-12;
          if (same) m = c;
        }
        const int om = ords[m].oct;
        const int k = S.ofk[(size_t)(om ^ ox) * nbf + sf];
        for (int b = 0; b < B; ++b) {
          const double vv = outv[(size_t)(gs.ob_first[om * B + b] + member[m]) * S.n_out_stride + k];
          tab[((size_t)b * Mf + a) * nbf + sf] = vv / (ords[m].w * std::fabs(ords[m].s[d])) * wall_scale(adj, b, d);
        }
      }
    }
  };
  // second-order correction of every position of every group from the stored
  // field, through the library's stencil table (as the correction kernel).
  // The emulated sweep carries f = den * u (the kernels carry w0 * f), so the
  // coefficient of axis d is -t0 v_b s_d / 2
  std::vector<int> stencil;
  std::vector<double> cc;
  if (second) {
    stencil = corr_stencil(hi, S);
    cc.assign((size_t)gs.band.size() * 3, 0.0);
    for (size_t g = 0; g < gs.band.size(); ++g) {
      const int a = gs.ords[g];
      if (a < 0) continue;
      for (int d = 0; d < dim; ++d) cc[g * 3 + d] = -t0 * v[gs.band[g]] * ords[a].s[d] / 2.0;
    }
  }
  auto correction = [&]() {
    const int W3 = 3 * dim;
    for (size_t g = 0; g < gs.band.size(); ++g) {
      const int o = gs.oct[g];
      const int band = gs.band[g];
      const int urow = has_spec ? band * Mf + std::max(0, gs.ords[g]) : band;
      const double* u = so_fld.data() + g * ppo;
      for (long long p = 0; p < ppo; ++p) {
        const int* e = stencil.data() + ((size_t)o * ppo + p) * W3;
        double corr = 0.0;
        if (e[0] != kNoCell) {
          const double uc = u[p];
          for (int d = 0; d < dim; ++d) {
            const int en = e[3 * d], eu = e[3 * d + 1], euu = e[3 * d + 2];
            const double un = en >= 0 ? u[en] : 0.0, uu = eu >= 0 ? u[eu] : 0.0;
            const double fd = en >= 0 ? 0.5 * (uc + un) : (eu >= 0 ? 1.5 * uc - 0.5 * uu : uc);
            const double fu = eu >= 0 ? 0.5 * (uc + uu)
                                      : (eu <= -2 ? ubf[(size_t)urow * nbf + (-eu - 2)] : (en >= 0 ? 1.5 * uc - 0.5 * un : uc));
            double du = 0.0;
            if (eu >= 0) {
              const double fuu = euu >= 0 ? 0.5 * (uu + u[euu])
                                          : (euu <= -2 ? ubf[(size_t)urow * nbf + (-euu - 2)] : 1.5 * uu - 0.5 * uc);
              du = 0.5 * (uu + uc) - fuu;
            }
            const double dd = ((o >> d) & 1) ? du - (fd - fu) : (fd - fu) - du;
            corr += cc[g * 3 + d] / hi.h[d] * dd;
          }
        }
        so_corr[g * ppo + p] = corr;
      }
    }
  };
  if (second) {
    // the first correction: the equilibrium field of the initial state
    for (size_t g = 0; g < gs.band.size(); ++g) {
      const int o = gs.oct[g];
      for (int c = 0; c < ncell; ++c) {
        const int p = S.pos[(size_t)o * ncell + c];
        if (hi.active[c] && p >= 0) so_fld[g * ppo + p] = X[c];
      }
    }
    correction();
  }
  std::vector<double> acc0, acc1;
  for (int it = 0; it < iters; ++it) {
    run_sweep(X, Q, coef, false, ubf, acc0, acc1, nullptr, nullptr, nullptr, nullptr);
    update_walls(false, ubf);
    if (second) correction();
    X = acc0;
  }
  if (argc > 2 && !second) {
    // adjoint with dJ/dT read from argv[2] (ncell doubles)
    std::vector<double> g(ncell);
    FILE* fg = fopen(argv[2], "rb");
    fread(g.data(), 8, ncell, fg);
    fclose(fg);
    std::vector<double> store((size_t)gs.band.size() * ncell * G, 0.0);
    run_sweep(X, Q, coef, false, ubf, acc0, acc1, &store, nullptr, nullptr, nullptr);
    std::vector<double> ca;
    group_coefficients(gs, ords, hi, v, tau, C, t0, true, ca);
    std::vector<double> ubfa(ubf.size(), 0.0), lam = g, dumQ(ncell, 0.0);
    for (int it = 0; it < iters; ++it) {
      run_sweep(lam, dumQ, ca, true, ubfa, acc0, acc1, nullptr, nullptr, nullptr, nullptr);
      update_walls(true, ubfa);
      for (int c = 0; c < ncell; ++c) lam[c] = hi.active[c] ? g[c] + acc0[c] : 0.0;
    }
    std::vector<double> tg(2 * gs.band.size(), 0.0);
    run_sweep(lam, dumQ, ca, true, ubfa, acc0, acc1, nullptr, &store, &X, &tg);
    double D = 0.0;
    for (int b = 0; b < B; ++b) D += C[b] / tau[b];
    double L = 0.0;
    for (int c = 0; c < ncell; ++c) if (hi.active[c]) L += lam[c] * X[c];
    std::vector<double> T1(B, 0.0), T2(B, 0.0);
    for (size_t k2 = 0; k2 < gs.band.size(); ++k2) { T1[gs.band[k2]] += tg[2 * k2]; T2[gs.band[k2]] += tg[2 * k2 + 1]; }
    for (int b = 0; b < B; ++b) printf("dtau %.17g\n", (1.0 / tau[b]) * ((t0 / tau[b]) * T1[b] - T2[b] + C[b] / (tau[b] * D) * L));
    for (int c = 0; c < ncell; ++c) printf("dQ %.17g\n", acc1[c]);
    return 0;
  }
  for (int c = 0; c < ncell; ++c) printf("%.17g\n", hi.active[c] ? X[c] + Tref : 0.0);
  return 0;
}
