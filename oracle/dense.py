"""Brute-force discrete fixed point for tiny grids (TEST INFRASTRUCTURE ONLY).

Assembles, as one dense linear system, every equation that the converged
source iteration satisfies, and solves it directly:

  * for every (band b, direction a, active cell c), the first-order upwind
    finite-volume balance (paper Methods: Eq. eq:fvm-1 with the upwind face value
    of the upwind cell, uniform Cartesian cells so S/V = 1/h_d):
        sum_faces v_b (s_a . n_f)/h_d e_face = -(e - C_b T_c/(4 pi))/tau_b
                                               + Q_c C_b / (4 pi sum_b C_b)
    where e_face is e_c on outflow faces, the upwind neighbour's e on interior
    inflow faces, C_b T_w/(4 pi) on isothermal inflow faces (Eq. 5), the
    unknown wall value eb_{b,f} on diffuse inflow faces, and on specular
    inflow faces the same cell's e along the mirror direction
    s' = s - 2 n (s.n) (Eq. 7);
  * for every active cell, the lattice-temperature definition (Eq. updatee0_t)
        (sum_b C_b/tau_b) T_c = sum_b sum_a w_a e_{b,a,c} / tau_b ;
  * for every diffuse face f and band b, the diffuse-reflection condition
    (Eq. 6 with the discrete half-range normalisation)
        eb_{b,f} sum_{s.n<0} w |s.n| = sum_{s.n>0} w (s.n) e_{b,a,c(f)} .

With order = 2 the face value of the balance is the paper's second-order one
(Methods, "Spatial discretization"): on a face whose upwind side is a cell u,
e_face = e_u + grad e_u . d_u, d_u the vector from u's centre to the face
centre, grad e_u by Green-Gauss over u's faces (interior face: the mean of the
two cells; an isothermal face the ordinate enters through: its wall value; any
other boundary face: the linear extrapolation from u and the neighbour across
the opposite face, or u's value when that is a boundary too); a face whose upwind
side is a wall carries the wall value. Here these are assembled directly as
linear forms of the unknowns, without the deferred-correction iteration the
oracle uses.

The unknowns are absolute energies and temperatures, so this also checks that
the deviational form used elsewhere is exact. Complex parameters are accepted,
which gives complex-step derivatives of any output to machine precision.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def _geometry(p):
    n0, n1, n2 = p.n
    act = np.flatnonzero(p.mask)
    index = -np.ones(p.ncell, dtype=np.int64)
    index[act] = np.arange(act.size)
    return act, index


def _neighbour(p, c, f):
    n0, n1, n2 = p.n
    idx = [c % n0, (c // n0) % n1, c // (n0 * n1)]
    d, side = f // 2, f % 2
    idx[d] += 1 if side else -1
    if idx[d] < 0 or idx[d] >= p.n[d]:
        return -1
    nb = idx[0] + n0 * (idx[1] + n1 * idx[2])
    return nb if p.mask[nb] else -1


def _mirror(p, a, d):
    # index of the direction equal to s_a with its axis-d component negated
    want = np.array(p.s[a], dtype=np.float64)
    want[d] = -want[d]
    hit = np.flatnonzero(np.all(np.abs(np.asarray(p.s) - want) <= 1e-12, axis=1))
    if hit.size == 0:
        raise ValueError("quadrature has no mirror of direction %d across axis %d" % (a, d))
    return int(hit[0])


def solve_dense(p, tau=None, Q=None, return_all=False, order=1):
    """Direct solve of the discrete fixed point (first- or second-order
    faces). Returns T over all cells (absolute; 0 on inactive cells), or
    (T, e, eb, faces) with return_all."""
    tau = np.asarray(p.tau if tau is None else tau)
    Q = np.asarray(p.Q if Q is None else Q)
    dtype = np.result_type(tau.dtype, Q.dtype, np.asarray(p.h).dtype, np.float64)
    B, M, dim = p.B, p.M, p.dim
    act, index = _geometry(p)
    Na = act.size
    # boundary faces
    faces = []
    for c in act:
        for f in range(2 * dim):
            if _neighbour(p, c, f) < 0:
                faces.append((c, f, int(p.face_bc[c, f])))
    diff = [k for k, (c, f, bc) in enumerate(faces) if p.bc_kind[bc] == 1]
    dslot = {k: i for i, k in enumerate(diff)}
    fslot = {(c, f): k for k, (c, f, bc) in enumerate(faces)}
    nE = B * M * Na
    nT = Na
    nD = B * len(diff)
    N = nE + nT + nD
    A = np.zeros((N, N), dtype=dtype)
    rhs = np.zeros(N, dtype=dtype)
    Csum = p.C.sum()
    D = (p.C / tau).sum()

    def ie(b, a, ci):
        return (b * M + a) * Na + ci

    def iT(ci):
        return nE + ci

    def iD(b, k):
        return nE + nT + b * len(diff) + dslot[k]

    def wall(b, a, c, f):
        # wall value of ordinate a entering through boundary face (c, f), as
        # ({unknown: coefficient}, constant)
        k = fslot[(c, f)]
        bc = faces[k][2]
        if p.bc_kind[bc] == 0:
            return {}, p.C[b] * p.bc_T[bc] / FOUR_PI
        if p.bc_kind[bc] == 2:
            return {ie(b, _mirror(p, a, f // 2), index[c]): 1.0}, 0.0
        return {iD(b, k): 1.0}, 0.0

    def green_gauss(b, a, c, d):
        # (e_f+ - e_f-) / h_d over cell c's two faces normal to axis d
        lin, cst = {}, 0.0
        for side, sg in ((1, 1.0), (0, -1.0)):
            f = 2 * d + side
            nb = _neighbour(p, c, f)
            sn = p.s[a][d] if side else -p.s[a][d]
            if nb >= 0:
                terms, k0 = {ie(b, a, index[c]): 0.5, ie(b, a, index[nb]): 0.5}, 0.0
            elif sn < 0 and p.bc_kind[int(p.face_bc[c, f])] == 0:
                terms, k0 = wall(b, a, c, f)
            else:
                ob = _neighbour(p, c, f ^ 1)
                terms = ({ie(b, a, index[c]): 1.5, ie(b, a, index[ob]): -0.5} if ob >= 0
                         else {ie(b, a, index[c]): 1.0})
                k0 = 0.0
            for key, v in terms.items():
                lin[key] = lin.get(key, 0.0) + sg * v / p.h[d]
            cst += sg * k0 / p.h[d]
        return lin, cst

    for b in range(B):
        for a in range(M):
            s = p.s[a]
            for ci, c in enumerate(act):
                r = ie(b, a, ci)
                # -(e - C T/4pi)/tau moved to the left: + e/tau - C T/(4 pi tau)
                A[r, r] += 1.0 / tau[b]
                A[r, iT(ci)] += -p.C[b] / (FOUR_PI * tau[b])
                rhs[r] += Q[c] * p.C[b] / (FOUR_PI * Csum)
                if order == 2:
                    for f in range(2 * dim):
                        d = f // 2
                        sn = s[d] if f % 2 else -s[d]
                        if sn == 0.0:
                            continue
                        coef = p.v[b] * sn / p.h[d]
                        nb = _neighbour(p, c, f)
                        if sn > 0:
                            up, dist = c, (0.5 if f % 2 else -0.5) * p.h[d]
                        elif nb >= 0:
                            up, dist = nb, (-0.5 if f % 2 else 0.5) * p.h[d]
                        else:
                            terms, k0 = wall(b, a, c, f)
                            for key, v in terms.items():
                                A[r, key] += coef * v
                            rhs[r] -= coef * k0
                            continue
                        A[r, ie(b, a, index[up])] += coef
                        lin, cst = green_gauss(b, a, up, d)
                        for key, v in lin.items():
                            A[r, key] += coef * dist * v
                        rhs[r] -= coef * dist * cst
                    continue
                for f in range(2 * dim):
                    d = f // 2
                    sn = s[d] if f % 2 else -s[d]
                    if sn == 0.0:
                        continue
                    coef = p.v[b] * sn / p.h[d]
                    if sn > 0:
                        A[r, r] += coef
                    else:
                        nb = _neighbour(p, c, f)
                        if nb >= 0:
                            A[r, ie(b, a, index[nb])] += coef
                        else:
                            k = fslot[(c, f)]
                            bc = faces[k][2]
                            if p.bc_kind[bc] == 0:
                                rhs[r] -= coef * p.C[b] * p.bc_T[bc] / FOUR_PI
                            elif p.bc_kind[bc] == 2:
                                A[r, ie(b, _mirror(p, a, d), ci)] += coef
                            else:
                                A[r, iD(b, k)] += coef
    for ci in range(Na):
        r = iT(ci)
        A[r, r] = D
        for b in range(B):
            for a in range(M):
                A[r, ie(b, a, ci)] -= p.w[a] / tau[b]
    for k in diff:
        c, f, bc = faces[k]
        ci = index[c]
        d = f // 2
        sn = np.array([p.s[a][d] if f % 2 else -p.s[a][d] for a in range(M)])
        half_in = float((p.w * np.where(sn < 0, -sn, 0.0)).sum())
        for b in range(B):
            r = iD(b, k)
            A[r, r] = half_in
            for a in range(M):
                if sn[a] > 0:
                    A[r, ie(b, a, ci)] -= p.w[a] * sn[a]
    x = np.linalg.solve(A, rhs)
    T = np.zeros(p.ncell, dtype=dtype)
    T[act] = x[nE:nE + nT]
    if not return_all:
        return T
    e = np.zeros((B, M, p.ncell), dtype=dtype)
    e[:, :, act] = x[:nE].reshape(B, M, Na)
    eb = x[nE + nT:].reshape(B, len(diff)) if diff else np.zeros((B, 0), dtype=dtype)
    return T, e, eb, faces


def complex_step_grad(p, loss, wrt="tau", idx=None, hstep=1e-30):
    """d loss(T) / d tau_b (wrt='tau') or d loss / d Q_c (wrt='Q') by the complex
    step: Im(loss(T(theta + i h e_k))) / h, exact to rounding for analytic loss."""
    base = np.asarray(p.tau if wrt == "tau" else p.Q, dtype=np.float64)
    idx = range(base.size) if idx is None else idx
    out = []
    for k in idx:
        th = base.astype(np.complex128)
        th[k] += 1j * hstep
        T = solve_dense(p, tau=th) if wrt == "tau" else solve_dense(p, Q=th)
        out.append(loss(T).imag / hstep)
    return np.array(out)


def complex_step_dscale(p, loss, hstep=1e-30):
    """d loss(T) / d s for a common factor s on every cell size (all lengths of
    the geometry scaled, s = 1), by the complex step on the cell sizes."""
    h = tuple(complex(hd) * (1.0 + 1j * hstep) for hd in p.h)
    T = solve_dense(p.replace(h=h))
    return loss(T).imag / hstep
