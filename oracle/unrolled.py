"""Unrolled FP64 source iteration in plain PyTorch CPU ops (TEST INFRASTRUCTURE ONLY).

Reverse-mode automatic differentiation through a fixed number of iterations
of the paper's scheme gives the gradient of the loss with respect to the
per-band relaxation times and the per-cell heat source; as the iteration
converges this approaches the gradient of the fixed point, which is what the
library's adjoint computes.

Each iteration follows the paper's Methods section in absolute variables:
  * for every (band l, direction a) the first-order upwind finite-volume matrix
    A (Eq. A_matrix: diagonal 1/tau_l + sum of outflow v.n S/V, off-diagonal
    -v|s_d|/h_d to the active upwind neighbour) is solved against
    b = e0/tau + Q_l/(4 pi) + inflow from isothermal walls (Eq. 5), i.e. the
    exact inner solve of Eq. Axb with first-order faces;
  * T_L = sum_l sum_a w_a e/tau_l / sum_l C_l/tau_l (Eq. updatee0_t).
The dense batched LU factorisation and solve of torch.linalg are the only
library steps. Isothermal walls only (no diffuse reflection). Small grids only.
"""
from __future__ import annotations

import math

import numpy as np
import torch

FOUR_PI = 4.0 * math.pi


def _neighbour(p, c, f):
    n0, n1, n2 = p.n
    idx = [c % n0, (c // n0) % n1, c // (n0 * n1)]
    d = f // 2
    idx[d] += 1 if f % 2 else -1
    if idx[d] < 0 or idx[d] >= p.n[d]:
        return -1
    nb = idx[0] + n0 * (idx[1] + n1 * idx[2])
    return nb if p.mask[nb] else -1


class Unrolled:
    """Differentiable source iteration for one small problem with isothermal walls."""

    def __init__(self, p):
        assert all(k == 0 for k in p.bc_kind), "isothermal walls only"
        self.p = p
        self.act = np.flatnonzero(p.mask)
        self.idx = -np.ones(p.ncell, dtype=np.int64)
        self.idx[self.act] = np.arange(self.act.size)
        N, M, dim = self.act.size, p.M, p.dim
        # per direction: upwind couplings and isothermal inflow factors (geometry only)
        self.coup = []      # list over a of (rows, cols, axis)
        self.inflow = []    # list over a of (rows, axis, wall temperature)
        for a in range(M):
            s = p.s[a]
            rows, cols, ax = [], [], []
            irows, iax, iT = [], [], []
            for ci, c in enumerate(self.act):
                for d in range(dim):
                    if s[d] == 0.0:
                        continue
                    f = 2 * d + (0 if s[d] > 0 else 1)  # inflow face on axis d
                    nb = _neighbour(p, c, f)
                    if nb >= 0:
                        rows.append(ci)
                        cols.append(self.idx[nb])
                        ax.append(d)
                    else:
                        irows.append(ci)
                        iax.append(d)
                        iT.append(p.bc_T[p.face_bc[c, f]])
            self.coup.append((np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64),
                              np.array(ax, dtype=np.int64)))
            self.inflow.append((np.array(irows, dtype=np.int64), np.array(iax, dtype=np.int64),
                                np.array(iT, dtype=np.float64)))

    def run(self, tau, Q, n_iters, T_init=None):
        """Returns T over the active cells after n_iters iterations (torch, FP64)."""
        p = self.p
        B, M, N, dim = p.B, p.M, self.act.size, p.dim
        v = torch.tensor(p.v, dtype=torch.float64)
        C = torch.tensor(p.C, dtype=torch.float64)
        w = torch.tensor(p.w, dtype=torch.float64)
        s = torch.tensor(p.s, dtype=torch.float64)
        h = torch.tensor(p.h, dtype=torch.float64)
        Csum = C.sum()
        D = (C / tau).sum()
        # A for every (l, a): batched dense matrices
        A = torch.zeros(B, M, N, N, dtype=torch.float64)
        rhs_wall = torch.zeros(B, M, N, dtype=torch.float64)
        eye = torch.eye(N, dtype=torch.float64)
        for a in range(M):
            diag = 1.0 / tau + v * sum(abs(float(s[a, d])) / float(h[d]) for d in range(dim))
            A[:, a] = diag[:, None, None] * eye
            rows, cols, ax = self.coup[a]
            for r_, c_, d_ in zip(rows, cols, ax):
                A[:, a, r_, c_] = -v * abs(float(s[a, d_])) / float(h[d_])
            irows, iax, iT = self.inflow[a]
            for r_, d_, Tw in zip(irows, iax, iT):
                rhs_wall[:, a, r_] += v * abs(float(s[a, d_])) / float(h[d_]) * C * Tw / FOUR_PI
        LU, piv = torch.linalg.lu_factor(A)
        Qa = Q[torch.as_tensor(self.act)]
        src = (C / Csum)[:, None] * Qa[None, :] / FOUR_PI                    # [B, N]
        T = (torch.full((N,), p.T_ref, dtype=torch.float64) if T_init is None
             else torch.as_tensor(T_init, dtype=torch.float64)[torch.as_tensor(self.act)])
        for _ in range(n_iters):
            e0 = C[:, None] * T[None, :] / FOUR_PI                           # [B, N]
            b = (e0 / tau[:, None] + src)[:, None, :] + rhs_wall             # [B, M, N]
            e = torch.linalg.lu_solve(LU, piv, b.unsqueeze(-1)).squeeze(-1)   # [B, M, N]
            T = torch.einsum("a,lan,l->n", w, e, 1.0 / tau) / D
        return T


def grad_unrolled(p, loss, n_iters, wrt=("tau", "Q")):
    """dJ/dtau [B] and dJ/dQ [ncell] by reverse mode through n_iters iterations."""
    un = Unrolled(p)
    tau = torch.tensor(p.tau, dtype=torch.float64, requires_grad=True)
    Q = torch.tensor(p.Q, dtype=torch.float64, requires_grad=True)
    T = un.run(tau, Q, n_iters)
    Tfull = torch.zeros(p.ncell, dtype=torch.float64).index_put((torch.as_tensor(un.act),), T)
    J = loss(Tfull)
    J.backward()
    return tau.grad.numpy().copy(), Q.grad.numpy().copy(), Tfull.detach().numpy()
