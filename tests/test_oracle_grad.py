"""Pins of the gradient references (CPU).

The unrolled PyTorch source iteration must reproduce the C oracle's iterates,
and its reverse-mode gradient must match the complex-step derivative of the
brute-force dense fixed point (exact to rounding) once the iteration has
converged. The transpose identity <u, L^-1 v> = <L^-T u, v> of one upwind
sweep pins the transposed sweep the adjoint relies on.
"""
import numpy as np
import pytest
import torch

import bte_inputs as bi
import oracle
from oracle import dense, unrolled


def _case():
    return bi.square_2d(6, L=0.05e-6, n_bands=3, n_theta=1, n_phi=1)


def test_unrolled_matches_c_oracle():
    p = _case()
    un = unrolled.Unrolled(p)
    for n in (1, 7, 40):
        T = un.run(torch.tensor(p.tau), torch.tensor(p.Q), n).numpy()
        r = oracle.solve(p, tol=0.0, max_iters=n)
        assert np.abs(T - r["T"]).max() < 1e-12 * np.abs(r["T"] - 300).max()


def test_unrolled_gradient_matches_complex_step():
    p = _case()
    r = oracle.solve(p, tol=1e-14, max_iters=2000)
    probes = np.array([7, 14, 21, 28])
    target = r["T"][probes] + 0.01

    def lossnp(T):
        return ((T[probes] - target) ** 2).mean()

    def losst(T):
        return ((T[torch.as_tensor(probes)] - torch.as_tensor(target)) ** 2).mean()

    gt, gq, _ = unrolled.grad_unrolled(p, losst, 300)
    cs_tau = dense.complex_step_grad(p, lossnp, "tau")
    idx = list(range(0, p.ncell, 5))
    cs_Q = dense.complex_step_grad(p, lossnp, "Q", idx=idx)
    assert np.abs(gt - cs_tau).max() < 1e-8 * np.abs(cs_tau).max()
    assert np.abs(gq[idx] - cs_Q).max() < 1e-9 * np.abs(cs_Q).max()


def test_complex_step_matches_central_difference():
    """The complex step itself against a plain central difference of the
    dense solve (independent of any derivative code)."""
    p = _case()
    probes = np.array([3, 20])

    def lossnp(T):
        return ((T[probes] - 300.0) ** 2).sum()

    cs = dense.complex_step_grad(p, lossnp, "tau", idx=[0, 2])
    for k, b in enumerate([0, 2]):
        h = 1e-4 * p.tau[b]
        tp, tm = p.tau.copy(), p.tau.copy()
        tp[b] += h
        tm[b] -= h
        fd = (lossnp(dense.solve_dense(p, tau=tp)) - lossnp(dense.solve_dense(p, tau=tm))) / (2 * h)
        assert abs(fd - cs[k]) < 1e-5 * abs(cs[k])


@pytest.mark.parametrize("a", [0, 3, 5])
def test_transpose_sweep_identity(a):
    """For one ordinate, L = A (first-order upwind matrix): the transposed
    operator is the same recurrence swept along -s with zero inflow."""
    p = _case()
    un = unrolled.Unrolled(p)
    N = un.act.size
    b = 1
    s = p.s[a]
    A = np.zeros((N, N))
    diag = 1.0 / p.tau[b] + sum(p.v[b] * abs(s[d]) / p.h[d] for d in range(p.dim))
    A[np.arange(N), np.arange(N)] = diag
    rows, cols, ax = un.coup[a]
    for r_, c_, d_ in zip(rows, cols, ax):
        A[r_, c_] = -p.v[b] * abs(s[d_]) / p.h[d_]
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(N), rng.standard_normal(N)
    # L^-T u by sweeping along -s: the reversed direction's matrix is A^T
    ar = int(np.argmin(np.linalg.norm(p.s + s, axis=1)))
    Ar = np.zeros((N, N))
    Ar[np.arange(N), np.arange(N)] = diag
    rows, cols, ax = un.coup[ar]
    for r_, c_, d_ in zip(rows, cols, ax):
        Ar[r_, c_] = -p.v[b] * abs(p.s[ar][d_]) / p.h[d_]
    assert np.abs(Ar - A.T).max() == 0.0
    lhs = u @ np.linalg.solve(A, v)
    rhs = np.linalg.solve(Ar, u) @ v
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


@pytest.mark.parametrize("make", [
    lambda: bi.film_1d(n_cells=12, L=24e-9, n_mu=6, Q=np.linspace(0, 1e18, 12)),
    lambda: bi.random_box_2d(5, 4, seed=2, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 1)),
    lambda: bi.random_box_2d(5, 4, seed=2, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2)),
])
def test_length_scale_complex_step_matches_c_oracle_differences(make):
    """The complex-step derivative of the dense fixed point with respect to a
    common factor on every cell size against central differences of the C
    oracle's converged solve with scaled cell sizes."""
    p = make()
    r = oracle.solve(p, tol=1e-14, max_iters=20000)
    act = np.flatnonzero(p.mask)
    probes = act[[1, 4, 7]]
    target = r["T"][probes] + 0.02

    def loss(T):
        return ((T[probes] - target) ** 2).mean()

    cs = dense.complex_step_dscale(p, loss)
    eps = 1e-5
    Jp = loss(oracle.solve(p.replace(h=tuple(hd * (1 + eps) for hd in p.h)), tol=1e-14, max_iters=20000)["T"])
    Jm = loss(oracle.solve(p.replace(h=tuple(hd * (1 - eps) for hd in p.h)), tol=1e-14, max_iters=20000)["T"])
    fd = (Jp - Jm) / (2 * eps)
    assert abs(cs) > 0
    assert abs(fd - cs) < 1e-6 * abs(cs)
