"""GPU parity of the hand-written adjoint (dJ/dtau_b, dJ/dQ_c).

References: reverse mode through the unrolled PyTorch-CPU oracle (run far past
convergence, so it equals the fixed-point gradient to rounding), complex-step
derivatives of the dense fixed point, and central finite differences of the
GPU FP64 forward solve on the inverse-problem workload.
"""
import numpy as np
import pytest

import bte_inputs as bi
from oracle import dense, unrolled

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _loss_parts(p, probes, target):
    pr = torch.as_tensor(probes)
    tg = torch.as_tensor(target, dtype=torch.float64)

    def loss_t(T):
        return ((T[pr.to(T.device)] - tg.to(T.device)) ** 2).mean()

    return loss_t


def _gpu_grads(bte, p, loss_t, precision="fp64", tol=1e-13):
    s = bte.Solver(p, precision=precision)
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
    T, _, rep = s.solve(Q, tol=tol, check_every=4, store_state=True)
    Tl = T.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(loss_t(Tl), Tl)
    dtau, dQ, rep_a = s.adjoint(g.contiguous(), tol=tol, check_every=4)
    torch.cuda.synchronize()
    out = dtau, dQ.cpu().numpy(), T.detach().cpu().numpy(), rep, rep_a
    s.close()
    return out


def test_adjoint_matches_unrolled_and_complex_step(hip_lib):
    p = bi.square_2d(8, L=0.06e-6, n_bands=3, n_theta=1, n_phi=1)
    probes = np.array([9, 18, 27, 36, 45])
    base = unrolled.Unrolled(p).run(torch.tensor(p.tau), torch.tensor(p.Q), 400).numpy()
    target = base[probes] + 0.05
    loss_t = _loss_parts(p, probes, target)
    dtau, dQ, T, rep, rep_a = _gpu_grads(hip_lib, p, loss_t)
    assert rep["status"] == "ok" and rep_a["status"] == "ok"
    gt, gq, _ = unrolled.grad_unrolled(p, loss_t, 400)
    assert np.abs(dtau - gt).max() < 1e-8 * np.abs(gt).max()
    assert np.abs(dQ - gq).max() < 1e-8 * np.abs(gq).max()
    cs = dense.complex_step_grad(p, lambda TT: ((TT[probes] - target) ** 2).mean(), "tau")
    assert np.abs(dtau - cs).max() < 1e-8 * np.abs(cs).max()


def test_adjoint_nongray_rectangle(hip_lib):
    base = bi.square_2d(20, L=0.15e-6, n_bands=5, n_theta=2, n_phi=1)
    n = (20, 13, 1)
    mask = np.ones(20 * 13, dtype=np.uint8)
    p = base.replace(n=n, mask=mask, face_bc=bi.face_bc_from_mask(n, 2, mask, lambda i, j, k, f: 0),
                     Q=base.Q[: 20 * 13].copy())
    rng = np.random.default_rng(3)
    probes = np.sort(rng.choice(p.ncell, 12, replace=False))
    target = 300.0 + rng.uniform(0, 5, size=12)
    loss_t = _loss_parts(p, probes, target)
    dtau, dQ, T, rep, rep_a = _gpu_grads(hip_lib, p, loss_t)
    gt, gq, _ = unrolled.grad_unrolled(p, loss_t, 600)
    assert np.abs(dtau - gt).max() < 1e-8 * np.abs(gt).max()
    assert np.abs(dQ - gq).max() < 1e-8 * np.abs(gq).max()


def test_autograd_function(hip_lib):
    p = bi.square_2d(10, L=0.08e-6, n_bands=3, n_theta=1, n_phi=1)
    s = hip_lib.Solver(p, precision="fp64")
    tau = torch.tensor(p.tau, dtype=torch.float64, requires_grad=True)
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda", requires_grad=True)
    T = hip_lib.BTESolve.apply(s, tau, Q, dict(tol=1e-13, check_every=4))
    J = ((T[torch.tensor([11, 22, 55], device="cuda")] - 301.0) ** 2).sum()
    J.backward()
    loss_t = _loss_parts(p, np.array([11, 22, 55]), np.full(3, 301.0))
    gt, gq, _ = unrolled.grad_unrolled(p, lambda TT: 3 * loss_t(TT), 400)
    assert np.abs(tau.grad.numpy() - gt).max() < 1e-8 * np.abs(gt).max()
    assert np.abs(Q.grad.cpu().numpy() - gq).max() < 1e-8 * np.abs(gq).max()


def test_adjoint_vs_central_differences_inverse_case(hip_lib):
    """Inverse-problem workload at reduced size: FD of the GPU FP64 forward on
    seeded tau and Q parameters near the probes."""
    p = bi.square_2d(48, L=0.25e-6, n_bands=15, n_theta=2, n_phi=2)
    case = bi.adjoint_case(p, n_probes=16, n_fd_tau=3, n_fd_Q=5)
    s = hip_lib.Solver(p, precision="fp64")
    Qt = torch.tensor(case["Q_true"], device="cuda")
    s.set_tau(case["tau_true"])
    Tstar, _, _ = s.solve(Qt, tol=1e-13, check_every=8)
    s.set_tau(p.tau)
    probes = torch.tensor(case["probes"], device="cuda")
    target = Tstar[probes].clone()

    def J_of(tau, Q):
        s.set_tau(tau)
        T, _, _ = s.solve(torch.tensor(Q, device="cuda"), tol=1e-13, check_every=8)
        return float(((T[probes] - target) ** 2).mean())

    Q0 = torch.tensor(p.Q, device="cuda")
    s.set_tau(p.tau)
    T, _, _ = s.solve(Q0, tol=1e-13, check_every=8, store_state=True)
    Tl = T.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(((Tl[probes] - target) ** 2).mean(), Tl)
    dtau, dQ, _ = s.adjoint(g.contiguous(), tol=1e-13, check_every=8)
    dQ = dQ.cpu().numpy()
    for b in case["fd_tau"]:
        hstep = 1e-4 * p.tau[b]
        tp, tm = p.tau.copy(), p.tau.copy()
        tp[b] += hstep
        tm[b] -= hstep
        fd = (J_of(tp, p.Q) - J_of(tm, p.Q)) / (2 * hstep)
        assert abs(fd - dtau[b]) < 1e-5 * abs(dtau).max(), (b, fd, dtau[b])
    for c in case["fd_Q"]:
        hstep = 1e-3 * p.Q.max()
        qp, qm = p.Q.copy(), p.Q.copy()
        qp[c] += hstep
        qm[c] -= hstep
        fd = (J_of(p.tau, qp) - J_of(p.tau, qm)) / (2 * hstep)
        assert abs(fd - dQ[c]) < 1e-5 * np.abs(dQ).max(), (c, fd, dQ[c])
    s.close()


def test_adjoint_requires_stored_state(hip_lib):
    p = bi.square_2d(8, L=0.06e-6, n_bands=2, n_theta=1, n_phi=1)
    s = hip_lib.Solver(p, precision="fp64")
    Q = torch.tensor(p.Q, device="cuda")
    s.solve(Q, tol=1e-10)
    with pytest.raises(hip_lib.BTEError) as ei:
        s.adjoint(torch.zeros(p.ncell, dtype=torch.float64, device="cuda"))
    assert ei.value.status == hip_lib.BTE_ERR_STATE
    s.close()


def test_adjoint_rejects_diffuse_walls(hip_lib):
    p = bi.random_box_2d(9, 7, seed=0, kinds=(0, 1))
    s = hip_lib.Solver(p, precision="fp64")
    Q = torch.tensor(p.Q, device="cuda")
    s.solve(Q, tol=1e-8, store_state=True)
    with pytest.raises(hip_lib.BTEError) as ei:
        s.adjoint(torch.zeros(p.ncell, dtype=torch.float64, device="cuda"))
    assert ei.value.status == hip_lib.BTE_ERR_INVALID
    s.close()
