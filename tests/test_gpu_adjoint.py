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


def _gpu_grads(bte, p, loss_t, precision="fp64", tol=1e-13, plan=None, max_iters=100000):
    s = bte.Solver(p, precision=precision, plan=plan)
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
    # a capped FP32 run may stop on its rounding floor: the report says so
    T, _, rep = s.solve(Q, tol=tol, check_every=4, store_state=True, max_iters=max_iters,
                        allow_not_converged=max_iters < 100000)
    Tl = T.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(loss_t(Tl), Tl)
    dtau, dQ, rep_a = s.adjoint(g.contiguous(), tol=tol, check_every=4, max_iters=max_iters,
                                allow_not_converged=max_iters < 100000)
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
    # the length-scale gradient needs an adjoint since the last solve
    with pytest.raises(hip_lib.BTEError) as ei:
        s.adjoint_dscale()
    assert ei.value.status == hip_lib.BTE_ERR_STATE
    s.solve(Q, tol=1e-10, store_state=True)
    s.adjoint(torch.zeros(p.ncell, dtype=torch.float64, device="cuda"), tol=1e-10)
    assert s.adjoint_dscale() == 0.0  # zero objective gradient
    s.solve(Q, tol=1e-10)
    with pytest.raises(hip_lib.BTEError):
        s.adjoint_dscale()
    s.close()


@pytest.mark.parametrize("kind,plan", [(1, None), (1, dict(G=2, R=1, P=1, NR=1)), (2, None),
                                       (2, dict(G=1, R=2, P=1, NR=1))])
def test_adjoint_with_reflecting_walls_matches_complex_step(hip_lib, kind, plan):
    """Diffuse (kind 1) or specular (kind 2) walls on every face but the
    isothermal bottom, hole faces included: the transposed sweeps carry the
    adjoint of the lagged wall values."""
    p = bi.random_box_2d(7, 6, seed=3, n_bands=2, n_theta=1, n_phi=1, kinds=(0, kind))
    probes = np.flatnonzero(p.mask)[[2, 9, 17, 23]]
    T0 = dense.solve_dense(p)
    target = T0[probes] + 0.05
    loss_t = _loss_parts(p, probes, target)
    dtau, dQ, T, rep, rep_a = _gpu_grads(hip_lib, p, loss_t, plan=plan)
    assert rep["status"] == "ok" and rep_a["status"] == "ok"

    def loss(TT):
        return ((TT[probes] - target) ** 2).mean()

    act = np.flatnonzero(p.mask)
    gt = dense.complex_step_grad(p, loss, "tau")
    gq = dense.complex_step_grad(p, loss, "Q", idx=list(act))
    assert np.abs(dtau - gt).max() < 1e-8 * np.abs(gt).max()
    assert np.abs(dQ[act] - gq).max() < 1e-8 * np.abs(gq).max()


@pytest.mark.parametrize("kind", [1, 2])
def test_adjoint_3d_reflecting_walls_matches_complex_step(hip_lib, kind):
    p = bi.random_box_3d(4, 3, 5, seed=5, n_bands=2, n_theta=1, n_phi=1, kinds=(0, kind))
    probes = np.flatnonzero(p.mask)[[1, 7, 20, 33, 41]]
    T0 = dense.solve_dense(p)
    target = T0[probes] - 0.03
    loss_t = _loss_parts(p, probes, target)
    dtau, dQ, T, rep, rep_a = _gpu_grads(hip_lib, p, loss_t)

    def loss(TT):
        return ((TT[probes] - target) ** 2).mean()

    act = np.flatnonzero(p.mask)
    gt = dense.complex_step_grad(p, loss, "tau")
    gq = dense.complex_step_grad(p, loss, "Q", idx=list(act))
    assert np.abs(dtau - gt).max() < 1e-8 * np.abs(gt).max()
    assert np.abs(dQ[act] - gq).max() < 1e-8 * np.abs(gq).max()


def _fd_check(bte, p, probes, target, fd_tau, fd_Q, rtol=1e-5):
    s = bte.Solver(p, precision="fp64")
    pr = torch.tensor(probes, device="cuda")
    tg = torch.tensor(target, device="cuda")

    def J_of(tau, Q):
        s.set_tau(tau)
        T, _, _ = s.solve(torch.tensor(Q, device="cuda"), tol=1e-13, check_every=8)
        return float(((T[pr] - tg) ** 2).mean())

    s.set_tau(p.tau)
    T, _, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=1e-13, check_every=8, store_state=True)
    Tl = T.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(((Tl[pr] - tg) ** 2).mean(), Tl)
    dtau, dQ, _ = s.adjoint(g.contiguous(), tol=1e-13, check_every=8)
    dQ = dQ.cpu().numpy()
    for b in fd_tau:
        hstep = 1e-4 * p.tau[b]
        tp, tm = p.tau.copy(), p.tau.copy()
        tp[b] += hstep
        tm[b] -= hstep
        fd = (J_of(tp, p.Q) - J_of(tm, p.Q)) / (2 * hstep)
        assert abs(fd - dtau[b]) < rtol * abs(dtau).max(), (b, fd, dtau[b])
    for c in fd_Q:
        hstep = 1e-3 * p.Q.max()
        qp, qm = p.Q.copy(), p.Q.copy()
        qp[c] += hstep
        qm[c] -= hstep
        fd = (J_of(p.tau, qp) - J_of(p.tau, qm)) / (2 * hstep)
        assert abs(fd - dQ[c]) < rtol * np.abs(dQ).max(), (c, fd, dQ[c])
    s.close()


def test_adjoint_vs_central_differences_specular_square(hip_lib):
    """The paper's 2D inverse setting: isothermal bottom, specular walls on the
    other sides; FD of the GPU FP64 forward on tau and Q entries."""
    p = bi.random_box_2d(40, 40, seed=7, n_bands=15, n_theta=2, n_phi=2, hole=False, kinds=(0, 2), Q0=1e19)
    rng = np.random.default_rng(8)
    act = np.flatnonzero(p.mask)
    probes = np.sort(rng.choice(act, 20, replace=False))
    target = 300.0 + rng.uniform(0.0, 2.0, size=20)
    _fd_check(hip_lib, p, probes, target, fd_tau=[0, 7, 14], fd_Q=list(rng.choice(act, 4, replace=False)))


def test_adjoint_vs_central_differences_finfet_mixed(hip_lib):
    p = bi.finfet_3d_mixed(scale=8, n_bands=3, n_theta=2, n_phi=2)
    rng = np.random.default_rng(9)
    act = np.flatnonzero(p.mask)
    probes = np.sort(rng.choice(act, 12, replace=False))
    target = 300.0 + rng.uniform(0.0, 1.0, size=12)
    _fd_check(hip_lib, p, probes, target, fd_tau=[0, 2], fd_Q=list(rng.choice(act[p.Q[act] > 0], 3, replace=False)))


@pytest.mark.parametrize("make", [
    lambda: bi.film_1d(n_cells=12, L=24e-9, n_mu=6, Q=np.linspace(0, 1e18, 12)),
    lambda: bi.random_box_2d(7, 6, seed=3, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 1)),
    lambda: bi.random_box_2d(7, 6, seed=3, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2)),
    lambda: bi.random_box_3d(4, 3, 5, seed=5, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 1)),
])
def test_length_scale_gradient_matches_complex_step(hip_lib, make):
    """dJ/ds for a common factor s on every cell size (L dJ/dL) against the
    complex step on the cell sizes of the dense fixed point."""
    p = make()
    act = np.flatnonzero(p.mask)
    probes = act[[1, 4, 7]]
    T0 = dense.solve_dense(p)
    target = T0[probes] + 0.02
    s = hip_lib.Solver(p, precision="fp64")
    T, _, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=1e-13, check_every=4, store_state=True)
    g = torch.zeros(p.ncell, dtype=torch.float64, device="cuda")
    g[torch.tensor(probes, device="cuda")] = 2.0 * (T[torch.tensor(probes, device="cuda")]
                                                    - torch.tensor(target, device="cuda")) / probes.size
    s.adjoint(g, tol=1e-13, check_every=4)
    ds = s.adjoint_dscale()
    s.close()
    cs = dense.complex_step_dscale(p, lambda TT: ((TT[probes] - target) ** 2).mean())
    assert abs(ds - cs) < 1e-8 * abs(cs)


def test_film_thickness_inverse(hip_lib):
    """Results, "1D inverse problem for system size": a gray silicon-like film
    (200 cells, 32 directions, tau of Kn = 1 at 100 nm) observed at 20 evenly
    spaced cells; starting from 50 nm, 25 steps of a normalised gradient descent
    on log L with an exponentially decaying step recover the 100 nm film."""
    n, L_true = 200, 100e-9
    base = bi.film_1d(n_cells=n, L=L_true, Kn=1.0)
    obs = torch.tensor(np.linspace(0, n - 1, 20).round().astype(int), device="cuda")
    s = hip_lib.Solver(base, precision="fp64")
    Q = torch.tensor(base.Q, device="cuda")

    def run(L, grad):
        s.close()
        s.__init__(base.replace(h=(L / n,) * 3), precision="fp64")
        T, _, _ = s.solve(Q, tol=1e-12, check_every=8, store_state=grad)
        return T

    T_obs = run(L_true, False)[obs].clone()
    L0 = 50e-9
    x, v = 0.0, 0.0
    for k in range(25):
        L = L0 * np.exp(x)
        T = run(L, True)
        g = torch.zeros(n, dtype=torch.float64, device="cuda")
        g[obs] = 2.0 * (T[obs] - T_obs)
        s.adjoint(g, tol=1e-12, check_every=8)
        dJdx = s.adjoint_dscale()  # = L dJ/dL = dJ/d(log L)
        v = 0.999 * v + 0.001 * dJdx * dJdx
        x -= 0.25 * 0.85 ** k * dJdx / np.sqrt(v / (1 - 0.999 ** (k + 1)))
    s.close()
    assert abs(L0 * np.exp(x) / L_true - 1.0) < 0.01


@pytest.mark.parametrize("kinds", [None, (0, 2)])
def test_adjoint_fp32_sweeps_match_fp64(hip_lib, kinds):
    """FP32 sweeps (FP64 sums) in the forward and the adjoint iterations give
    dJ/dtau and dJ/dQ within 1e-3 of the largest component of the FP64 ones;
    with isothermal walls (15-band square) and with specular walls."""
    if kinds is None:
        p = bi.square_2d(48, L=0.25e-6, n_bands=15, n_theta=2, n_phi=2)
    else:
        p = bi.random_box_2d(48, 40, seed=3, n_bands=15, n_theta=2, n_phi=2, hole=False, kinds=kinds, Q0=1e19)
    rng = np.random.default_rng(21)
    act = np.flatnonzero(p.mask)
    probes = np.sort(rng.choice(act, 16, replace=False))
    target = 300.0 + rng.uniform(0.0, 1.0, size=16)
    loss_t = _loss_parts(p, probes, target)
    d64, q64, _, _, _ = _gpu_grads(hip_lib, p, loss_t, precision="fp64", tol=1e-12)
    d32, q32, _, _, r32 = _gpu_grads(hip_lib, p, loss_t, precision="fp32", tol=1e-7, max_iters=20000)
    assert np.abs(d32 - d64).max() < 1e-3 * np.abs(d64).max()
    assert np.abs(q32 - q64).max() < 1e-3 * np.abs(q64).max()


def test_heat_source_inverse_with_specular_walls(hip_lib):
    """Results, "2D inverse problem for heat source intensity": a 100 nm square
    (32 x 32 cells, 15 bands) with an isothermal 300 K bottom and specular walls
    elsewhere, heated in a 10 nm x 20 nm box near the top; the temperatures of 20
    evenly spaced bottom-row cells recover the box's intensity (1e19 W/m^3) from
    half of it with dJ/dQ summed over the box, in 25 normalised gradient steps
    with an exponentially decaying step."""
    n, L = 32, 100e-9
    h = L / n
    mask = np.ones(n * n, dtype=np.uint8)
    fbc = bi.face_bc_from_mask((n, n, 1), 2, mask, lambda i, j, k, f: 0 if (f == 2 and j == 0) else 1)
    v, tau, C = bi.band_table_synthetic(15)
    s_, w_ = bi.quad_octant_gl(2, 2, polar_axis=2)
    X, Y = np.meshgrid((np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h, indexing="xy")
    box = ((np.abs(X - 0.5 * L) <= 5e-9) & (Y >= L - 25e-9) & (Y <= L - 5e-9)).reshape(-1)
    assert box.sum() > 0
    p = bi.Problem("source_inverse", 2, (n, n, 1), (h, h, h), mask, fbc,
                   np.array([bi.BC_ISOTHERMAL, bi.BC_SPECULAR], dtype=np.int32), np.array([300.0, 300.0]),
                   v, tau, C, s_, w_, 1e19 * box.astype(np.float64), 300.0)
    obs = torch.tensor(np.linspace(0, n - 1, 20).round().astype(int), device="cuda")  # bottom row j = 0
    boxt = torch.tensor(box, device="cuda")
    s = hip_lib.Solver(p, precision="fp64")

    def solve(I, grad):
        T, _, _ = s.solve(torch.tensor(I * box.astype(np.float64), device="cuda"), tol=1e-12, check_every=8,
                          store_state=grad)
        return T

    T_obs = solve(1e19, False)[obs].clone()
    x, vv = 0.5, 0.0  # intensity in units of 1e19 W/m^3
    for k in range(25):
        T = solve(x * 1e19, True)
        g = torch.zeros(p.ncell, dtype=torch.float64, device="cuda")
        g[obs] = 2.0 * (T[obs] - T_obs)
        _, dQ, _ = s.adjoint(g, tol=1e-12, check_every=8)
        dJdx = float(dQ[boxt].sum()) * 1e19
        vv = 0.999 * vv + 0.001 * dJdx * dJdx
        x -= 0.25 * 0.85 ** k * dJdx / np.sqrt(vv / (1 - 0.999 ** (k + 1)))
    s.close()
    assert abs(x - 1.0) < 0.01
