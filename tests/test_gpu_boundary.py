"""GPU checks of the C ABI beyond parity: a caller-owned workspace, the
relaxation times passed per solve, the reference temperature, the autotune
cache, the non-finite flag and a warm start (Methods, "Forward and inverse
modeling workflow"; "Iterative matrix formulation and solution scheme",
Eq. 22). FP64 parity bar 1e-10 of max|T - T_ref| against the FP64 oracle."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b, p):
    act = p.mask > 0
    return np.abs(a[act] - b[act]).max() / np.abs(b[act] - p.T_ref).max()


def _box():
    return bi.random_box_2d(40, 33, seed=2, n_bands=4, n_theta=2, n_phi=1, kinds=(0, 1))


def test_workspace_bound_solve_equals_own_memory(hip_lib):
    p = _box()
    Q = torch.tensor(p.Q, device="cuda")
    a = hip_lib.Solver(p, precision="fp64")
    Ta, qa, _ = a.solve(Q, tol=0.0, max_iters=12, check_every=4)
    b = hip_lib.Solver(p, precision="fp64")
    n0, n1 = b.workspace_bytes(False), b.workspace_bytes(True)
    assert 0 < n0 < n1
    # garbage in the workspace: the library clears what it needs
    ws = torch.full((n0,), 255, dtype=torch.uint8, device="cuda")
    b.bind_workspace(ws)
    Tb, qb, _ = b.solve(Q, tol=0.0, max_iters=12, check_every=4)
    assert torch.equal(Ta, Tb) and torch.equal(qa, qb)
    r = oracle.solve(p, tol=0.0, max_iters=12)
    assert _rel(Tb.cpu().numpy(), r["T"], p) < 1e-10
    # no room for the adjoint's angular field in this workspace
    with pytest.raises(hip_lib.BTEError) as ei:
        b.solve(Q, tol=0.0, max_iters=2, store_state=True)
    assert ei.value.status == hip_lib.BTE_ERR_WORKSPACE
    # too small altogether
    with pytest.raises(hip_lib.BTEError) as ei:
        b.bind_workspace(torch.empty(n0 - 4096, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == hip_lib.BTE_ERR_WORKSPACE
    # with room for it: solve and adjoint equal the own-memory handle's
    ws1 = torch.full((n1,), 7, dtype=torch.uint8, device="cuda")
    b.bind_workspace(ws1)
    g = torch.zeros(p.ncell, dtype=torch.float64, device="cuda")
    g[::7] = 1.0
    Ta, _, _ = a.solve(Q, tol=1e-12, check_every=4, store_state=True)
    Tb, _, _ = b.solve(Q, tol=1e-12, check_every=4, store_state=True)
    assert torch.equal(Ta, Tb)
    da, qa, _ = a.adjoint(g, tol=1e-12, check_every=4)
    db, qb, _ = b.adjoint(g, tol=1e-12, check_every=4)
    assert np.array_equal(da, db) and torch.equal(qa, qb)
    a.close()
    b.close()


def test_workspace_plan_change_that_does_not_fit(hip_lib):
    """Fewer ordinate groups per workgroup need more partial-sum rows: with the
    workspace sized for the current plan the change is refused and the handle
    keeps working with its plan."""
    p = _box()
    Q = torch.tensor(p.Q, device="cuda")
    s = hip_lib.Solver(p, precision="fp64", plan=dict(G=1, P=2))
    ws = torch.empty(s.workspace_bytes(False), dtype=torch.uint8, device="cuda")
    s.bind_workspace(ws)
    before = s.plan()
    with pytest.raises(hip_lib.BTEError) as ei:
        s.set_plan(P=1)
    assert ei.value.status == hip_lib.BTE_ERR_WORKSPACE
    assert s.plan() == before
    T, _, _ = s.solve(Q, tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    # unbinding goes back to the library's own memory
    s.bind_workspace(None)
    s.set_plan(P=1)
    T, _, _ = s.solve(Q, tol=0.0, max_iters=6, check_every=3)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    s.close()


def test_bound_workspace_solve_allocates_no_device_memory(hip_lib):
    p = bi.square_2d(192, L=0.5e-6, n_bands=6, n_theta=2, n_phi=2)
    Q = torch.tensor(p.Q, device="cuda")
    warm = hip_lib.Solver(p, precision="fp32")
    warm.solve(Q, tol=0.0, max_iters=2, use_graph=False)
    warm.close()
    s = hip_lib.Solver(p, precision="fp32")
    need = s.workspace_bytes(False)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    s.bind_workspace(ws)
    s.solve(Q, tol=0.0, max_iters=4, check_every=2, use_graph=False)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert need > 8 << 20
    assert free0 - free1 < need // 8, (free0 - free1, need)
    s.close()


def test_tau_per_solve(hip_lib):
    p = bi.square_2d(24, L=0.1e-6, n_bands=4, n_theta=2, n_phi=1)
    Q = torch.tensor(p.Q, device="cuda")
    s = hip_lib.Solver(p, precision="fp64")
    tau2 = p.tau * np.linspace(0.6, 1.7, p.B)
    T1, _, _ = s.solve(Q, tau=tau2, tol=0.0, max_iters=10, check_every=5)
    r2 = oracle.solve(p, tau=tau2, tol=0.0, max_iters=10)
    assert _rel(T1.cpu().numpy(), r2["T"], p) < 1e-10
    # NULL keeps the tau of the last solve
    T2, _, _ = s.solve(Q, tol=0.0, max_iters=10, check_every=5)
    assert torch.equal(T1, T2)
    T3, _, _ = s.solve(Q, tau=p.tau, tol=0.0, max_iters=10, check_every=5)
    r1 = oracle.solve(p, tol=0.0, max_iters=10)
    assert _rel(T3.cpu().numpy(), r1["T"], p) < 1e-10
    # a state kept for the adjoint belongs to its tau
    s.solve(Q, tol=1e-10, store_state=True)
    s.set_tau(tau2)
    with pytest.raises(hip_lib.BTEError) as ei:
        s.adjoint(torch.zeros(p.ncell, dtype=torch.float64, device="cuda"))
    assert ei.value.status == hip_lib.BTE_ERR_STATE
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reference_temperature_is_exact(hip_lib, prec):
    """The deviational form is exact for any T_ref (the equations are linear in
    (e, T)): from the same initial temperature every T_ref gives the same
    iterates, up to rounding. T_ref <= 0 takes the mean isothermal wall
    temperature."""
    p = _box()
    Q = torch.tensor(p.Q, device="cuda")
    Ti = torch.full((p.ncell,), 301.0, dtype=torch.float64, device="cuda")
    r = oracle.solve(p, T_init=np.full(p.ncell, 301.0), tol=0.0, max_iters=15)
    s = hip_lib.Solver(p, precision=prec)
    bar = 1e-10 if prec == "fp64" else 1e-4
    for T_ref in (300.0, 0.0, 296.5):
        T, _, _ = s.solve(Q, T_init=Ti, tol=0.0, max_iters=15, check_every=5, T_ref=T_ref)
        assert _rel(T.cpu().numpy(), r["T"], p) < bar, T_ref
    s.close()


def test_autotune_cache(hip_lib, tmp_path):
    p = bi.square_2d(64, L=0.2e-6, n_bands=3, n_theta=2, n_phi=1)
    Q = torch.tensor(p.Q, device="cuda")
    path = tmp_path / "plans.txt"
    s = hip_lib.Solver(p, precision="fp32")
    T1, _, rep = s.solve(Q, tol=1e-6, autotune_cache=str(path))
    assert rep["status"] == "ok"
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and " plan " in lines[0]
    key, vals = lines[0].split(" plan ")
    pl = s.plan()
    assert [int(x) for x in vals.split()] == [pl[k] for k in ("G", "R", "P", "C", "NR")]
    # a fresh handle takes the stored plan without tuning again
    s2 = hip_lib.Solver(p, precision="fp32", plan=dict(G=2, P=1))
    T2, _, _ = s2.solve(Q, tol=1e-6, autotune_cache=str(path))
    assert path.read_text().splitlines() == lines and s2.plan() == pl
    # the last matching line wins: a hand-written entry is applied
    path.write_text(lines[0] + "\n" + key + " plan 1 1 1 8 1\n")
    s3 = hip_lib.Solver(p, precision="fp32")
    T3, _, _ = s3.solve(Q, tol=1e-6, autotune_cache=str(path))
    assert s3.plan() == dict(G=1, R=1, P=1, C=8, NR=1)
    r = oracle.solve(p, tol=1e-6)
    for T in (T1, T2, T3):
        assert _rel(T.cpu().numpy(), r["T"], p) < 1e-4
    # another problem has another key
    q = bi.square_2d(40, L=0.2e-6, n_bands=3, n_theta=2, n_phi=1)
    s4 = hip_lib.Solver(q, precision="fp32")
    s4.solve(torch.tensor(q.Q, device="cuda"), tol=1e-6, autotune_cache=str(path))
    assert len(path.read_text().splitlines()) == 3
    for x in (s, s2, s3, s4):
        x.close()


def test_autotune_batch_handle_takes_no_source(hip_lib):
    ps = [bi.square_2d(n, L=0.1e-6, n_bands=2, n_theta=1, n_phi=1) for n in (12, 20)]
    bs = hip_lib.BatchSolver(ps, precision="fp32")
    Q = torch.tensor(ps[0].Q, device="cuda")
    st = hip_lib.bte_autotune(bs._h, hip_lib._ptr(Q), 2, hip_lib._stream(None), None)
    assert st == hip_lib.BTE_ERR_STATE
    pl = bs.autotune(n_iters=2)
    Qs = [torch.tensor(p.Q, device="cuda") for p in ps]
    Ts, _, reps = bs.solve(Qs, tol=1e-6)
    for p, T, rp in zip(ps, Ts, reps):
        assert rp["status"] == "ok"
        # the oracle stopped by the same rule at the same tolerance
        r = oracle.solve(p, tol=1e-6)
        assert _rel(T.cpu().numpy(), r["T"], p) < 1e-4, pl
    bs.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_source_is_reported(hip_lib, prec):
    p = bi.square_2d(16, L=0.1e-6, n_bands=3, n_theta=1, n_phi=1)
    Qbad = p.Q.copy()
    Qbad[37] = np.nan
    s = hip_lib.Solver(p, precision=prec)
    with pytest.raises(hip_lib.BTEError) as ei:
        s.solve(torch.tensor(Qbad, device="cuda"), tol=1e-10, max_iters=64)
    assert ei.value.status == hip_lib.BTE_ERR_NONFINITE
    # the handle still solves the finite problem afterwards
    T, _, rep = s.solve(torch.tensor(p.Q, device="cuda"), tol=1e-9)
    assert rep["status"] == "ok"
    r = oracle.solve(p, tol=1e-12)
    assert _rel(T.cpu().numpy(), r["T"], p) < (1e-8 if prec == "fp64" else 1e-4)
    s.close()


def test_warm_start_resumes_the_iteration(hip_lib):
    """With isothermal walls the iteration's whole state is the temperature: k
    iterations, then a solve from their result, give the n-iteration result
    (to the rounding of T - T_ref); with diffuse walls the resumed run reaches
    the same fixed point."""
    p = bi.square_2d(48, L=0.2e-6, n_bands=5, n_theta=2, n_phi=1)
    Q = torch.tensor(p.Q, device="cuda")
    s = hip_lib.Solver(p, precision="fp64")
    Tn, _, _ = s.solve(Q, tol=0.0, max_iters=20, check_every=4)
    Tk, _, _ = s.solve(Q, tol=0.0, max_iters=8, check_every=4)
    Tr, _, _ = s.solve(Q, T_init=Tk.clone(), tol=0.0, max_iters=12, check_every=4)
    assert _rel(Tr.cpu().numpy(), Tn.cpu().numpy(), p) < 1e-13
    s.close()
    q = _box()
    Qq = torch.tensor(q.Q, device="cuda")
    s = hip_lib.Solver(q, precision="fp64")
    Tc, _, rc = s.solve(Qq, tol=1e-13, check_every=8)
    Tk, _, _ = s.solve(Qq, tol=0.0, max_iters=10, check_every=5)
    Tr, _, rr = s.solve(Qq, T_init=Tk.clone(), tol=1e-13, check_every=8)
    assert rc["status"] == "ok" and rr["status"] == "ok"
    assert rr["iters"] < rc["iters"]
    assert _rel(Tr.cpu().numpy(), Tc.cpu().numpy(), q) < 1e-10
    s.close()


def test_autograd_gradient_belongs_to_its_forward(hip_lib):
    """A second solve on the same solver between a forward pass and its
    backward pass does not change the backward's gradient."""
    from oracle import unrolled
    p = bi.square_2d(10, L=0.08e-6, n_bands=3, n_theta=1, n_phi=1)
    s = hip_lib.Solver(p, precision="fp64")
    tau = torch.tensor(p.tau, dtype=torch.float64, requires_grad=True)
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda", requires_grad=True)
    probes = torch.tensor([11, 22, 55], device="cuda")
    T = hip_lib.BTESolve.apply(s, tau, Q, dict(tol=1e-13, check_every=4))
    J = ((T[probes] - 301.0) ** 2).sum()
    # another forward at other parameters on the same solver
    s.solve(torch.tensor(p.Q * 0.5, device="cuda"), tau=p.tau * 1.3, tol=1e-10, store_state=True)
    J.backward()
    pr = torch.tensor([11, 22, 55])
    gt, gq, _ = unrolled.grad_unrolled(p, lambda TT: ((TT[pr.to(TT.device)] - 301.0) ** 2).sum(), 400)
    assert np.abs(tau.grad.numpy() - gt).max() < 1e-8 * np.abs(gt).max()
    assert np.abs(Q.grad.cpu().numpy() - gq).max() < 1e-8 * np.abs(gq).max()
    s.close()
