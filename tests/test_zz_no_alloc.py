"""bte_solve_noalloc (the solve for callers that cannot allocate device
memory) against bte_solve: two calls in a row, the second with a smaller
problem, each equal to the ordinary solve on its own handle; a handle whose
arrays another handle's call displaced solves correctly again; the refusals
(too large for the static workspace, a handle with memory of its own)."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b, p):
    act = p.mask > 0
    return np.abs(a[act] - b[act]).max() / np.abs(b[act] - p.T_ref).max()


def _pair(hip_lib, p, prec):
    Q = torch.tensor(p.Q, device="cuda")
    ref = hip_lib.Solver(p, precision=prec)
    T0, q0, r0 = ref.solve(Q, tol=0.0, max_iters=10, check_every=5)
    ref.close()
    s = hip_lib.Solver(p, precision=prec)  # fresh: no device memory of its own
    assert s.workspace_bytes(False) < 64 << 20
    T1 = torch.empty(p.ncell, dtype=torch.float64, device="cuda")
    q1 = torch.empty(p.ncell * p.dim, dtype=torch.float64, device="cuda")
    r1 = s.solve_noalloc(Q, T1, q1, tol=0.0, max_iters=10, check_every=5)
    assert r1["iters"] == r0["iters"] == 10
    return s, Q, T0, q0, T1, q1


def test_solve_noalloc_matches_solve(hip_lib):
    big = bi.square_2d(96, L=0.4e-6, n_bands=15, n_theta=8, n_phi=2)
    small = bi.random_box_2d(30, 23, seed=5, n_bands=4, n_theta=2, n_phi=1, kinds=(0, 1))
    sb, Qb, T0, q0, T1, q1 = _pair(hip_lib, big, "fp32")
    assert torch.equal(T0, T1) and torch.equal(q0, q1.view(-1, 2))
    ss, Qs, T0s, q0s, T1s, q1s = _pair(hip_lib, small, "fp64")
    assert torch.equal(T0s, T1s) and torch.equal(q0s, q1s.view(-1, 2))
    r = oracle.solve(small, tol=0.0, max_iters=10)
    assert _rel(T1s.cpu().numpy(), r["T"], small) < 1e-10
    # the big handle's arrays were displaced by the small one's call: it
    # rebinds and solves the same again
    T2 = torch.empty_like(T1)
    sb.solve_noalloc(Qb, T2, tol=0.0, max_iters=10, check_every=5)
    assert torch.equal(T2, T0)
    # converged, with the stop test, on the small problem again
    T3 = torch.empty_like(T1s)
    rep = ss.solve_noalloc(Qs, T3, tol=1e-12, check_every=8)
    assert rep["status"] == "ok"
    r = oracle.solve(small, tol=1e-13, max_iters=20000)
    assert _rel(T3.cpu().numpy(), r["T"], small) < 1e-9
    sb.close()
    ss.close()


def test_solve_noalloc_refusals(hip_lib):
    p = bi.square_2d(256)
    s = hip_lib.Solver(p, precision="fp32")
    assert s.workspace_bytes(False) > 64 << 20
    T = torch.empty(p.ncell, dtype=torch.float64, device="cuda")
    Q = torch.tensor(p.Q, device="cuda")
    with pytest.raises(hip_lib.BTEError) as ei:
        s.solve_noalloc(Q, T, tol=0.0, max_iters=2)
    assert ei.value.status == hip_lib.BTE_ERR_WORKSPACE
    s.close()
    q = bi.square_2d(16, L=0.1e-6, n_bands=2, n_theta=1, n_phi=1)
    s = hip_lib.Solver(q, precision="fp64")
    Qq = torch.tensor(q.Q, device="cuda")
    s.solve(Qq, tol=0.0, max_iters=2)  # the handle now holds memory of its own
    T = torch.empty(q.ncell, dtype=torch.float64, device="cuda")
    with pytest.raises(hip_lib.BTEError) as ei:
        s.solve_noalloc(Qq, T, tol=0.0, max_iters=2)
    assert ei.value.status == hip_lib.BTE_ERR_STATE
    s.close()
