"""GPU parity with specularly reflecting walls (Eq. 7): the HIP library against
the FP64 oracle, which takes the mirror direction's outgoing value at the same
cell, lagged one iteration. Same bars as the other parity tests: FP64 1e-10 and
FP32 1e-4 of max|T - T_ref|."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve_gpu(bte, p, precision="fp64", plan=None, **opt):
    s = bte.Solver(p, precision=precision, plan=plan)
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
    T, q, rep = s.solve(Q, **opt)
    torch.cuda.synchronize()
    out = T.cpu().numpy(), q.cpu().numpy(), rep, s.plan()
    s.close()
    return out


def _rel(a, b, p):
    act = p.mask > 0
    scale = np.abs(b[act] - p.T_ref).max()
    return np.abs(a[act] - b[act]).max() / scale


def _film_specular():
    p = bi.film_1d(n_cells=200, n_mu=32, Q=np.linspace(0.0, 1e18, 200))
    return p.replace(bc_kind=np.array([bi.BC_ISOTHERMAL, bi.BC_SPECULAR], dtype=np.int32))


def test_film_1d_specular_fp64(hip_lib):
    p = _film_specular()
    T, q, rep, _ = _solve_gpu(hip_lib, p, tol=0.0, max_iters=15, check_every=5)
    r = oracle.solve(p, tol=0.0, max_iters=15)
    assert _rel(T, r["T"], p) < 1e-10
    assert np.abs(q - r["q"]).max() < 1e-10 * np.abs(r["q"]).max()


@pytest.mark.parametrize("plan", [dict(G=1, R=1, P=1, NR=1), dict(G=1, R=1, P=2, NR=2),
                                  dict(G=1, R=2, P=2, NR=1), dict(G=1, R=1, P=2, NR=4)])
def test_masked_2d_specular_fp64(hip_lib, plan):
    """Specular walls on every face but the isothermal bottom, hole faces
    included; strips in sequence and pipelined, one to four rows per lane."""
    p = bi.multi_hole_2d(50, 150, seed=4, n_bands=2, n_theta=2, n_phi=1, kinds=(0, 2))
    T, q, rep, _ = _solve_gpu(hip_lib, p, plan=plan, tol=0.0, max_iters=9, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=9, threads=oracle.num_threads())
    assert _rel(T, r["T"], p) < 1e-10
    assert np.abs(q - r["q"]).max() < 1e-10 * np.abs(r["q"]).max()


def test_mixed_walls_2d_fp64(hip_lib):
    """Isothermal, diffuse and specular faces in one problem."""
    p = bi.random_box_2d(40, 33, seed=2, n_bands=3, n_theta=2, n_phi=2, kinds=(0, 2))
    fbc = bi.face_bc_from_mask(p.n, 2, p.mask, lambda i, j, k, f: 0 if (f == 2 and j == 0) else (1 if f < 2 else 2))
    p = p.replace(face_bc=fbc, bc_kind=np.array([0, 1, 2], dtype=np.int32), bc_T=np.array([305.0, 300.0, 300.0]))
    T, q, rep, _ = _solve_gpu(hip_lib, p, plan=dict(G=1, R=1, P=2, NR=1), tol=0.0, max_iters=10, check_every=5)
    r = oracle.solve(p, tol=0.0, max_iters=10)
    assert _rel(T, r["T"], p) < 1e-10


def test_specular_2d_fp32_converged(hip_lib):
    p = bi.random_box_2d(96, 80, seed=5, n_bands=15, n_theta=4, n_phi=2, kinds=(0, 2))
    T, q, rep, plan = _solve_gpu(hip_lib, p, precision="fp32", tol=1e-7, check_every=8, max_iters=20000)
    r = oracle.solve(p, tol=1e-10, max_iters=20000, threads=oracle.num_threads())
    assert r["status"] == "converged"
    assert plan["G"] == 1
    assert _rel(T, r["T"], p) < 1e-4


@pytest.mark.parametrize("plan", [None, dict(G=1, P=2, C=16)])
def test_box_3d_specular_fp64(hip_lib, plan):
    p = bi.random_box_3d(11, 9, 13, seed=1, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2))
    T, q, rep, used = _solve_gpu(hip_lib, p, plan=plan, tol=0.0, max_iters=7, check_every=7)
    r = oracle.solve(p, tol=0.0, max_iters=7)
    assert used["G"] == 1
    assert _rel(T, r["T"], p) < 1e-10


def test_finfet_mixed_walls_fp64(hip_lib):
    """The FinFET-like domain with specular base surfaces, diffuse fin walls and
    isothermal substrate bottom and fin top."""
    p = bi.finfet_3d_mixed(scale=8, n_bands=3, n_theta=2, n_phi=2)
    T, q, rep, _ = _solve_gpu(hip_lib, p, tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6)
    assert _rel(T, r["T"], p) < 1e-10


def test_finfet_mixed_walls_fp32_converged(hip_lib):
    p = bi.finfet_3d_mixed(scale=4, n_bands=4, n_theta=2, n_phi=2)
    T, q, rep, _ = _solve_gpu(hip_lib, p, precision="fp32", tol=1e-7, check_every=8, max_iters=20000)
    r = oracle.solve(p, tol=1e-10, max_iters=20000, threads=oracle.num_threads())
    assert r["status"] == "converged"
    assert _rel(T, r["T"], p) < 1e-4


def test_specular_plans_need_one_ordinate_per_group(hip_lib):
    p = bi.random_box_2d(20, 16, seed=1, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2))
    s = hip_lib.Solver(p, precision="fp64")
    try:
        assert s.plan()["G"] == 1
        with pytest.raises(hip_lib.BTEError, match="G = 1"):
            s.set_plan(G=2)
        assert s.plan()["G"] == 1
        Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
        best = s.autotune(Q, n_iters=2)
        assert best["G"] == 1
        T, _, rep = s.solve(Q, tol=0.0, max_iters=4, check_every=4, store_state=True)
        assert rep["iters"] == 4
    finally:
        s.close()
