"""Second-order faces by deferred correction (Methods, "Spatial
discretization"; Eq. rhs_b) on the GPU against the FP64 oracle with the same
reconstruction: fixed iteration counts at 1e-10 of max|T - T_ref| (FP64),
converged at 1e-9 (FP64) and 1e-4 (FP32 sweeps), the 1D film of the paper's
grid study, masked 2D boxes and 3D boxes, the staircase and the FinFET-like
mask with isothermal, diffuse and specular walls, several kernel shapes (3D:
the rows-per-lane layout)."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b, p):
    act = p.mask > 0
    return np.abs(a[act] - b[act]).max() / np.abs(b[act] - p.T_ref).max()


def _solver(hip_lib, p, prec="fp64", plan=None):
    s = hip_lib.Solver(p, precision=prec)
    s.set_order(2)
    if plan:
        s.set_plan(**plan)
    assert s.plan()["G"] == 1
    return s


@pytest.mark.parametrize("n", [50, 200])
def test_film_second_order_fixed_iterations(hip_lib, n):
    p = bi.film_1d(n_cells=n)
    s = _solver(hip_lib, p)
    T, q, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=0.0, max_iters=9, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=9, order=2)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    qs = np.abs(r["q"]).max()
    assert np.abs(q.cpu().numpy() - r["q"]).max() < 1e-10 * qs
    s.close()


def test_film_second_order_converged(hip_lib):
    p = bi.film_1d()
    s = _solver(hip_lib, p)
    T, _, rep = s.solve(torch.tensor(p.Q, device="cuda"), tol=1e-12, check_every=4)
    r = oracle.solve(p, tol=1e-12, order=2)
    assert rep["status"] == "ok" and abs(rep["iters"] - r["iters"]) <= 4
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-9
    # and it is not the first-order solution
    r1 = oracle.solve(p, tol=1e-12)
    assert _rel(T.cpu().numpy(), r1["T"], p) > 1e-4
    s.close()


@pytest.mark.parametrize("kinds,plan", [((0, 1), None), ((0, 1), dict(NR=2, P=1)), ((0, 2), None),
                                        ((0, 0), dict(NR=1, P=2))])
def test_masked_2d_second_order_fixed_iterations(hip_lib, kinds, plan):
    p = bi.multi_hole_2d(37, 70, seed=6, n_bands=3, n_theta=2, n_phi=1, kinds=kinds)
    s = _solver(hip_lib, p, plan=plan)
    T, q, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6, order=2)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    act = p.mask > 0
    qs = np.abs(r["q"][act]).max()
    assert np.abs(q.cpu().numpy()[act] - r["q"][act]).max() < 1e-10 * qs
    s.close()


def test_square_second_order_converged_fp64_and_fp32(hip_lib):
    p = bi.square_2d(64, L=0.25e-6, n_bands=6, n_theta=2, n_phi=2)
    r = oracle.solve(p, tol=1e-12, order=2)
    for prec, tol, bar in (("fp64", 1e-12, 1e-9), ("fp32", 1e-7, 1e-4)):
        s = _solver(hip_lib, p, prec)
        T, _, rep = s.solve(torch.tensor(p.Q, device="cuda"), tol=tol, check_every=8, max_iters=5000)
        assert rep["status"] == "ok", (prec, rep)
        assert _rel(T.cpu().numpy(), r["T"], p) < bar, prec
        s.close()


def test_second_order_batch_matches_single(hip_lib):
    ps = [bi.square_2d(n, L=0.1e-6, n_bands=3, n_theta=2, n_phi=1) for n in (20, 33)]
    bs = hip_lib.BatchSolver(ps, precision="fp64")
    assert hip_lib.bte_set_order(bs._h, 2) == hip_lib.BTE_OK
    Qs = [torch.tensor(p.Q, device="cuda") for p in ps]
    Ts, _, _ = bs.solve(Qs, tol=0.0, max_iters=7, check_every=7)
    for p, T in zip(ps, Ts):
        r = oracle.solve(p, tol=0.0, max_iters=7, order=2)
        assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    bs.close()


# 3D: (geometry, plans); the FP64 rows layout takes up to eight waves with one
# row per lane, or four with two
PLANS3 = [None, dict(G=1, P=1, NR=1), dict(G=1, P=2, NR=2), dict(G=1, P=8, NR=1)]


@pytest.mark.parametrize("kinds", [(0, 1), (0, 2), (0, 0)], ids=["diffuse", "specular", "isothermal"])
@pytest.mark.parametrize("plan", PLANS3, ids=["default", "p1nr1", "p2nr2", "p8nr1"])
def test_box_3d_second_order_fixed_iterations(hip_lib, kinds, plan):
    p = bi.random_box_3d(11, 9, 13, seed=1, n_bands=2, n_theta=2, n_phi=1, kinds=kinds)
    s = _solver(hip_lib, p, plan=plan)
    assert s.plan()["NR"] >= 1
    T, q, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6, order=2)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    act = p.mask > 0
    qs = np.abs(r["q"][act]).max()
    assert np.abs(q.cpu().numpy()[act] - r["q"][act]).max() < 1e-10 * qs
    s.close()


@pytest.mark.parametrize("make", [lambda: bi.staircase_3d(bi.BC_DIFFUSE, n_bands=2, n_theta=2, n_phi=1),
                                  lambda: bi.staircase_3d(bi.BC_SPECULAR, n_bands=2, n_theta=2, n_phi=1),
                                  lambda: bi.finfet_3d(scale=8, n_bands=3, n_theta=2, n_phi=2),
                                  lambda: bi.finfet_3d_mixed(scale=4, n_bands=2, n_theta=1, n_phi=1)],
                         ids=["staircase_diffuse", "staircase_specular", "finfet8", "finfet4_mixed"])
def test_masks_3d_second_order_fixed_iterations(hip_lib, make):
    p = make()
    s = _solver(hip_lib, p)
    T, q, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=0.0, max_iters=5, check_every=5)
    r = oracle.solve(p, tol=0.0, max_iters=5, order=2)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    act = p.mask > 0
    qs = np.abs(r["q"][act]).max()
    assert np.abs(q.cpu().numpy()[act] - r["q"][act]).max() < 1e-10 * qs
    s.close()


def test_finfet_quarter_all_bands_second_order(hip_lib):
    """The FinFET-like mask at a quarter of its size per axis with all 15 bands
    and 128 directions (the bench's band and direction counts), FP64 at 1e-10
    and FP32 sweeps at 1e-4, three iterations."""
    p = bi.finfet_3d(scale=4)
    assert p.B == 15 and p.M == 128
    r = oracle.solve(p, tol=0.0, max_iters=3, order=2, threads=oracle.num_threads())
    act = p.mask > 0
    for prec, bar in (("fp64", 1e-10), ("fp32", 1e-4)):
        s = _solver(hip_lib, p, prec)
        T, q, _ = s.solve(torch.tensor(p.Q, device="cuda"), tol=0.0, max_iters=3, check_every=3)
        assert _rel(T.cpu().numpy(), r["T"], p) < bar, prec
        qs = np.abs(r["q"][act]).max()
        assert np.abs(q.cpu().numpy()[act] - r["q"][act]).max() < bar * qs, prec
        s.close()


def test_box_3d_second_order_converged_fp64_and_fp32(hip_lib):
    p = bi.random_box_3d(12, 10, 9, seed=4, n_bands=3, n_theta=2, n_phi=2, kinds=(0, 1))
    r = oracle.solve(p, tol=1e-12, order=2)
    r1 = oracle.solve(p, tol=1e-12)
    # (FP32: the successive-change stop at 1e-6 sits ~1e-5 from the fixed point)
    for prec, tol, bar, plan in (("fp64", 1e-12, 1e-9, None), ("fp32", 1e-6, 1e-4, dict(G=1, P=8, NR=2))):
        s = _solver(hip_lib, p, prec, plan=plan)
        T, _, rep = s.solve(torch.tensor(p.Q, device="cuda"), tol=tol, check_every=8, max_iters=5000)
        assert rep["status"] == "ok", (prec, rep)
        assert _rel(T.cpu().numpy(), r["T"], p) < bar, prec
        # and it is not the first-order solution
        assert _rel(T.cpu().numpy(), r1["T"], p) > 10 * bar, prec
        s.close()


def test_second_order_refusals(hip_lib):
    # 3D: the pencil layout has no second-order sweep; asking for second order
    # on a pencil plan moves the handle to the rows layout, and a pencil plan
    # is refused afterwards
    p3 = bi.random_box_3d(6, 5, 4, seed=1, n_bands=2, n_theta=1, n_phi=1)
    s = hip_lib.Solver(p3, precision="fp64", plan=dict(G=2, P=2, NR=-1))
    assert s.plan()["NR"] == 0
    s.set_order(2)
    assert s.plan()["NR"] >= 1 and s.plan()["G"] == 1
    with pytest.raises(hip_lib.BTEError) as ei:
        s.set_plan(G=1, P=2, NR=-1)
    assert ei.value.status == hip_lib.BTE_ERR_INVALID
    assert s.plan()["NR"] >= 1
    s.close()
    p = bi.square_2d(12, L=0.1e-6, n_bands=2, n_theta=1, n_phi=1)
    s = _solver(hip_lib, p)
    with pytest.raises(hip_lib.BTEError):
        s.set_plan(G=2)
    assert s.plan()["G"] == 1
    Q = torch.tensor(p.Q, device="cuda")
    with pytest.raises(hip_lib.BTEError) as ei:
        s.solve(Q, tol=1e-8, store_state=True)
    assert ei.value.status == hip_lib.BTE_ERR_STATE
    # back to first order: the ordinary solve and its adjoint work again
    s.set_order(1)
    T, _, _ = s.solve(Q, tol=0.0, max_iters=5, check_every=5)
    r = oracle.solve(p, tol=0.0, max_iters=5)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    s.close()
