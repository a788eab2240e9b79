"""GPU parity of the 3D rows-per-lane sweep (the default 3D layout) across its
shapes, against the FP64 oracle at 1e-10 of max|T - T_ref| (fixed iteration
counts, both paths).

Geometries: the staircase (blocks of 8 columns whose plane ranges differ and
overlap by one or two planes, with diffuse or specular walls), a box with
odd-length axes (a partial last lane with two rows per lane), boxes 4 and 3
cells thick, the FinFET at a quarter of its size per axis; plans with 1 to 8
waves per workgroup and 1 or 2 rows per lane, and the pencil layout."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(bte, p, plan=None, iters=5, precision="fp64"):
    s = bte.Solver(p, precision=precision, plan=plan)
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
    T, q, rep = s.solve(Q, tol=0.0, max_iters=iters, check_every=iters)
    torch.cuda.synchronize()
    out = T.cpu().numpy(), q.cpu().numpy(), s.plan()
    s.close()
    return out


def _check(p, T, q, r, bar=1e-10):
    act = p.mask > 0
    scale = np.abs(r["T"][act] - p.T_ref).max()
    assert np.abs(T[act] - r["T"][act]).max() < bar * scale
    qs = np.abs(r["q"]).max()
    assert np.abs(q[act] - r["q"][act]).max() < bar * qs


# (eight waves with two rows per lane need more LDS than a workgroup has in
# FP64; the FP32 test below takes that shape)
PLANS = [None, dict(G=1, P=1, NR=1), dict(G=1, P=2, NR=2), dict(G=1, P=4, NR=1), dict(G=1, P=8, NR=1),
         dict(G=1, P=2, NR=-1)]


@pytest.mark.parametrize("kind", [bi.BC_DIFFUSE, bi.BC_SPECULAR])
@pytest.mark.parametrize("plan", PLANS, ids=["default", "p1nr1", "p2nr2", "p4nr1", "p8nr1", "pencil"])
def test_staircase_plans_fp64(hip_lib, kind, plan):
    p = bi.staircase_3d(kind, n_bands=2, n_theta=2, n_phi=1)
    T, q, got = _run(hip_lib, p, plan=plan, iters=5)
    r = oracle.solve(p, tol=0.0, max_iters=5)
    _check(p, T, q, r)
    if plan is not None:
        assert got["P"] == plan["P"]
        assert got["NR"] == (0 if plan["NR"] < 0 else plan["NR"])


@pytest.mark.parametrize("kind", [bi.BC_DIFFUSE, bi.BC_SPECULAR])
def test_staircase_eight_waves_fp32(hip_lib, kind):
    p = bi.staircase_3d(kind, n_bands=2, n_theta=2, n_phi=1)
    T, q, got = _run(hip_lib, p, plan=dict(G=1, P=8, NR=2), iters=5, precision="fp32")
    assert got["P"] == 8 and got["NR"] == 2
    r = oracle.solve(p, tol=0.0, max_iters=5)
    _check(p, T, q, r, bar=1e-4)


def test_eight_waves_two_rows_fp64_rejected(hip_lib):
    p = bi.staircase_3d(bi.BC_DIFFUSE, n_bands=2, n_theta=2, n_phi=1)
    s = hip_lib.Solver(p, precision="fp64")
    with pytest.raises(hip_lib.BTEError, match="LDS"):
        s.set_plan(G=1, P=8, NR=2)
    s.close()


@pytest.mark.parametrize("kinds", [(0, 1), (0, 2)], ids=["diffuse", "specular"])
def test_odd_axes_two_rows(hip_lib, kinds):
    """Two rows per lane on a box whose every axis has odd length: the last
    lane's second row lies outside the grid whichever axis the lanes run
    along, and its partial sums must not land on a cell of the next line."""
    p = bi.random_box_3d(11, 9, 13, seed=1, n_bands=2, n_theta=2, n_phi=1, kinds=kinds)
    r = oracle.solve(p, tol=0.0, max_iters=5)
    for plan, prec, bar in ((dict(G=1, P=1, NR=2), "fp64", 1e-10), (dict(G=1, P=2, NR=2), "fp64", 1e-10),
                            (dict(G=1, P=4, NR=2), "fp64", 1e-10), (dict(G=1, P=8, NR=2), "fp32", 1e-4)):
        T, q, got = _run(hip_lib, p, plan=plan, iters=5, precision=prec)
        assert got["NR"] == 2
        _check(p, T, q, r, bar=bar)


def test_thin_boxes_fp64(hip_lib):
    """Boxes 4 and 3 cells thick: the plane axis needs at least 4 cells, so
    the 3-cell axis can only be the step or lane axis."""
    for nz in (4, 3):
        p = bi.random_box_3d(19, 70, nz, seed=7, n_bands=2, n_theta=1, n_phi=1, hole=(nz == 4))
        T, q, got = _run(hip_lib, p, iters=4)
        r = oracle.solve(p, tol=0.0, max_iters=4)
        _check(p, T, q, r)


def test_finfet_quarter_plans_fp64(hip_lib):
    p = bi.finfet_3d(scale=4, n_bands=3, n_theta=2, n_phi=2)
    r = oracle.solve(p, tol=0.0, max_iters=4)
    for plan in (None, dict(G=1, P=2, NR=1)):
        T, q, _ = _run(hip_lib, p, plan=plan, iters=4)
        _check(p, T, q, r)


def test_staircase_fp32_converged(hip_lib):
    """FP32 sweeps to tol 1e-6 against the oracle stopped by the same rule at
    the same tolerance (the successive-change test stops up to tol/(1 - rho)
    from the fixed point, which both sides share)."""
    p = bi.staircase_3d(bi.BC_DIFFUSE, n_bands=2, n_theta=2, n_phi=1)
    s = hip_lib.Solver(p, precision="fp32")
    Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
    T, q, rep = s.solve(Q, tol=1e-6, check_every=1, max_iters=20000)
    s.close()
    assert rep["status"] == "ok"
    r = oracle.solve(p, tol=1e-6)
    act = p.mask > 0
    scale = np.abs(r["T"][act] - p.T_ref).max()
    assert np.abs(T.cpu().numpy()[act] - r["T"][act]).max() < 1e-4 * scale
