"""GPU parity: the HIP sweep library against the FP64 oracle.

Every case runs both paths on the same seeded inputs, either for the same
fixed number of iterations (tol = 0) or both converged far below the
comparison tolerance. FP64 bar: 1e-10 relative to the imposed temperature
scale max|T - T_ref|. FP32 bar: 1e-4 of the same scale.
"""
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
    out = T.cpu().numpy(), q.cpu().numpy(), rep
    s.close()
    return out


def _rel(a, b, p):
    act = p.mask > 0
    scale = np.abs(b[act] - p.T_ref).max()
    return np.abs(a[act] - b[act]).max() / scale


def test_film_1d_fixed_iterations(hip_lib):
    p = bi.film_1d()
    T, q, rep = _solve_gpu(hip_lib, p, tol=0.0, max_iters=12, check_every=1)
    r = oracle.solve(p, tol=0.0, max_iters=12)
    assert rep["iters"] == 12
    assert _rel(T, r["T"], p) < 1e-10
    assert np.abs(q[:, 0] - r["q"][:, 0]).max() < 1e-10 * np.abs(r["q"]).max()


def test_film_1d_converged(hip_lib):
    p = bi.film_1d()
    T, q, rep = _solve_gpu(hip_lib, p, tol=1e-10, check_every=1)
    r = oracle.solve(p, tol=1e-10)
    assert rep["status"] == "ok"
    assert rep["iters"] == r["iters"]
    assert _rel(T, r["T"], p) < 1e-10


@pytest.mark.parametrize("plan", [dict(G=1, R=1, P=1, NR=1), dict(G=2, R=2, P=1, NR=1),
                                  dict(G=1, R=1, P=2, NR=2), dict(G=2, R=1, P=2, NR=4),
                                  dict(G=1, R=2, P=2, NR=1)])
def test_square_2d_fp64_plans(hip_lib, plan):
    """Strips processed in sequence and pipelined across waves, a partial last
    strip, one to four rows per lane, one to four waves per workgroup."""
    p = bi.square_2d(100, L=0.4e-6, n_bands=4, n_theta=2, n_phi=2)
    T, q, rep = _solve_gpu(hip_lib, p, plan=plan, tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6)
    assert _rel(T, r["T"], p) < 1e-10
    qs = np.abs(r["q"]).max()
    assert np.abs(q - r["q"]).max() < 1e-10 * qs
    off = p.mask == 0
    assert (T[off] == 0).all() and (q[off] == 0).all()  # inactive cells are written as zeros


def test_rectangle_ragged_fp64(hip_lib):
    p = bi.square_2d(70, L=0.3e-6, n_bands=3, n_theta=2, n_phi=1)
    # ragged rectangle: drop rows so ny is not a multiple of 64
    n = (70, 37, 1)
    mask = np.ones(70 * 37, dtype=np.uint8)
    fbc = bi.face_bc_from_mask(n, 2, mask, lambda i, j, k, f: 0)
    p = p.replace(n=n, mask=mask, face_bc=fbc, Q=p.Q[: 70 * 37].copy())
    T, q, rep = _solve_gpu(hip_lib, p, plan=dict(G=2, R=1, P=1, NR=1), tol=0.0, max_iters=5, check_every=5)
    r = oracle.solve(p, tol=0.0, max_iters=5)
    assert _rel(T, r["T"], p) < 1e-10


@pytest.mark.parametrize("plan", [dict(G=2, R=1, P=1, NR=1), dict(G=1, R=1, P=2, NR=2)])
@pytest.mark.parametrize("seed,kinds", [(0, (0, 1)), (1, (0, 0))])
def test_masked_2d_with_diffuse_walls_fp64(hip_lib, seed, kinds, plan):
    p = bi.random_box_2d(23, 19, seed=seed, n_bands=3, n_theta=2, n_phi=1, kinds=kinds)
    T, q, rep = _solve_gpu(hip_lib, p, plan=plan, tol=0.0, max_iters=9, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=9)
    assert _rel(T, r["T"], p) < 1e-10


@pytest.mark.parametrize("plan", [dict(G=1, R=2, P=1, NR=4), dict(G=2, R=1, P=2, NR=2)])
def test_multi_hole_2d_diffuse_fp64(hip_lib, plan):
    """Holes inside a lane's rows, across lanes and beside strip boundaries;
    diffuse walls on every face but the bottom."""
    p = bi.multi_hole_2d(50, 300, seed=4, n_bands=2, n_theta=2, n_phi=1)
    T, q, rep = _solve_gpu(hip_lib, p, plan=plan, tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6, threads=oracle.num_threads())
    assert _rel(T, r["T"], p) < 1e-10
    qs = np.abs(r["q"]).max()
    assert np.abs(q - r["q"]).max() < 1e-10 * qs
    off = p.mask == 0
    assert off.any() and (T[off] == 0).all() and (q[off] == 0).all()  # inactive cells are written as zeros


def test_square_2d_converged_fp64(hip_lib):
    p = bi.square_2d(64, L=0.25e-6, n_bands=5, n_theta=4, n_phi=2)
    T, q, rep = _solve_gpu(hip_lib, p, tol=1e-13, check_every=4)
    r = oracle.solve(p, tol=1e-13)
    assert rep["status"] == "ok"
    assert _rel(T, r["T"], p) < 1e-10


def test_square_2d_fp32_tolerance(hip_lib):
    p = bi.square_2d(96, L=0.5e-6, n_bands=15, n_theta=4, n_phi=2)
    T, q, rep = _solve_gpu(hip_lib, p, precision="fp32", tol=1e-7, check_every=8)
    r = oracle.solve(p, tol=1e-10)
    assert _rel(T, r["T"], p) < 1e-4


def test_box_3d_fp64(hip_lib):
    p = bi.random_box_3d(11, 9, 13, seed=1, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 1))
    T, q, rep = _solve_gpu(hip_lib, p, tol=0.0, max_iters=7, check_every=7)
    r = oracle.solve(p, tol=0.0, max_iters=7)
    assert _rel(T, r["T"], p) < 1e-10


def test_finfet_small_fp64(hip_lib):
    p = bi.finfet_3d(scale=8, n_bands=3, n_theta=2, n_phi=2)
    T, q, rep = _solve_gpu(hip_lib, p, tol=0.0, max_iters=6, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=6)
    assert _rel(T, r["T"], p) < 1e-10
