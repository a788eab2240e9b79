"""Full-size cases: the 2D bench workload (256 x 256, 15 bands, 128 directions)
against the oracle element by element at a fixed iteration count, in the
kernel shape the bench uses; the 3D FinFET-like domain at half size against
the oracle and at full size through properties that hold at any size
(monotone, non-negative source iteration from T_ref under a non-negative
source with walls at T_ref; linearity in the source; FP32 vs FP64)."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b, p):
    act = p.mask > 0
    return np.abs(a[act] - b[act]).max() / np.abs(b[act] - p.T_ref).max()


@pytest.fixture(scope="module")
def square_full():
    p = bi.square_2d(256)
    r = oracle.solve(p, tol=0.0, max_iters=4, threads=oracle.num_threads())
    return p, r


def test_square_full_fp32_bench_shape(hip_lib, square_full):
    p, r = square_full
    s = hip_lib.Solver(p, precision="fp32")
    Q = torch.tensor(p.Q, device="cuda")
    s.autotune(Q, n_iters=3)
    T, q, rep = s.solve(Q, tol=0.0, max_iters=4, check_every=4)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-5
    qs = np.abs(r["q"]).max()
    assert np.abs(q.cpu().numpy() - r["q"]).max() < 1e-4 * qs
    s.close()


def test_square_full_fp64(hip_lib, square_full):
    p, r = square_full
    s = hip_lib.Solver(p, precision="fp64")
    Q = torch.tensor(p.Q, device="cuda")
    T, q, rep = s.solve(Q, tol=0.0, max_iters=4, check_every=2)
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-10
    s.close()


def test_finfet_half_size_fp32(hip_lib):
    p = bi.finfet_3d(scale=2, n_bands=15, n_theta=4, n_phi=4)
    s = hip_lib.Solver(p, precision="fp32")
    T, q, rep = s.solve(torch.tensor(p.Q, device="cuda"), tol=0.0, max_iters=3, check_every=3)
    r = oracle.solve(p, tol=0.0, max_iters=3, threads=oracle.num_threads())
    assert _rel(T.cpu().numpy(), r["T"], p) < 1e-4
    s.close()


def test_finfet_full_properties(hip_lib):
    p = bi.finfet_3d(scale=1)
    act = p.mask > 0
    Q = torch.tensor(p.Q, device="cuda")
    s32 = hip_lib.Solver(p, precision="fp32")
    prev = np.zeros(p.ncell)
    for n in (1, 2, 4):
        T, _, _ = s32.solve(Q, tol=0.0, max_iters=n, check_every=n)
        dT = T.cpu().numpy()[act] - p.T_ref
        assert np.isfinite(dT).all()
        assert dT.min() >= -1e-5 * dT.max()          # non-negative
        assert (dT - prev[act] >= -1e-5 * dT.max()).all()  # monotone in n
        prev = np.zeros(p.ncell)
        prev[act] = dT
    # linearity in Q at a fixed iteration count (FP64)
    s64 = hip_lib.Solver(p, precision="fp64")
    Q2 = torch.roll(Q, 1000)
    T1, _, _ = s64.solve(Q, tol=0.0, max_iters=3, check_every=3)
    T2, _, _ = s64.solve(Q2, tol=0.0, max_iters=3, check_every=3)
    T3, _, _ = s64.solve(2.0 * Q - Q2, tol=0.0, max_iters=3, check_every=3)
    a, b, c = (x.cpu().numpy()[act] - p.T_ref for x in (T1, T2, T3))
    assert np.abs(c - (2 * a - b)).max() < 1e-10 * np.abs(c).max()
    # FP32 sweeps agree with FP64 at the same iteration count
    T32, _, _ = s32.solve(Q, tol=0.0, max_iters=3, check_every=3)
    assert np.abs(T32.cpu().numpy()[act] - p.T_ref - a).max() < 1e-4 * np.abs(a).max()
    s32.close()
    s64.close()


def test_determinism_fp64(hip_lib):
    p = bi.square_2d(128, L=0.5e-6, n_bands=6, n_theta=2, n_phi=2)
    s = hip_lib.Solver(p, precision="fp64")
    Q = torch.tensor(p.Q, device="cuda")
    T1, q1, _ = s.solve(Q, tol=0.0, max_iters=5, check_every=5)
    T1 = T1.clone()
    T2, q2, _ = s.solve(Q, tol=0.0, max_iters=5, check_every=5)
    assert torch.equal(T1, T2)
    s.close()


def test_plans_agree_fp64(hip_lib):
    """Every kernel shape gives the same per-cell expression: equal to rounding."""
    p = bi.square_2d(130, L=0.5e-6, n_bands=4, n_theta=2, n_phi=2)
    Q = torch.tensor(p.Q, device="cuda")
    ref = None
    for plan in (dict(G=1, R=1, P=1, NR=1), dict(G=2, R=3, P=1, NR=1), dict(G=2, R=2, P=2, NR=1),
                 dict(G=1, R=1, P=2, NR=4), dict(G=2, R=1, P=2, NR=2)):
        s = hip_lib.Solver(p, precision="fp64", plan=plan)
        T, _, _ = s.solve(Q, tol=0.0, max_iters=3, check_every=3)
        T = T.cpu().numpy()
        if ref is None:
            ref = T
        else:
            assert np.abs(T - ref).max() < 1e-13 * np.abs(ref - 300).max()
        s.close()


def test_oversized_plan_rejected(hip_lib):
    """A plan whose LDS carve-up exceeds the per-workgroup limit is an input error."""
    p = bi.square_2d(130, L=0.5e-6, n_bands=4, n_theta=2, n_phi=2)
    with pytest.raises(hip_lib.BTEError, match="LDS"):
        hip_lib.Solver(p, precision="fp64", plan=dict(G=2, R=1, P=4, NR=4))


def test_plan_wave_limit_rejected(hip_lib):
    """The 1D/2D kernel takes at most four waves per workgroup (R*P <= 4)."""
    p = bi.square_2d(130, L=0.5e-6, n_bands=4, n_theta=2, n_phi=2)
    with pytest.raises(hip_lib.BTEError, match="R\\*P <= 4"):
        hip_lib.Solver(p, precision="fp32", plan=dict(G=1, R=2, P=4, NR=1))
