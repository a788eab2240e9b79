"""GPU tests of the batched persistent solver: every instance of a batch must
equal its single-instance solve and the oracle, with per-instance convergence
and retirement."""
import numpy as np
import pytest

import bte_inputs as bi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _small_batch(n=6, seed=11):
    insts = bi.batch_instances(n_inst=n, seed=seed, nx_range=(12, 40), ny_range=(10, 70),
                               Kn_range=(0.1, 5.0), n_bands=4, n_theta=2, n_phi=1)
    return insts


def test_batch_matches_single_and_oracle_fp64(hip_lib):
    insts = _small_batch()
    bs = hip_lib.BatchSolver(insts, precision="fp64", plan=dict(G=2, R=1, P=2, NR=2))
    Qs = [torch.tensor(p.Q, device="cuda") for p in insts]
    Ts, qs, reps = bs.solve(Qs, tol=1e-12, check_every=4)
    torch.cuda.synchronize()
    iters = [r["iters"] for r in reps]
    assert all(r["status"] == "ok" for r in reps)
    assert len(set(iters)) > 1  # uneven convergence: instances retire independently
    for k, p in enumerate(insts):
        s = hip_lib.Solver(p, precision="fp64", plan=dict(G=2, R=1, P=2, NR=2))
        T1, _, r1 = s.solve(Qs[k], tol=1e-12, check_every=4)
        assert r1["iters"] == reps[k]["iters"]
        a = Ts[k].cpu().numpy()
        b = T1.cpu().numpy()
        assert np.array_equal(a, b)
        ro = oracle.solve(p, tol=1e-13)
        assert np.abs(a - ro["T"]).max() < 1e-9 * np.abs(ro["T"] - 300).max()
        s.close()


def test_batch_fixed_iterations_fp32(hip_lib):
    insts = _small_batch(n=5, seed=12)
    bs = hip_lib.BatchSolver(insts, precision="fp32")
    Qs = [torch.tensor(p.Q, device="cuda") for p in insts]
    Ts, qs, reps = bs.solve(Qs, tol=0.0, max_iters=10, check_every=5)
    for k, p in enumerate(insts):
        ro = oracle.solve(p, tol=0.0, max_iters=10)
        sc = np.abs(ro["T"] - 300).max()
        assert np.abs(Ts[k].cpu().numpy() - ro["T"]).max() < 1e-4 * sc


def test_batch_adjoint_matches_single(hip_lib):
    insts = _small_batch(n=4, seed=13)
    plan = dict(G=2, R=1, P=2, NR=2)
    bs = hip_lib.BatchSolver(insts, precision="fp64", plan=plan)
    Qs = [torch.tensor(p.Q, device="cuda") for p in insts]
    Ts, _, _ = bs.solve(Qs, tol=1e-12, check_every=4, store_state=True)
    gs = [torch.ones(p.ncell, dtype=torch.float64, device="cuda") / p.ncell for p in insts]
    dtau_b, dQ_b, reps = bs.adjoint(gs, tol=1e-12, check_every=4)
    for k, p in enumerate(insts):
        s = hip_lib.Solver(p, precision="fp64", plan=plan)
        s.solve(Qs[k], tol=1e-12, check_every=4, store_state=True)
        dtau, dQ, _ = s.adjoint(gs[k], tol=1e-12, check_every=4)
        assert np.abs(dtau_b[k] - dtau).max() <= 1e-12 * np.abs(dtau).max()
        assert np.abs(dQ_b[k].cpu().numpy() - dQ.cpu().numpy()).max() <= 1e-12 * dQ.abs().max().item()
        s.close()


def test_batch_with_reflecting_walls_matches_single(hip_lib):
    """A batch mixing diffuse-walled and specular-walled instances (bottom edge
    isothermal): the batched forward and adjoint (with the wall-value adjoint
    and the length-scale gradient) equal the single-instance ones."""
    base = _small_batch(n=4, seed=17)
    insts = []
    for k, p in enumerate(base):
        fbc = bi.face_bc_from_mask(p.n, 2, p.mask, lambda i, j, kk, f: 0 if (f == 2 and j == 0) else 1)
        kind = bi.BC_DIFFUSE if k % 2 == 0 else bi.BC_SPECULAR
        insts.append(p.replace(face_bc=fbc, bc_kind=np.array([bi.BC_ISOTHERMAL, kind], dtype=np.int32),
                               bc_T=np.array([305.0, 300.0])))
    plan = dict(G=1, R=1, P=2, NR=1)
    bs = hip_lib.BatchSolver(insts, precision="fp64", plan=plan)
    Qs = [torch.tensor(p.Q, device="cuda") for p in insts]
    Ts, _, reps = bs.solve(Qs, tol=1e-12, check_every=4, store_state=True)
    assert all(r["status"] == "ok" for r in reps)
    gs = [torch.ones(p.ncell, dtype=torch.float64, device="cuda") / p.ncell for p in insts]
    dtau_b, dQ_b, _ = bs.adjoint(gs, tol=1e-12, check_every=4)
    ds_b = bs.adjoint_dscale()
    for k, p in enumerate(insts):
        s = hip_lib.Solver(p, precision="fp64", plan=plan)
        T1, _, r1 = s.solve(Qs[k], tol=1e-12, check_every=4, store_state=True)
        assert r1["iters"] == reps[k]["iters"]
        assert np.abs(Ts[k].cpu().numpy() - T1.cpu().numpy()).max() <= 1e-12 * 5.0
        ro = oracle.solve(p, tol=1e-13, max_iters=100000)
        act = p.mask > 0
        assert np.abs(T1.cpu().numpy()[act] - ro["T"][act]).max() < 1e-9 * np.abs(ro["T"][act] - 300).max()
        dtau, dQ, _ = s.adjoint(gs[k], tol=1e-12, check_every=4)
        assert np.abs(dtau_b[k] - dtau).max() <= 1e-10 * np.abs(dtau).max()
        assert np.abs(dQ_b[k].cpu().numpy() - dQ.cpu().numpy()).max() <= 1e-10 * dQ.abs().max().item()
        assert abs(ds_b[k] - s.adjoint_dscale()) <= 1e-10 * abs(ds_b[k])
        s.close()
