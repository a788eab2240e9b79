"""Writes sampled converged oracle values under tests/golden/ for GPU parity
tests whose oracle solve takes minutes (run from the repository root:
python tests/golden/make_golden_samples.py). Calls only the FP64 oracle and
the seeded input generators.

square256_samples.txt: the 2D nongray square of the throughput workload
(256 x 256 cells, 1 um, 15 bands, 8 x 2 directions per octant, seeded
Gaussian hot spot, isothermal 300 K edges), converged to 1e-10 on both
residuals of Eq. 22; T and q at 1024 seeded cells, and the largest |T - T_ref| and |q|.

batch_lowkn_samples.txt: the two lowest-Knudsen instances of the seeded
batch that the GPU tests use (indices 144, Kn = 0.0100, and 131, Kn = 0.0282,
of batch_instances()), converged to 1e-12, and stopped by the same rule at
1e-6 (the tolerance of the batch workload); T at 512 seeded cells each, and
the largest |T - T_ref|.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import bte_inputs as bi  # noqa: E402
import oracle  # noqa: E402

BATCH_LOWKN = (144, 131)


def sample_cells(p, n, seed):
    act = np.flatnonzero(p.mask)
    return np.sort(np.random.default_rng(seed).choice(act, size=min(n, act.size), replace=False))


def main():
    p = bi.square_2d()
    r = oracle.solve(p, tol=1e-10, max_iters=100000)
    assert r["status"] == "converged"
    cells = sample_cells(p, 1024, 7)
    with open(os.path.join(HERE, "square256_samples.txt"), "w") as f:
        f.write("# converged oracle (tol 1e-10) on the 256^2 nongray square, 15 bands, 128 directions\n")
        act = p.mask > 0
        f.write(f"# iterations {r['iters']}; columns: cell T_L(K) q_x q_y (W/m^2); "
                "written by tests/golden/make_golden_samples.py\n")
        f.write(f"# max|T - T_ref| {np.abs(r['T'][act] - p.T_ref).max():.15e} "
                f"max|q| {np.linalg.norm(r['q'][act], axis=1).max():.15e}\n")
        for c in cells:
            f.write(f"{c:d} {r['T'][c]:.15e} {r['q'][c, 0]:.15e} {r['q'][c, 1]:.15e}\n")
    ps = bi.batch_instances()
    with open(os.path.join(HERE, "batch_lowkn_samples.txt"), "w") as f:
        f.write("# oracle on the lowest-Kn instances of batch_instances(), stopped at tol 1e-12 and at 1e-6\n")
        f.write("# columns: instance tolerance cell T_L(K); written by tests/golden/make_golden_samples.py\n")
        for i in BATCH_LOWKN:
            q = ps[i]
            cells = sample_cells(q, 512, 8 + i)
            for tol in (1e-12, 1e-6):
                r = oracle.solve(q, tol=tol, max_iters=400000)
                assert r["status"] == "converged"
                f.write(f"# instance {i} tol {tol:.0e} Kn {q.Kn:.6f} n {q.n[0]}x{q.n[1]} iterations {r['iters']} "
                        f"max|T - T_ref| {np.abs(r['T'][q.mask > 0] - q.T_ref).max():.15e}\n")
                for c in cells:
                    f.write(f"{i:d} {tol:.0e} {c:d} {r['T'][c]:.15e}\n")


if __name__ == "__main__":
    main()
