"""Writes the stored oracle values under tests/golden/ (run from the repository
root: python tests/golden/make_golden.py). Calls only the FP64 oracle and the
seeded input generators.

film_1d_kn1.txt: the converged lattice temperature of the 1D gray cross-plane
film (Results, "1D cross-plane phonon transport": 100 nm, Kn = 1, thermalizing
walls at 301 K and 299 K), 200 cells, 32-point Gauss-Legendre directions,
first-order upwind faces, tolerance 1e-12 on the residuals of Eq. 22.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import bte_inputs as bi  # noqa: E402
import oracle  # noqa: E402


def main():
    p = bi.film_1d()
    r = oracle.solve(p, tol=1e-12, max_iters=100000)
    assert r["status"] == "converged"
    with open(os.path.join(HERE, "film_1d_kn1.txt"), "w") as f:
        f.write("# converged T_L (K) of the 1D film, 200 cells, Kn = 1, 32 GL directions, first-order faces\n")
        f.write(f"# iterations {r['iters']}; written by tests/golden/make_golden.py from the FP64 oracle\n")
        for t in r["T"]:
            f.write(f"{t:.15e}\n")


if __name__ == "__main__":
    main()
