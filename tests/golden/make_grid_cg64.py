"""Writes grid_cg64.txt: the CG ground truth of Omega_vv = ((alpha L + I)^{-1})_vv on
64 seeded non-isolated vertices of the 1000 x 1000 grid with 12% of its edges
removed (seed 0), at alpha = 0.5, 1 and 2 -- the ground-truth protocol of the
experiments (Section 6.1: conjugate gradients to a relative residual of 1e-9
per unit vector e_v).

Calls only the oracle (and the shared seeded input generators).  Run from the
repository root:  python3 tests/golden/make_grid_cg64.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_cg64.txt")


def main():
    g = inputs.grid_removed(1000, 1000, 0.12, 0)
    deg = np.diff(g.row_ptr)
    live = np.flatnonzero(deg > 0)
    vs = np.sort(np.random.default_rng(1000).choice(live, 64, replace=False))
    with open(OUT, "w") as f:
        f.write("# Omega_vv of 64 seeded non-isolated vertices of the 1000 x 1000 grid with 12% of\n")
        f.write("# its edges removed (inputs.grid_removed(1000, 1000, 0.12, 0)) at alpha = 0.5, 1, 2:\n")
        f.write("# binary64 Jacobi-CG of the oracle to a relative residual of 1e-9 per e_v\n")
        f.write("# (Section 6.1's ground-truth protocol).\n")
        f.write("# written by tests/golden/make_grid_cg64.py (oracle only)\n")
        f.write("# alpha vertex degree omega_vv\n")
        for alpha in (0.5, 1.0, 2.0):
            om = oracle.omega_diag_cg(g, alpha, vs, rtol=1e-9)
            for v, o in zip(vs, om):
                f.write(f"{alpha} {int(v)} {int(deg[v])} {float(o).hex()}\n")


if __name__ == "__main__":
    main()
