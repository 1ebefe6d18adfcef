"""Writes rmat22_cg64.txt: the CG ground truth of Omega_vv = ((alpha L + I)^{-1})_vv
on 64 seeded non-isolated vertices of the R-MAT graph n = 2^22, edge factor 8,
seed 0, alpha = 1 -- the ground-truth protocol of the experiments (Section 6.1:
conjugate gradients to a relative residual of 1e-9 per unit vector e_v).

Calls only the oracle (and the shared seeded input generators).  Run from the
repository root:  python3 tests/golden/make_rmat22_cg64.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat22_cg64.txt")


def main():
    g = inputs.rmat(1 << 22, 8, 0)
    deg = np.diff(g.row_ptr)
    live = np.flatnonzero(deg > 0)
    vs = np.sort(np.random.default_rng(22).choice(live, 64, replace=False))
    om = oracle.omega_diag_cg(g, 1.0, vs, rtol=1e-9)
    with open(OUT, "w") as f:
        f.write("# Omega_vv of 64 seeded non-isolated vertices of R-MAT n = 2^22, edge factor 8,\n")
        f.write("# seed 0 (inputs.rmat), alpha = 1: binary64 Jacobi-CG of the oracle to a\n")
        f.write("# relative residual of 1e-9 per e_v (Section 6.1's ground-truth protocol).\n")
        f.write("# written by tests/golden/make_rmat22_cg64.py (oracle only)\n")
        f.write(f"# n {g.n} nnz {g.col_idx.size}\n")
        f.write("# vertex degree omega_vv\n")
        for v, o in zip(vs, om):
            f.write(f"{int(v)} {int(deg[v])} {float(o).hex()}\n")


if __name__ == "__main__":
    main()
