"""The committed oracle fixtures are what their scripts say: the R-MAT 2^22
and grid CG ground truths hold 64 distinct non-isolated vertices whose Omega_vv
lies in the interval every Omega_vv must (1 / (1 + alpha d_v) <= Omega_vv <= 1),
and on the grid Omega_vv falls as alpha grows (Omega = (alpha L + I)^{-1}: its
diagonal is non-increasing in alpha)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_rmat22_cg64_fixture_shape_and_bounds():
    vs, deg, om = [], [], []
    with open(os.path.join(HERE, "golden", "rmat22_cg64.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b, c = line.split()
            vs.append(int(a))
            deg.append(int(b))
            om.append(float.fromhex(c))
    vs, deg, om = np.array(vs), np.array(deg), np.array(om)
    assert vs.size == 64 and np.unique(vs).size == 64 and (np.diff(vs) > 0).all()
    assert (vs >= 0).all() and (vs < 1 << 22).all()
    assert (deg >= 1).all()
    alpha = 1.0
    assert (om >= 1.0 / (1.0 + alpha * deg) - 1e-9).all()
    assert (om < 1.0).all()


def test_grid_cg64_fixture_shape_bounds_and_monotone():
    rows = {}
    with open(os.path.join(HERE, "golden", "grid_cg64.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, v, d, o = line.split()
            rows.setdefault(float(a), []).append((int(v), int(d), float.fromhex(o)))
    assert sorted(rows) == [0.5, 1.0, 2.0]
    prev = None
    for alpha in (0.5, 1.0, 2.0):
        vs = np.array([r[0] for r in rows[alpha]])
        deg = np.array([r[1] for r in rows[alpha]])
        om = np.array([r[2] for r in rows[alpha]])
        assert vs.size == 64 and np.unique(vs).size == 64
        assert (deg >= 1).all() and (deg <= 4).all()
        assert (om >= 1.0 / (1.0 + alpha * deg) - 1e-9).all() and (om < 1.0).all()
        if prev is not None:
            assert np.array_equal(prev[0], vs)
            assert (om <= prev[1] + 1e-9).all()
        prev = (vs, om)
