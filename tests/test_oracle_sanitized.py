"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only), run on a few small graphs through a plain C driver:
no sanitizer report, and the same trees, counts and estimates as the
ordinary build loaded through ctypes."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import inputs
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "helpers", "oracle_san_driver.c")


@pytest.fixture(scope="module")
def san_driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    out = str(tmp_path_factory.mktemp("san") / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           DRIVER, oracle.SRC_PATH, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _run(exe, tmp_path, g, alpha, seed, stream, t0, count):
    path = str(tmp_path / "g.bin")
    w = getattr(g, "weights", None)
    with open(path, "wb") as f:
        f.write(struct.pack("<iqidQIII", g.n, g.col_idx.size, 1 if w is not None else 0, alpha,
                            seed, stream, t0, count))
        f.write(np.ascontiguousarray(g.row_ptr, np.int32).tobytes())
        f.write(np.ascontiguousarray(g.col_idx, np.int32).tobytes())
        if w is not None:
            f.write(np.ascontiguousarray(w, np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-2000:]
    lines = r.stdout.split("\n")
    trees = [tuple(int(x) for x in ln.split()) for ln in lines[:count]]
    tail = dict(ln.split() for ln in lines[count:] if ln.strip())
    return trees, {k: int(v) for k, v in tail.items()}


CASES = [
    ("er200", lambda: inputs.erdos_renyi(200, 0.03, 1), 1.0, 3, 0, 5, 20),
    ("grid_w", lambda: inputs.with_weights(inputs.grid_removed(15, 20, 0.12, 2), 4), 2.0, 1, 7, 0, 12),
    ("ba500", lambda: inputs.barabasi_albert(500, 3, 5), 0.5, 9, 0, 40, 10),
    ("isolated", lambda: inputs.from_edge_list(7, [(0, 1), (2, 3)]), 1.0, 0, 0, 0, 6),
    ("path", lambda: inputs.from_edge_list(60, [(i, i + 1) for i in range(59)]), 0.1, 2, 1, 3, 8),
]


@pytest.mark.parametrize("name,make,alpha,seed,stream,t0,count", CASES, ids=[c[0] for c in CASES])
def test_sanitized_oracle_matches(san_driver, tmp_path, name, make, alpha, seed, stream, t0, count):
    g = make()
    trees, tot = _run(san_driver, tmp_path, g, alpha, seed, stream, t0, count)
    ref = oracle.sample(g, alpha, seed, t0, count, stream=stream, per_tree=True)
    assert [t[0] for t in trees] == [int(x) for x in ref.digests]
    assert [t[1] for t in trees] == [int(x) for x in ref.steps]
    assert [t[2] for t in trees] == [int(x) for x in ref.roots]
    assert tot["R"] == int(ref.R.sum())
    assert tot["visits"] == int(ref.visits.sum())
    assert tot["parents"] == int(ref.parents.astype(np.uint32).astype(np.uint64).sum())
    d, _, _ = oracle.estimate(ref.R, max(count, 1))
    assert tot["est"] == int(d.view(np.uint64).sum(dtype=np.uint64))
    assert tot["tau"] == oracle.tau(g.m, g.n, 0.1, 0.1)
