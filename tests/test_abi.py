"""The C-ABI library on a host without a GPU: it loads, exports every symbol
that include/fc.h declares, and its host-only logic (tau, argument checks,
error strings) behaves as documented.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_2101_06192_amd as fc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "fc.h")).read()
    return sorted(set(re.findall(r"FC_API\s+[\w\s\*]+?\b(fc_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert len(names) >= 10
    L = fc.lib()
    for name in names:
        assert hasattr(L, name), name


def test_binding_names_match_header():
    # every declared entry point has a ctypes signature in the binding
    L = fc.lib()
    for name in _declared_symbols():
        assert getattr(L, name).argtypes is not None, name


@pytest.mark.parametrize("m,n,eps,delta,kappa", [
    (5012, 1000, 0.1, 0.1, 0.0), (999985, 200000, 0.1, 0.1, 0.0),
    (1758240, 1000000, 0.1, 0.1, 0.0), (999985, 200000, 0.05, 0.01, 0.5),
    (0, 1, 0.5, 0.5, 0.0), (3, 1000, 0.2, 0.3, 0.25)])
def test_tau_matches_oracle(m, n, eps, delta, kappa):
    assert fc.tau(m, n, eps, delta, kappa) == oracle.tau(m, n, eps, delta, kappa)


@pytest.mark.parametrize("args", [
    (10, 10, 0.0, 0.1, 0.0), (10, 10, 1.0, 0.1, 0.0), (10, 10, 0.1, 0.0, 0.0),
    (10, 10, 0.1, 1.0, 0.0), (10, 10, 0.1, 0.1, 1.0), (10, 0, 0.1, 0.1, 0.0),
    (-1, 10, 0.1, 0.1, 0.0), (10, 10, float("nan"), 0.1, 0.0)])
def test_tau_rejects_invalid(args):
    with pytest.raises(fc.FCError) as e:
        fc.tau(*args)
    assert e.value.code == fc.FC_ERR_ARG


def test_tau_null_output():
    assert fc.lib().fc_tau(10, 10, 0.1, 0.1, 0.0, None) == fc.FC_ERR_ARG


def test_error_strings():
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = fc.error_string(code)
        assert s and s != "unknown error code"
    assert fc.error_string(-99) == "unknown error code"
    assert fc.lib().fc_last_error(None) == b"no context"


def test_null_context_arguments():
    L = fc.lib()
    assert L.fc_create(None, 0, None) == fc.FC_ERR_ARG
    assert L.fc_destroy(None) == fc.FC_OK
    assert L.fc_set_stream(None, None) == fc.FC_ERR_ARG
    assert L.fc_set_option(None, b"coop_threads", 256) == fc.FC_ERR_ARG
    st = fc.fc_stats()
    gs = fc.fc_graph(1, 0, ctypes.c_void_p(1), None, None, 0)
    ps = fc.fc_params(1.0, 0.1, 0.1, 0.0, 0, 1, 0, 0, 0)
    assert L.fc_sample(None, ctypes.byref(gs), ctypes.byref(ps), 0, 1, None, None, None,
                       None, None, None, ctypes.byref(st)) == fc.FC_ERR_ARG
    assert L.fc_diag_estimate(None, ctypes.byref(gs), ctypes.byref(ps), None, None,
                              ctypes.byref(st)) == fc.FC_ERR_ARG


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert fc.lib().fc_create(ctypes.byref(h), 0, None) == fc.FC_ERR_HIP
    assert not h.value


def test_struct_layouts():
    # field offsets must agree with the C declarations in include/fc.h
    assert ctypes.sizeof(fc.fc_graph) == 48
    assert fc.fc_graph.nnz.offset == 8 and fc.fc_graph.weights.offset == 32
    assert fc.fc_graph.mem.offset == 40
    assert ctypes.sizeof(fc.fc_params) == 56
    assert fc.fc_params.seed.offset == 32 and fc.fc_params.flags.offset == 52
    assert ctypes.sizeof(fc.fc_stats) == 136 and fc.fc_stats.ms_predraw.offset == 128
    assert ctypes.sizeof(fc.fc_job) == 88 and fc.fc_job.root_counts.offset == 72


def test_struct_layouts_match_the_c_compiler(tmp_path):
    # every ctypes field offset and struct size against offsetof / sizeof from
    # a C program compiled against include/fc.h
    structs = [fc.fc_graph, fc.fc_params, fc.fc_stats, fc.fc_job]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fc.h"', 'int main(void) {']
    for st in structs:
        name = st.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, (name, f)
