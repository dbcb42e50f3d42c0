"""The C-ABI library on the CPU: it loads, exports every symbol that
include/nbx.h declares, and its host-only entry points (GLL rule,
derivative matrix, brick numbering, argument validation) agree with the
oracle.  Nothing here touches a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import synthetic as S
import paper_2011_04981_amd as nbx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nbx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbx_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = nbx.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version():
    L = nbx.lib()
    assert L.nbx_status_str(0) == b"ok"
    assert L.nbx_status_str(-5) == b"CG breakdown"
    assert L.nbx_version() >= 100


@pytest.mark.parametrize("N", list(range(2, 17)))
def test_gll_and_derivative_match_oracle(N):
    xi, w = nbx.gll(N)
    oxi, ow = O.gll(N)
    np.testing.assert_allclose(xi, oxi, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, ow, rtol=1e-14, atol=0)
    D = nbx.deriv(N)
    oD = O.deriv(N)
    assert np.abs(D - oD).max() <= 1e-13 * np.abs(oD).max()


def test_gll_rejects_bad_sizes():
    L = nbx.lib()
    buf = np.zeros(32)
    p = buf.ctypes.data_as(C.c_void_p)
    assert L.nbx_gll(1, p, p) == -1
    assert L.nbx_gll(17, p, p) == -1
    assert L.nbx_gll(4, None, p) == -1


@pytest.mark.parametrize("dims,N", [((1, 1, 1), 2), ((3, 2, 4), 5), ((4, 4, 4), 10)])
def test_brick_ids_match_oracle(dims, N):
    gid, bnd = nbx.brick_ids(*dims, N)
    ogid, obnd = O.brick_ids(S.Brick(*dims, N))
    np.testing.assert_array_equal(gid, ogid)
    np.testing.assert_array_equal(bnd, obnd)


def test_ax_argument_validation_without_gpu():
    """Invalid sizes and null pointers are rejected before any HIP call;
    E == 0 is a no-op."""
    L = nbx.lib()
    dummy = C.c_void_p(16)
    assert L.nbx_ax(0, dummy, dummy, dummy, 1, 1, C.c_void_p(32), None) == -1   # N < 2
    assert L.nbx_ax(0, dummy, dummy, dummy, 17, 1, C.c_void_p(32), None) == -1  # N > 16
    assert L.nbx_ax(0, dummy, dummy, dummy, 4, -1, C.c_void_p(32), None) == -1  # E < 0
    assert L.nbx_ax(0, None, dummy, dummy, 4, 3, C.c_void_p(32), None) == -1    # null u
    assert L.nbx_ax(0, dummy, dummy, dummy, 4, 3, dummy, None) == -1            # u == w
    assert L.nbx_ax(0, dummy, dummy, dummy, 4, 0, C.c_void_p(32), None) == 0    # E == 0
    assert L.nbx_ax(7, dummy, dummy, dummy, 4, 3, C.c_void_p(32), None) == -2   # precision
    assert L.nbx_problem_create(None, None, 4, 1, None, None, None) == -1
    assert L.nbx_pcg(None, None, None, None, None, None) == -1
    assert L.nbx_dssum(None, 0, None, 1, None) == -1


def test_gs_create_rejects_bad_arguments_without_gpu():
    L = nbx.lib()
    h = C.c_void_p()
    assert L.nbx_gs_create(None, -1, None, C.byref(h), None) == -1
    assert L.nbx_gs_create(None, 5, None, C.byref(h), None) == -1
    assert L.nbx_gs_create(None, 5, None, None, None) == -1


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus above 1 exits with status 2 and
    a JSON line that says so, before anything touches a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
