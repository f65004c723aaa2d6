"""The C-ABI library builds for gfx950, loads, exports every declared entry
point and rejects bad arguments on the host (no GPU work is started)."""
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import pytest

from tests.helpers import header_functions

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gep_ci.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2511_01927_amd import gep_ci, build
    if not os.path.exists(gep_ci.LIB_PATH):
        build.build()
    return gep_ci.load()


def test_exports_match_header(lib):
    from paper_2511_01927_amd import gep_ci
    declared = header_functions(HEADER)
    assert sorted(gep_ci.EXPORTS) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", gep_ci.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_code_object_is_gfx950(lib):
    from paper_2511_01927_amd import gep_ci
    data = open(gep_ci.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_opts_defaults(lib):
    from paper_2511_01927_amd import gep_ci
    import ctypes as C
    o = gep_ci.gep_opts()
    lib.gep_opts_default(C.byref(o))
    assert o.max_refine == 1 and o.solve_tol == 1e-9 and o.max_iter == 100000 and o.seed == 1
    assert o.row_group == 0 and o.rows_per_block == 0 and o.use_graph == 1


def _solve_status(A, B, contours, N=16, M=4, L=8, tol=1e-8, **kw):
    from paper_2511_01927_amd import gep_ci
    try:
        gep_ci.gep_ci_solve(A, B, contours, N, M, L, tol, stream=0, **kw)
    except gep_ci.GepError as e:
        return e.status, str(e)
    return 0, ""


def test_argument_errors_are_reported(lib):
    from workloads import pencils
    A, B = pencils.fem1d(50)
    good = np.array([[100.0, 50.0, 60.0, 140.0]])
    assert _solve_status(A, B, good, N=15)[0] == -1            # odd node count
    assert _solve_status(A, B, good, M=0)[0] == -1
    assert _solve_status(A, B, good, L=0)[0] == -1
    assert _solve_status(A, B, good, tol=0.0)[0] == -1
    assert _solve_status(A, B, good, row_group=3)[0] == -1
    assert _solve_status(A, B, good, rows_per_block=-1)[0] == -1
    assert _solve_status(A, B, good, solver=4)[0] == -1           # no such solver
    bad = np.array([[100.0, 10.0, 60.0, 140.0]])               # window outside the circle
    assert _solve_status(A, B, bad)[0] == -1
    assert _solve_status(A, B, np.array([[100.0, -1.0, 99.0, 100.0]]))[0] == -1
    # non-symmetric A
    An = A.tolil()
    An[0, 1] = An[0, 1] * 1.5
    assert _solve_status(An.tocsr(), B, good)[0] == -2
    # B with a negative diagonal entry
    Bn = B.tolil()
    Bn[3, 3] = -1.0
    assert _solve_status(A, Bn.tocsr(), good)[0] == -3
    # NaN value
    Ab = A.copy()
    Ab.data[5] = np.nan
    assert _solve_status(Ab, B, good)[0] == -1
    # unsorted column indices
    Au = A.copy()
    Au.indices[[0, 1]] = Au.indices[[1, 0]]
    assert _solve_status(Au, B, good)[0] == -1


def test_strerror(lib):
    assert lib.gep_strerror(0) == b"ok"
    assert b"symmetric" in lib.gep_strerror(-2)
