"""GPU parity of the multi-shift COCG solves (solver="multishift",
multishift.hip), through the C ABI.

For B = beta I the shifted systems (z_j B - A) y = B v of one contour's
nodes are shifts of one another and share a Krylov space per right-hand
side; one seed recurrence per column of the contour's block serves every
node.  Checked here:

* a constant-coefficient 7-point 3D pencil (lumped mass h^3 I) against
  its closed-form spectrum;
* a log-normal-coefficient 7-point pencil against the oracle, with blocks
  of 32 (one 64-column seed tile for two circles) and 48 (two seed tiles,
  the second one ragged);
* agreement with the Jacobi-COCG solver on the same pencil;
* an iteration cap that stops the seeds early: the unconverged columns are
  counted and no pair is reported converged above tol;
* the rejections: a consistent-mass B (off-diagonal entries), a diagonal
  but non-constant B, and a batch.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import inertia
from workloads import configs, pencils
from tests.test_gpu_solve import assert_pairs_match, _converged
from tests.test_gpu_wide import _fd7_var

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _check_ms_stats(st):
    assert st["solver_run"] == "multishift"
    assert st["multishift_iters"] > 0 and st["multishift_unconverged"] == 0
    assert st["cocg_iters"] == 0 and st["band_factorisations"] == 0


def test_multishift_fd7_closed_form(lib):
    """Constant coefficient, 8^3 nodes: eigenvalues are sums of three 1D
    finite-difference eigenvalues (scaled by the lumped mass)."""
    m = 8
    A, B = pencils.fd7_3d(m)
    h = 1.0 / (m + 1)
    l1 = 4.0 / h ** 2 * np.sin(np.arange(1, m + 1) * np.pi * h / 2.0) ** 2
    ev = np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())
    gaps = [i + 1 for i in range(20, 100) if ev[i + 1] - ev[i] > 1e-9 * ev[i + 1]]
    first, last = gaps[0] + 1, gaps[-1]
    lo, hi = configs.gap_window(ev, first, last)
    cont = configs.uniform_contours(lo, hi, 2, 0.1)
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 48, 1e-8, seed=4, solver="multishift")
    ref = ev[first - 1:last]
    assert got["evals"].size == ref.size
    assert np.max(np.abs(got["evals"] - ref) / ref) <= 1e-10
    assert np.max(got["resid"]) <= 1e-8
    _check_ms_stats(got["stats"])


@pytest.mark.parametrize("block", [32, 48])
def test_multishift_fd7_variable_coefficient_vs_oracle(lib, block):
    """12^3 nodes, log-normal coefficient, two circles: 2 x block seed columns."""
    A, B, cont, win = _fd7_var()
    got = lib.gep_ci_solve(A, B, cont, 32, 4, block, 1e-8, seed=8, solver="multishift")
    ref = oracle.oracle_ci_solve(A, B, cont, 32, 4, block, 1e-8, seed=8)
    assert_pairs_match(got, *_converged(ref), B)
    assert got["evals"].size == inertia.count_in(A, B, *win)
    _check_ms_stats(got["stats"])


def test_multishift_agrees_with_cocg(lib):
    A, B, cont, _ = _fd7_var(m=10, seed=17, first=21, last=50, k=2)
    ms = lib.gep_ci_solve(A, B, cont, 16, 4, 32, 1e-8, seed=3, solver="multishift")
    cg = lib.gep_ci_solve(A, B, cont, 16, 4, 32, 1e-8, seed=3, solver="cocg")
    assert ms["evals"].size == cg["evals"].size > 0
    assert np.max(np.abs(ms["evals"] - cg["evals"]) / np.abs(cg["evals"])) <= 1e-10
    _check_ms_stats(ms["stats"])


def test_multishift_rejects_non_scalar_mass(lib):
    w = configs.config_fem1d(n=400, first=31, last=40, n_nodes=16, moments=4, block=8, seed=7)
    with pytest.raises(lib.GepError, match="beta I"):
        lib.gep_ci_solve(w.A, w.B, w.contours, 16, 4, 8, 1e-8, seed=7, solver="multishift")
    A, B, cont, _ = _fd7_var(m=8, seed=5, first=11, last=30, k=1)
    d = B.diagonal() * (1.0 + 1e-3 * np.arange(B.shape[0]) / B.shape[0])
    with pytest.raises(lib.GepError, match="diagonal is not constant"):
        lib.gep_ci_solve(A, sp.diags(d, format="csr"), cont, 16, 4, 8, 1e-8, seed=7, solver="multishift")
    with pytest.raises(lib.GepError, match="single pencils"):
        lib.gep_ci_solve_batch([(A, B, cont), (A, B, cont)], 16, 4, 8, 1e-8, seed=7, solver="multishift")


def test_multishift_iteration_cap_reports_unconverged(lib):
    A, B, cont, _ = _fd7_var(m=8, seed=5, first=11, last=30, k=1)
    got = lib.gep_ci_solve(A, B, cont, 16, 4, 16, 1e-8, seed=7, solver="multishift", max_iter=3)
    st = got["stats"]
    assert st["solver_run"] == "multishift" and st["multishift_iters"] % 3 == 0   # 3 per pass
    assert st["multishift_unconverged"] > 0
    assert np.all(got["resid"][got["converged"]] <= 1e-8)
    assert got["status"] in (0, lib.GEP_WNOCONV, lib.GEP_WSATURATED)
