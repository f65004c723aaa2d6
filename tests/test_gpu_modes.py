"""GPU parity of the solver modes beyond one moment-based pass, through the
C ABI: FEAST subspace iteration (GEP_FEAST: one moment, passes with
V <- Ritz vectors) against the closed form and against the oracle run as
the same iteration (one moment, refinement passes); the m smallest
eigenpairs (gep_ci_solve_smallest, no upper end given) against the
closed-form 1D and square-grid spectra and a brute-force dense solve of a
variable-coefficient pencil."""
import numpy as np
import pytest

import oracle
from oracle import dense
from workloads import configs, pencils
from tests.test_gpu_solve import assert_pairs_match, _converged, _var2d
from tests.test_gpu_paths import _q1_vectors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _sines(n, js, B):
    i = np.arange(1, n + 1)
    X = np.stack([np.sin(i * j * np.pi / (n + 1)) for j in js], axis=1)
    return X / np.sqrt(np.einsum("ij,ij->j", X, B @ X))[None, :]


@pytest.mark.parametrize("solver", ["band", "cocg"])
def test_feast_fem1d_closed_form_and_oracle(lib, solver):
    w = configs.config_fem1d(n=2000, n_nodes=16, moments=4, block=32)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 16, 4, 32, w.tol, seed=w.seed, solver=solver,
                           method="feast", max_refine=8)
    st = got["stats"]
    assert st["method"] == "feast"
    assert st["contours"][0]["passes"] >= 2
    ref = configs.line_eigs(2000)[100:120]
    assert_pairs_match(got, ref, _sines(2000, range(101, 121), w.B), w.B)
    orc = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 1, 32, w.tol, seed=w.seed, max_refine=8)
    assert_pairs_match(got, *_converged(orc), w.B)


def test_feast_variable_coefficient_vs_oracle(lib):
    w = _var2d()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, 48, w.tol, seed=w.seed,
                           method="feast", max_refine=8)
    orc = oracle.oracle_ci_solve(w.A, w.B, w.contours, w.n_nodes, 1, 48, w.tol, seed=w.seed, max_refine=8)
    assert_pairs_match(got, *_converged(orc), w.B)


@pytest.mark.parametrize("solver", ["band", "cocg"])
def test_smallest_fem1d(lib, solver):
    n = 400
    A, B = pencils.fem1d(n)
    pen = lib.Pencil(A, B)
    got = pen.solve_smallest(25, lower=0.0, per_contour=20, n_nodes=32, moments=4, block=16, tol=1e-8,
                             seed=3, solver=solver)
    assert got["status"] in (0, lib.GEP_WSATURATED)
    ref = configs.line_eigs(n)[:25]
    assert_pairs_match(got, ref, _sines(n, range(1, 26), B), B)


def test_smallest_square_grid(lib):
    m = 30
    A, B = pencils.q1_2d(m, m)
    ev = configs.q1_2d_eigs(m, m)
    k = next(k for k in range(40, 60) if ev[k] - ev[k - 1] > 1e-9 * ev[k])   # cut in a gap
    pen = lib.Pencil(A, B)
    got = pen.solve_smallest(k, lower=0.0, per_contour=25, n_nodes=32, moments=4, block=24, tol=1e-8, seed=5)
    ref = ev[:k]
    assert_pairs_match(got, ref, _q1_vectors(m, m, B, ref), B)
    assert got["stats"]["rounds"] >= 1


def test_smallest_variable_coefficient_vs_bruteforce(lib):
    w = _var2d(nx=24, ny=22, seed=13)
    lam, X = dense.dense_bruteforce(w.A, w.B)
    k = next(k for k in range(30, 50) if lam[k] - lam[k - 1] > 1e-6 * lam[k])
    pen = lib.Pencil(w.A, w.B)
    got = pen.solve_smallest(k, lower=0.0, per_contour=20, n_nodes=32, moments=4, block=24, tol=1e-8, seed=2)
    assert_pairs_match(got, lam[:k], X[:, :k], w.B)
