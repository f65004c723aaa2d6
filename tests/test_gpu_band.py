"""Banded L D L^T solves of the shifted systems (solver="band") through the
C ABI: eigenpairs against closed forms and the oracle for half bandwidths
below the panel width, between one and two 64-wide update tiles, and above;
solver statistics (factorisations, pivots, residual after refinement); the
automatic choice and the rejection of pencils whose band is too wide.

Bar: as in test_gpu_solve (count, 1e-10 relative eigenvalues, residual
<= 1e-8, eigenvectors up to sign / cluster bases)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import configs, pencils

from test_gpu_solve import assert_pairs_match, _converged, _var2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _check_band_stats(got, n_systems):
    st = got["stats"]
    assert st["band_factorisations"] == n_systems, st["band_factorisations"]
    assert st["band_pivot_flags"] == 0
    assert st["band_unconverged"] == 0
    assert st["band_relres_max"] <= 1e-9
    assert st["cocg_iters"] == 0


@pytest.mark.parametrize("nx,ny", [(70, 12), (31, 29)])
def test_band_constant_q1_closed_form(lib, nx, ny):
    """Constant-coefficient Q1 on nx x ny interior nodes: half bandwidth nx+1
    (71: two 64-row update tiles; 32: one), eigenvalues from the closed form."""
    eig = configs.q1_2d_eigs(nx, ny)
    w = configs.config_q1_2d(nx=nx, ny=ny, first=21, last=60, k=2, n_nodes=32, moments=4, block=16, seed=4)
    lo, hi = w.window
    ref = eig[(eig >= lo) & (eig < hi)]
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           solver="band")
    assert got["evals"].size == ref.size
    assert np.max(np.abs(got["evals"] - ref) / ref) <= 1e-10
    assert np.max(got["resid"]) <= 1e-8
    _check_band_stats(got, len(w.contours) * w.n_nodes // 2)


@pytest.mark.parametrize("nx,ny,kernels", [(399, 12, "auto"), (499, 8, "auto"), (499, 8, "narrow")])
def test_band_wide_bands_closed_form(lib, nx, ny, kernels):
    """Half bandwidths 400 and 500: past the blocked sweeps' limit (register
    window sweeps instead) and, at 500, past the one-thread-per-row panel:
    the automatic choice takes the wide-band kernels there, "narrow" keeps
    the one-work-group panel in global memory."""
    eig = configs.q1_2d_eigs(nx, ny)
    w = configs.config_q1_2d(nx=nx, ny=ny, first=21, last=60, k=2, n_nodes=16, moments=4, block=16, seed=6)
    lo, hi = w.window
    ref = eig[(eig >= lo) & (eig < hi)]
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           solver="band", band_kernels=kernels)
    assert got["evals"].size == ref.size
    assert np.max(np.abs(got["evals"] - ref) / ref) <= 1e-10
    assert np.max(got["resid"]) <= 1e-8
    _check_band_stats(got, len(w.contours) * w.n_nodes // 2)


def test_band_variable_coefficient_vs_oracle(lib):
    """kappa = exp(GRF) on 31 x 29 (n = 899, the last panel is short)."""
    w = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, solver="band")
    ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5)
    assert_pairs_match(got, *_converged(ref), w.B)
    _check_band_stats(got, 2 * 16)


def test_band_1d_below_panel_width(lib):
    """Tridiagonal pencil: half bandwidth 1, far below the 16-column panel."""
    w = configs.fem1d_2000()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           solver="band")
    lam_ref = configs.line_eigs(2000)[100:120]
    assert got["evals"].size == 20
    assert np.max(np.abs(got["evals"] - lam_ref) / lam_ref) <= 1e-10
    _check_band_stats(got, 8)


def test_band_batch_of_uneven_pencils(lib):
    """Band widths 1, 32 and 71 in one batch; problem p draws V from seed + p."""
    w1 = configs.config_fem1d(n=401, first=31, last=40, n_nodes=16, moments=4, block=16, seed=11)
    w2 = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    w3 = configs.config_q1_2d(nx=70, ny=12, first=21, last=40, k=1, n_nodes=16, moments=4, block=16, seed=4)
    probs = [(w.A, w.B, w.contours) for w in (w1, w2, w3)]
    got = lib.gep_ci_solve_batch(probs, 16, 4, 16, 1e-8, seed=3, solver="band")
    for p, w in enumerate((w1, w2, w3)):
        ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 4, 16, 1e-8, seed=3 + p)
        assert_pairs_match(got[p], *_converged(ref), w.B)
        assert got[p]["stats"]["band_pivot_flags"] == 0


def test_band_automatic_choice_and_wide_band(lib):
    """Automatic choice: band for narrow pencils, COCG when the band is wider
    than the automatic limit; solver="band" rejects a band wider than the
    kept maximum."""
    w = configs.config_fem1d(n=400, first=31, last=40, n_nodes=16, moments=4, block=8, seed=7)
    auto = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed)
    assert auto["stats"]["band_factorisations"] > 0 and auto["stats"]["cocg_iters"] == 0
    # a symmetric coupling between rows 0 and n-1 widens the band to n-1
    n = 5000
    A, B = pencils.fem1d(n)
    E = sp.csr_matrix(([1e-3, 1e-3], ([0, n - 1], [n - 1, 0])), shape=(n, n))
    Aw = (A + E).tocsr()
    Aw.sort_indices()
    c = np.array([[1e5, 5e4, 6e4, 1.4e5]])
    got = lib.gep_ci_solve(Aw, B, c, 16, 2, 8, 1e-8, seed=1, max_iter=32, max_refine=0)
    assert got["stats"]["band_factorisations"] == 0 and got["stats"]["cocg_iters"] > 0
    with pytest.raises(lib.GepError) as e:
        lib.gep_ci_solve(Aw, B, c, 16, 2, 8, 1e-8, seed=1, solver="band")
    assert e.value.status == -1


@pytest.mark.parametrize("which", ["fem1d", "q1"])
def test_band_timing_statistics(lib, which):
    """Per-kernel timing on (the bench's mode): sampled HIP events around the
    factorisation launches, including steps whose window update is empty
    (half bandwidth 1), give finite per-class times and launch counts."""
    if which == "fem1d":
        w = configs.fem1d_2000()
    else:
        w = configs.config_q1_2d(nx=70, ny=12, first=21, last=40, k=1, n_nodes=16, moments=4, block=16, seed=4)
    P = lib.Pencil(w.A, w.B)
    got = P.solve(w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, solver="band", timing=True)
    st = got["stats"]
    km, kl = st["kernel_ms"], st["kernel_launches"]
    steps = st["band_panel_steps"]
    assert kl["band_panel"] == steps and kl["band_update"] == steps - 1 and kl["band_update_next"] == steps - 1
    for k in ("band_panel", "band_update", "band_update_next", "band_solve"):
        assert np.isfinite(km[k]) and km[k] >= 0.0, (k, km[k])
    assert km["band_panel"] > 0.0 and km["band_solve"] > 0.0
    assert np.max(got["resid"]) <= 1e-8


def test_band_diagonal_pencil(lib):
    """Half bandwidth 0 (diagonal A and B): no coupling between panels, the
    factorisation is the diagonal itself; eigenvalues a_ii / b_ii exactly."""
    n = 600
    rng = np.random.default_rng(21)
    lam = np.arange(1.0, n + 1.0)
    b = rng.uniform(1.0, 2.0, n)
    A = sp.diags(lam * b).tocsr()
    B = sp.diags(b).tocsr()
    lo, hi = configs.gap_window(lam, 101, 120)
    c = configs.uniform_contours(lo, hi, 2, 0.1)
    got = lib.gep_ci_solve(A, B, c, 16, 4, 8, 1e-8, seed=3, solver="band")
    ref = lam[100:120]
    assert got["evals"].size == ref.size
    assert np.max(np.abs(got["evals"] - ref) / ref) <= 1e-10
    assert np.max(got["resid"]) <= 1e-8
    _check_band_stats(got, 2 * 8)
