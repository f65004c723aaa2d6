"""GPU parity of the wide-band / FP32 banded solves (band_wide.hip), through
the C ABI.

The wide-band kernels factor every system whose half bandwidth exceeds
1024 (3D grids in natural order) and every FP32 factor (mixed precision:
FP32 factors, FP64 residual refinement).  Here they are also forced onto
narrow pencils (band_kernels="wide") so that the oracle can check them:
1D and 2D pencils against closed forms, variable-coefficient 2D and 3D
pencils against the oracle, a 27-point 3D pencil, a square grid with
exact doubles, a memory cap that factors the systems in groups, and a
constant-coefficient 3D pencil of half bandwidth 1089 (past the
register-panel kernels) against its closed-form spectrum.
"""
import numpy as np
import pytest

import oracle
from oracle import inertia
from workloads import configs, pencils
from tests.test_gpu_solve import assert_pairs_match, _converged, _var2d
from tests.test_gpu_paths import _q1_vectors, _q1_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _check_band_stats(st, fp32):
    assert st["band_factorisations"] > 0 and st["cocg_iters"] == 0
    assert st["band_pivot_flags"] == 0 and st["band_unconverged"] == 0
    assert st["band_relres_max"] <= 1e-9
    assert st["precision"] == ("mixed" if fp32 else "fp64")
    if fp32:
        assert st["band_refinements"] >= 1


PRECS = ["fp64", "mixed"]


@pytest.mark.parametrize("prec", PRECS)
def test_wide_fem1d_2000_closed_form(lib, prec):
    w = configs.fem1d_2000()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           solver="band", band_kernels="wide", precision=prec)
    ref = configs.line_eigs(2000)[100:120]
    i = np.arange(1, 2001)
    X = np.stack([np.sin(i * j * np.pi / 2001) for j in range(101, 121)], axis=1)
    X /= np.sqrt(np.einsum("ij,ij->j", X, w.B @ X))[None, :]
    assert_pairs_match(got, ref, X, w.B)
    _check_band_stats(got["stats"], prec == "mixed")


@pytest.mark.parametrize("prec", PRECS)
def test_wide_q1_closed_form(lib, prec):
    A, B, cont, ref = _q1_case(70, 12, 41, 90, 2, 32)
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 32, 1e-8, seed=21, solver="band", band_kernels="wide",
                           precision=prec)
    assert_pairs_match(got, ref, _q1_vectors(70, 12, B, ref), B)
    _check_band_stats(got["stats"], prec == "mixed")


@pytest.mark.parametrize("prec", PRECS)
def test_wide_variable_coefficient_2d_vs_oracle(lib, prec):
    w = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, solver="band",
                           band_kernels="wide", precision=prec)
    ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5)
    assert_pairs_match(got, *_converged(ref), w.B)
    assert got["evals"].size == inertia.count_in(w.A, w.B, *w.window)
    _check_band_stats(got["stats"], prec == "mixed")


def _fd7_var(m=12, seed=31, first=41, last=80, k=2):
    g = pencils.grf((m + 2,) * 3, seed=seed)
    A, B = pencils.fd7_3d(m, np.exp(g))
    lam = np.linalg.eigvalsh(A.toarray() / B.diagonal()[0])
    lo, hi = 0.5 * (lam[first - 2] + lam[first - 1]), 0.5 * (lam[last - 1] + lam[last])
    cont = configs.uniform_contours(lo, hi, k, 0.1)
    return A, B, cont, (lo, hi)


@pytest.mark.parametrize("prec", PRECS)
def test_wide_fd7_3d_variable_coefficient_vs_oracle(lib, prec):
    """12^3 nodes, half bandwidth 144, log-normal coefficient."""
    A, B, cont, win = _fd7_var()
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 32, 1e-8, seed=8, solver="band", band_kernels="wide",
                           precision=prec)
    ref = oracle.oracle_ci_solve(A, B, cont, 32, 4, 32, 1e-8, seed=8)
    assert_pairs_match(got, *_converged(ref), B)
    assert got["evals"].size == inertia.count_in(A, B, *win)
    _check_band_stats(got["stats"], prec == "mixed")


@pytest.mark.parametrize("prec", PRECS)
def test_wide_q1_3d_closed_form(lib, prec):
    """27-point trilinear pencil on 8^3 (half bandwidth 73)."""
    m = 8
    A, B = pencils.q1_3d(m)
    l1 = configs.line_eigs(m)
    ev = np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())
    gaps = [i + 1 for i in range(30, 120) if ev[i + 1] - ev[i] > 1e-9 * ev[i + 1]]
    first, last = gaps[0] + 1, gaps[-1]
    lo, hi = configs.gap_window(ev, first, last)
    cont = configs.uniform_contours(lo, hi, 2, 0.1)
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 48, 1e-8, seed=4, solver="band", band_kernels="wide",
                           precision=prec)
    ref = ev[first - 1:last]
    assert got["evals"].size == ref.size
    assert np.max(np.abs(got["evals"] - ref) / ref) <= 1e-10
    assert np.max(got["resid"]) <= 1e-8
    _check_band_stats(got["stats"], prec == "mixed")


@pytest.mark.parametrize("prec", PRECS)
def test_wide_square_grid_doubles(lib, prec):
    A, B, cont, ref = _q1_case(48, 48, 61, 121, 2, 32)
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 32, 1e-8, seed=12, solver="band", band_kernels="wide",
                           precision=prec)
    assert_pairs_match(got, ref, _q1_vectors(48, 48, B, ref), B)
    _check_band_stats(got["stats"], prec == "mixed")


@pytest.mark.parametrize("prec", PRECS)
def test_wide_groups_of_systems(lib, prec):
    """At most 5 systems factored at once: the 32 systems of the pass are
    factored, solved and refined in 7 groups; the results equal the
    one-group solve."""
    w = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    free = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, solver="band",
                            band_kernels="wide", precision=prec)
    capped = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, solver="band",
                              band_kernels="wide", precision=prec, band_group=5)
    assert capped["stats"]["band_factorisations"] == free["stats"]["band_factorisations"] == 32
    assert_pairs_match(capped, free["evals"], free["evecs"], w.B)
    _check_band_stats(capped["stats"], prec == "mixed")


def _fd1d_eigs(m):
    h = 1.0 / (m + 1)
    return 4.0 / h ** 2 * np.sin(np.arange(1, m + 1) * np.pi * h / 2) ** 2


@pytest.mark.parametrize("prec", PRECS)
def test_wide_band_past_register_panels_closed_form(lib, prec):
    """Constant-coefficient 7-point pencil on 33^3 nodes: half bandwidth 1089,
    factored by the wide-band kernels with the automatic choice."""
    m = 33
    A, B = pencils.fd7_3d(m)
    l1 = _fd1d_eigs(m)
    ev = np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())
    gaps = [i + 1 for i in range(60, 140) if ev[i + 1] - ev[i] > 1e-9 * ev[i + 1]]
    first, last = gaps[0] + 1, gaps[-1]
    lo, hi = configs.gap_window(ev, first, last)
    cont = configs.uniform_contours(lo, hi, 1, 0.1)
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 64, 1e-8, seed=6, precision=prec)
    ref = ev[first - 1:last]
    st = got["stats"]
    assert st["solver_run"] == "band"
    assert got["evals"].size == ref.size
    assert np.max(np.abs(got["evals"] - ref) / ref) <= 1e-10
    assert np.max(got["resid"]) <= 1e-8
    _check_band_stats(st, prec == "mixed")
