"""GPU parity at the benchmark's full sizes, in the launch configuration it
times (device-resident pencil on the caller's stream, default options).

* 2D Q1 300x300 (n = 90,000; 4 circles x 32 nodes, 4 moments, block 64;
  banded factors): every returned pair against the closed form (count,
  eigenvalues within 1e-10, eigenvector subspaces per cluster), and every
  residual recomputed on the CPU in FP64 from the returned vectors.
* 3D 7-point 64^3 (n = 262,144; log-normal coefficient; FP32 factors with
  FP64 refinement): too large for the oracle's sparse LU, so properties
  that hold at any size, on every returned pair: the residual recomputed on
  the CPU, unit B-norms and the B-orthogonality that the residuals imply,
  eigenvalues inside the keep windows.
* The 64-pencil uneven batch: pairs that miss tol come back flagged (and
  are at most 1% of the pairs); for the six smallest pencils the count of
  converged pairs inside their windows by Sylvester inertia (the oracle's
  LDL^T of A - sigma B) and their residuals recomputed on the CPU; for every
  pencil residuals and B-normalisation on a sample of converged pairs.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import inertia
from workloads import configs
from tests.test_gpu_paths import _q1_vectors
from tests.test_gpu_solve import assert_pairs_match

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _cpu_residuals(A, B, lam, X, vectors=False):
    """||A x - lambda B x|| / (||A||_1 ||x||) in FP64 on the CPU (and the
    residual vectors' norms, unscaled, when asked)."""
    anorm = spla.norm(A, 1)
    R = A @ X - (B @ X) * lam[None, :]
    rn = np.linalg.norm(R, axis=0)
    rel = rn / (anorm * np.linalg.norm(X, axis=0))
    return (rel, rn) if vectors else rel


def _check_b_orthogonality(X, B, lam, rn):
    """Unit B-norms, and for i != j the bound that follows from the residuals
    r = A x - lambda B x of any two approximate pairs of a symmetric pencil:
    (lambda_j - lambda_i) x_i^T B x_j = x_j^T r_i - x_i^T r_j, so
    |x_i^T B x_j| <= (||x_j|| ||r_i|| + ||x_i|| ||r_j||) / |lambda_i - lambda_j|.
    Pairs of different circles are computed apart and are only as orthogonal
    as that bound allows; pairs of one circle come out of one Rayleigh-Ritz
    step and are orthogonal to rounding."""
    G = X.T @ (B @ X)
    assert np.abs(np.diag(G) - 1.0).max() <= 1e-10
    xn = np.linalg.norm(X, axis=0)
    gap = np.abs(lam[:, None] - lam[None, :])
    np.fill_diagonal(gap, np.inf)
    bound = (xn[None, :] * rn[:, None] + xn[:, None] * rn[None, :]) / gap
    off = np.abs(G - np.diag(np.diag(G)))
    assert np.all(off <= 1.01 * bound + 1e-12), np.max(off - bound)


def test_headline_q1_300x300_full_size(lib):
    import torch
    w = configs.q1_2d_300()
    ev = configs.q1_2d_eigs(300, 300)
    lo, hi = w.window
    ref = ev[(ev >= lo) & (ev < hi)]
    stream = torch.cuda.current_stream()
    pen = lib.Pencil(w.A, w.B, stream=stream)
    got = pen.solve(w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, stream=stream)
    assert got["stats"]["solver_run"] == "band"
    assert_pairs_match(got, ref, _q1_vectors(300, 300, w.B, ref), w.B)
    res = _cpu_residuals(w.A, w.B, got["evals"], got["evecs"])
    assert res.max() <= 1e-8, res.max()


def test_fd7_64cube_mixed_full_size(lib):
    import torch
    w = configs.fd7_3d_64()
    stream = torch.cuda.current_stream()
    pen = lib.Pencil(w.A, w.B, stream=stream)
    got = pen.solve(w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, stream=stream,
                    precision="mixed")
    st = got["stats"]
    assert st["precision"] == "mixed" and st["band_unconverged"] == 0
    lam, X = got["evals"], got["evecs"]
    assert lam.size >= 500   # ~500 by Weyl's law over the window
    lo, hi = w.window
    assert lam.min() >= lo * (1 - 1e-12) and lam.max() < hi * (1 + 1e-12)
    assert np.all(np.diff(lam) >= 0)
    res, rn = _cpu_residuals(w.A, w.B, lam, X, vectors=True)
    assert res.max() <= 1e-8, res.max()
    _check_b_orthogonality(X, w.B, lam, rn)


def test_batch64_full_size(lib):
    import torch
    bt = configs.q1_batch64()
    stream = torch.cuda.current_stream()
    bp = lib.BatchPencil([(w.A, w.B) for w in bt.problems], stream=stream)
    out = bp.solve([w.contours for w in bt.problems], bt.n_nodes, bt.moments, bt.block, bt.tol,
                   seed=bt.seed, stream=stream)
    assert len(out) == len(bt.problems)
    rng = np.random.default_rng(0)
    total = flagged = 0
    for w, r in zip(bt.problems, out):
        lam, X = r["evals"], r["evecs"]
        ok = r["resid"] <= 1e-8
        # pairs that miss tol after the refinement pass come back flagged
        assert np.array_equal(r["converged"], ok), w.name
        total += lam.size
        flagged += int(np.sum(~ok))
        lo, hi = w.window
        assert lam.size > 0 and lam.min() >= lo * (1 - 1e-12) and lam.max() < hi * (1 + 1e-12)
        good = np.flatnonzero(ok)
        pick = rng.choice(good, size=min(8, good.size), replace=False)
        res = _cpu_residuals(w.A, w.B, lam[pick], X[:, pick])
        assert res.max() <= 1e-8, (w.name, res.max())
        d = np.einsum("ij,ij->j", X[:, pick], w.B @ X[:, pick])
        assert np.abs(d - 1.0).max() <= 1e-10
    assert flagged <= 0.01 * total, (flagged, total)
    small = sorted(range(len(bt.problems)), key=lambda b: bt.problems[b].n)[:6]
    for b in small:
        w, r = bt.problems[b], out[b]
        ok = r["converged"]
        assert int(np.sum(ok)) == inertia.count_in(w.A, w.B, *w.window), w.name
        res = _cpu_residuals(w.A, w.B, r["evals"][ok], r["evecs"][:, ok])
        assert res.max() <= 1e-8, (w.name, res.max())
