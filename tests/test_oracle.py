"""Pins of the CPU oracle against mathematics that does not come from the oracle.

* known-answer SplitMix64 outputs (published generator) and Box-Muller
  distribution tests for the random block;
* the trapezoid filter closed form: for a diagonal pencil the moments are
  S_k = diag(t^k / (1 + t^N)) V exactly, t = (lambda - c)/R (this follows
  from the residue theorem applied to the nodes, the roots of zeta^N = -1);
* closed-form spectra and eigenvectors of the 1D FEM pencil at full size;
* brute-force dense solves (self-written Cholesky + Jacobi, itself checked
  against LAPACK) and Sylvester-inertia counts for variable coefficients;
* metamorphic invariances (scaling, shift, symmetric permutation);
* planted mistakes in the quadrature are shown to break the filter pin.
"""
import os

import numpy as np
import scipy.sparse as sp
import scipy.stats as st
import pytest

import oracle
from oracle import cirr, dense, inertia, rng
from workloads import pencils, configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- random block
def test_splitmix64_known_answers():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        ref = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    got = rng.splitmix64(0, np.arange(len(ref), dtype=np.uint64))
    assert [int(x) for x in got] == ref


def test_gaussian_block_distribution_and_layout():
    V = rng.gaussian_block(50_000, 4, seed=7)
    x = V.ravel()
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    assert st.kstest(x, "norm").pvalue > 1e-3
    # the cosine and sine branches of one Box-Muller pair are uncorrelated
    flat = V.T.ravel()
    assert abs(np.corrcoef(flat[0::2], flat[1::2])[0, 1]) < 0.01
    # column-major counter order: column l starts at counter l*n
    V2 = rng.gaussian_block(10, 3, seed=7)
    V3 = rng.gaussian_block(30, 1, seed=7)
    assert np.array_equal(V2.T.ravel(), V3.ravel())
    assert np.all(rng.uniform01(7, np.arange(100_000, dtype=np.uint64)) > 0)


# ---------------------------------------------------------------- quadrature
def _diag_pencil(n=40, seed=0):
    r = np.random.default_rng(seed)
    lam = np.sort(r.uniform(0.0, 10.0, n))
    b = r.uniform(0.5, 2.0, n)
    return sp.diags(lam * b).tocsr(), sp.diags(b).tocsr(), lam


def _filter_pin_error(N=16, M=4, c=5.0, R=1.7):
    A, B, lam = _diag_pencil()
    V = rng.gaussian_block(A.shape[0], 3, seed=5)
    S = cirr.contour_moments(A, B, V, c, R, N, M)
    t = (lam - c) / R
    err = 0.0
    for k in range(M):
        ref = (t ** k / (1.0 + t ** N))[:, None] * V
        err = max(err, np.max(np.abs(S[:, k * 3:(k + 1) * 3] - ref)))
    return err


def test_filter_closed_form():
    for N in (8, 16, 32):
        assert _filter_pin_error(N=N, M=min(N - 1, 6)) < 1e-12


def test_quadrature_nodes_are_conjugate_pairs():
    z, w, zeta = cirr.quadrature(3.0, 2.0, 16)
    assert np.allclose(zeta ** 16, -1.0, atol=1e-14)
    assert np.allclose(z[::-1], np.conj(z), atol=1e-14)
    assert np.all(np.abs(z.imag) > 0)


def test_planted_mistake_weights_break_filter_pin(monkeypatch):
    good = cirr.quadrature

    def bad(center, radius, n_nodes):       # weight without the zeta factor
        z, w, zeta = good(center, radius, n_nodes)
        return z, radius / n_nodes + 0 * w, zeta

    monkeypatch.setattr(cirr, "quadrature", bad)
    with pytest.raises(AssertionError):
        assert _filter_pin_error() < 1e-12


def test_planted_mistake_nodes_break_filter_pin(monkeypatch):
    def bad(center, radius, n_nodes):       # nodes shifted by half a step
        j = np.arange(1, n_nodes + 1)
        zeta = np.exp(1j * np.pi * (2 * j - 1) / n_nodes + 0.3j * np.pi / n_nodes)
        return center + radius * zeta, radius * zeta / n_nodes, zeta

    monkeypatch.setattr(cirr, "quadrature", bad)
    with pytest.raises(AssertionError):
        assert _filter_pin_error() < 1e-12


# ---------------------------------------------------------------- residual
def test_residual_closed_form():
    A, B, lam = _diag_pencil(n=10)
    x = np.zeros((10, 1))
    x[2, 0] = 1.0
    x[5, 0] = 1e-3
    rho = cirr.residuals(A, B, np.array([lam[2]]), x)
    b = B.diagonal()
    # r = 1e-3 * (lam_5 - lam_2) * b_5 e_5
    ref = 1e-3 * (lam[5] - lam[2]) * b[5] / (np.max(lam * b) * np.sqrt(1 + 1e-6))
    assert abs(rho[0] - ref) < 1e-14 * ref


# ---------------------------------------------------------------- brute force
def test_dense_bruteforce_against_lapack_and_closed_form():
    r = np.random.default_rng(1)
    n = 30
    g = r.standard_normal((n, n))
    a = g + g.T
    h = r.standard_normal((n, n))
    b = h @ h.T + n * np.eye(n)
    lam, X = dense.dense_bruteforce(a, b)
    import scipy.linalg as sla
    ref = sla.eigh(a, b, eigvals_only=True)
    assert np.max(np.abs(lam - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.allclose(X.T @ b @ X, np.eye(n), atol=1e-12)
    assert np.allclose(a @ X, b @ X * lam[None, :], atol=1e-10)
    A1, B1 = pencils.fem1d(40)
    lam1, _ = dense.dense_bruteforce(A1, B1)
    assert np.max(np.abs(lam1 - configs.line_eigs(40)) / lam1) < 1e-12


def test_inertia_counts_closed_form():
    A, B = pencils.fem1d(300)
    lam = configs.line_eigs(300)
    for sigma in (50.0, 1e4, 3.3e5, 1e7):
        assert inertia.count_below(A, B, sigma) == int(np.sum(lam < sigma))


# ---------------------------------------------------------------- CI oracle
def test_oracle_fem1d_full_size_closed_form():
    w = configs.fem1d_2000()
    res = oracle.oracle_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block,
                                 w.tol, seed=w.seed)
    ref = configs.line_eigs(2000)[100:120]
    assert res["evals"].size == 20
    assert np.max(np.abs(res["evals"] - ref) / ref) <= 1e-10
    assert np.max(res["resid"]) <= 1e-8
    # eigenvectors: B-normalised discrete sines
    i = np.arange(1, 2001)
    for k, j in enumerate(range(101, 121)):
        v = np.sin(i * j * np.pi / 2001)
        v /= np.sqrt(v @ (w.B @ v))
        assert abs(v @ (w.B @ res["evecs"][:, k])) >= 1 - 1e-8
    X = res["evecs"]
    assert np.allclose(X.T @ (w.B @ X), np.eye(20), atol=1e-8)
    assert inertia.count_in(w.A, w.B, *w.window) == 20


def _small_variable_case(nx=14, ny=12, seed=21):
    g = pencils.grf((ny + 1, nx + 1), seed=seed)
    A, B = pencils.q1_2d(nx, ny, np.exp(g))
    lam, X = dense.dense_bruteforce(A, B)
    # a window over eigenvalues 31..70 cut at the two widest nearby gaps
    lo = 0.5 * (lam[29] + lam[30])
    hi = 0.5 * (lam[69] + lam[70])
    return A, B, lam, X, lo, hi


def test_oracle_variable_coefficient_vs_bruteforce():
    A, B, lam, X, lo, hi = _small_variable_case()
    cont = configs.uniform_contours(lo, hi, 3, 0.1)
    res = oracle.oracle_ci_solve(A, B, cont, 32, 4, 12, 1e-8, seed=3)
    ref = lam[(lam >= lo) & (lam < hi)]
    assert res["evals"].size == ref.size == inertia.count_in(A, B, lo, hi)
    assert np.max(np.abs(res["evals"] - ref) / np.abs(ref)) <= 1e-10
    assert np.max(res["resid"]) <= 1e-8


def test_oracle_invariances():
    A, B, lam, X, lo, hi = _small_variable_case(nx=10, ny=9, seed=4)
    cont = configs.uniform_contours(lo, hi, 2, 0.1)
    base = oracle.oracle_ci_solve(A, B, cont, 32, 4, 12, 1e-8, seed=9)["evals"]
    # scaling A -> a A, B -> b B maps lambda -> (a/b) lambda
    a_, b_ = 3.0, 0.25
    c2 = cont.copy()
    c2 *= a_ / b_
    scaled = oracle.oracle_ci_solve(a_ * A, b_ * B, c2, 32, 4, 12, 1e-8, seed=9)["evals"]
    assert np.allclose(scaled, base * a_ / b_, rtol=1e-10)
    # shift A -> A + s B maps lambda -> lambda + s
    s = 1000.0
    c3 = cont.copy()
    c3[:, [0, 2, 3]] += s
    shifted = oracle.oracle_ci_solve((A + s * B).tocsr(), B, c3, 32, 4, 12, 1e-8, seed=9)["evals"]
    assert np.allclose(shifted, base + s, rtol=1e-10)
    # symmetric permutation leaves the spectrum unchanged
    p = np.random.default_rng(0).permutation(A.shape[0])
    P = sp.eye(A.shape[0], format="csr")[p]
    perm = oracle.oracle_ci_solve((P @ A @ P.T).tocsr(), (P @ B @ P.T).tocsr(), cont, 32, 4, 12,
                                  1e-8, seed=9)["evals"]
    assert np.allclose(perm, base, rtol=1e-10)


def test_oracle_saturation_flag():
    w = configs.fem1d_2000()
    res = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 1, 4, 1e-8, seed=1, max_refine=0)
    assert res["info"][0]["saturated"]
    ok = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 4, 16, 1e-8, seed=1)
    assert not ok["info"][0]["saturated"]
