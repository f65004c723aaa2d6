"""Pins of the oracle's merge, refinement and sign steps.

* de-duplication across contours (the merge step of the CI pipeline):
  planted pairs with known answers -- one eigenvector found by two
  contours (merged, the smaller residual kept), an exact double eigenvalue
  of one contour (never merged), a double found by two contours in rotated
  bases (the better contour's basis kept), two orthogonal vectors of a
  double split over two contours (both kept), equal vectors at values that
  differ beyond the tolerance (both kept); end to end, contours whose keep
  windows overlap return every eigenvalue of the union exactly once, against
  the closed-form 1D spectrum and the closed-form square-grid spectrum with
  its exact doubles;
* the FEAST-type refinement pass: with 8 trapezoid nodes one CIRR pass
  leaves kept pairs above tol on the 1D n = 2000 pencil, and the second
  pass reaches the closed form;
* the sign rule: returned eigenvectors equal the B-normalised closed-form
  sines with the sign of their first largest-modulus entry (mirror-
  symmetric modes have exactly tied entries).
"""
import numpy as np
import pytest

import oracle
from oracle import cirr, dense
from workloads import configs, pencils


def _fem_pairs(n=60):
    A, B = pencils.fem1d(n)
    lam, X = dense.dense_bruteforce(A, B)
    return A, B, lam, X


def test_dedupe_simple_duplicate_keeps_smaller_residual():
    A, B, lam, X = _fem_pairs()
    x = X[:, 10]
    noise = 1e-11 * np.random.default_rng(1).standard_normal(x.size)
    for rho in ([3e-12, 1e-12], [1e-12, 3e-12]):
        l2, X2, r2, c2 = cirr.dedupe(np.array([lam[10], lam[10] * (1 + 1e-12)]),
                                     np.stack([x, -x + noise], axis=1), np.array(rho),
                                     np.array([0, 1], dtype=np.int32), B)
        assert l2.size == 1
        assert r2[0] == min(rho)
        assert c2[0] == int(np.argmin(rho))


def _square_double(m=6):
    """A 2D eigenspace of the square Q1 grid (exactly double eigenvalue)."""
    A, B = pencils.q1_2d(m, m)
    lam, X = dense.dense_bruteforce(A, B)
    for i in range(lam.size - 1):
        if abs(lam[i + 1] - lam[i]) <= 1e-10 * lam[i] and (i + 2 == lam.size or lam[i + 2] - lam[i] > 1e-6 * lam[i]):
            return A, B, lam[i], X[:, i], X[:, i + 1]
    raise AssertionError("no double eigenvalue")


def test_dedupe_never_merges_one_contours_double():
    A, B, l, v1, v2 = _square_double()
    l2, X2, r2, c2 = cirr.dedupe(np.array([l, l]), np.stack([v1, v2], axis=1), np.array([1e-12, 2e-12]),
                                 np.array([0, 0], dtype=np.int32), B)
    assert l2.size == 2


def test_dedupe_double_found_by_two_contours_in_rotated_bases():
    A, B, l, v1, v2 = _square_double()
    w1, w2 = (v1 + v2) / np.sqrt(2), (v1 - v2) / np.sqrt(2)
    lam = np.array([l, l, l, l])
    X = np.stack([v1, w1, v2, w2], axis=1)
    cid = np.array([0, 1, 0, 1], dtype=np.int32)
    rho = np.array([1e-12, 5e-13, 2e-12, 4e-13])     # contour 1's worst residual is smaller
    l2, X2, r2, c2 = cirr.dedupe(lam, X, rho, cid, B)
    assert l2.size == 2
    assert set(c2.tolist()) == {1}
    # the kept pair is B-orthonormal and spans the eigenspace
    G = X2.T @ (B @ X2)
    assert np.allclose(G, np.eye(2), atol=1e-10)
    P = np.stack([v1, v2], axis=1)
    s = np.linalg.svd(X2.T @ (B @ P), compute_uv=False)
    assert s.min() >= 1 - 1e-10


def test_dedupe_keeps_orthogonal_vectors_of_a_split_double():
    A, B, l, v1, v2 = _square_double()
    l2, X2, r2, c2 = cirr.dedupe(np.array([l, l]), np.stack([v1, v2], axis=1), np.array([1e-12, 1e-12]),
                                 np.array([0, 1], dtype=np.int32), B)
    assert l2.size == 2


def test_dedupe_needs_equal_values():
    A, B, lam, X = _fem_pairs()
    x = X[:, 20]
    l2, X2, r2, c2 = cirr.dedupe(np.array([lam[20], lam[20] * (1 + 1e-6)]), np.stack([x, x], axis=1),
                                 np.array([1e-12, 1e-12]), np.array([0, 1], dtype=np.int32), B)
    assert l2.size == 2


def _overlapping(lo1, hi1, lo2, hi2):
    """Two circles whose keep windows [lo1, hi1) and [lo2, hi2) overlap."""
    return np.array([[(lo1 + hi1) / 2, 0.5 * (hi1 - lo1), lo1, hi1],
                     [(lo2 + hi2) / 2, 0.5 * (hi2 - lo2), lo2, hi2]])


def test_oracle_overlapping_windows_fem1d_closed_form():
    n = 400
    A, B = pencils.fem1d(n)
    ev = configs.line_eigs(n)
    lo1, hi1 = configs.gap_window(ev, 31, 45)
    lo2, hi2 = configs.gap_window(ev, 40, 52)
    cont = _overlapping(lo1, hi1, lo2, hi2)
    res = oracle.oracle_ci_solve(A, B, cont, 32, 4, 16, 1e-8, seed=3)
    ref = ev[30:52]
    assert res["evals"].size == ref.size == 22
    assert np.max(np.abs(res["evals"] - ref) / ref) <= 1e-10
    assert np.max(res["resid"]) <= 1e-8
    # both contours found eigenvalues 40..45: the merge really ran
    raw = [oracle.oracle_ci_solve(A, B, cont[k:k + 1], 32, 4, 16, 1e-8, seed=3)["evals"].size for k in range(2)]
    assert sum(raw) == 22 + 6


def test_oracle_overlapping_windows_square_grid_doubles():
    m = 14
    A, B = pencils.q1_2d(m, m)
    ev = configs.q1_2d_eigs(m, m)
    lam_bf, X_bf = dense.dense_bruteforce(A, B)
    lo1, hi1 = configs.gap_window(ev, 21, 39)
    lo2, hi2 = configs.gap_window(ev, 31, 50)
    cont = _overlapping(lo1, hi1, lo2, hi2)
    res = oracle.oracle_ci_solve(A, B, cont, 32, 4, 24, 1e-8, seed=4)
    ref = ev[20:50]
    assert res["evals"].size == ref.size
    assert np.max(np.abs(res["evals"] - ref) / ref) <= 1e-10
    X = res["evecs"]
    assert np.allclose(X.T @ (B @ X), np.eye(X.shape[1]), atol=1e-8)
    # every eigenspace (doubles included) is returned with a full basis
    sel = (lam_bf >= lo1) & (lam_bf < hi2)
    s = np.linalg.svd(X.T @ (B @ X_bf[:, sel]), compute_uv=False)
    assert s.min() >= 1 - 1e-8
    assert np.sum(np.diff(ref) <= 1e-10 * ref[1:]) >= 5     # the window holds exact doubles


def test_oracle_refinement_pass_reaches_closed_form():
    w = configs.config_fem1d(n=2000, n_nodes=8, moments=4, block=16)
    ref = configs.line_eigs(2000)[100:120]
    one = oracle.oracle_ci_solve(w.A, w.B, w.contours, 8, 4, 16, w.tol, seed=w.seed, max_refine=0)
    assert np.max(one["resid"]) > w.tol           # a single CIRR pass misses tol here
    res = oracle.oracle_ci_solve(w.A, w.B, w.contours, 8, 4, 16, w.tol, seed=w.seed)
    assert res["info"][0]["passes"] == 2
    assert res["evals"].size == 20
    assert np.max(np.abs(res["evals"] - ref) / ref) <= 1e-10
    assert np.max(res["resid"]) <= w.tol


def _sine_with_sign_rule(n, j, B):
    i = np.arange(1, n + 1)
    v = np.sin(i * j * np.pi / (n + 1))
    v /= np.sqrt(v @ (B @ v))
    a = np.abs(v)
    first = int(np.nonzero(a >= (1 - 1e-4) * a.max())[0][0])
    return v * np.sign(v[first])


def test_sign_rule_against_closed_form_sines():
    n = 400
    w = configs.config_fem1d(n=n, first=31, last=52, n_nodes=16, moments=4, block=24, seed=6)
    res = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 4, 24, 1e-8, seed=6)
    assert res["evals"].size == 22
    for k, j in enumerate(range(31, 53)):
        v = _sine_with_sign_rule(n, j, w.B)
        assert np.abs(res["evecs"][:, k] - v).max() <= 1e-8 * np.abs(v).max(), j


def test_sign_rule_breaks_mirror_ties_by_lowest_index():
    n = 50
    A, B = pencils.fem1d(n)
    i = np.arange(1, n + 1)
    v = np.sin(i * 2 * np.pi / (n + 1))          # antisymmetric: v[n-1-i] = -v[i]
    top = np.flatnonzero(np.abs(v) >= np.abs(v).max() * (1 - 1e-12))
    assert top.size == 2
    lo, hi = top
    for bump in (1 + 1e-7, 1 - 1e-7):
        u = v.copy()
        u[hi] *= bump                  # a computed vector's error picks either entry as the max
        out = cirr._normalise(u[:, None], B)[:, 0]
        assert out[lo] > 0


def test_planted_mistakes_break_the_merge_pins(monkeypatch):
    """Without the merge, or with a value-only merge, the overlapping-window
    pins fail: duplicates survive, or the square grid's doubles collapse."""
    m = 14
    A, B = pencils.q1_2d(m, m)
    ev = configs.q1_2d_eigs(m, m)
    cont = _overlapping(*configs.gap_window(ev, 21, 39), *configs.gap_window(ev, 31, 50))
    ref = ev[20:50]

    def no_merge(lam, X, rho, cid, B, **kw):
        return lam, X, rho, cid

    def value_merge(lam, X, rho, cid, B, rel=1e-8, **kw):
        order = np.argsort(lam, kind="stable")
        lam, X, rho, cid = lam[order], X[:, order], rho[order], cid[order]
        keep = np.ones(lam.size, dtype=bool)
        keep[1:] = np.diff(lam) > rel * np.abs(lam[1:])
        return lam[keep], X[:, keep], rho[keep], cid[keep]

    for bad in (no_merge, value_merge):
        monkeypatch.setattr(cirr, "dedupe", bad)
        res = oracle.oracle_ci_solve(A, B, cont, 32, 4, 24, 1e-8, seed=4)
        assert res["evals"].size != ref.size, bad.__name__


def test_oracle_feast_iteration_reaches_closed_form():
    """One moment and refinement passes (V <- Ritz vectors) is FEAST subspace
    iteration; with a subspace larger than the window's count it converges
    to the closed form, and a single pass does not."""
    w = configs.config_fem1d(n=2000, n_nodes=16, moments=4, block=32)
    ref = configs.line_eigs(2000)[100:120]
    one = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 1, 32, w.tol, seed=w.seed, max_refine=0)
    assert one["evals"].size != 20 or np.max(one["resid"]) > w.tol
    res = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 1, 32, w.tol, seed=w.seed, max_refine=8)
    assert res["info"][0]["passes"] >= 2
    assert res["evals"].size == 20
    assert np.max(np.abs(res["evals"] - ref) / ref) <= 1e-10
    assert np.max(res["resid"]) <= w.tol
