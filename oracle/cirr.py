"""Plain FP64 CIRR oracle: what the contour-integral hot path computes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's CI pipeline (Appendix "Numerical Implementation of CI
Methods": quadrature equation, Alg. "Standard CI pipeline with contour
partitioning and orthogonalization", and the moment matrices S_m of the
moment-based family), for a real symmetric pencil with B SPD (Sec. 3.1):

1. draw the block V (n x L) and form B V;
2. at EVERY trapezoid node z_j of every circle, solve (z_j B - A) Y_j = B V
   with a sparse complex LU (SciPy SuperLU) -- no conjugate halving;
3. accumulate the moments S_m = sum_j w_j zeta_j^m Y_j, m = 0..M-1;
4. orthonormalise span[S_0 .. S_{M-1}] (Euclidean SVD, rank cut 1e-12);
5. Rayleigh-Ritz: A_k = Q^T A Q, B_k = Q^T B Q, dense eigh(A_k, B_k),
   Ritz vectors X = Q U, keep lambda in the contour's keep window;
6. residuals, one FEAST-type refinement pass if any kept pair misses tol;
7. merge / de-duplicate across contours, normalise and sort.

Readings of points the paper leaves open (all listed in the design notes):
nodes zeta_j = exp(i pi (2j-1)/N) (no node on the real axis), weights
w_j = R zeta_j / N (trapezoid rule for the contour integral (1/2 pi i) dz), moment base
zeta^m = ((z - c)/R)^m instead of raw z^m (same span, better conditioned),
real Gaussian V shared by all contours, residual
||A x - lambda B x||_2 / (||A||_inf ||x||_2), half-open keep windows,
refinement V <- all Ritz vectors with one moment, sign: largest-|.| entry
positive (ties within 1e-4 relative go to the lowest index), duplicates
across contours merged by value cluster and B-projection.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl
from threadpoolctl import threadpool_limits

from .rng import gaussian_block


def quadrature(center: float, radius: float, n_nodes: int):
    """Trapezoid nodes and weights on a circle (Appendix, quadrature equation).

    zeta_j = exp(i pi (2j - 1) / N), z_j = c + R zeta_j, w_j = R zeta_j / N,
    j = 1..N.  Returns (z, w, zeta) as complex arrays of length N.
    """
    j = np.arange(1, n_nodes + 1)
    zeta = np.exp(1j * np.pi * (2 * j - 1) / n_nodes)
    return center + radius * zeta, radius * zeta / n_nodes, zeta


def filter_value(center: float, radius: float, n_nodes: int, lam) -> np.ndarray:
    """Value at real lam of the rational filter that the quadrature applies to
    the spectrum (Appendix, quadrature equation): f(lam) = Re sum_j w_j /
    (z_j - lam), about 1 well inside the circle, 1/2 on it and about 0 outside.
    Used for the boundary-proximity check of the robustness safeguards
    (Appendix, robustness under mild distribution shifts)."""
    z, w, _ = quadrature(center, radius, n_nodes)
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    return np.real((w[None, :] / (z[None, :] - lam[:, None])).sum(axis=1))


def inf_norm(A) -> float:
    """Maximum absolute row sum of a sparse matrix."""
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))


def residuals(A, B, lam: np.ndarray, X: np.ndarray) -> np.ndarray:
    """rho_i = ||A x_i - lambda_i B x_i||_2 / (||A||_inf ||x_i||_2)."""
    if X.shape[1] == 0:
        return np.zeros(0)
    R = A @ X - (B @ X) * lam[None, :]
    return np.linalg.norm(R, axis=0) / (inf_norm(A) * np.linalg.norm(X, axis=0))


_SHARED = {}


def _pair_moments(args):
    """Moments contributed by the conjugate node pair (j, N+1-j) of one circle.

    Both nodes are solved with their own LU; the pair's imaginary parts cancel
    for a real pencil and real V, and the real part is returned together with
    the size of the cancelled imaginary part (a check of the quadrature).
    The pencil and B V are read from the fork-inherited _SHARED table.
    """
    c, R, N, M, jpair = args
    A, B, BV = _SHARED["A"], _SHARED["B"], _SHARED["BV"]
    z, w, zeta = quadrature(c, R, N)
    n, L = BV.shape
    acc = np.zeros((n, L * M), dtype=np.complex128)
    with threadpool_limits(1):
        for j in jpair:
            K = (z[j] * B - A).tocsc()
            lu = spl.splu(K, permc_spec="MMD_AT_PLUS_A")
            Y = lu.solve(BV.astype(np.complex128))
            for m in range(M):
                acc[:, m * L:(m + 1) * L] += (w[j] * zeta[j] ** m) * Y
    return acc.real.copy(), float(np.linalg.norm(acc.imag)), float(np.linalg.norm(acc.real))


def contour_moments(A, B, V, center, radius, n_nodes, moments, workers=1, progress=None):
    """S = [S_0 ... S_{M-1}] (n x L*M, real) for one circle, all N nodes solved."""
    if n_nodes % 2:
        raise ValueError("the oracle pairs conjugate nodes: N must be even")
    _SHARED.update(A=A, B=B, BV=B @ V)
    tasks = [(center, radius, n_nodes, moments, (j, n_nodes - 1 - j))
             for j in range(n_nodes // 2)]
    pool = None
    if workers > 1:
        pool = ProcessPoolExecutor(max_workers=min(workers, len(tasks)),
                                   mp_context=mp.get_context("fork"))
    it = pool.map(_pair_moments, tasks) if pool is not None else map(_pair_moments, tasks)
    S = None
    im2 = 0.0
    re2 = 0.0
    for part, im, re in it:
        if progress is not None:
            progress("node pair solved")
        S = part if S is None else S + part
        im2 += im * im
        re2 += re * re
    if pool is not None:
        pool.shutdown()
    _SHARED.clear()
    if np.sqrt(im2) > 1e-10 * max(np.sqrt(re2), 1e-300):
        raise AssertionError("conjugate node pairs did not cancel the imaginary part")
    return S


def orth(S: np.ndarray, rank_tol: float = 1e-12):
    """Orthonormal basis of range(S) from the SVD, singular values > rank_tol * s_1.

    Also returns s_min / s_1 over all columns of S: when even the weakest
    direction keeps a weight above SATURATION (1e-3), more eigenvectors carry
    filter weight than S has columns and eigenvalues may be missed.
    """
    U, s, _ = np.linalg.svd(S, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return U[:, :0], 0, 0.0
    r = int(np.sum(s > rank_tol * s[0]))
    return U[:, :r], r, float(s[-1] / s[0])


SATURATION = 1e-3


def rayleigh_ritz(A, B, Q):
    """Reduced GEP Q^T A Q u = theta Q^T B Q u, Ritz vectors X = Q U (B-orthonormal)."""
    AQ = A @ Q
    BQ = B @ Q
    TA = Q.T @ AQ
    TB = Q.T @ BQ
    TA = 0.5 * (TA + TA.T)
    TB = 0.5 * (TB + TB.T)
    theta, U = sla.eigh(TA, TB)
    return theta, Q @ U


SIGN_TIE = 1e-4


def _normalise(X: np.ndarray, B) -> np.ndarray:
    """B-normalise each column and make its largest-|.| entry positive.

    Entries whose modulus is within a relative SIGN_TIE of the column's
    largest count as tied, and the lowest index among them decides the sign:
    eigenvectors of mirror-symmetric pencils have pairs of entries of exactly
    equal modulus, which the errors of a computed eigenvector (about the
    residual over the spectral gap, 1e-7 for pairs accepted at residual
    1e-8) would otherwise order at random.
    """
    X = X / np.sqrt(np.einsum("ij,ij->j", X, B @ X))[None, :]
    a = np.abs(X)
    top = a.max(axis=0)
    idx = np.argmax(a >= (1.0 - SIGN_TIE) * top[None, :], axis=0)
    sgn = np.sign(X[idx, np.arange(X.shape[1])])
    sgn[sgn == 0] = 1.0
    return X * sgn[None, :]


def _solve_contour(A, B, V0, c, R, lo, hi, N, M, tol, max_refine, rank_tol, workers, progress=None):
    V, Mcur = V0, M
    info = {"passes": 0, "rank": [], "saturated": False}
    for p in range(max_refine + 1):
        S = contour_moments(A, B, V, c, R, N, Mcur, workers, progress)
        Q, r, smin = orth(S, rank_tol)
        info["rank"].append(r)
        if p == 0 and smin > SATURATION:
            info["saturated"] = True
        theta, X = rayleigh_ritz(A, B, Q)
        rho = residuals(A, B, theta, X)
        info["passes"] = p + 1
        keep = (theta >= lo) & (theta < hi)
        if np.all(rho[keep] <= tol) or p == max_refine:
            break
        V, Mcur = X, 1
    return theta[keep], X[:, keep], rho[keep], info


def dedupe(lam, X, rho, cid, B, rel: float = 1e-8, overlap: float = 0.9):
    """Merge the pairs that several contours found for the same eigenvalue.

    Values are grouped into clusters (ascending, consecutive values within
    rel * |lambda| of each other).  In a cluster holding pairs of several
    contours, the contour whose cluster pairs have the smallest worst
    residual (lowest id on ties) keeps all of them; the other contours' pairs
    follow in ascending residual, and a pair is dropped when its B-orthogonal
    projection onto the span of the pairs kept so far has B-norm >= overlap
    times its own (it repeats an eigenvector already returned).  Pairs of one
    contour are never merged with each other: an exact multiple eigenvalue
    keeps all its vectors.
    """
    order = np.argsort(lam, kind="stable")
    lam, X, rho, cid = lam[order], X[:, order], rho[order], cid[order]
    keep = np.ones(lam.size, dtype=bool)
    BX = B @ X
    start = 0
    while start < lam.size:
        end = start + 1
        while end < lam.size and lam[end] - lam[end - 1] <= rel * max(abs(lam[end]), abs(lam[end - 1])):
            end += 1
        idx = np.arange(start, end)
        owners = sorted(set(cid[idx].tolist()), key=lambda k: (rho[idx][cid[idx] == k].max(), k))
        if len(owners) > 1:
            kept = [int(i) for i in idx if cid[i] == owners[0]]
            for k in owners[1:]:
                mine = sorted((int(i) for i in idx if cid[i] == k), key=lambda i: (rho[i], i))
                for i in mine:
                    G = X[:, kept].T @ BX[:, kept]
                    b = X[:, kept].T @ BX[:, i]
                    proj2 = float(b @ np.linalg.solve(G, b))
                    if proj2 >= overlap ** 2 * float(X[:, i] @ BX[:, i]):
                        keep[i] = False
                    else:
                        kept.append(i)
        start = end
    return lam[keep], X[:, keep], rho[keep], cid[keep]


def oracle_ci_solve(A, B, contours, n_nodes: int, moments: int, block: int, tol: float = 1e-8,
                    seed: int | None = 1, V: np.ndarray | None = None, max_refine: int = 1,
                    rank_tol: float = 1e-12, workers: int = 1, progress=None):
    """All eigenpairs of (A, B) inside the contours' keep windows.

    contours: array (K, 4) of [centre, radius, keep_lo, keep_hi]; keep windows
    are half-open.  Returns a dict with ascending ``evals``, B-normalised
    ``evecs`` (n x m), ``resid`` (rho), ``contour`` ids and per-contour info.
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    B = sp.csr_matrix(B, dtype=np.float64)
    n = A.shape[0]
    contours = np.atleast_2d(np.asarray(contours, dtype=np.float64))
    if V is None:
        V = gaussian_block(n, block, seed)
    lams, Xs, rhos, cids, infos = [], [], [], [], []
    for k, (c, R, lo, hi) in enumerate(contours):
        lam, X, rho, info = _solve_contour(A, B, V, c, R, lo, hi, n_nodes, moments, tol,
                                           max_refine, rank_tol, workers, progress)
        lams.append(lam)
        Xs.append(X)
        rhos.append(rho)
        cids.append(np.full(lam.size, k, dtype=np.int32))
        infos.append(info)
    lam = np.concatenate(lams)
    X = np.concatenate(Xs, axis=1) if Xs else np.zeros((n, 0))
    rho = np.concatenate(rhos)
    cid = np.concatenate(cids)
    lam, X, rho, cid = dedupe(lam, X, rho, cid, B)
    X = _normalise(X, B) if X.shape[1] else X
    rho = residuals(A, B, lam, X)
    return {"evals": lam, "evecs": X, "resid": rho, "contour": cid, "info": infos}


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))
