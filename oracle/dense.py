"""Brute-force dense eigensolver for small symmetric-definite pencils.

Solves A v = lambda B v (Sec. 3.1, Eq. GEP, real symmetric A and symmetric
positive definite B) by the textbook reduction: Cholesky B = L L^T, the
standard symmetric problem C = L^-1 A L^-T, cyclic Jacobi rotations on C
(Golub and Van Loan, Matrix Computations, Sec. 8.5), and back-substitution
v = L^-T y.  Everything is written out here (no LAPACK eigensolver) so that
it can serve as an independent check of the CI oracle.  Intended for n <= 300.
"""
from __future__ import annotations

import numpy as np


def cholesky(b: np.ndarray) -> np.ndarray:
    """Lower-triangular L with L L^T = b (column-by-column Cholesky-Banachiewicz)."""
    n = b.shape[0]
    low = np.zeros_like(b, dtype=np.float64)
    for j in range(n):
        d = b[j, j] - low[j, :j] @ low[j, :j]
        if not d > 0.0:
            raise np.linalg.LinAlgError("matrix is not positive definite")
        low[j, j] = np.sqrt(d)
        low[j + 1:, j] = (b[j + 1:, j] - low[j + 1:, :j] @ low[j, :j]) / low[j, j]
    return low


def forward_solve(low: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve L y = rhs for lower-triangular L (rhs may have several columns)."""
    y = np.array(rhs, dtype=np.float64, copy=True)
    n = low.shape[0]
    for i in range(n):
        y[i] = (y[i] - low[i, :i] @ y[:i]) / low[i, i]
    return y


def backward_solve_t(low: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve L^T x = rhs for lower-triangular L."""
    x = np.array(rhs, dtype=np.float64, copy=True)
    n = low.shape[0]
    for i in range(n - 1, -1, -1):
        x[i] = (x[i] - low[i + 1:, i] @ x[i + 1:]) / low[i, i]
    return x


def jacobi_eigh(c: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic Jacobi eigen-decomposition of a symmetric matrix.

    Sweeps over all (p, q), p < q, annihilating c[p, q] with the rotation whose
    tangent is the smaller root of t^2 + 2 tau t - 1 = 0, tau = (c_qq - c_pp)/(2 c_pq),
    until the off-diagonal Frobenius norm is <= tol * ||c||_F.
    Returns ascending eigenvalues and orthonormal eigenvectors (columns).
    """
    a = np.array(c, dtype=np.float64, copy=True)
    a = 0.5 * (a + a.T)
    n = a.shape[0]
    v = np.eye(n)
    fro = np.linalg.norm(a)
    for _ in range(max_sweeps):
        off = np.sqrt(max(np.sum(a * a) - np.sum(np.diag(a) ** 2), 0.0))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = a[p, q]
                if apq == 0.0:
                    continue
                diff = a[q, q] - a[p, p]
                if abs(diff) > 1e150 * abs(apq):
                    t = apq / diff               # tau huge: t = 1/(2 tau) to first order
                else:
                    tau = diff / (2.0 * apq)
                    t = np.sign(tau) / (abs(tau) + np.sqrt(1.0 + tau * tau)) if tau != 0 else 1.0
                cs = 1.0 / np.sqrt(1.0 + t * t)
                sn = t * cs
                ap = a[:, p].copy()
                aq = a[:, q].copy()
                a[:, p] = cs * ap - sn * aq
                a[:, q] = sn * ap + cs * aq
                rp = a[p, :].copy()
                rq = a[q, :].copy()
                a[p, :] = cs * rp - sn * rq
                a[q, :] = sn * rp + cs * rq
                vp = v[:, p].copy()
                vq = v[:, q].copy()
                v[:, p] = cs * vp - sn * vq
                v[:, q] = sn * vp + cs * vq
    w = np.diag(a).copy()
    order = np.argsort(w, kind="stable")
    return w[order], v[:, order]


def dense_bruteforce(A, B):
    """All eigenpairs of the pencil (A, B): ascending lambda, B-orthonormal X."""
    a = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    b = B.toarray() if hasattr(B, "toarray") else np.asarray(B, dtype=np.float64)
    low = cholesky(b)
    # C = L^-1 A L^-T, built from two triangular solves
    t = forward_solve(low, a)          # L^-1 A
    cmat = forward_solve(low, t.T)     # L^-1 (L^-1 A)^T = L^-1 A L^-T
    lam, y = jacobi_eigh(cmat)
    x = backward_solve_t(low, y)
    return lam, x
