"""Exact eigenvalue counts of a symmetric-definite pencil by Sylvester inertia.

The paper names eigenvalue-counting techniques among the contour-selection
tools (Sec. 3.2, "Motivation"; the Sylvester-inertia approach it cites).
For symmetric A and SPD B, the number of eigenvalues below sigma equals the
number of negative eigenvalues of A - sigma B, which by Sylvester's law of
inertia equals the number of negative eigenvalues of the block-diagonal
factor D in A - sigma B = L D L^T.  Dense LDL^T (Bunch-Kaufman, SciPy) is
used, so this is meant for n up to a few thousand.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def count_below(A, B, sigma: float) -> int:
    """Number of eigenvalues of (A, B) strictly below sigma."""
    a = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    b = B.toarray() if hasattr(B, "toarray") else np.asarray(B, dtype=np.float64)
    _, d, _ = sla.ldl(a - sigma * b, lower=True)
    neg = 0
    i = 0
    n = d.shape[0]
    while i < n:
        if i + 1 < n and d[i + 1, i] != 0.0:
            neg += int(np.sum(np.linalg.eigvalsh(d[i:i + 2, i:i + 2]) < 0.0))
            i += 2
        else:
            neg += int(d[i, i] < 0.0)
            i += 1
    return neg


def count_in(A, B, lo: float, hi: float) -> int:
    """Number of eigenvalues in [lo, hi) (exact when neither end is an eigenvalue)."""
    return count_below(A, B, hi) - count_below(A, B, lo)
