"""Seeded synthetic pencils (A, B) that stand in for the paper's FEM workloads.

The paper builds its generalized eigenproblems from Galerkin finite-element
discretisations of PDEs whose coefficient fields are Gaussian random fields
(Sec. 3.1 "Problem Formulation"; Appendix "From Partial Differential Equation
to GEPs"; dataset appendix, thermal-diffusion and EM-cavity domains).  Its
datasets are not released, so these generators produce pencils with the same
structure: Dirichlet problems on the unit interval / square / cube, interior
nodes only, h = 1/(m+1) per direction.

This module is input generation only.  It holds none of the contour-integral
method's arithmetic and is shared by the oracle, the tests and the benchmark.
All matrices are returned as scipy.sparse CSR with sorted column indices,
int64 row pointers and int32 column indices, both triangles stored.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _csr(mat) -> sp.csr_matrix:
    m = sp.csr_matrix(mat)
    m.sum_duplicates()
    m.sort_indices()
    m.indptr = m.indptr.astype(np.int64)
    m.indices = m.indices.astype(np.int32)
    return m


def _line_mats(m: int):
    """1D linear-FEM stiffness and mass on m interior nodes, h = 1/(m+1)."""
    h = 1.0 / (m + 1)
    e = np.ones(m)
    k = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]) / h
    ms = sp.diags([e[:-1], 4 * e, e[:-1]], [-1, 0, 1]) * (h / 6.0)
    return k, ms


def fem1d(n: int):
    """Linear FEM for -u'' = lambda u on (0,1), Dirichlet, n interior nodes.

    K = tridiag(-1, 2, -1)/h and M = h tridiag(1, 4, 1)/6 with h = 1/(n+1).
    """
    if n < 2:
        raise ValueError("fem1d needs n >= 2")
    k, m = _line_mats(n)
    return _csr(k), _csr(m)


def q1_2d(nx: int, ny: int, kappa=None):
    """Bilinear (Q1) FEM for -div(kappa grad u) = lambda u on the unit square.

    Dirichlet boundary, nx*ny interior nodes numbered i = ix + nx*iy.
    ``kappa`` is None (kappa = 1) or an array of shape (ny+1, nx+1) holding
    one value per element (cell centre).  The mass matrix is the consistent
    Q1 mass with unit coefficient, so both matrices have the 9-point pattern.
    """
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    ex, ey = nx + 1, ny + 1
    if kappa is None:
        kap = np.ones((ey, ex))
    else:
        kap = np.asarray(kappa, dtype=np.float64)
        if kap.shape != (ey, ex):
            raise ValueError(f"kappa must have shape {(ey, ex)}")
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    # local node order: (a, b) with a the x offset, b the y offset
    kx, mx = k1 / hx, m1 * hx
    ky, my = k1 / hy, m1 * hy
    ke = np.zeros((4, 4))
    me = np.zeros((4, 4))
    offs = [(a, b) for b in range(2) for a in range(2)]
    for p, (ap, bp) in enumerate(offs):
        for q, (aq, bq) in enumerate(offs):
            ke[p, q] = kx[ap, aq] * my[bp, bq] + mx[ap, aq] * ky[bp, bq]
            me[p, q] = mx[ap, aq] * my[bp, bq]
    jy, jx = np.meshgrid(np.arange(ey), np.arange(ex), indexing="ij")
    jx, jy, kv = jx.ravel(), jy.ravel(), kap.ravel()
    rows, cols, kvals, mvals = [], [], [], []
    for p, (ap, bp) in enumerate(offs):
        gx_p, gy_p = jx + ap - 1, jy + bp - 1  # interior index of the local node
        ok_p = (gx_p >= 0) & (gx_p < nx) & (gy_p >= 0) & (gy_p < ny)
        for q, (aq, bq) in enumerate(offs):
            gx_q, gy_q = jx + aq - 1, jy + bq - 1
            ok = ok_p & (gx_q >= 0) & (gx_q < nx) & (gy_q >= 0) & (gy_q < ny)
            rows.append((gx_p + nx * gy_p)[ok])
            cols.append((gx_q + nx * gy_q)[ok])
            kvals.append(kv[ok] * ke[p, q])
            mvals.append(np.full(int(ok.sum()), me[p, q]))
    r, c = np.concatenate(rows), np.concatenate(cols)
    n = nx * ny
    a = sp.coo_matrix((np.concatenate(kvals), (r, c)), shape=(n, n))
    b = sp.coo_matrix((np.concatenate(mvals), (r, c)), shape=(n, n))
    return _csr(a), _csr(b)


def fd7_3d(m: int, kappa=None):
    """7-point finite differences for -div(kappa grad u) on the unit cube.

    Dirichlet boundary, m^3 interior nodes numbered i = ix + m*(iy + m*iz).
    ``kappa`` is None or a nodal field of shape (m+2, m+2, m+2) indexed
    [z, y, x] including boundary nodes; face coefficients are harmonic means
    of the two nodal values.  Scaled by h^3 so that the lumped mass is
    B = h^3 I.
    """
    h = 1.0 / (m + 1)
    if kappa is None:
        kap = np.ones((m + 2,) * 3)
    else:
        kap = np.asarray(kappa, dtype=np.float64)
        if kap.shape != (m + 2,) * 3:
            raise ValueError(f"kappa must have shape {(m + 2,) * 3}")
    n = m ** 3
    iz, iy, ix = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    idx = ix + m * (iy + m * iz)
    kc = kap[iz + 1, iy + 1, ix + 1]
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for dx, dy, dz in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        kn = kap[iz + 1 + dz, iy + 1 + dy, ix + 1 + dx]
        kf = 2.0 * kc * kn / (kc + kn)
        diag += kf * h
        jx, jy, jz = ix + dx, iy + dy, iz + dz
        ok = (jx >= 0) & (jx < m) & (jy >= 0) & (jy < m) & (jz >= 0) & (jz < m)
        rows.append(idx[ok])
        cols.append((jx + m * (jy + m * jz))[ok])
        vals.append(-kf[ok] * h)
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    a = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    b = sp.identity(n, format="csr") * h ** 3
    return _csr(a), _csr(b)


def q1_3d(m: int, kappa=None):
    """Trilinear (Q1) FEM, 27-point K and consistent M, on the unit cube.

    Dirichlet boundary, m^3 interior nodes numbered i = ix + m*(iy + m*iz).
    ``kappa`` is None or an element field of shape (m+1, m+1, m+1) [z, y, x].
    """
    h = 1.0 / (m + 1)
    ne = m + 1
    if kappa is None:
        kap = np.ones((ne,) * 3)
    else:
        kap = np.asarray(kappa, dtype=np.float64)
        if kap.shape != (ne,) * 3:
            raise ValueError(f"kappa must have shape {(ne,) * 3}")
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * (h / 6.0)
    offs = [(a, b, c) for c in range(2) for b in range(2) for a in range(2)]
    ke = np.zeros((8, 8))
    me = np.zeros((8, 8))
    for p, (ap, bp, cp) in enumerate(offs):
        for q, (aq, bq, cq) in enumerate(offs):
            mxx, myy, mzz = m1[ap, aq], m1[bp, bq], m1[cp, cq]
            ke[p, q] = k1[ap, aq] * myy * mzz + mxx * k1[bp, bq] * mzz + mxx * myy * k1[cp, cq]
            me[p, q] = mxx * myy * mzz
    jz, jy, jx = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    jx, jy, jz, kv = jx.ravel(), jy.ravel(), jz.ravel(), kap.ravel()
    n = m ** 3
    rows, cols, kvals, mvals = [], [], [], []
    for p, (ap, bp, cp) in enumerate(offs):
        gx, gy, gz = jx + ap - 1, jy + bp - 1, jz + cp - 1
        okp = (gx >= 0) & (gx < m) & (gy >= 0) & (gy < m) & (gz >= 0) & (gz < m)
        ip = gx + m * (gy + m * gz)
        for q, (aq, bq, cq) in enumerate(offs):
            hx_, hy_, hz_ = jx + aq - 1, jy + bq - 1, jz + cq - 1
            ok = okp & (hx_ >= 0) & (hx_ < m) & (hy_ >= 0) & (hy_ < m) & (hz_ >= 0) & (hz_ < m)
            rows.append(ip[ok])
            cols.append((hx_ + m * (hy_ + m * hz_))[ok])
            kvals.append(kv[ok] * ke[p, q])
            mvals.append(np.full(int(ok.sum()), me[p, q]))
    r, c = np.concatenate(rows), np.concatenate(cols)
    a = sp.coo_matrix((np.concatenate(kvals), (r, c)), shape=(n, n))
    b = sp.coo_matrix((np.concatenate(mvals), (r, c)), shape=(n, n))
    return _csr(a), _csr(b)


def grf(shape, seed: int, ell: float = 0.1, sigma: float = 1.0) -> np.ndarray:
    """Gaussian random field on a unit-box grid, squared-exponential covariance.

    Synthesised spectrally with numpy's PCG64 generator: white noise is
    filtered in Fourier space by the square root of the covariance spectrum
    exp(-(2 pi |k| ell)^2 / 4) and the sample is rescaled to zero mean and
    standard deviation ``sigma``.  Returns log-coefficients g; the coefficient
    field is exp(g).
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    freqs = np.meshgrid(*[np.fft.fftfreq(s, d=1.0 / s) for s in shape], indexing="ij")
    k2 = sum(f * f for f in freqs)
    filt = np.exp(-((2.0 * np.pi * ell) ** 2) * k2 / 4.0)
    g = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g *= sigma / sd
    return g
