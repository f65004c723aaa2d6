"""Pins of the input generators against closed-form discrete spectra.

The pencils are the inputs of every parity test, so their spectra are
checked against the separable closed forms of the constant-coefficient
discretisations (dense LAPACK eigensolves at small n as the reference):

* 1D linear FEM: lambda_j = (12/h^2) sin^2(theta_j/2) / (2 + cos theta_j),
  theta_j = j pi/(n+1);
* Q1 on a tensor grid: K = K1 (x) M1 + M1 (x) K1, M = M1 (x) M1, so the
  eigenvalues are sums of the 1D ones;
* 7-point FD with B = h^3 I: lambda = sum_d (4/h^2) sin^2(theta_d/2);
* 27-point trilinear FEM: sums of three 1D FEM eigenvalues.
"""
import numpy as np
import scipy.linalg as sla
import pytest

from workloads import pencils, configs


def _fem1d_closed(m):
    h = 1.0 / (m + 1)
    th = np.arange(1, m + 1) * np.pi / (m + 1)
    return 12.0 / h ** 2 * np.sin(th / 2) ** 2 / (2.0 + np.cos(th))


def _fd1d_closed(m):
    h = 1.0 / (m + 1)
    th = np.arange(1, m + 1) * np.pi / (m + 1)
    return 4.0 / h ** 2 * np.sin(th / 2) ** 2


def _gep(A, B):
    return sla.eigh(A.toarray(), B.toarray(), eigvals_only=True)


def test_fem1d_closed_form():
    A, B = pencils.fem1d(57)
    ref = _fem1d_closed(57)
    got = _gep(A, B)
    assert np.max(np.abs(got - ref) / ref) < 1e-12
    # eigenvectors are discrete sines
    j = 5
    th = j * np.pi / 58
    v = np.sin(np.arange(1, 58) * th)
    lam = ref[j - 1]
    r = A @ v - lam * (B @ v)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(A @ v)


def test_q1_2d_closed_form_rectangular():
    nx, ny = 11, 7
    A, B = pencils.q1_2d(nx, ny)
    ref = np.sort((_fem1d_closed(nx)[None, :] + _fem1d_closed(ny)[:, None]).ravel())
    got = _gep(A, B)
    assert np.max(np.abs(got - ref) / ref) < 1e-12
    assert np.allclose(ref, configs.q1_2d_eigs(nx, ny), rtol=1e-14)
    # 9-point pattern, symmetric
    assert A.nnz == B.nnz == (3 * nx - 2) * (3 * ny - 2)
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()


def test_q1_2d_variable_coefficient_is_spd_and_scales():
    nx, ny = 9, 8
    g = pencils.grf((ny + 1, nx + 1), seed=3)
    A, B = pencils.q1_2d(nx, ny, np.exp(g))
    a = A.toarray()
    assert np.allclose(a, a.T, atol=1e-13 * abs(a).max())
    assert np.linalg.eigvalsh(a).min() > 0
    # kappa -> 2 kappa doubles every eigenvalue
    A2, B2 = pencils.q1_2d(nx, ny, 2 * np.exp(g))
    assert np.allclose(_gep(A2, B2), 2 * _gep(A, B), rtol=1e-12)


def test_fd7_3d_closed_form():
    m = 5
    A, B = pencils.fd7_3d(m)
    l1 = _fd1d_closed(m)
    ref = np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())
    got = _gep(A, B)
    assert np.max(np.abs(got - ref) / ref) < 1e-12
    assert abs(B - B.T).max() == 0 and B.nnz == m ** 3


def test_q1_3d_closed_form():
    m = 4
    A, B = pencils.q1_3d(m)
    l1 = _fem1d_closed(m)
    ref = np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())
    got = _gep(A, B)
    assert np.max(np.abs(got - ref) / ref) < 1e-12
    # interior rows of the 27-point stencil have 27 entries
    assert np.max(np.diff(A.indptr)) == 27


def test_grf_moments_and_seed():
    g = pencils.grf((32, 32, 32), seed=11)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12
    assert np.array_equal(g, pencils.grf((32, 32, 32), seed=11))
    assert not np.array_equal(g, pencils.grf((32, 32, 32), seed=12))


def test_headline_windows():
    w = configs.fem1d_2000()
    lam = _fem1d_closed(2000)
    lo, hi = w.window
    assert np.sum((lam >= lo) & (lam < hi)) == 20
    assert w.contours.shape == (1, 4)
    c, R, klo, khi = w.contours[0]
    assert abs(c - (lo + hi) / 2) < 1e-9 and abs(R - (hi - lo) / 2) < 1e-9


@pytest.mark.slow
def test_q1_300_window_count():
    lam = configs.q1_2d_eigs(300, 300)
    lo, hi = configs.gap_window(lam, 1002, 1200)
    assert np.sum((lam >= lo) & (lam < hi)) == 199
    cont = configs.uniform_contours(lo, hi, 4, 0.1)
    assert np.allclose(cont[1:, 2], cont[:-1, 3])
