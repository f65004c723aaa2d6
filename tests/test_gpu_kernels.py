"""Kernel-level parity of the HIP library against plain numpy / the oracle.

Each kernel is called through the C ABI on seeded inputs whose sizes span
several tiles and a ragged tail, and compared element by element with a
float64 CPU computation.
"""
import numpy as np
import pytest

from tests.helpers import to_tiled, from_tiled

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _pencils():
    from workloads import pencils
    g = pencils.grf((38, 31), seed=5)
    return {"fem1d_2000": pencils.fem1d(2000), "q1_30x37_var": pencils.q1_2d(30, 37, np.exp(g)),
            "fd7_9": pencils.fd7_3d(9)}


@pytest.mark.parametrize("name", ["fem1d_2000", "q1_30x37_var", "fd7_9"])
@pytest.mark.parametrize("W", [64, 192])
def test_spmm_shifted_fp64(dev, name, W):
    import torch
    from paper_2511_01927_amd import gep_ci
    A, B = _pencils()[name]
    n = A.shape[0]
    rng = np.random.default_rng(W + n)
    X = rng.standard_normal((n, W)) + 1j * rng.standard_normal((n, W))
    z = rng.uniform(-5, 5, W) * np.abs(A).max() / np.abs(B).max() + 1j * rng.uniform(0.1, 3, W)
    ref = (B @ X) * z[None, :] - A @ X
    P = gep_ci.Pencil(A, B)
    Xd = _t(to_tiled(X).view(np.float64), dev)
    Yd = torch.zeros_like(Xd)
    zd = _t(z.astype(np.complex128).view(np.float64), dev)
    pq = torch.zeros(2 * W, dtype=torch.float64, device=dev)
    gep_ci.gep_spmm_shifted(P, zd, Xd, Yd, W, pq=pq, stream=0)
    Y = from_tiled(Yd.cpu().numpy().view(np.complex128), n, W)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err < 1e-14, err
    pq_ref = np.sum(X * ref, axis=0)
    pqg = pq.cpu().numpy().view(np.complex128)
    assert np.abs(pqg - pq_ref).max() <= 1e-12 * np.abs(pq_ref).max()


def test_spmm_shifted_fp32(dev):
    import torch
    from paper_2511_01927_amd import gep_ci
    A, B = _pencils()["q1_30x37_var"]
    n = A.shape[0]
    W = 128
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((n, W)) + 1j * rng.standard_normal((n, W))).astype(np.complex64)
    z = rng.uniform(0, 300, W) + 1j * rng.uniform(1, 30, W)
    ref = (B @ X.astype(np.complex128)) * z[None, :] - A @ X.astype(np.complex128)
    P = gep_ci.Pencil(A, B)
    Xd = _t(to_tiled(X).view(np.float32), dev)
    Yd = torch.zeros_like(Xd)
    zd = _t(z.astype(np.complex128).view(np.float64), dev)
    gep_ci.gep_spmm_shifted_f32(P, zd, Xd, Yd, W, stream=0)
    Y = from_tiled(Yd.cpu().numpy().view(np.complex64), n, W)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err


@pytest.mark.parametrize("k", [1, 70, 130])
def test_spmm_real(dev, k):
    import torch
    from paper_2511_01927_amd import gep_ci
    A, B = _pencils()["q1_30x37_var"]
    n = A.shape[0]
    X = np.random.default_rng(k).standard_normal((n, k))
    P = gep_ci.Pencil(A, B)
    Xd = _t(X, dev)
    YA = torch.zeros_like(Xd)
    YB = torch.zeros_like(Xd)
    gep_ci.gep_spmm_real(P, Xd, k, k, YA, YB, stream=0)
    assert np.abs(YA.cpu().numpy() - A @ X).max() <= 1e-14 * np.abs(A @ X).max()
    assert np.abs(YB.cpu().numpy() - B @ X).max() <= 1e-14 * np.abs(B @ X).max()


@pytest.mark.parametrize("n,k1,k2", [(1000, 64, 64), (4099, 200, 130), (37, 5, 3), (90001, 256, 256)])
def test_gram_mfma(dev, n, k1, k2):
    import torch
    from paper_2511_01927_amd import gep_ci
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, k1))
    Y = rng.standard_normal((n, k2))
    G = torch.zeros((k1, k2), dtype=torch.float64, device=dev)
    gep_ci.gep_gram(_t(X, dev), k1, _t(Y, dev), k2, n, k1, k2, G, stream=0)
    ref = X.T @ Y
    assert np.abs(G.cpu().numpy() - ref).max() <= 1e-13 * np.sqrt(n) * 10


@pytest.mark.parametrize("n,k,m", [(1000, 64, 64), (4099, 150, 77), (5, 3, 2), (90001, 256, 200)])
def test_gemm_tall_mfma(dev, n, k, m):
    import torch
    from paper_2511_01927_amd import gep_ci
    rng = np.random.default_rng(n + k)
    X = rng.standard_normal((n, k))
    T = rng.standard_normal((k, m))
    Cm = torch.zeros((n, m), dtype=torch.float64, device=dev)
    gep_ci.gep_gemm_tall(_t(X, dev), k, _t(T, dev), m, n, k, m, Cm, m, stream=0)
    ref = X @ T
    assert np.abs(Cm.cpu().numpy() - ref).max() <= 1e-13 * np.sqrt(k) * 10


@pytest.mark.parametrize("k", [1, 2, 17, 33, 65, 100, 256, 500])
def test_sym_eig_jacobi(dev, k):
    import torch
    from paper_2511_01927_amd import gep_ci
    rng = np.random.default_rng(k)
    g = rng.standard_normal((k, k))
    A = g + g.T
    # a graded spectrum like a Gram matrix
    if k >= 17:
        Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
        A = Q @ np.diag(10.0 ** rng.uniform(-14, 0, k)) @ Q.T
        A = 0.5 * (A + A.T)
    Ad = _t(A, dev)
    w = torch.zeros(k, dtype=torch.float64, device=dev)
    V = torch.zeros((k, k), dtype=torch.float64, device=dev)
    gep_ci.gep_sym_eig(Ad, w, V, k, 1, stream=0)
    wh, Vh = w.cpu().numpy(), V.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    assert np.abs(wh - ref).max() <= 1e-14 * scale * max(1, k) ** 0.5
    assert np.abs(Vh.T @ Vh - np.eye(k)).max() <= 1e-13 * max(1, k)
    assert np.abs(A @ Vh - Vh * wh[None, :]).max() <= 1e-13 * scale * max(1, k)


def test_sym_eig_batch_and_clusters(dev):
    """Three matrices in one call: exactly repeated eigenvalues (clusters of
    four), a diagonal matrix (nothing to rotate) and a graded spectrum; per
    matrix the eigenvalues match, V is orthonormal and A V = V diag(w)."""
    import torch
    from paper_2511_01927_amd import gep_ci
    k = 96
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    lam = np.repeat(np.arange(1.0, k // 4 + 1), 4)
    A0 = Q @ np.diag(lam) @ Q.T
    A1 = np.diag(rng.uniform(-1, 1, k))
    Q2, _ = np.linalg.qr(rng.standard_normal((k, k)))
    A2 = Q2 @ np.diag(10.0 ** rng.uniform(-12, 0, k)) @ Q2.T
    mats = [0.5 * (M + M.T) for M in (A0, A1, A2)]
    Ad = _t(np.stack(mats), dev)
    w = torch.zeros(3 * k, dtype=torch.float64, device=dev)
    V = torch.zeros((3, k, k), dtype=torch.float64, device=dev)
    gep_ci.gep_sym_eig(Ad, w, V, k, 3, stream=0)
    wh, Vh = w.cpu().numpy().reshape(3, k), V.cpu().numpy()
    for b, A in enumerate(mats):
        ref = np.linalg.eigvalsh(A)
        scale = np.abs(ref).max()
        assert np.abs(wh[b] - ref).max() <= 1e-14 * scale * k ** 0.5
        assert np.abs(Vh[b].T @ Vh[b] - np.eye(k)).max() <= 1e-13 * k
        assert np.abs(A @ Vh[b] - Vh[b] * wh[b][None, :]).max() <= 1e-13 * scale * k


def test_gaussian_block_matches_oracle_generator(dev):
    import torch
    from paper_2511_01927_amd import gep_ci
    from oracle import rng
    n, L = 1001, 7
    V = torch.zeros((n, L), dtype=torch.float64, device=dev)
    gep_ci.gep_gaussian_block(12345, n, L, V, stream=0)
    ref = rng.gaussian_block(n, L, 12345)
    assert np.abs(V.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()
