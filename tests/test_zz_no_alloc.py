"""gep_gram_noalloc: the Gram product with its split-K partials in the
library's static device scratch instead of a per-call allocation.

Checked through the C ABI against gep_gram (same kernels, same split plan,
so the results agree bit for bit) on two calls in a row, the second with a
smaller input, so the second call reads a scratch that still holds the
first call's partials.  Also checked against a float64 numpy product.
"""
import numpy as np
import pytest

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


def _both(dev, n, k1, k2, seed):
    import torch
    from paper_2511_01927_amd import gep_ci
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, k1))
    Y = rng.standard_normal((n, k2))
    Xd, Yd = _t(X, dev), _t(Y, dev)
    G0 = torch.full((k1, k2), np.nan, dtype=torch.float64, device=dev)
    G1 = torch.full((k1, k2), np.nan, dtype=torch.float64, device=dev)
    gep_ci.gep_gram(Xd, k1, Yd, k2, n, k1, k2, G0, stream=0)
    gep_ci.gep_gram_noalloc(Xd, k1, Yd, k2, n, k1, k2, G1, stream=0)
    g0, g1 = G0.cpu().numpy(), G1.cpu().numpy()
    return g0, g1, X.T @ Y


@pytest.mark.parametrize("sizes", [((90001, 256, 256), (4099, 150, 77)),
                                   ((70000, 64, 64), (1000, 33, 64))])
def test_gram_noalloc_matches_gram_two_calls(dev, sizes):
    for i, (n, k1, k2) in enumerate(sizes):
        g0, g1, ref = _both(dev, n, k1, k2, seed=100 + 7 * i + n)
        assert np.isfinite(g1).all()
        assert np.array_equal(g0, g1), (i, n, k1, k2, np.abs(g0 - g1).max())
        assert np.abs(g1 - ref).max() <= 1e-13 * np.sqrt(n) * 10


def test_gram_noalloc_rejects_oversized(dev):
    import torch
    from paper_2511_01927_amd import gep_ci
    # k1 = k2 = 4096: even one split needs 16 Mi doubles of partials (> 8 Mi)
    k = 4096
    X = torch.zeros((8, k), dtype=torch.float64, device=dev)
    G = torch.zeros((k, k), dtype=torch.float64, device=dev)
    with pytest.raises(gep_ci.GepError) as e:
        gep_ci.gep_gram_noalloc(X, k, X, k, 8, k, k, G, stream=0)
    assert e.value.status == -1
    assert "scratch" in str(e.value)
