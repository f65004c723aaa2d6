"""Pins of the learned-contour oracles (density MLP in float64, KDE contours)
and of the pure helpers of the learned pipeline."""
import math

import numpy as np
import pytest

from oracle import density, kde


def test_gelu_values():
    # GELU(z) = z Phi(z): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    z = np.array([0.0, 1.0, -1.0, 3.0])
    g = density.gelu(z)
    assert abs(g[0]) == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + 0.15865525393145707) < 1e-15
    assert abs(density.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_density_gradients_match_finite_differences():
    r = np.random.default_rng(0)
    dims = [(6, 5), (5,), (5, 5), (5,), (5, 3), (3,)]
    params = [r.standard_normal(d) * 0.7 for d in dims]
    X = r.standard_normal((4, 6))
    T = r.standard_normal((4, 3))
    loss, grads = density.loss_and_grads(params, X, T)
    h = 1e-6
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        gf = g.reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp, _ = density.loss_and_grads(params, X, T)
            flat[i] = old - h
            lm, _ = density.loss_and_grads(params, X, T)
            flat[i] = old
            assert abs((lp - lm) / (2 * h) - gf[i]) < 1e-7 * max(1.0, abs(gf[i]))


def test_kde_cuts_in_gaps_and_bounds_counts():
    lam = np.concatenate([np.linspace(0, 1, 30), np.linspace(2, 3, 30), np.linspace(4, 5, 30)])
    # a kernel narrower than the gaps (w = 200 for an interval of width 6)
    ivs = kde.kde_intervals(lam, nmin=10, nmax=50, w=200.0, window=(-0.5, 5.5))
    assert len(ivs) == 3
    cuts = [ivs[0][1], ivs[1][1]]
    assert 1.0 < cuts[0] < 2.0 and 3.0 < cuts[1] < 4.0
    assert abs(cuts[0] - 1.5) < 1e-12 and abs(cuts[1] - 3.5) < 1e-12
    assert ivs[0][0] == -0.5 and ivs[-1][1] == 5.5


def _g_scan(inside, s, e, w):
    """Sparsity G(t) = sum_k exp(-w ((t - x_k) / (e - s))^2) at every midpoint
    between consecutive distinct sorted predictions (the interval's interior
    candidates), scanned directly."""
    mids = [0.5 * (a + b) for a, b in zip(inside[:-1], inside[1:]) if b > a]
    g = [float(np.sum(np.exp(-w * ((t - np.asarray(inside)) / (e - s)) ** 2))) for t in mids]
    return np.asarray(mids), np.asarray(g)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kde_cut_is_the_plain_argmin_when_it_leaves_nmin_each_side(seed):
    """Sec. 4.2, Alg. "Adaptive Contour Construction via KDE": the interval is
    split at the minimum of G.  The reading here restricts candidates to
    midpoints that leave N_min predictions on each side; whenever the plain
    argmin over all interior midpoints already does, the cut is that argmin.
    One split (N_max = n - 1) exposes the cut as the shared interval end."""
    r = np.random.default_rng(seed)
    lam = np.sort(np.concatenate([r.uniform(0.0, 1.0, 40), r.uniform(1.6, 3.0, 50)]))
    # a kernel narrow against the gap, so G is least inside it and not at the ends
    s, e, w, nmin = -0.1, 3.1, 200.0, 10
    mids, g = _g_scan(list(lam), s, e, w)
    t_star = mids[int(np.argmin(g))]
    left = int(np.sum(lam < t_star))
    assert nmin <= left <= lam.size - nmin   # the plain argmin is admissible here
    ivs = kde.kde_intervals(lam, nmin=nmin, nmax=lam.size - 1, w=w, window=(s, e))
    assert len(ivs) == 2 and ivs[0][1] == ivs[1][0]
    assert abs(ivs[0][1] - t_star) <= 1e-15 * max(1.0, abs(t_star))


def test_kde_cut_skips_an_argmin_that_leaves_too_few():
    """The plain argmin of G sits next to the interval's end (a lone
    prediction far from the rest), leaving fewer than N_min on one side; the
    cut then goes to the admissible midpoint of least G."""
    lam = np.sort(np.concatenate([np.linspace(0.0, 1.0, 60), [2.9]]))
    s, e, w, nmin = -0.05, 3.0, 10.0, 10
    mids, g = _g_scan(list(lam), s, e, w)
    t_plain = mids[int(np.argmin(g))]
    assert np.sum(lam > t_plain) < nmin       # the plain argmin is not admissible
    ok = np.array([nmin <= np.sum(lam < t) <= lam.size - nmin for t in mids])
    t_adm = mids[ok][int(np.argmin(g[ok]))]
    ivs = kde.kde_intervals(lam, nmin=nmin, nmax=lam.size - 1, w=w, window=(s, e))
    assert len(ivs) == 2
    assert abs(ivs[0][1] - t_adm) <= 1e-15 * max(1.0, abs(t_adm))


def test_kde_default_weight_keeps_counts_in_range():
    r = np.random.default_rng(3)
    lam = np.sort(r.uniform(0, 10, 237))
    ivs = kde.kde_intervals(lam, nmin=10, nmax=50, w=10.0, window=(0.0, 10.0))
    counts = [np.sum((lam >= s) & ((lam <= e) if i == len(ivs) - 1 else (lam < e))) for i, (s, e) in enumerate(ivs)]
    assert sum(counts) == lam.size and max(counts) <= 50 and min(counts) >= 10
    assert all(a[1] == b[0] for a, b in zip(ivs[:-1], ivs[1:]))


def test_kde_merges_small_intervals():
    # a lone cluster of 4 predictions must be merged into a neighbour
    lam = np.concatenate([np.linspace(0, 1, 40), np.linspace(1.4, 1.5, 4), np.linspace(3, 4, 40)])
    ivs = kde.kde_intervals(lam, nmin=10, nmax=50, w=10.0, window=(-0.1, 4.1))
    counts = [np.sum((lam >= s) & ((lam <= e) if i == len(ivs) - 1 else (lam < e))) for i, (s, e) in enumerate(ivs)]
    assert min(counts) >= 10 and max(counts) <= 50
    assert sum(counts) == lam.size


def test_kde_circle_geometry_and_unsplittable():
    c = kde.kde_contours([1.0, 2.0, 3.0], nmin=1, nmax=5, alpha=0.5, window=(0.0, 4.0))
    assert c == [(2.0, 3.0, 0.0, 4.0)]
    # all predictions equal: cannot be split, kept as one interval
    assert len(kde.kde_intervals([1.0] * 80, nmin=1, nmax=50, window=(0.0, 2.0))) == 1
    # no window: initial interval is the hull widened by beta (max - min)
    ivs = kde.kde_intervals([0.0, 1.0, 2.0], nmin=1, nmax=50, beta=0.1)
    assert ivs == [(-0.2, 2.2)]


def test_quantile_points_and_histogram_helpers():
    from paper_2511_01927_amd import learned
    hist = np.ones(10, dtype=np.float32)
    pts = learned.quantile_points(hist, (0.0, 10.0), expected=20.0)
    assert pts.size == 20 and np.allclose(pts, np.arange(20) * 0.5 + 0.25)
    h = learned.histogram_target(np.array([0.5, 0.6, 9.5]), (0.0, 10.0), 10, expected=10.0)
    assert h[0] == 2.0 and h[9] == 1.0 and h.sum() == 3.0
    g = np.arange(64.0).reshape(8, 8)
    f = learned.field_features(g, side=4)
    assert f.shape == (16,) and abs(f[0] - np.mean(g[:2, :2])) < 1e-6
