"""Pins of the oracle's quadrature filter (boundary-proximity check).

The N-node trapezoid rule on offset nodes zeta_j = exp(i pi (2j - 1) / N)
applies the rational filter f(c + r t) = 1 / (1 + t^N) to a real eigenvalue
at relative position t (a classical closed form: the zeta_j are the roots of
zeta^N = -1).  Special cases: f = 1 at the centre, 1/2 on the circle, and
f(c + r t) = f(c - r t) for even N.
"""
import numpy as np
import pytest

from oracle.cirr import filter_value


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64])
def test_filter_matches_closed_form(N):
    c, r = 37.5, 4.25
    t = np.concatenate([np.linspace(-2.5, 2.5, 41), [0.0, 0.999, 1.0, 1.001]])
    got = filter_value(c, r, N, c + r * t)
    want = 1.0 / (1.0 + t ** N)
    assert np.max(np.abs(got - want)) <= 1e-13


def test_filter_special_values():
    for N in (8, 32):
        assert abs(filter_value(2.0, 1.5, N, 2.0)[0] - 1.0) <= 1e-15
        np.testing.assert_allclose(filter_value(2.0, 1.5, N, [0.5, 3.5]), [0.5, 0.5], atol=1e-14)
        x = np.array([0.3, 0.8, 1.2])
        np.testing.assert_allclose(filter_value(2.0, 1.5, N, 2.0 + 1.5 * x),
                                   filter_value(2.0, 1.5, N, 2.0 - 1.5 * x), atol=1e-14)


def test_filter_transition_band_narrows_with_nodes():
    # the band where 0.1 < f < 0.9 shrinks as N grows: |t| in ((1/9)^(1/N), 9^(1/N))
    for N in (8, 16, 32):
        lo, hi = (1 / 9) ** (1 / N), 9 ** (1 / N)
        f = filter_value(0.0, 1.0, N, [lo * 0.999, lo * 1.001, hi * 0.999, hi * 1.001])
        assert f[0] > 0.9 > f[1] and f[2] > 0.1 > f[3]
