"""Counter-based Gaussian block V for the CI method (Alg. 1, "draw a random block").

The paper draws a random block V per contour without fixing its law; the
reading used here is real i.i.d. N(0, 1) entries, one block shared by all
contours.  Entry e of the column-major n-by-L block comes from:

* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) evaluated at counter e:
  z = seed + (e + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the published
  finaliser z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
  z *= 0x94D049BB133111EB; z ^= z >> 31.
* a uniform in (0, 1]: u = ((z >> 11) + 1) * 2^-53.
* Box-Muller (1958) on the pair p = e // 2 with u1 = u(2p), u2 = u(2p + 1):
  even e takes sqrt(-2 ln u1) cos(2 pi u2), odd e takes the sine branch.

This is an independent implementation of the same published definition the
GPU library implements; the two share no code.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output at each counter (uint64 array)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1] from the top 53 bits of SplitMix64."""
    z = splitmix64(seed, counters)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def gaussian_block(n: int, L: int, seed: int) -> np.ndarray:
    """Real n-by-L block of N(0, 1) entries, column-major counter order."""
    total = n * L
    e = np.arange(total, dtype=np.uint64)
    p = e // np.uint64(2)
    u1 = uniform01(seed, np.uint64(2) * p)
    u2 = uniform01(seed, np.uint64(2) * p + np.uint64(1))
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    g = np.where((e & np.uint64(1)) == 0, rad * np.cos(ang), rad * np.sin(ang))
    return g.reshape(L, n).T.copy()
