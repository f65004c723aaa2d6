"""KDE contour construction, written out plainly (TEST INFRASTRUCTURE ONLY).

Follows the paper's adaptive contour design (Sec. 4.2: interval sparsity
function G_k(t), recursive splitting at its minimum until each interval
holds at most N_max predicted eigenvalues, merging of intervals with fewer
than N_min, circles with centre (s+e)/2 and radius (1+alpha)(e-s)/2) and its
Alg. "Adaptive Contour Construction via KDE", with these readings of open
points: the initial interval is the target window when given, else
[min - eps, max + eps] with eps = beta (max - min); split candidates are the
midpoints between consecutive distinct predictions inside the interval
(the ends are excluded) that leave at least N_min predictions on each
side when such a midpoint exists; ties go to the lower G, then to the candidate
nearest the centre; an interval whose predictions cannot be split is kept;
a small interval merges with the neighbour holding fewer predictions (the
left one on ties) and the merged interval is split again above N_max;
keep windows are half-open except the last.
"""
from __future__ import annotations

import math


def _members(lam, s, e, last):
    return [x for x in lam if s <= x and (x <= e if last else x < e)]


def _cut(lam, s, e, last, w, nmin):
    inside = _members(lam, s, e, last)
    n = len(inside)
    # candidates: midpoints between consecutive distinct predictions that leave
    # at least nmin predictions on each side (all midpoints if none does)
    cands = [i for i in range(n - 1) if inside[i + 1] > inside[i] and i + 1 >= nmin and n - i - 1 >= nmin]
    if not cands:
        cands = [i for i in range(n - 1) if inside[i + 1] > inside[i]]
    best = None
    for i in cands:
        a, b = inside[i], inside[i + 1]
        t = 0.5 * (a + b)
        g = 0.0
        for x in inside:
            d = (t - x) / (e - s)
            g += math.exp(-w * d * d)
        key = (g, abs(t - 0.5 * (s + e)))
        if best is None or key < best[0]:
            best = (key, t)
    return None if best is None else best[1]


def _split(lam, s, e, last, nmax, w, nmin, out):
    n = len(_members(lam, s, e, last))
    t = _cut(lam, s, e, last, w, nmin) if n > nmax else None
    if t is None:
        out.append((s, e))
        return
    _split(lam, s, t, False, nmax, w, nmin, out)
    _split(lam, t, e, last, nmax, w, nmin, out)


def kde_intervals(lam_hat, nmin=10, nmax=50, w=10.0, beta=0.0, window=None):
    lam = sorted(float(x) for x in lam_hat)
    if window is not None:
        s0, e0 = float(window[0]), float(window[1])
    else:
        if not lam:
            return []
        eps = beta * (lam[-1] - lam[0])
        s0, e0 = lam[0] - eps, lam[-1] + eps
    ivs = []
    _split(lam, s0, e0, True, nmax, w, nmin, ivs)
    ivs.sort()

    def cnt(i):
        return len(_members(lam, ivs[i][0], ivs[i][1], i == len(ivs) - 1))

    for _ in range(4 * len(ivs) + 8):
        if len(ivs) < 2:
            break
        small = [i for i in range(len(ivs)) if cnt(i) < nmin]
        if not small:
            break
        b = small[0]
        nl = cnt(b - 1) if b > 0 else math.inf
        nr = cnt(b + 1) if b + 1 < len(ivs) else math.inf
        a = b - 1 if nl <= nr else b
        last = a + 2 == len(ivs)
        s, e = ivs[a][0], ivs[a + 1][1]
        parts = []
        _split(lam, s, e, last, nmax, w, nmin, parts)
        parts.sort()
        ivs[a:a + 2] = parts
    return ivs


def kde_contours(lam_hat, nmin=10, nmax=50, w=10.0, alpha=0.1, beta=0.0, window=None):
    """[(centre, radius, keep_lo, keep_hi)] for the KDE intervals."""
    return [((s + e) / 2, (1 + alpha) * (e - s) / 2, s, e)
            for s, e in kde_intervals(lam_hat, nmin, nmax, w, beta, window)]
