"""Learned contours: spectral-density prior + KDE contour construction.

The paper's Deepcontour framework (Alg. "The Deepcontour Framework"):
discretise the coefficient field, predict the spectrum with a trained
network (Sec. 4.1), build contours with KDE (Sec. 4.2, Alg. "Adaptive
Contour Construction via KDE"), then run the CI solver.  Here:

* the network is the library's BF16-matrix-core MLP (``gep_density_*``) that
  maps a block-averaged downsample of log(kappa) (16 x 16 for 2D fields,
  8^3 for 3D ones, the latter by ``gep_field_downsample`` on the GPU) to a
  histogram of the eigenvalues over a target window, in units of the mean
  count per bin;
* labels come from this library's own CI solves (``gep_ci_solve_batch``);
* predicted eigenvalue positions are the histogram's quantile points, fed to
  ``gep_kde_contours``;
* every learned solve is judged by the solver: contours whose subspace is
  saturated, whose pairs miss the residual bar, or that found more than 20%
  fewer eigenvalues than predicted fall back to uniform contours over their
  interval (the scouting-free baseline).

Only marshalling and O(#eigenvalues) bookkeeping run in Python; the solves,
the network and KDE run in the library.
"""
from __future__ import annotations

import math

import numpy as np

from . import gep_ci

FEATURE_SIDE = 16


def field_features(g: np.ndarray, side: int = FEATURE_SIDE) -> np.ndarray:
    """Block-average a 2D log-coefficient field onto a side x side grid (float32)."""
    g = np.asarray(g, dtype=np.float64)
    ny, nx = g.shape
    yi = (np.arange(ny) * side // ny)
    xi = (np.arange(nx) * side // nx)
    out = np.zeros((side, side))
    cnt = np.zeros((side, side))
    np.add.at(out, (yi[:, None], xi[None, :]), g)
    np.add.at(cnt, (yi[:, None], xi[None, :]), 1.0)
    return (out / np.maximum(cnt, 1)).astype(np.float32).ravel()


def field_features_3d(g: np.ndarray, side: int = 8) -> np.ndarray:
    """Block-average a 3D log-coefficient field onto side^3 cells on the GPU
    (gep_field_downsample); returns float32 features ordered [z][y][x]."""
    import torch
    dev = torch.device("cuda:0")
    gd = torch.from_numpy(np.ascontiguousarray(g, dtype=np.float32)).to(dev)
    out = torch.zeros(side ** 3, dtype=torch.float32, device=dev)
    gep_ci.gep_field_downsample(gd, side, out)
    return out.cpu().numpy()


def weyl_count_3d(kappa: np.ndarray, lam) -> np.ndarray:
    """Weyl's law for -div(kappa grad u) = lambda u on the unit cube:
    N(lambda) ~ lambda^(3/2) mean(kappa^(-3/2)) / (6 pi^2)."""
    m = float(np.mean(np.asarray(kappa, dtype=np.float64) ** -1.5))
    return np.asarray(lam, dtype=np.float64) ** 1.5 * m / (6.0 * math.pi ** 2)


def weyl_window_3d(kappa: np.ndarray, first: int, last: int):
    """Window [lambda(first), lambda(last)] by the 3D Weyl law."""
    m = float(np.mean(np.asarray(kappa, dtype=np.float64) ** -1.5))
    lam = lambda k: (6.0 * math.pi ** 2 * k / m) ** (2.0 / 3.0)
    return lam(first), lam(last)


def weyl_window_2d(kappa: np.ndarray, first: int, last: int):
    """Window [lambda(first), lambda(last)] by Weyl's law N(lam) ~ lam mean(1/kappa) / (4 pi)."""
    m = float(np.mean(1.0 / kappa))
    return 4.0 * math.pi * first / m, 4.0 * math.pi * last / m


def histogram_target(evals: np.ndarray, window, n_bins: int, expected: float) -> np.ndarray:
    """Eigenvalue counts per bin of the window, divided by the mean count per bin."""
    h, _ = np.histogram(evals, bins=n_bins, range=window)
    return (h / (expected / n_bins)).astype(np.float32)


def quantile_points(hist: np.ndarray, window, expected: float) -> np.ndarray:
    """Predicted eigenvalue positions: the (j - 1/2)/N quantiles of the histogram density."""
    counts = np.maximum(hist.astype(np.float64), 0.0) * (expected / hist.size)
    total = counts.sum()
    m = int(round(total))
    if m <= 0:
        return np.zeros(0)
    edges = np.linspace(window[0], window[1], hist.size + 1)
    cdf = np.concatenate([[0.0], np.cumsum(counts)])
    targets = (np.arange(m) + 0.5) * total / m
    return np.interp(targets, cdf, edges)


class SpectralPrior:
    """Density network + training loop on the library's kernels."""

    def __init__(self, n_bins=32, hidden=256, max_batch=256, seed=1, device=None, din=None):
        import torch
        self.torch = torch
        self.dev = device or torch.device("cuda:0")
        self.n_bins = n_bins
        self.net = gep_ci.DensityNet(din or FEATURE_SIDE * FEATURE_SIDE, hidden, n_bins, max_batch, seed)
        self.max_batch = max_batch

    def train(self, X: np.ndarray, T: np.ndarray, epochs=200, batch=32, lr=1e-3, seed=0, log=None):
        torch = self.torch
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(self.dev)
        Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(self.dev)
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        hist = []
        for ep in range(epochs):
            perm = rng.permutation(n)
            tot = 0.0
            for b0 in range(0, n, batch):
                idx = torch.from_numpy(perm[b0:b0 + batch]).to(self.dev)
                xb = Xd.index_select(0, idx).contiguous()
                tb = Td.index_select(0, idx).contiguous()
                tot += self.net.grads(xb, tb) * xb.shape[0]
                self.net.adam(lr=lr)
            hist.append(tot / n)
            if log and (ep % 50 == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {hist[-1]:.4f}")
        return hist

    def predict(self, X: np.ndarray) -> np.ndarray:
        torch = self.torch
        out = []
        for b0 in range(0, X.shape[0], self.max_batch):
            xb = np.ascontiguousarray(X[b0:b0 + self.max_batch], dtype=np.float32)
            Xd = torch.from_numpy(xb).to(self.dev)
            Y = torch.zeros((xb.shape[0], self.n_bins), dtype=torch.float32, device=self.dev)
            self.net.forward(Xd, Y)
            out.append(Y.cpu().numpy())
        return np.concatenate(out) if out else np.zeros((0, self.n_bins), dtype=np.float32)

    def loss(self, X, T) -> float:
        P = self.predict(X)
        return float(np.mean((P - T) ** 2))


def learned_contours(hist, window, expected, nmin=10, nmax=50, w=10.0, alpha=0.1):
    """KDE contours over the window from a predicted histogram, with predicted counts."""
    lam_hat = quantile_points(hist, window, expected)
    cont = gep_ci.gep_kde_contours(lam_hat, nmin=nmin, nmax=nmax, w=w, alpha=alpha, window=window)
    counts = np.array([np.sum((lam_hat >= lo) & (lam_hat < hi)) for _, _, lo, hi in cont])
    if len(counts):
        counts[-1] += int(np.sum(lam_hat == window[1]))
    return cont, counts


def uniform_contours(window, k, alpha=0.1):
    lo, hi = window
    cuts = np.linspace(lo, hi, k + 1)
    return np.array([[(a + b) / 2, (1 + alpha) * (b - a) / 2, a, b] for a, b in zip(cuts[:-1], cuts[1:])])


def blocks_for(counts, moments, factor=2.5, step=8, cap=None):
    """Per-contour block sizes: L_k * moments >= factor * count_k, rounded up to `step`."""
    b = [max(step, step * math.ceil(factor * max(int(c), 1) / moments / step)) for c in counts]
    return [min(x, cap) for x in b] if cap else b


def solve_with_fallback(A, B, contours, predicted, n_nodes, moments, block, tol, fallback_k=2,
                        **kw):
    """Solve on the given contours; re-solve flagged contours on uniform sub-contours.

    A contour is flagged when its subspace is saturated, when a kept pair
    misses tol, or when it found fewer eigenvalues than predicted by more than
    20% (and by more than 2): a missed eigenvalue shows as a shortfall, while
    more pairs than predicted in an unsaturated subspace of converged pairs
    means the prediction was low, not that the solve failed.  Returns (result,
    n_fallback).
    """
    res = gep_ci.gep_ci_solve(A, B, contours, n_nodes, moments, block, tol, **kw)
    flagged = []
    for k, c in enumerate(res["stats"]["contours"]):
        mine = res["contour"] == k
        found = int(np.sum(mine))
        bad_pairs = bool(np.any(~res["converged"][mine]))
        miss = predicted is not None and found < predicted[k] - max(2, 0.2 * predicted[k])
        if c["saturated"] or bad_pairs or miss:
            flagged.append(k)
    if not flagged:
        return res, 0
    sub = np.concatenate([uniform_contours((contours[k][2], contours[k][3]), fallback_k) for k in flagged])
    kw2 = dict(kw)
    kw2.pop("blocks", None)
    res2 = gep_ci.gep_ci_solve(A, B, sub, n_nodes, moments, block, tol, **kw2)
    keep = ~np.isin(res["contour"], flagged)
    merged = {
        "evals": np.concatenate([res["evals"][keep], res2["evals"]]),
        "evecs": np.concatenate([res["evecs"][:, keep], res2["evecs"]], axis=1),
        "resid": np.concatenate([res["resid"][keep], res2["resid"]]),
        "contour": np.concatenate([res["contour"][keep], res2["contour"] + len(contours)]),
        "converged": np.concatenate([res["converged"][keep], res2["converged"]]),
        "filter": np.concatenate([res["filter"][keep], res2["filter"]]),
        "status": max(res["status"], res2["status"]),
        "stats": {"first": res["stats"], "fallback": res2["stats"],
                  "cocg_iters": res["stats"]["cocg_iters"] + res2["stats"]["cocg_iters"],
                  "columns": res["stats"]["columns"] + res2["stats"]["columns"]},
    }
    order = np.argsort(merged["evals"], kind="stable")
    for key in ("evals", "resid", "contour", "converged", "filter"):
        merged[key] = merged[key][order]
    merged["evecs"] = merged["evecs"][:, order]
    return merged, len(flagged)


def resolve_flagged(res, pencils_, contours_list, predicted, n_nodes, moments, block, tol, fallback_k=2, **kw):
    """Per problem p, the contours of the first-pass result res[p] that are
    flagged (saturated, a kept pair above tol, or more than 20% and 2 fewer
    eigenvalues than predicted) re-solved on uniform sub-contours on that
    problem's Pencil.  Returns (per-problem dicts with evals, resid, contour,
    converged, stats; number of flagged contours)."""
    out, nflag = [], 0
    for p, r in enumerate(res):
        conts = np.asarray(contours_list[p])
        flagged = []
        cs = r["stats"].get("contours", [])
        for k in range(len(conts)):
            mine = r["contour"] == k
            found = int(np.sum(mine))
            sat = k < len(cs) and bool(cs[k]["saturated"])
            bad = bool(np.any(~r["converged"][mine]))
            miss = predicted is not None and found < predicted[p][k] - max(2, 0.2 * predicted[p][k])
            if sat or bad or miss:
                flagged.append(k)
        nflag += len(flagged)
        keep = ~np.isin(r["contour"], flagged)
        ev, rs, cv, cid = r["evals"][keep], r["resid"][keep], r["converged"][keep], r["contour"][keep]
        if flagged:
            sub = np.concatenate([uniform_contours((conts[k][2], conts[k][3]), fallback_k) for k in flagged])
            kw2 = {key: v for key, v in kw.items() if key != "blocks"}
            r2 = pencils_[p].solve(sub, n_nodes, moments, block, tol, **kw2)
            ev = np.concatenate([ev, r2["evals"]])
            rs = np.concatenate([rs, r2["resid"]])
            cv = np.concatenate([cv, r2["converged"]])
            cid = np.concatenate([cid, r2["contour"] + len(conts)])
        o = np.argsort(ev, kind="stable")
        out.append({"evals": ev[o], "resid": rs[o], "converged": cv[o], "contour": cid[o], "stats": r["stats"]})
    return out, nflag


def batch_with_fallback(bp, pencils_, contours_list, predicted, n_nodes, moments, block, tol, blocks=None,
                        fallback_k=2, **kw):
    """Batched solve of every problem's contours on a BatchPencil, then the
    flagged contours of each problem re-solved on its own Pencil
    (resolve_flagged)."""
    res = bp.solve(contours_list, n_nodes, moments, block, tol, blocks=blocks, **kw)
    return resolve_flagged(res, pencils_, contours_list, predicted, n_nodes, moments, block, tol,
                           fallback_k=fallback_k, **kw)
