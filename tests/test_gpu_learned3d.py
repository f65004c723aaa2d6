"""Learned contours on 3D pencils (27-point trilinear FEM, log-normal
coefficients), through the C ABI.

* the network's input, block averages of the coefficient field on the
  GPU (gep_field_downsample), against numpy;
* the gain of the trained spectral prior over uniform contours at equal
  accuracy: the prior is trained on eigenvalues from this library's own
  solves of 64 random 16^3 fields, and on held-out fields (three at 16^3
  and one at 20^3, a finer grid than any it saw) both strategies must miss
  no eigenpair of a brute-force reference; the uniform circles get their
  per-circle block sizes from the Weyl law over each circle's interval,
  the learned ones from the predicted histogram, with the same rule, so
  what the learned contours gain is the prediction's.
"""
import math
import time

import numpy as np
import pytest

from workloads import pencils

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _block_average(g, side):
    sh = g.shape
    idx = [np.arange(n) * side // n for n in sh]
    out = np.zeros((side,) * len(sh))
    cnt = np.zeros_like(out)
    grids = np.meshgrid(*idx, indexing="ij")
    np.add.at(out, tuple(grids), g)
    np.add.at(cnt, tuple(grids), 1.0)
    return (out / cnt).ravel()


@pytest.mark.parametrize("shape,side", [((17, 17, 17), 8), ((21, 19, 23), 8), ((41, 37), 16), ((9, 9, 9), 9)])
def test_field_downsample_vs_numpy(lib, shape, side):
    import torch
    g = np.random.default_rng(sum(shape)).standard_normal(shape).astype(np.float32)
    gd = torch.from_numpy(g).to("cuda:0")
    out = torch.zeros(side ** len(shape), dtype=torch.float32, device="cuda:0")
    lib.gep_field_downsample(gd, side, out)
    ref = _block_average(g.astype(np.float64), side)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-6


def _instance(m, seed, first, last):
    from paper_2511_01927_amd import learned
    g = pencils.grf((m + 1,) * 3, seed=seed)
    kap = np.exp(g)
    A, B = pencils.q1_3d(m, kap)
    return A, B, g, kap, learned.weyl_window_3d(kap, first, last)


def _reference(A, B, win):
    L = np.linalg.cholesky(B.toarray())
    C = np.linalg.solve(L, np.linalg.solve(L, A.toarray()).T)
    lam = np.linalg.eigvalsh(0.5 * (C + C.T))
    return lam[(lam >= win[0]) & (lam < win[1])]


def test_learned_contours_3d_gain_over_uniform(lib):
    from paper_2511_01927_amd import learned
    first, last, nbins, side = 60, 220, 64, 8
    expected = last - first
    feats, targs, probs = [], [], []
    for s in range(300, 364):
        A, B, g, kap, win = _instance(16, s, first, last)
        probs.append((A, B, learned.uniform_contours(win, 5)))
        feats.append(learned.field_features_3d(g, side))
    res = lib.gep_ci_solve_batch(probs, 32, 4, 48, 1e-8, seed=1, max_refine=1)
    for (A, B, c), r_ in zip(probs, res):
        win = (c[0][2], c[-1][3])
        targs.append(learned.histogram_target(r_["evals"][r_["resid"] <= 1e-8], win, nbins, expected))
    X, T = np.array(feats), np.array(targs)
    prior = learned.SpectralPrior(n_bins=nbins, hidden=256, max_batch=64, seed=11, din=side ** 3)
    hist = prior.train(X, T, epochs=200, batch=16, lr=1e-3)
    assert hist[-1] < 0.5 * hist[0]
    f, M = 2.5, 4
    tot = {k: {"pairs": 0, "s": 0.0, "columns": 0, "missed": 0, "fallbacks": 0} for k in ("learned", "uniform")}
    for m, s in ((16, 900), (16, 901), (16, 902), (20, 903)):
        A, B, g, kap, win = _instance(m, s, first, last)
        ref = _reference(A, B, win)
        h = prior.predict(learned.field_features_3d(g, side)[None, :])[0]
        cont, pred = learned.learned_contours(h, win, expected, nmin=10, nmax=50, w=10.0, alpha=0.1)
        bl = learned.blocks_for(pred, M, factor=f)
        ku = max(1, math.ceil(expected / 40))
        uc = learned.uniform_contours(win, ku)
        pu = np.array([learned.weyl_count_3d(kap, b) - learned.weyl_count_3d(kap, a) for _, _, a, b in uc])
        bu = learned.blocks_for(pu, M, factor=f)
        runs = {}
        for name, c, p, b in (("learned", cont, pred, bl), ("uniform", uc, pu, bu)):
            best = None
            for rep in range(3):
                t0 = time.perf_counter()
                r_, nf = learned.solve_with_fallback(A, B, c, p, 32, M, max(b), 1e-8, seed=3, blocks=b)
                d = time.perf_counter() - t0
                best = d if best is None else min(best, d)
            runs[name] = (r_, nf, best)
        for name, (r_, nf, d) in runs.items():
            good = r_["evals"][r_["resid"] <= 1e-8]
            hit = sum(np.any(np.abs(good - x) <= 1e-10 * abs(x)) for x in ref)
            t = tot[name]
            t["pairs"] += int(hit)
            t["s"] += d
            t["columns"] += int(r_["stats"]["columns"])
            t["missed"] += int(ref.size - hit)
            t["fallbacks"] += nf
    for name, t in tot.items():
        print(f"{name}: {t['pairs']} pairs, {t['pairs'] / t['s']:.1f} eigenpairs/s, {t['columns']} columns, "
              f"{t['missed']} missed, {t['fallbacks']} fallbacks")
    # equal accuracy: neither misses an eigenpair
    assert tot["learned"]["missed"] == 0 and tot["uniform"]["missed"] == 0
    assert tot["learned"]["pairs"] == tot["uniform"]["pairs"]
    # the prediction's gain: fewer shifted-system columns and a higher rate
    assert tot["learned"]["columns"] < tot["uniform"]["columns"]
    assert tot["learned"]["pairs"] / tot["learned"]["s"] >= tot["uniform"]["pairs"] / tot["uniform"]["s"]


def test_batched_fallback_matches_single_pencil_solves(lib):
    """learned.batch_with_fallback (one batched mixed-precision solve, flagged
    contours re-solved per pencil) returns the converged eigenvalues of plain
    FP64 single-pencil solves of the same contours, pencil by pencil."""
    from paper_2511_01927_amd import learned
    from workloads import configs
    insts = [configs.learned_instance(m, s, 60, 140) for m, s in ((12, 950), (14, 951))]
    pens = [lib.Pencil(A, B) for A, B, *_ in insts]
    bp = lib.BatchPencil([(A, B) for A, B, *_ in insts])
    conts, preds, blocks = [], [], []
    for A, B, g, kap, win in insts:
        c = learned.uniform_contours(win, 2)
        p = [learned.weyl_count_3d(kap, b) - learned.weyl_count_3d(kap, a) for _, _, a, b in c]
        conts.append(c)
        preds.append(p)
        blocks.append(learned.blocks_for(p, 4, factor=2.5))
    bmax = max(max(b) for b in blocks)
    got, nflag = learned.batch_with_fallback(bp, pens, conts, preds, 32, 4, bmax, 1e-8, blocks=blocks,
                                             precision="mixed", seed=3)
    for i, pen in enumerate(pens):
        ref = pen.solve(conts[i], 32, 4, bmax, 1e-8, seed=3, precision="fp64")
        a = np.sort(ref["evals"][ref["resid"] <= 1e-8])
        b = np.sort(got[i]["evals"][got[i]["resid"] <= 1e-8])
        assert a.size > 20 and a.size == b.size, (i, a.size, b.size, nflag)
        np.testing.assert_allclose(b, a, rtol=1e-10)
