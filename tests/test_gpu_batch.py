"""GPU parity of batched solves of uneven pencils through a packed batch
pencil (gep_pencil_create_batch + gep_ci_solve_pencil_batch): a reduced
instance of the uneven-batch configuration (variable-coefficient Q1 pencils
of different sizes, aspect ratios and window counts), every problem against
its own oracle solve and its Sylvester-inertia count; a repeated solve on
the same pencil (kept workspace) gives the same pairs."""
import numpy as np
import pytest

import oracle
from oracle import inertia
from workloads import configs
from tests.test_gpu_solve import assert_pairs_match, _converged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


@pytest.mark.parametrize("solver", ["band", "cocg"])
def test_uneven_batch_pencil_vs_oracle(lib, solver):
    bt = configs.config_q1_batch(count=4, seed0=4100, nmin=1200, nmax=3500, cmin=20, cmax=70)
    assert len({w.n for w in bt.problems}) == 4
    bp = lib.BatchPencil([(w.A, w.B) for w in bt.problems])
    assert bp.n_problems == 4
    conts = [w.contours for w in bt.problems]
    got = bp.solve(conts, bt.n_nodes, bt.moments, bt.block, bt.tol, seed=bt.seed, solver=solver)
    again = bp.solve(conts, bt.n_nodes, bt.moments, bt.block, bt.tol, seed=bt.seed, solver=solver)
    for p, w in enumerate(bt.problems):
        ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, bt.n_nodes, bt.moments, bt.block, bt.tol,
                                     seed=bt.seed + p)
        assert_pairs_match(got[p], *_converged(ref), w.B)
        lo, hi = w.contours[0][2], w.contours[-1][3]
        assert got[p]["evals"].size == inertia.count_in(w.A, w.B, lo, hi)
        assert np.array_equal(got[p]["evals"], again[p]["evals"])
        assert all(c["problem"] == p for c in got[p]["stats"]["contours"])


def test_batch_pencil_needs_the_batch_entry_point(lib):
    bt = configs.config_q1_batch(count=2, seed0=4200, nmin=1000, nmax=1500, cmin=20, cmax=30)
    bp = lib.BatchPencil([(w.A, w.B) for w in bt.problems])
    with pytest.raises(lib.GepError) as e:
        lib.Pencil.solve(bp, bt.problems[0].contours, 32, 4, 32, 1e-8)
    assert e.value.status == -1


def test_batch_per_contour_blocks(lib):
    """Per-contour block sizes in a batched solve (the problems' entries one
    after another) give each problem the pairs of its own single-pencil solve
    with the same block sizes, and the statistics count the smaller blocks'
    columns."""
    bt = configs.config_q1_batch(count=3, seed0=4200, nmin=1200, nmax=2500, cmin=20, cmax=50)
    bp = lib.BatchPencil([(w.A, w.B) for w in bt.problems])
    conts = [w.contours for w in bt.problems]
    rng = np.random.default_rng(5)
    blocks = [rng.integers(bt.block * 3 // 4, bt.block + 1, size=len(c)) for c in conts]
    got = bp.solve(conts, bt.n_nodes, bt.moments, bt.block, bt.tol, seed=bt.seed, blocks=blocks)
    full = bp.solve(conts, bt.n_nodes, bt.moments, bt.block, bt.tol, seed=bt.seed)
    assert got[0]["stats"]["columns"] < full[0]["stats"]["columns"]
    for p, w in enumerate(bt.problems):
        one = lib.gep_ci_solve(w.A, w.B, w.contours, bt.n_nodes, bt.moments, bt.block, bt.tol,
                               seed=bt.seed + p, blocks=blocks[p])
        assert got[p]["evals"].size == one["evals"].size and np.all(got[p]["converged"])
        np.testing.assert_allclose(got[p]["evals"], one["evals"], rtol=1e-10)
    with pytest.raises(lib.GepError):
        bad = [b.copy() for b in blocks]
        bad[1][0] = bt.block + 1
        bp.solve(conts, bt.n_nodes, bt.moments, bt.block, bt.tol, seed=bt.seed, blocks=bad)
