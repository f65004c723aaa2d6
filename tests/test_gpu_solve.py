"""End-to-end parity of gep_ci_solve (HIP path, called through the C ABI)
against the CPU oracle and closed forms.

Bar: same eigenvalue count, eigenvalues within 1e-10 relative, residuals
||Ax - lambda Bx|| / (||A||_inf ||x||) <= 1e-8, eigenvectors equal up to
sign (simple eigenvalues: |x^T B x_ref| >= 1 - 1e-8) or, inside clusters
of (near-)equal eigenvalues where several bases are correct, all singular
values of X^T B X_ref >= 1 - 1e-8.
"""
import numpy as np
import pytest

import oracle
from workloads import configs, pencils

pytestmark = pytest.mark.gpu

REL = 1e-10
RES = 1e-8


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _clusters(lam, rel=1e-8):
    groups, cur = [], [0]
    for i in range(1, lam.size):
        if lam[i] - lam[i - 1] <= rel * abs(lam[i]):
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    if lam.size:
        groups.append(cur)
    return groups


def assert_pairs_match(got, lam_ref, X_ref, B):
    lam = got["evals"]
    assert lam.size == lam_ref.size, (lam.size, lam_ref.size)
    if lam.size == 0:
        return
    rel = np.max(np.abs(lam - lam_ref) / np.abs(lam_ref))
    assert rel <= REL, rel
    assert np.max(got["resid"]) <= RES, np.max(got["resid"])
    X = got["evecs"]
    BX = B @ X
    assert np.abs(np.einsum("ij,ij->j", X, BX) - 1.0).max() <= 1e-10
    for g in _clusters(lam_ref):
        s = np.linalg.svd(BX[:, g].T @ X_ref[:, g], compute_uv=False)
        assert s.min() >= 1 - 1e-8, (g, s)


def _converged(ref, tol=RES):
    """The oracle's converged pairs.  It also returns, flagged, Ritz pairs in
    a keep window that still miss tol after refinement (spurious values of
    the filter); those are not eigenpairs and are not compared."""
    ok = ref["resid"] <= tol
    return ref["evals"][ok], ref["evecs"][:, ok]


def _oracle_refs(w, **kw):
    ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol,
                                 seed=w.seed, **kw)
    return _converged(ref)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_small_fem1d_vs_oracle(lib, solver):
    w = configs.config_fem1d(n=400, first=31, last=40, n_nodes=16, moments=4, block=8, seed=7)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, solver=solver)
    lam, X = _oracle_refs(w)
    assert_pairs_match(got, lam, X, w.B)
    assert got["status"] in (0, lib.GEP_WSATURATED)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_fem1d_2000_closed_form(lib, solver):
    """1D linear-FEM pencil, n = 2000, eigenvalues 101..120, 16 nodes, 4 moments, 16 rhs."""
    w = configs.fem1d_2000()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, solver=solver)
    lam_ref = configs.line_eigs(2000)[100:120]
    i = np.arange(1, 2001)
    X_ref = np.stack([np.sin(i * j * np.pi / 2001) for j in range(101, 121)], axis=1)
    X_ref /= np.sqrt(np.einsum("ij,ij->j", X_ref, w.B @ X_ref))[None, :]
    assert_pairs_match(got, lam_ref, X_ref, w.B)
    lam_o, X_o = _oracle_refs(w)
    assert_pairs_match(got, lam_o, X_o, w.B)


def _var2d(nx=40, ny=37, seed=8, first=41, last=100, k=3):
    g = pencils.grf((ny + 1, nx + 1), seed=seed)
    A, B = pencils.q1_2d(nx, ny, np.exp(g))
    lam = np.linalg.eigvalsh(np.linalg.solve(np.linalg.cholesky(B.toarray()),
                                             np.linalg.solve(np.linalg.cholesky(B.toarray()), A.toarray()).T))
    lo, hi = 0.5 * (lam[first - 2] + lam[first - 1]), 0.5 * (lam[last - 1] + lam[last])
    cont = configs.uniform_contours(lo, hi, k, 0.1)
    return configs.Workload("var2d", A, B, cont, 32, 4, 32, seed + 100, window=(lo, hi))


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_variable_coefficient_2d_vs_oracle(lib, solver):
    w = _var2d()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, solver=solver)
    lam, X = _oracle_refs(w)
    assert_pairs_match(got, lam, X, w.B)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_explicit_rhs_and_device_inputs(lib, solver):
    import torch
    from oracle import rng
    w = configs.config_fem1d(n=600, first=41, last=52, n_nodes=16, moments=4, block=8, seed=3)
    V = rng.gaussian_block(w.n, w.block, w.seed)
    a = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed, solver=solver)
    b = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, rhs=V, solver=solver)
    assert np.abs(a["evals"] - b["evals"]).max() <= 1e-12 * np.abs(a["evals"]).max()
    dev = torch.device("cuda:0")
    def d(M):
        return (torch.from_numpy(M.indptr.astype(np.int64)).to(dev),
                torch.from_numpy(M.indices.astype(np.int32)).to(dev),
                torch.from_numpy(M.data.astype(np.float64)).to(dev))
    c = lib.gep_ci_solve(d(w.A), d(w.B), w.contours, w.n_nodes, w.moments, w.block, w.tol,
                         seed=w.seed, solver=solver)
    assert np.array_equal(a["evals"], c["evals"])


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_empty_contour(lib, solver):
    w = configs.config_fem1d(n=300, first=31, last=40, n_nodes=16, moments=2, block=8, seed=3)
    lam = configs.line_eigs(300)
    lo = 0.5 * (lam[30] + lam[31])
    c = np.array([[lo + 1e-3, 1e-3, lo, lo + 2e-3]])     # tiny circle inside a gap
    got = lib.gep_ci_solve(w.A, w.B, c, 16, 2, 8, 1e-8, seed=1, solver=solver)
    assert got["evals"].size == 0


def test_no_convergence_flag(lib):
    w = configs.config_fem1d(n=300, first=31, last=40, n_nodes=16, moments=4, block=8, seed=3)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           max_iter=3, max_refine=0, solver="cocg")
    assert got["status"] == lib.GEP_WNOCONV
    assert not got["converged"].all()


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_saturation_flag(lib, solver):
    w = configs.fem1d_2000()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 16, 1, 4, 1e-8, seed=1, max_refine=0, solver=solver)
    assert got["status"] in (lib.GEP_WSATURATED, lib.GEP_WNOCONV)
    assert any(c["saturated"] for c in got["stats"]["contours"])


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_two_contours_share_cut_without_duplicates(lib, solver):
    w = configs.config_fem1d(n=800, first=61, last=80, n_nodes=16, moments=4, block=16, seed=5)
    lo, hi = w.window
    cont = configs.uniform_contours(lo, hi, 2, 0.2)
    got = lib.gep_ci_solve(w.A, w.B, cont, 16, 4, 16, 1e-8, seed=5, solver=solver)
    ref = oracle.oracle_ci_solve(w.A, w.B, cont, 16, 4, 16, 1e-8, seed=5)
    assert_pairs_match(got, *_converged(ref), w.B)
    assert np.all(np.diff(got["evals"]) > 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_precisions_fem1d_2000(lib, prec):
    """FP32 COCG with FP64 residual replacement meets the same bar as FP64."""
    w = configs.fem1d_2000()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           precision=prec, solver="cocg")
    lam_o, X_o = _oracle_refs(w)
    assert_pairs_match(got, lam_o, X_o, w.B)
    assert got["stats"]["precision"] == prec


def test_mixed_variable_coefficient_2d_vs_oracle(lib):
    w = _var2d(seed=9)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           precision="mixed", solver="cocg")
    lam, X = _oracle_refs(w)
    assert_pairs_match(got, lam, X, w.B)
    assert got["stats"]["replacements"] > 0


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_batch_of_uneven_pencils_vs_oracle(lib, solver):
    """gep_ci_solve_batch: pencils of different sizes share the COCG launches;
    problem p draws V from seed + p and must match its own oracle solve."""
    w1 = configs.config_fem1d(n=400, first=31, last=40, n_nodes=16, moments=4, block=16, seed=11)
    w2 = _var2d(nx=30, ny=27, seed=4, first=21, last=40, k=2)
    w3 = configs.config_fem1d(n=900, first=51, last=62, n_nodes=16, moments=4, block=16, seed=11)
    probs = [(w.A, w.B, w.contours) for w in (w1, w2, w3)]
    got = lib.gep_ci_solve_batch(probs, 16, 4, 16, 1e-8, seed=11, solver=solver)
    for p, w in enumerate((w1, w2, w3)):
        ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 4, 16, 1e-8, seed=11 + p)
        assert_pairs_match(got[p], *_converged(ref), w.B)
        assert all(c["problem"] == p for c in got[p]["stats"]["contours"])


def test_graph_replay_equals_eager(lib):
    """Chunks of COCG iterations replayed from captured HIP graphs give the
    same result as eager launches (same kernels, grids and reductions)."""
    import torch
    w = _var2d(nx=32, ny=30, seed=6, first=31, last=60, k=2)
    s = torch.cuda.Stream()
    eager = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, use_graph=False, stream=s, solver="cocg")
    torch.cuda.synchronize()
    graph = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, use_graph=True, stream=s, solver="cocg")
    torch.cuda.synchronize()
    again = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, use_graph=True, solver="cocg")
    assert graph["stats"]["graph_captures"] > 0
    assert np.array_equal(eager["evals"], graph["evals"])
    assert np.array_equal(eager["resid"], graph["resid"])
    assert np.array_equal(eager["evals"], again["evals"])
    assert eager["stats"]["cocg_iters"] == graph["stats"]["cocg_iters"]


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_per_contour_block_sizes_vs_oracle(lib, solver):
    """opts.blocks: contour k solves with the first blocks[k] columns of V."""
    from oracle import rng
    w = configs.config_fem1d(n=800, first=61, last=80, n_nodes=16, moments=4, block=16, seed=5)
    cont = configs.uniform_contours(*w.window, 2, 0.2)
    blocks = [8, 16]
    got = lib.gep_ci_solve(w.A, w.B, cont, 16, 4, 16, 1e-8, seed=5, blocks=blocks, solver=solver)
    V = rng.gaussian_block(w.n, 16, 5)
    lams, Xs = [], []
    for k in range(2):
        ref = oracle.oracle_ci_solve(w.A, w.B, cont[k:k + 1], 16, 4, blocks[k], 1e-8, V=V[:, :blocks[k]])
        lam_k, X_k = _converged(ref)
        lams.append(lam_k)
        Xs.append(X_k)
    assert_pairs_match(got, np.concatenate(lams), np.concatenate(Xs, axis=1), w.B)


@pytest.mark.parametrize("prec", ["fp64"])
def test_row_groups_match_csr_and_oracle(lib, prec):
    """The COCG kernels walk 4-row groups (union of the rows' columns, zero
    padded coefficients) or plain CSR rows.  Each row's K p' is the same
    either way; the dot products are summed over different row sets per
    wave, so the two solves agree to the parity bar, not bit for bit.  The
    31 x 29 grid has n = 899 rows, so the last group is short."""
    w = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    assert w.n % 4 != 0
    r = {g: lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, precision=prec, row_group=g,
                             rows_per_block=16, solver="cocg")
         for g in (1, 4)}
    assert r[1]["evals"].size > 0
    assert_pairs_match(r[4], r[1]["evals"], r[1]["evecs"], w.B)
    ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5)
    assert_pairs_match(r[4], *_converged(ref), w.B)


def test_row_groups_in_a_batch_of_uneven_pencils(lib):
    """Groups never cross the pencils of a batch (sizes 899, 401, 703), and
    row blocks past a shorter pencil's end stay empty."""
    w1 = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    w2 = configs.config_fem1d(n=401, first=31, last=40, n_nodes=16, moments=4, block=16, seed=11)
    w3 = configs.config_fem1d(n=703, first=51, last=62, n_nodes=16, moments=4, block=16, seed=11)
    probs = [(w.A, w.B, w.contours) for w in (w1, w2, w3)]
    assert all(w.n % 4 for w in (w1, w2, w3))
    a = lib.gep_ci_solve_batch(probs, 16, 4, 16, 1e-8, seed=3, row_group=1, solver="cocg")
    b = lib.gep_ci_solve_batch(probs, 16, 4, 16, 1e-8, seed=3, row_group=4, solver="cocg")
    for p, w in enumerate((w1, w2, w3)):
        assert a[p]["evals"].size > 0
        assert_pairs_match(b[p], a[p]["evals"], a[p]["evecs"], w.B)
        ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 16, 4, 16, 1e-8, seed=3 + p)
        assert_pairs_match(b[p], *_converged(ref), w.B)


def test_row_groups_mixed_precision(lib):
    """FP32 recurrence on the 4-row group kernels vs plain CSR rows."""
    w = _var2d()
    r = {g: lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                             precision="mixed", row_group=g, solver="cocg")
         for g in (1, 4)}
    lam, X = _oracle_refs(w)
    for g in (1, 4):
        assert_pairs_match(r[g], lam, X, w.B)


def test_mixed_fp64_completion_of_stalled_columns(lib):
    """On this 31 x 29 problem the FP32 recurrence stalls on the shifted
    systems nearest the real axis; those columns are finished by the FP64
    recurrence from the folded solution, and every pair meets the bar."""
    w = _var2d(nx=31, ny=29, seed=9, first=31, last=60, k=2)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5, precision="mixed", solver="cocg")
    ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, 32, 4, 16, 1e-8, seed=5)
    assert_pairs_match(got, *_converged(ref), w.B)
    assert got["stats"]["fp64_columns"] > 0
    assert got["stats"]["cocg_iters"] < 2 * 100000
