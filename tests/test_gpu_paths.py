"""GPU parity of the paths the headline runs and of the solve's edge cases,
through the C ABI.

* the COCG direction kernel (the first kernel of every COCG iteration:
  P' = U + beta P, the bilinear P'^T K P') against SciPy, both row walks;
* the FEAST-type refinement pass (8 trapezoid nodes: one pass misses tol)
  against the closed form;
* contours with overlapping keep windows (the merge step) against the
  closed-form 1D and square-grid spectra;
* the sign rule: returned eigenvectors equal the closed-form sines with the
  sign of their first largest-modulus entry;
* a 48 x 48 square grid (exact double eigenvalues, several bases correct);
* the banded solver at the half bandwidths of the 2D headline (301: 384-row
  register panel, blocked sweeps over more than eight 32-row tiles) and 201;
* eigenvalue counts of the variable-coefficient pencil by Sylvester inertia;
* a device-memory cap that splits the contours into waves;
* the precision the statistics report for a mixed request.
"""
import numpy as np
import pytest

import oracle
from oracle import inertia
from workloads import configs, pencils
from tests.helpers import to_tiled, from_tiled
from tests.test_gpu_solve import assert_pairs_match, _converged, _var2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01927_amd import gep_ci
    gep_ci.load()
    return gep_ci


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("name", ["fem1d_2003", "q1_30x37_var", "fd7_9"])
@pytest.mark.parametrize("row_group", [1, 4])
def test_cocg_direction_kernel_vs_scipy(lib, name, row_group):
    g = pencils.grf((38, 31), seed=5)
    A, B = {"fem1d_2003": lambda: pencils.fem1d(2003),
            "q1_30x37_var": lambda: pencils.q1_2d(30, 37, np.exp(g)),
            "fd7_9": lambda: pencils.fd7_3d(9)}[name]()
    n, W = A.shape[0], 192
    rng = np.random.default_rng(n + row_group)
    cx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    U, P = cx(n, W), cx(n, W)
    beta = cx(W)
    z = 1e3 * cx(W)
    pen = lib.Pencil(A, B)
    Pn_d = _t(np.zeros(n * W * 2))
    pq_d = _t(np.zeros(2 * W))
    lib.gep_cocg_direction(pen, _t(z.view(np.float64)), _t(beta.view(np.float64)),
                           _t(to_tiled(U).view(np.float64)), _t(to_tiled(P).view(np.float64)),
                           Pn_d, W, pq_d, row_group=row_group, stream=0)
    Pn = from_tiled(Pn_d.cpu().numpy().view(np.complex128), n, W)
    ref = U + P * beta[None, :]
    scale = np.abs(U) + np.abs(P) * np.abs(beta)[None, :]
    assert np.all(np.abs(Pn - ref) <= 4e-16 * scale)
    KP = (B @ ref) * z[None, :] - A @ ref
    pq_ref = np.sum(ref * KP, axis=0)
    pq = pq_d.cpu().numpy().view(np.complex128)
    mag = np.sum(np.abs(ref) * (np.abs(B) @ np.abs(ref) * np.abs(z)[None, :] + np.abs(A) @ np.abs(ref)), axis=0)
    assert np.all(np.abs(pq - pq_ref) <= 1e-13 * mag)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_refinement_pass_closed_form(lib, solver):
    w = configs.config_fem1d(n=2000, n_nodes=8, moments=4, block=16)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 8, 4, 16, w.tol, seed=w.seed, solver=solver)
    assert got["stats"]["contours"][0]["passes"] == 2
    ref = configs.line_eigs(2000)[100:120]
    i = np.arange(1, 2001)
    X_ref = np.stack([np.sin(i * j * np.pi / 2001) for j in range(101, 121)], axis=1)
    X_ref /= np.sqrt(np.einsum("ij,ij->j", X_ref, w.B @ X_ref))[None, :]
    assert_pairs_match(got, ref, X_ref, w.B)
    assert got["status"] == 0


def _overlap(lo1, hi1, lo2, hi2):
    return np.array([[(lo1 + hi1) / 2, 0.5 * (hi1 - lo1), lo1, hi1],
                     [(lo2 + hi2) / 2, 0.5 * (hi2 - lo2), lo2, hi2]])


def _q1_vectors(nx, ny, B, lam_want):
    """Closed-form Q1 eigenvectors (tensor sines) for the wanted eigenvalues, ascending."""
    ex, ey = configs.line_eigs(nx), configs.line_eigs(ny)
    ix, iy = np.arange(1, nx + 1), np.arange(1, ny + 1)
    vals = (ex[None, :] + ey[:, None]).ravel()
    order = np.argsort(vals, kind="stable")
    sel = [o for o in order if lam_want[0] * (1 - 1e-12) <= vals[o] <= lam_want[-1] * (1 + 1e-12)]
    assert len(sel) == lam_want.size
    cols = []
    for o in sel:
        ky, kx = divmod(int(o), nx)
        v = np.outer(np.sin(iy * (ky + 1) * np.pi / (ny + 1)), np.sin(ix * (kx + 1) * np.pi / (nx + 1))).ravel()
        cols.append(v)
    X = np.stack(cols, axis=1)
    return X / np.sqrt(np.einsum("ij,ij->j", X, B @ X))[None, :]


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_overlapping_windows_merge(lib, solver):
    n = 400
    A, B = pencils.fem1d(n)
    ev = configs.line_eigs(n)
    cont = _overlap(*configs.gap_window(ev, 31, 45), *configs.gap_window(ev, 40, 52))
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 16, 1e-8, seed=3, solver=solver)
    ref = ev[30:52]
    i = np.arange(1, n + 1)
    X_ref = np.stack([np.sin(i * j * np.pi / (n + 1)) for j in range(31, 53)], axis=1)
    X_ref /= np.sqrt(np.einsum("ij,ij->j", X_ref, B @ X_ref))[None, :]
    assert_pairs_match(got, ref, X_ref, B)
    # square grid: exact doubles in the overlap, found by both contours
    m = 14
    A, B = pencils.q1_2d(m, m)
    ev = configs.q1_2d_eigs(m, m)
    cont = _overlap(*configs.gap_window(ev, 21, 39), *configs.gap_window(ev, 31, 50))
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 24, 1e-8, seed=4, solver=solver)
    ref = ev[20:50]
    assert_pairs_match(got, ref, _q1_vectors(m, m, B, ref), B)
    res = oracle.oracle_ci_solve(A, B, cont, 32, 4, 24, 1e-8, seed=4)
    assert_pairs_match(got, *_converged(res), B)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_sign_rule_vs_closed_form(lib, solver):
    n = 400
    w = configs.config_fem1d(n=n, first=31, last=52, n_nodes=16, moments=4, block=24, seed=6)
    got = lib.gep_ci_solve(w.A, w.B, w.contours, 16, 4, 24, 1e-8, seed=6, solver=solver)
    assert got["evals"].size == 22
    i = np.arange(1, n + 1)
    for k, j in enumerate(range(31, 53)):
        v = np.sin(i * j * np.pi / (n + 1))
        v /= np.sqrt(v @ (w.B @ v))
        a = np.abs(v)
        v *= np.sign(v[np.nonzero(a >= (1 - 1e-4) * a.max())[0][0]])
        # a flipped sign would differ by 2 max|v|; the vectors agree to ~1e-7
        assert np.abs(got["evecs"][:, k] - v).max() <= 1e-5 * a.max(), j


def _q1_case(nx, ny, first, last, k, L, N=32, M=4):
    A, B = pencils.q1_2d(nx, ny)
    ev = configs.q1_2d_eigs(nx, ny)
    lo, hi = configs.gap_window(ev, first, last)
    cont = configs.uniform_contours(lo, hi, k, 0.1)
    ref = ev[first - 1:last]
    return A, B, cont, ref


@pytest.mark.parametrize("solver", ["band", "cocg"])
def test_square_grid_48_exact_doubles(lib, solver):
    A, B, cont, ref = _q1_case(48, 48, 61, 121, 2, 32)
    assert np.sum(np.diff(ref) <= 1e-10 * ref[1:]) >= 10
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 32, 1e-8, seed=12, solver=solver)
    assert_pairs_match(got, ref, _q1_vectors(48, 48, B, ref), B)


@pytest.mark.parametrize("nx,first,last", [(300, 41, 100), (200, 41, 90)])
def test_band_headline_half_bandwidths(lib, nx, first, last):
    """Half bandwidth nx + 1: 301 is the 2D headline's (384-row register
    panel, blocked sweeps with more than eight 32-row tiles per step); 201
    takes the 256-row panel."""
    ny = 12
    A, B, cont, ref = _q1_case(nx, ny, first, last, 2, 64)
    got = lib.gep_ci_solve(A, B, cont, 32, 4, 64, 1e-8, seed=13, solver="band")
    st = got["stats"]
    assert st["band_factorisations"] == 2 * 16 and st["band_pivot_flags"] == 0
    assert st["band_unconverged"] == 0 and st["band_relres_max"] <= 1e-9
    assert_pairs_match(got, ref, _q1_vectors(nx, ny, B, ref), B)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_variable_coefficient_counts_by_inertia(lib, solver):
    w = _var2d()
    got = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                           solver=solver)
    lo, hi = w.window
    assert got["evals"].size == inertia.count_in(w.A, w.B, lo, hi)
    for k, (c, r, klo, khi) in enumerate(w.contours):
        mine = (got["evals"] >= klo) & (got["evals"] < khi)
        assert int(mine.sum()) == inertia.count_in(w.A, w.B, klo, khi)


@pytest.mark.parametrize("solver", ["cocg", "band"])
def test_memory_cap_splits_contours_into_waves(lib, solver):
    w = _var2d()
    free = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                            solver=solver)
    capped = lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                              solver=solver, mem_limit_bytes=1.0e8)
    assert free["stats"]["waves"] == 1
    assert capped["stats"]["waves"] == len(w.contours)
    assert_pairs_match(capped, free["evals"], free["evecs"], w.B)
    ref = oracle.oracle_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed)
    assert_pairs_match(capped, *_converged(ref), w.B)


def test_memory_cap_below_one_contour_is_an_error(lib):
    w = _var2d()
    with pytest.raises(lib.GepError) as e:
        lib.gep_ci_solve(w.A, w.B, w.contours, w.n_nodes, w.moments, w.block, w.tol, seed=w.seed,
                         solver="cocg", mem_limit_bytes=1.0e6)
    assert e.value.status == -4


def test_reported_precision_is_what_ran(lib):
    """A mixed request on a narrow-band pencil with the automatic solver
    choice: the statistics name the precision of the solves that ran."""
    w = configs.config_fem1d(n=400, first=31, last=40, n_nodes=16, moments=4, block=8, seed=7)
    cocg = lib.gep_ci_solve(w.A, w.B, w.contours, 16, 4, 8, 1e-8, seed=7, precision="mixed", solver="cocg")
    assert cocg["stats"]["precision"] == "mixed" and cocg["stats"]["fp32_passes"] >= 1
    band = lib.gep_ci_solve(w.A, w.B, w.contours, 16, 4, 8, 1e-8, seed=7, precision="fp64", solver="band")
    assert band["stats"]["precision"] == "fp64" and band["stats"]["solver_run"] == "band"
    assert band["stats"]["precision_requested"] == "fp64"
    auto = lib.gep_ci_solve(w.A, w.B, w.contours, 16, 4, 8, 1e-8, seed=7, precision="mixed")
    st = auto["stats"]
    assert st["precision_requested"] == "mixed"
    assert (st["precision"] == "mixed") == (st["fp32_passes"] > 0)


def test_device_eigenvectors_equal_host_copy(lib):
    """evecs="device" (gep_result_copy_evecs_device) returns, on the GPU, the
    same eigenvectors as the host copy of a second solve with the same seed
    (both sign-normalised), and "none" returns the rest unchanged."""
    import torch
    w = configs.config_fem1d(n=600, first=11, last=30, n_nodes=16, moments=4, block=16, seed=3)
    pen = lib.Pencil(w.A, w.B)
    host = pen.solve(w.contours, 16, 4, 16, 1e-8, seed=3)
    dev = pen.solve(w.contours, 16, 4, 16, 1e-8, seed=3, evecs="device")
    none = pen.solve(w.contours, 16, 4, 16, 1e-8, seed=3, evecs="none")
    assert host["evals"].size == 20 and none["evecs"] is None
    assert isinstance(dev["evecs"], torch.Tensor) and dev["evecs"].is_cuda
    assert tuple(dev["evecs"].shape) == host["evecs"].shape
    torch.cuda.synchronize()
    np.testing.assert_allclose(dev["evals"], host["evals"], rtol=1e-13)
    np.testing.assert_allclose(none["evals"], host["evals"], rtol=1e-13)
    got = dev["evecs"].cpu().numpy()
    assert np.abs(got - host["evecs"]).max() <= 1e-9 * np.abs(host["evecs"]).max()
    empty = pen.solve([[1e9, 1.0, 1e9 - 1.0, 1e9 + 1.0]], 16, 4, 16, 1e-8, seed=3, evecs="device")
    assert empty["evals"].size == 0 and tuple(empty["evecs"].shape) == (w.n, 0)


def test_band_factorisation_graph_replay(lib):
    """use_graph=2 captures the banded factorisation's launches once and
    replays them: a second solve on the same pencil replays the graph, and
    both agree with direct launches (same kernels, same order of arithmetic)."""
    w = _var2d(first=21, last=40, k=2)
    pen = lib.Pencil(w.A, w.B)
    args = (w.contours, w.n_nodes, w.moments, w.block, w.tol)
    ref = pen.solve(*args, seed=w.seed, solver="band")
    g1 = pen.solve(*args, seed=w.seed, solver="band", use_graph=2)
    g2 = pen.solve(*args, seed=w.seed, solver="band", use_graph=2)
    assert g1["stats"]["graph_captures"] >= 1 and g2["stats"]["graph_captures"] == 0
    assert ref["evals"].size == 20
    for r in (g1, g2):
        assert r["evals"].size == ref["evals"].size
        np.testing.assert_allclose(r["evals"], ref["evals"], rtol=1e-12)
        assert np.all(r["resid"] <= w.tol)


@pytest.mark.parametrize("alpha,near", [(0.0, True), (0.25, False)])
def test_boundary_proximity_filter(lib, alpha, near):
    """Per-pair quadrature filter values (gep_result_filter) against the
    oracle's filter at the returned eigenvalues, and the near-boundary count:
    keep windows that reach the circle (alpha 0) put pairs in the filter's
    transition band, a 25% margin keeps them out."""
    from oracle.cirr import filter_value
    n = 800
    A, B = pencils.fem1d(n)
    lam = configs.line_eigs(n)
    lo, hi = configs.gap_window(lam, 21, 36)
    cont = configs.uniform_contours(lo, hi, 1, alpha)
    r = lib.gep_ci_solve(A, B, cont, 32, 4, 16, 1e-8, seed=4)
    assert r["evals"].size == 16 and np.all(r["converged"])
    c, rad = cont[0][0], cont[0][1]
    want = filter_value(c, rad, 32, r["evals"])
    np.testing.assert_allclose(r["filter"], want, rtol=0, atol=1e-12)
    st = r["stats"]
    assert st["near_boundary_pairs"] == int(np.sum(want < 0.9))
    assert (st["near_boundary_pairs"] > 0) == near
    assert abs(st["filter_min"] - want.min()) <= 1e-6
