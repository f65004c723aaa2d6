"""ctypes binding of libgepci.so (the C ABI declared in include/gep_ci.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Host inputs are scipy CSR matrices / numpy arrays; device
inputs and outputs are torch CUDA (HIP) tensors, whose data pointers are
passed through unchanged.  There is no fallback: if the library is missing
or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgepci.so")

GEP_FP64 = 0
GEP_MIXED = 1
GEP_WNOCONV = 1
GEP_WSATURATED = 2


class GepError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gep status {status}: {msg}")
        self.status = status


class gep_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p)]


class gep_contour(C.Structure):
    _fields_ = [("center", C.c_double), ("radius", C.c_double), ("keep_lo", C.c_double),
                ("keep_hi", C.c_double)]


class gep_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("precision", C.c_int), ("max_refine", C.c_int),
                ("solve_tol", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int),
                ("stream", C.c_void_p), ("inputs_on_device", C.c_int), ("rhs", C.c_void_p),
                ("mem_limit_bytes", C.c_double), ("timing", C.c_int), ("rows_per_block", C.c_int),
                ("verbose", C.c_int), ("use_graph", C.c_int), ("blocks", C.c_void_p),
                ("row_group", C.c_int), ("solver", C.c_int), ("band_kernels", C.c_int),
                ("method", C.c_int), ("band_group", C.c_int)]


# every symbol declared in include/gep_ci.h
EXPORTS = [
    "gep_opts_default", "gep_ci_solve", "gep_result_count", "gep_result_copy",
    "gep_result_copy_evecs_device", "gep_result_filter",
    "gep_result_stats", "gep_result_free", "gep_strerror", "gep_last_error",
    "gep_pencil_create", "gep_pencil_free", "gep_pencil_info", "gep_ci_solve_pencil",
    "gep_spmm_shifted", "gep_cocg_direction", "gep_spmm_shifted_f32", "gep_spmm_real", "gep_gram", "gep_gram_noalloc",
    "gep_gemm_tall",
    "gep_sym_eig", "gep_gaussian_block", "gep_ci_solve_batch", "gep_kde_contours",
    "gep_density_create", "gep_density_free", "gep_density_forward", "gep_density_grads",
    "gep_density_adam", "gep_density_param", "gep_gemm_bf16", "gep_pencil_create_batch",
    "gep_pencil_problems", "gep_ci_solve_pencil_batch", "gep_ci_solve_smallest",
    "gep_field_downsample",
]

_lib = None


def load():
    """Load libgepci.so (built by ``paper_2511_01927_amd.build``) and declare signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2511_01927_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i64, i32, dbl = C.c_int64, C.c_int, C.c_double
    sig = {
        "gep_opts_default": (None, [C.POINTER(gep_opts)]),
        "gep_ci_solve": (i32, [C.POINTER(gep_csr), C.POINTER(gep_csr), C.POINTER(gep_contour), i32,
                               i32, i32, i32, dbl, C.POINTER(gep_opts), C.POINTER(P)]),
        "gep_ci_solve_pencil": (i32, [P, C.POINTER(gep_contour), i32, i32, i32, i32, dbl,
                                      C.POINTER(gep_opts), C.POINTER(P)]),
        "gep_result_count": (i32, [P, C.POINTER(i64), C.POINTER(i64)]),
        "gep_result_copy": (i32, [P, P, P, P, P, P]),
        "gep_result_copy_evecs_device": (i32, [P, P, P]),
        "gep_result_filter": (i32, [P, P]),
        "gep_result_stats": (i32, [P, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
        "gep_result_free": (None, [P]),
        "gep_strerror": (C.c_char_p, [i32]),
        "gep_last_error": (C.c_char_p, []),
        "gep_pencil_create": (i32, [C.POINTER(gep_csr), C.POINTER(gep_csr), i32, P, C.POINTER(P)]),
        "gep_pencil_free": (None, [P]),
        "gep_pencil_info": (i32, [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(dbl)]),
        "gep_spmm_shifted": (i32, [P, P, P, P, i64, P, P]),
        "gep_spmm_shifted_f32": (i32, [P, P, P, P, i64, P]),
        "gep_cocg_direction": (i32, [P, P, P, P, P, P, i64, P, i32, P]),
        "gep_spmm_real": (i32, [P, P, i64, i64, P, P, P]),
        "gep_gram": (i32, [P, i64, P, i64, i64, i64, i64, P, P]),
        "gep_gram_noalloc": (i32, [P, i64, P, i64, i64, i64, i64, P, P]),
        "gep_gemm_tall": (i32, [P, i64, P, i64, i64, i64, i64, P, i64, P]),
        "gep_sym_eig": (i32, [P, P, P, i64, i32, P]),
        "gep_gaussian_block": (i32, [C.c_uint64, i64, i64, P, P]),
        "gep_kde_contours": (i32, [P, i64, i32, i32, dbl, dbl, dbl, dbl, dbl, P, i32,
                                   C.POINTER(C.c_int)]),
        "gep_density_create": (i32, [i32, i32, i32, i32, C.c_uint64, C.POINTER(P)]),
        "gep_field_downsample": (i32, [P, i32, i32, i32, i32, P, P]),
        "gep_density_free": (None, [P]),
        "gep_density_forward": (i32, [P, P, i32, P, P]),
        "gep_density_grads": (i32, [P, P, P, i32, C.POINTER(dbl), P]),
        "gep_density_adam": (i32, [P, C.c_float, C.c_float, C.c_float, C.c_float, P]),
        "gep_density_param": (i32, [P, i32, i32, P, i32]),
        "gep_gemm_bf16": (i32, [P, i64, i64, P, i64, i64, P, i64, i32, i32, i32, P]),
        "gep_pencil_create_batch": (i32, [i32, C.POINTER(gep_csr), C.POINTER(gep_csr), i32, P, C.POINTER(P)]),
        "gep_pencil_problems": (i32, [P, C.POINTER(C.c_int)]),
        "gep_ci_solve_smallest": (i32, [P, i64, dbl, i32, i32, i32, i32, dbl, C.POINTER(gep_opts), C.POINTER(P)]),
        "gep_ci_solve_pencil_batch": (i32, [P, C.POINTER(C.POINTER(gep_contour)), C.POINTER(C.c_int), i32, i32,
                                            i32, dbl, C.POINTER(gep_opts), C.POINTER(P)]),
        "gep_ci_solve_batch": (i32, [i32, C.POINTER(gep_csr), C.POINTER(gep_csr),
                                     C.POINTER(C.POINTER(gep_contour)), C.POINTER(C.c_int), i32, i32,
                                     i32, dbl, C.POINTER(gep_opts), C.POINTER(P)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int, allow_warn: bool = False) -> int:
    if st < 0 or (st > 0 and not allow_warn):
        lib = load()
        raise GepError(st, f"{lib.gep_strerror(st).decode()}: {lib.gep_last_error().decode()}")
    return st


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class _HostCSR:
    """Keeps contiguous int64/int32/float64 host copies alive for a gep_csr."""

    def __init__(self, M):
        M = M.tocsr()
        self.rowptr = np.ascontiguousarray(M.indptr, dtype=np.int64)
        self.colind = np.ascontiguousarray(M.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(M.data, dtype=np.float64)
        self.s = gep_csr(M.shape[0], self.val.size, self.rowptr.ctypes.data,
                         self.colind.ctypes.data, self.val.ctypes.data)


class _DevCSR:
    """gep_csr over torch device tensors (rowptr int64, colind int32, val float64)."""

    def __init__(self, rowptr, colind, val):
        self.keep = (rowptr, colind, val)
        self.s = gep_csr(rowptr.numel() - 1, val.numel(), rowptr.data_ptr(), colind.data_ptr(),
                         val.data_ptr())


def _csr_arg(M):
    if isinstance(M, tuple):
        return _DevCSR(*M), 1
    return _HostCSR(M), 0


def _contours(contours):
    arr = np.atleast_2d(np.asarray(contours, dtype=np.float64))
    cs = (gep_contour * arr.shape[0])()
    for k, (c, r, lo, hi) in enumerate(arr):
        cs[k] = gep_contour(c, r, lo, hi)
    return cs, arr.shape[0]


def _opts(seed=1, precision="fp64", max_refine=1, solve_tol=1e-9, max_iter=100000, check_every=16,
          stream=None, on_device=0, rhs=None, mem_limit_bytes=0.0, timing=False, rows_per_block=0, verbose=0, use_graph=True, blocks=None,
          row_group=0, solver="auto", band_kernels=0, band_group=0, method="cirr"):
    lib = load()
    o = gep_opts()
    lib.gep_opts_default(C.byref(o))
    o.seed = seed
    o.precision = GEP_MIXED if precision == "mixed" else GEP_FP64
    o.max_refine = max_refine
    o.solve_tol = solve_tol
    o.max_iter = max_iter
    o.check_every = check_every
    o.stream = _stream_ptr(stream).value
    o.inputs_on_device = on_device
    keep = None
    if rhs is not None:
        if hasattr(rhs, "data_ptr"):
            o.rhs = rhs.data_ptr()
            o.inputs_on_device = 1
            keep = rhs
        else:
            keep = np.asfortranarray(rhs, dtype=np.float64)
            o.rhs = keep.ctypes.data
    o.mem_limit_bytes = mem_limit_bytes
    o.timing = 1 if timing else 0
    o.rows_per_block = rows_per_block
    o.verbose = verbose
    o.use_graph = int(use_graph)   # True = 1; 2 adds the banded factorisation
    o.row_group = row_group
    o.solver = {"auto": 0, "cocg": 1, "band": 2, "multishift": 3}[solver] if isinstance(solver, str) else int(solver)
    o.band_kernels = {"auto": 0, "narrow": 1, "wide": 2}[band_kernels] if isinstance(band_kernels, str) \
        else int(band_kernels)
    o.band_group = band_group
    o.method = {"cirr": 0, "feast": 1}[method] if isinstance(method, str) else int(method)
    if blocks is not None:
        bl = np.ascontiguousarray(blocks, dtype=np.int32)
        o.blocks = bl.ctypes.data
        keep = (keep, bl)
    return o, keep


def _collect(res_ptr, status, evecs="host", stream=None):
    """Result dict of a gep_result (freed here).  evecs: "host" (numpy n x m),
    "device" (torch float64 n x m on the solve's GPU, a column-major view) or
    "none" (not copied)."""
    lib = load()
    m = C.c_int64()
    n = C.c_int64()
    _check(lib.gep_result_count(res_ptr, C.byref(m), C.byref(n)))
    m, n = m.value, n.value
    ev = np.zeros(m)
    rho = np.zeros(m)
    cid = np.zeros(m, dtype=np.int32)
    conv = np.zeros(m, dtype=np.uint8)
    vec = None
    if evecs == "host":
        vec = np.empty((m, n))      # row j = eigenvector j  (column-major n x m)
    elif evecs == "device":
        import torch
        vec = torch.empty((m, n), dtype=torch.float64, device="cuda")
        if m:
            _check(lib.gep_result_copy_evecs_device(res_ptr, vec.data_ptr(), _stream_ptr(stream)))
    elif evecs != "none":
        lib.gep_result_free(res_ptr)
        raise ValueError(f"evecs must be 'host', 'device' or 'none', not {evecs!r}")
    _check(lib.gep_result_copy(res_ptr, ev.ctypes.data, vec.ctypes.data if evecs == "host" else None,
                               rho.ctypes.data, cid.ctypes.data, conv.ctypes.data))
    filt = np.ones(m)
    _check(lib.gep_result_filter(res_ptr, filt.ctypes.data))
    need = C.c_size_t()
    lib.gep_result_stats(res_ptr, None, 0, C.byref(need))
    buf = C.create_string_buffer(need.value)
    lib.gep_result_stats(res_ptr, buf, need.value, None)
    lib.gep_result_free(res_ptr)
    return {"evals": ev, "evecs": vec.T if vec is not None else None, "resid": rho, "contour": cid,
            "converged": conv.astype(bool), "filter": filt, "status": status,
            "stats": json.loads(buf.value.decode())}


def gep_ci_solve(A, B, contours, n_nodes, moments, block, tol, **kw):
    """Solve A x = lambda B x inside the contours' keep windows.

    A, B: scipy sparse matrices (host) or (rowptr, colind, val) torch device
    tensors.  Returns dict(evals, evecs (n x m), resid, contour, converged,
    status, stats).  Warnings (unconverged / saturated) are reported in
    ``status``; errors raise GepError.  ``evecs="device"`` returns the
    eigenvectors as a torch tensor on the GPU (copied on ``stream``),
    ``"none"`` skips them; the default ``"host"`` returns numpy.
    """
    lib = load()
    a, dev_a = _csr_arg(A)
    b, dev_b = _csr_arg(B)
    cs, K = _contours(contours)
    ev_mode = kw.pop("evecs", "host")
    o, keep = _opts(on_device=dev_a, **kw)
    if dev_a != dev_b:
        raise ValueError("A and B must both be host or both be device matrices")
    out = C.c_void_p()
    st = lib.gep_ci_solve(C.byref(a.s), C.byref(b.s), cs, K, n_nodes, moments, block, tol,
                          C.byref(o), C.byref(out))
    _check(st, allow_warn=True)
    return _collect(out, st, ev_mode, kw.get("stream"))


def gep_ci_solve_batch(problems, n_nodes, moments, block, tol, **kw):
    """Solve a batch of independent pencils in one set of launches.

    problems: list of (A, B, contours) with host scipy matrices.  Returns a
    list of result dicts (as gep_ci_solve), problem p using seed + p.
    """
    lib = load()
    P = len(problems)
    hosts = [(_HostCSR(a), _HostCSR(b)) for a, b, _ in problems]
    As = (gep_csr * P)(*[h[0].s for h in hosts])
    Bs = (gep_csr * P)(*[h[1].s for h in hosts])
    conts = [_contours(c) for _, _, c in problems]
    cptr = (C.POINTER(gep_contour) * P)(*[C.cast(c[0], C.POINTER(gep_contour)) for c in conts])
    nks = (C.c_int * P)(*[c[1] for c in conts])
    ev_mode = kw.pop("evecs", "host")
    o, keep = _opts(**kw)
    outs = (C.c_void_p * P)()
    st = lib.gep_ci_solve_batch(P, As, Bs, cptr, nks, n_nodes, moments, block, tol, C.byref(o), outs)
    _check(st, allow_warn=True)
    return [_collect(C.c_void_p(outs[p]), st, ev_mode, kw.get("stream")) for p in range(P)]


class BatchPencil:
    """Several pencils packed once, device-resident (gep_pencil_create_batch)."""

    def __init__(self, pairs, stream=None):
        lib = load()
        hosts = [(_HostCSR(a), _HostCSR(b)) for a, b in pairs]
        P = len(hosts)
        As = (gep_csr * P)(*[h[0].s for h in hosts])
        Bs = (gep_csr * P)(*[h[1].s for h in hosts])
        h = C.c_void_p()
        _check(lib.gep_pencil_create_batch(P, As, Bs, 0, _stream_ptr(stream), C.byref(h)))
        self.h = h
        cnt = C.c_int()
        _check(lib.gep_pencil_problems(h, C.byref(cnt)))
        self.n_problems = cnt.value

    def solve(self, contours_list, n_nodes, moments, block, tol, **kw):
        """contours_list[p]: the circles of problem p; returns a list of result dicts.
        blocks (optional): per problem, its contours' block sizes."""
        lib = load()
        P = self.n_problems
        if len(contours_list) != P:
            raise ValueError(f"{P} problems, {len(contours_list)} contour sets")
        if kw.get("blocks") is not None:
            kw["blocks"] = np.concatenate([np.asarray(b, dtype=np.int32).ravel() for b in kw["blocks"]])
        conts = [_contours(c) for c in contours_list]
        cptr = (C.POINTER(gep_contour) * P)(*[C.cast(c[0], C.POINTER(gep_contour)) for c in conts])
        nks = (C.c_int * P)(*[c[1] for c in conts])
        ev_mode = kw.pop("evecs", "host")
        o, keep = _opts(**kw)
        outs = (C.c_void_p * P)()
        st = lib.gep_ci_solve_pencil_batch(self.h, cptr, nks, n_nodes, moments, block, tol, C.byref(o), outs)
        _check(st, allow_warn=True)
        return [_collect(C.c_void_p(outs[p]), st, ev_mode, kw.get("stream")) for p in range(P)]

    def free(self):
        if getattr(self, "h", None):
            load().gep_pencil_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Pencil:
    """A packed, device-resident pencil (gep_pencil_create)."""

    def __init__(self, A, B, stream=None):
        lib = load()
        a, dev = _csr_arg(A)
        b, _ = _csr_arg(B)
        h = C.c_void_p()
        _check(lib.gep_pencil_create(C.byref(a.s), C.byref(b.s), dev, _stream_ptr(stream), C.byref(h)))
        self.h = h
        n = C.c_int64()
        nnz = C.c_int64()
        ainf = C.c_double()
        lib.gep_pencil_info(h, C.byref(n), C.byref(nnz), C.byref(ainf))
        self.n, self.nnz, self.a_inf = n.value, nnz.value, ainf.value

    def solve(self, contours, n_nodes, moments, block, tol, **kw):
        lib = load()
        cs, K = _contours(contours)
        ev_mode = kw.pop("evecs", "host")
        o, keep = _opts(**kw)
        out = C.c_void_p()
        st = lib.gep_ci_solve_pencil(self.h, cs, K, n_nodes, moments, block, tol, C.byref(o),
                                     C.byref(out))
        _check(st, allow_warn=True)
        return _collect(out, st, ev_mode, kw.get("stream"))

    def solve_smallest(self, m, lower=0.0, per_contour=50, n_nodes=32, moments=4, block=32, tol=1e-8, **kw):
        """The m smallest eigenpairs with eigenvalue >= lower (gep_ci_solve_smallest)."""
        lib = load()
        ev_mode = kw.pop("evecs", "host")
        o, keep = _opts(**kw)
        out = C.c_void_p()
        st = lib.gep_ci_solve_smallest(self.h, m, lower, per_contour, n_nodes, moments, block, tol,
                                       C.byref(o), C.byref(out))
        _check(st, allow_warn=True)
        return _collect(out, st, ev_mode, kw.get("stream"))

    def free(self):
        if getattr(self, "h", None):
            load().gep_pencil_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---- component entry points on torch device tensors --------------------------
def gep_spmm_shifted(pencil: Pencil, shifts, X, Y, W: int, pq=None, stream=None):
    _check(load().gep_spmm_shifted(pencil.h, shifts.data_ptr(), X.data_ptr(), Y.data_ptr(), W,
                                   pq.data_ptr() if pq is not None else None, _stream_ptr(stream)))


def gep_cocg_direction(pencil: Pencil, shifts, beta, U, P, Pn, W: int, pq, row_group=4, stream=None):
    _check(load().gep_cocg_direction(pencil.h, shifts.data_ptr(), beta.data_ptr(), U.data_ptr(),
                                     P.data_ptr(), Pn.data_ptr(), W, pq.data_ptr(), row_group,
                                     _stream_ptr(stream)))


def gep_spmm_shifted_f32(pencil: Pencil, shifts, X, Y, W: int, stream=None):
    _check(load().gep_spmm_shifted_f32(pencil.h, shifts.data_ptr(), X.data_ptr(), Y.data_ptr(), W,
                                       _stream_ptr(stream)))


def gep_spmm_real(pencil: Pencil, X, k: int, ld: int, YA=None, YB=None, stream=None):
    _check(load().gep_spmm_real(pencil.h, X.data_ptr(), k, ld,
                                YA.data_ptr() if YA is not None else None,
                                YB.data_ptr() if YB is not None else None, _stream_ptr(stream)))


def gep_gram(X, ld1, Y, ld2, n, k1, k2, G, stream=None):
    _check(load().gep_gram(X.data_ptr(), ld1, Y.data_ptr(), ld2, n, k1, k2, G.data_ptr(),
                           _stream_ptr(stream)))


def gep_gram_noalloc(X, ld1, Y, ld2, n, k1, k2, G, stream=None):
    _check(load().gep_gram_noalloc(X.data_ptr(), ld1, Y.data_ptr(), ld2, n, k1, k2, G.data_ptr(),
                                   _stream_ptr(stream)))


def gep_gemm_tall(X, ldx, T, ldt, n, k, m, Cm, ldc, stream=None):
    _check(load().gep_gemm_tall(X.data_ptr(), ldx, T.data_ptr(), ldt, n, k, m, Cm.data_ptr(), ldc,
                                _stream_ptr(stream)))


def gep_sym_eig(A, w, V, k, batch=1, stream=None):
    _check(load().gep_sym_eig(A.data_ptr(), w.data_ptr(), V.data_ptr(), k, batch, _stream_ptr(stream)))


def gep_gaussian_block(seed, n, L, V, stream=None):
    _check(load().gep_gaussian_block(seed, n, L, V.data_ptr(), _stream_ptr(stream)))


# ---- learned contours -----------------------------------------------------------
def gep_kde_contours(lam_hat, nmin=10, nmax=50, w=10.0, alpha=0.1, beta=0.0, window=None):
    """KDE contour construction; returns an array (K, 4) of centre, radius, keep_lo, keep_hi."""
    lib = load()
    lam = np.ascontiguousarray(lam_hat, dtype=np.float64)
    lo, hi = (window if window is not None else (float("nan"), float("nan")))
    cnt = C.c_int()
    _check(lib.gep_kde_contours(lam.ctypes.data, lam.size, nmin, nmax, w, alpha, beta, lo, hi, None,
                                0, C.byref(cnt)))
    buf = (gep_contour * max(cnt.value, 1))()
    _check(lib.gep_kde_contours(lam.ctypes.data, lam.size, nmin, nmax, w, alpha, beta, lo, hi, buf,
                                cnt.value, C.byref(cnt)))
    return np.array([[c.center, c.radius, c.keep_lo, c.keep_hi] for c in buf[:cnt.value]]).reshape(-1, 4)


def gep_field_downsample(g, side, out, stream=None):
    """Block averages of a device FP32 field (nz, ny, nx) or (ny, nx) onto side^3 (side^2) cells."""
    shape = tuple(g.shape)
    nz, ny, nx = (1,) + shape if len(shape) == 2 else shape
    _check(load().gep_field_downsample(g.data_ptr(), nz, ny, nx, side, out.data_ptr(), _stream_ptr(stream)))


class DensityNet:
    """Handle on gep_density (device-resident MLP with BF16 matrix-core GEMMs)."""

    def __init__(self, din, dhidden, dout, max_batch, seed=1):
        lib = load()
        h = C.c_void_p()
        _check(lib.gep_density_create(din, dhidden, dout, max_batch, seed, C.byref(h)))
        self.h, self.din, self.dh, self.dout = h, din, dhidden, dout
        self.shapes = [(din, dhidden), (dhidden,), (dhidden, dhidden), (dhidden,), (dhidden, dout), (dout,)]

    def forward(self, X, Y, stream=None):
        _check(load().gep_density_forward(self.h, X.data_ptr(), X.shape[0], Y.data_ptr(), _stream_ptr(stream)))

    def grads(self, X, T, stream=None):
        loss = C.c_double()
        _check(load().gep_density_grads(self.h, X.data_ptr(), T.data_ptr(), X.shape[0], C.byref(loss),
                                        _stream_ptr(stream)))
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(load().gep_density_adam(self.h, lr, beta1, beta2, eps, _stream_ptr(stream)))

    def param(self, which, grad=False):
        a = np.zeros(self.shapes[which], dtype=np.float32)
        _check(load().gep_density_param(self.h, which, 1 if grad else 0, a.ctypes.data, 0))
        return a

    def set_param(self, which, value):
        a = np.ascontiguousarray(value, dtype=np.float32).reshape(self.shapes[which])
        _check(load().gep_density_param(self.h, which, 0, a.ctypes.data, 1))

    def free(self):
        if getattr(self, "h", None):
            load().gep_density_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def gep_gemm_bf16(A, sam, sak, B, sbk, sbn, Cm, ldc, M, N, K, stream=None):
    _check(load().gep_gemm_bf16(A.data_ptr(), sam, sak, B.data_ptr(), sbk, sbn, Cm.data_ptr(), ldc, M, N, K,
                                _stream_ptr(stream)))
