"""Named synthetic workloads: pencil, target window, contours and solver sizes.

Windows for the constant-coefficient pencils are placed at midpoints of
spectral gaps using the separable closed form of the discrete spectrum (the
1D linear-FEM eigenvalues and, for tensor-product Q1 elements, their sums);
this only chooses inputs and is not part of the solve.  Contours are circles
built from intervals as the paper does (Sec. 4.2: centre at the interval
midpoint, radius (1 + alpha) times the half-width).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import pencils


@dataclass
class Workload:
    name: str
    A: object
    B: object
    contours: np.ndarray          # (K, 4): centre, radius, keep_lo, keep_hi
    n_nodes: int
    moments: int
    block: int
    seed: int
    tol: float = 1e-8
    window: tuple = (0.0, 0.0)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]


def line_eigs(m: int) -> np.ndarray:
    """Discrete spectrum of the 1D linear-FEM pencil on m interior nodes, ascending."""
    h = 1.0 / (m + 1)
    th = np.arange(1, m + 1) * np.pi / (m + 1)
    return 12.0 / h ** 2 * np.sin(th / 2) ** 2 / (2.0 + np.cos(th))


def q1_2d_eigs(nx: int, ny: int) -> np.ndarray:
    """Discrete spectrum of the constant-coefficient Q1 pencil, ascending."""
    return np.sort((line_eigs(nx)[None, :] + line_eigs(ny)[:, None]).ravel())


def gap_window(eigs: np.ndarray, first: int, last: int):
    """Window holding sorted eigenvalues first..last (1-based, inclusive), ends at gap midpoints."""
    for i in (first - 2, last - 1):
        if not eigs[i + 1] - eigs[i] > 1e-9 * abs(eigs[i + 1]):
            raise ValueError(f"no spectral gap after eigenvalue {i + 1}: choose another window end")
    lo = 0.5 * (eigs[first - 2] + eigs[first - 1])
    hi = 0.5 * (eigs[last - 1] + eigs[last])
    return float(lo), float(hi)


def uniform_contours(lo: float, hi: float, k: int, alpha: float) -> np.ndarray:
    """Split [lo, hi) into k equal keep windows, one circle per window."""
    cuts = np.linspace(lo, hi, k + 1)
    out = np.zeros((k, 4))
    for i in range(k):
        s, e = cuts[i], cuts[i + 1]
        out[i] = [(s + e) / 2, (1 + alpha) * (e - s) / 2, s, e]
    return out


def config_fem1d(n: int = 2000, first: int = 101, last: int = 120, n_nodes: int = 16,
                 moments: int = 4, block: int = 16, seed: int = 1001) -> Workload:
    """1D linear-FEM pencil, one circle whose diameter is the gap-to-gap window."""
    A, B = pencils.fem1d(n)
    lo, hi = gap_window(line_eigs(n), first, last)
    cont = uniform_contours(lo, hi, 1, 0.0)
    return Workload(f"fem1d_n{n}", A, B, cont, n_nodes, moments, block, seed, window=(lo, hi),
                    meta={"first": first, "last": last})


def config_q1_2d(nx: int = 300, ny: int = 300, first: int = 1002, last: int = 1200, k: int = 4,
                 alpha: float = 0.1, n_nodes: int = 32, moments: int = 4, block: int = 64,
                 seed: int = 1002) -> Workload:
    """Constant-coefficient Q1 pencil, gap-to-gap window split into k uniform circles."""
    A, B = pencils.q1_2d(nx, ny)
    lo, hi = gap_window(q1_2d_eigs(nx, ny), first, last)
    cont = uniform_contours(lo, hi, k, alpha)
    return Workload(f"q1_2d_{nx}x{ny}", A, B, cont, n_nodes, moments, block, seed, window=(lo, hi),
                    meta={"first": first, "last": last})


# The two headline configurations: a 1D linear-FEM pencil (n = 2000, the
# eigenvalues 101..120, one circle, 16 nodes, 4 moments, 16 right-hand sides)
# and a 300 x 300 Q1 pencil (n = 90000, eigenvalues 1002..1200 split over four
# uniform circles, 32 nodes, 4 moments, 64 right-hand sides).
def fem1d_2000() -> Workload:
    return config_fem1d()


def q1_2d_300() -> Workload:
    return config_q1_2d()


def weyl_index_to_lambda(kappa_nodes: np.ndarray, index: float, dim: int = 3) -> float:
    """Invert Weyl's law for -div(kappa grad u) = lambda u on the unit box.

    N(lambda) ~ c_d lambda^{d/2} * mean(kappa^{-d/2}) with c_3 = 1/(6 pi^2),
    c_2 = 1/(4 pi).  Used only to place target windows on variable-coefficient
    pencils whose spectrum has no closed form.
    """
    if dim == 3:
        c = 1.0 / (6.0 * np.pi ** 2)
    else:
        c = 1.0 / (4.0 * np.pi)
    m = float(np.mean(kappa_nodes ** (-dim / 2.0)))
    return float((index / (c * m)) ** (2.0 / dim))


def config_fd7_3d(m: int = 64, first: int = 2000, last: int = 2500, k: int = 4,
                  alpha: float = 0.1, n_nodes: int = 32, moments: int = 8, block: int = 64,
                  sigma: float = 1.0, field_seed: int = 2003, seed: int = 1003) -> Workload:
    """7-point FD diffusion pencil on m^3 nodes, log-normal kappa, lumped mass B = h^3 I.

    The window covers roughly the eigenvalue indices first..last by Weyl's law
    (the actual count is whatever the pencil has there) and is split into k
    uniform circles.
    """
    g = pencils.grf((m + 2,) * 3, seed=field_seed, sigma=sigma)
    kap = np.exp(g)
    A, B = pencils.fd7_3d(m, kap)
    lo = weyl_index_to_lambda(kap, first)
    hi = weyl_index_to_lambda(kap, last)
    cont = uniform_contours(lo, hi, k, alpha)
    return Workload(f"fd7_3d_{m}", A, B, cont, n_nodes, moments, block, seed, window=(lo, hi),
                    meta={"first": first, "last": last, "sigma": sigma, "field_seed": field_seed})


# 3D configuration: 7-point variable-coefficient diffusion on 64^3 (n = 262144),
# log-normal coefficient (sigma = 1), lumped mass, ~500 interior eigenvalues over
# 4 uniform circles, 32 nodes, 8 moments, 64 right-hand sides (the shifted
# systems are solved by banded factors, whose cost grows with the number of
# circles, so the window is cut into four circles of ~150 eigenvalues each;
# 8 moments give each a 512-dimensional subspace at no extra solve cost).
def fd7_3d_64() -> Workload:
    return config_fd7_3d()


@dataclass
class Batch:
    """A batch of independent pencils, each with its own circles."""
    name: str
    problems: list                # list of Workload
    n_nodes: int
    moments: int
    block: int
    seed: int                     # problem p draws its right-hand sides from seed + p
    tol: float = 1e-8
    meta: dict = field(default_factory=dict)


def config_q1_batch(count: int = 64, seed0: int = 4000, nmin: int = 5000, nmax: int = 200000,
                    cmin: int = 20, cmax: int = 300, per_contour: int = 50, alpha: float = 0.1,
                    sigma: float = 1.0, n_nodes: int = 32, moments: int = 4, block: int = 32,
                    seed: int = 1004) -> Batch:
    """Batch of variable-coefficient 2D Q1 pencils of uneven sizes.

    Instance b (generator seeded with seed0 + b): n log-uniform in
    [nmin, nmax], aspect ratio nx / ny uniform in [0.5, 2], element
    coefficient exp(GRF) with standard deviation sigma (field seed seed0 + b),
    a target count c ~ U{cmin..cmax} of eigenvalues placed by Weyl's law at
    the interior indices [2c, 3c), and ceil(c / per_contour) uniform circles.
    """
    probs = []
    for b in range(count):
        rng = np.random.default_rng(seed0 + b)
        n = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        ar = float(rng.uniform(0.5, 2.0))
        nx = max(8, int(round(np.sqrt(n * ar))))
        ny = max(8, int(round(n / nx)))
        c = int(rng.integers(cmin, cmax + 1))
        g = pencils.grf((ny + 1, nx + 1), seed=seed0 + b, sigma=sigma)
        kap = np.exp(g)
        A, B = pencils.q1_2d(nx, ny, kap)
        lo = weyl_index_to_lambda(kap, 2 * c, dim=2)
        hi = weyl_index_to_lambda(kap, 3 * c, dim=2)
        k = int(np.ceil(c / per_contour))
        cont = uniform_contours(lo, hi, k, alpha)
        probs.append(Workload(f"q1_{nx}x{ny}_b{b}", A, B, cont, n_nodes, moments, block, seed + b,
                              window=(lo, hi), meta={"target_count": c, "nx": nx, "ny": ny}))
    return Batch(f"q1_batch{count}", probs, n_nodes, moments, block, seed,
                 meta={"seed0": seed0, "nmin": nmin, "nmax": nmax})


# Batch configuration: 64 uneven 2D Q1 pencils (n log-uniform in [5k, 200k],
# log-normal coefficients with sigma 1), 20-300 eigenvalues each over
# ceil(count / 50) circles, 32 nodes, 4 moments, 32 right-hand sides.
def q1_batch64() -> Batch:
    return config_q1_batch()



# Learned-contour comparison: 3D 27-point trilinear FEM pencils with
# log-normal coefficients (sigma 1).  The spectral prior trains on 64 random
# 16^3 fields (field seeds 300..363); the comparison runs on held-out fields
# on finer grids (the prior's transfer to grids it never saw).  Every instance
# targets the Weyl-law indices [60, 220) of its own coefficient field.
LEARNED_TRAIN = [(24, s) for s in range(300, 364)]
LEARNED_EVAL = [(32, 900), (32, 901), (36, 902), (36, 903), (40, 904), (40, 905)]
LEARNED_FIRST, LEARNED_LAST = 60, 220


def learned_instance(m: int, seed: int, first: int = LEARNED_FIRST, last: int = LEARNED_LAST):
    """(A, B, log-coefficient field, coefficient field, Weyl window) of one
    3D instance on an m^3 element grid."""
    g = pencils.grf((m + 1,) * 3, seed=seed)
    kap = np.exp(g)
    A, B = pencils.q1_3d(m, kap)
    m_ = float(np.mean(kap ** -1.5))
    lam = lambda k: (6.0 * np.pi ** 2 * k / m_) ** (2.0 / 3.0)
    return A, B, g, kap, (lam(first), lam(last))
