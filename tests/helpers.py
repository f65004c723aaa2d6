"""Test helpers: layouts of the library's device buffers, built with numpy."""
import numpy as np

TILE = 64


def to_tiled(X: np.ndarray) -> np.ndarray:
    """n x W complex -> tiled [W/64][n][64] complex (interleaved re/im in memory)."""
    n, W = X.shape
    assert W % TILE == 0
    return np.ascontiguousarray(X.reshape(n, W // TILE, TILE).transpose(1, 0, 2))


def from_tiled(Xt: np.ndarray, n: int, W: int) -> np.ndarray:
    return np.ascontiguousarray(Xt.reshape(W // TILE, n, TILE).transpose(1, 0, 2).reshape(n, W))


def header_functions(path: str):
    """Names of the functions declared in a C header (gep_* identifiers followed by '(')."""
    import re
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gep_[a-z0-9_]+)\s*\(", txt)))
