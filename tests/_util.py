"""Helpers shared by the tests (layout marshalling only, no arithmetic of the method)."""
import numpy as np


def pack(full: np.ndarray) -> np.ndarray:
    """[M, 2, N, N] full matrices -> packed layout [2, P, M] (upper triangle,
    row-major, trajectory innermost), as the library stores the state."""
    M, _, N, _ = full.shape
    iu = np.triu_indices(N)
    return np.ascontiguousarray(np.transpose(full[:, :, iu[0], iu[1]], (1, 2, 0)))


def unpack(packed: np.ndarray, N: int) -> np.ndarray:
    """Packed [2, P, M] -> full [M, 2, N, N] (conjugates below the diagonal)."""
    _, P, M = packed.shape
    iu = np.triu_indices(N)
    out = np.zeros((M, 2, N, N), dtype=packed.dtype)
    t = np.transpose(packed, (2, 0, 1))
    out[:, :, iu[0], iu[1]] = t
    out[:, :, iu[1], iu[0]] = np.conj(t)
    return out


def unpack_s2(S2: np.ndarray, D: int) -> np.ndarray:
    iu = np.triu_indices(D)
    out = np.zeros(S2.shape[:-1] + (D, D))
    out[..., iu[0], iu[1]] = S2
    out[..., iu[1], iu[0]] = S2
    return out
