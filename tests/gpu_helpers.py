"""Helpers shared by the GPU tests: column-major device buffers and oracle mapping."""
from __future__ import annotations

import numpy as np

EXP_ZERO, EXP_NONFINITE = -32768, 32767


def to_device(mat: np.ndarray, ld: int | None = None):
    """Column-major complex numpy matrix -> (torch buffer, ld).  Padding rows hold NaN
    garbage so that a kernel reading outside the logical matrix would show up."""
    import torch

    rows, cols = mat.shape
    ld = max(1, rows) if ld is None else ld
    dt = torch.complex128 if mat.dtype == np.complex128 else torch.complex64
    host = np.full((max(cols, 1), ld), complex(np.nan, np.nan), dtype=mat.dtype)
    host[:cols, :rows] = mat.T
    return torch.from_numpy(host).to("cuda"), ld


def from_device(buf, rows: int, cols: int, ld: int) -> np.ndarray:
    host = buf.cpu().numpy()
    return np.asfortranarray(host[:cols, :rows].T)


def stored(op_mat: np.ndarray, op: str) -> np.ndarray:
    """The matrix to store so that op(stored) == op_mat."""
    if op == "N":
        return op_mat
    if op == "T":
        return np.asfortranarray(op_mat.T)
    return np.asfortranarray(op_mat.conj().T)


def oracle_exp(mu, flags, flag_ok=1, flag_zero=0):
    out = np.array(mu, dtype=np.int64).copy()
    out[flags == flag_zero] = EXP_ZERO
    out[(flags != flag_zero) & (flags != flag_ok)] = EXP_NONFINITE
    return out.astype(np.int16)
