"""Seeded synthetic inputs shaped like the paper's test matrices.

This module holds no arithmetic of the emulation method: it only draws
matrices.  Both the GPU path's tests/benchmarks and the CPU oracle consume
what it produces, so the two sides see identical inputs.

Value distribution (Section IV-A, accuracy experiments): the real and the
imaginary part of every entry are drawn independently as

    (u - 0.5) * exp(phi * g),   u ~ U[0, 1),  g ~ N(0, 1),

where phi controls the dynamic range of the entries.  The paper draws u from
(0, 1]; numpy's generator draws from [0, 1), a difference of measure zero
that does not change the distribution.

Layout: BLAS column-major.  ``complex_matrix(rows, cols, ...)`` returns a
Fortran-ordered numpy array whose leading dimension is ``rows``.
"""
from __future__ import annotations

import numpy as np


def seed_for(config_id: int, rep: int, which: str) -> int:
    """Seed convention: 1000*config + 10*rep + {A:0, B:1, C:2, x:3}."""
    return 1000 * int(config_id) + 10 * int(rep) + {"A": 0, "B": 1, "C": 2, "x": 3}[which]


def complex_matrix(rows: int, cols: int, phi: float, seed: int,
                   dtype=np.complex128) -> np.ndarray:
    """Host matrix (rows x cols, column-major) with Re/Im = (u-0.5)*exp(phi*g)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (2, cols, rows)  # generated row-major over (part, col, row) => column-major matrix
    u = rng.random(shape)
    g = rng.standard_normal(shape)
    x = (u - 0.5) * np.exp(phi * g)
    z = np.empty((cols, rows), dtype=np.complex128)
    z.real = x[0]
    z.imag = x[1]
    out = z.T  # (rows, cols) view, Fortran-ordered
    if dtype == np.complex64:
        out = out.astype(np.complex64, order="F")
    return out


def integer_matrix(rows: int, cols: int, bits: int, seed: int) -> np.ndarray:
    """Complex matrix whose Re/Im parts are random integers with |x| < 2**bits."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lim = 1 << bits
    re = rng.integers(-lim + 1, lim, size=(cols, rows)).astype(np.float64)
    im = rng.integers(-lim + 1, lim, size=(cols, rows)).astype(np.float64)
    z = np.empty((cols, rows), dtype=np.complex128)
    z.real = re
    z.imag = im
    return z.T


def skewed(mat: np.ndarray, row_exp: np.ndarray | None = None,
           col_exp: np.ndarray | None = None) -> np.ndarray:
    """Scale rows/columns by exact powers of two: diag(2^r) * mat * diag(2^c)."""
    out = np.array(mat, order="F", copy=True)
    if row_exp is not None:
        out = np.ldexp(out.real, row_exp[:, None]) + 1j * np.ldexp(out.imag, row_exp[:, None])
    if col_exp is not None:
        out = np.ldexp(out.real, col_exp[None, :]) + 1j * np.ldexp(out.imag, col_exp[None, :])
    return np.asfortranarray(out.astype(mat.dtype))


def complex_matrix_torch(rows: int, cols: int, phi: float, seed: int,
                         dtype=None, device="cuda"):
    """Device matrix with the same distribution, drawn by torch's device generator.

    Used for the large workloads, where drawing on the host would dominate the
    run.  Returns a torch tensor of shape (cols, rows) (row-major), i.e. the
    column-major (rows x cols) matrix.  Rows/columns needed by the CPU oracle
    are copied back from the device.
    """
    import torch

    dtype = dtype or torch.complex128
    real_dtype = torch.float64 if dtype == torch.complex128 else torch.float32
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    x = torch.empty((2, cols, rows), dtype=torch.float64, device=device)
    g = torch.empty((2, cols, rows), dtype=torch.float64, device=device)
    x.uniform_(0.0, 1.0, generator=gen)
    g.normal_(0.0, 1.0, generator=gen)
    x.sub_(0.5).mul_(torch.exp(g.mul_(phi)))
    del g
    out = torch.complex(x[0].to(real_dtype), x[1].to(real_dtype))
    del x
    return out.contiguous()
