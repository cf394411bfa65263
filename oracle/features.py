"""CPU reference of the statistics fed to the moduli-count predictor (FP64).

TEST INFRASTRUCTURE ONLY (compared with the library's feature kernel).

The statistics come from the same per-row quantities the scaling step of the
paper uses (Section III-B: the row maximum and a sum of squares), so they
are cheap to collect next to it.  A "row" is a row of op(A) or a column of
op(B), taken as its 2k real numbers (real and imaginary parts).  For a
nonzero row with largest magnitude M, e = floor(log2 M),
    l2 = 0.5 log2 sum (|x| / 2^e)^2,   l1 = log2 sum |x| / 2^e,
both independent of a power-of-two scaling of the row.  Zero rows are left
out of the statistics (all-zero operand: zeros).

Feature vector (20 entries):
  0 log2 m, 1 log2 n, 2 log2 k,
  3-6   A rows l2: min, max, mean, population std
  7-10  A rows l1: min, max, mean, std
  11-14 B columns l2: min, max, mean, std
  15-18 B columns l1: min, max, mean, std
  19    fraction of zero entries among the 2(m + n)k reals of op(A), op(B)
"""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 20


def _row_stats(rows):
    """rows: (r, k) complex array -> (l2, l1) arrays over the nonzero rows, zero count."""
    re = np.abs(np.asarray(rows).real).astype(np.float64)
    im = np.abs(np.asarray(rows).imag).astype(np.float64)
    mags = np.concatenate([re, im], axis=1)
    zeros = int(np.count_nonzero(mags == 0))
    mx = mags.max(axis=1) if mags.shape[1] else np.zeros(mags.shape[0])
    nz = mx > 0
    e = np.floor(np.log2(mx[nz]))
    # exact power-of-two normalisation
    scaled = mags[nz] * np.ldexp(1.0, -e.astype(int))[:, None]
    l2 = 0.5 * np.log2(np.sum(scaled * scaled, axis=1))
    l1 = np.log2(np.sum(scaled, axis=1))
    return l2, l1, zeros


def _four(v):
    if v.size == 0:
        return [0.0, 0.0, 0.0, 0.0]
    return [float(v.min()), float(v.max()), float(v.mean()), float(v.std())]


def features(A, B):
    """A: (m, k) = op(A), B: (k, n) = op(B) (complex)."""
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    n = B.shape[1]
    l2a, l1a, za = _row_stats(A)
    l2b, l1b, zb = _row_stats(B.T)
    f = [math.log2(m), math.log2(n), math.log2(k)]
    f += _four(l2a) + _four(l1a) + _four(l2b) + _four(l1b)
    f.append((za + zb) / (2.0 * (m + n) * k))
    return np.array(f, dtype=np.float64)
