"""CPU reference of the statistics fed to the moduli-count predictor.

TEST INFRASTRUCTURE ONLY (compared with the library's feature kernels).

The statistics are the integer sums of the fast-mode scaling step (Section
III-B: a row's largest magnitude and a sum of squares) plus the matching sum
of magnitudes, so the library collects them in the pass that computes the
scaling exponents.  A "row" is a row of op(A) or a column of op(B), taken as
its 2k real numbers (real and imaginary parts).  For a nonzero finite row with
largest magnitude M, e = floor(log2 M) and, with F = 20 fraction bits,

    sigma = sum ceil(|x| 2^(F - e))^2,   tau = sum ceil(|x| 2^(F - e)),
    l2 = 0.5 log2 sigma - F,             l1 = log2 tau - F,

integers computed exactly (every nonzero |x| contributes at least 1 to tau),
independent of a power-of-two scaling of the row.  Zero rows and rows holding
inf or NaN are left out of the statistics; zero reals are counted in all rows.

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
F = 20  # fraction bits of the scaling statistics


def _ceil_scaled(row, e):
    """ceil(|x| 2^(F - e)) for the magnitudes of one row, as exact integers: a scaled
    value >= 1 is an exact double (a power-of-two scaling of x below 2^(F + 1)); a
    nonzero value below 1 has ceiling 1, also when the scaling underflows."""
    scaled = np.ldexp(row, F - int(e))
    return np.where(row > 0, np.maximum(np.ceil(scaled), 1.0), 0.0).astype(np.uint64)


def _row_stats(rows):
    """rows: (r, k) complex array -> (l2, l1) over the nonzero finite rows, zero count."""
    rows = np.asarray(rows)
    mags = np.concatenate([np.abs(rows.real), np.abs(rows.imag)], axis=1).astype(np.float64)
    zeros = int(np.count_nonzero(mags == 0))
    l2, l1 = [], []
    for r in range(mags.shape[0]):
        row = mags[r]
        if not np.all(np.isfinite(row)) or not np.any(row > 0):
            continue
        e = math.frexp(float(row.max()))[1] - 1   # floor(log2 max)
        c = _ceil_scaled(row, e)
        sigma = int(np.sum(c * c, dtype=np.uint64))
        tau = int(np.sum(c, dtype=np.uint64))
        l2.append(0.5 * math.log2(sigma) - F)
        l1.append(math.log2(tau) - F)
    return np.array(l2), np.array(l1), zeros


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
