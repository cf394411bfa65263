"""The FP64 residue rule of the product kernel's epilogue, checked on the host.

The epilogue reduces INT32 values x (an accumulator of k <= 2^17 products of
symmetric residues, possibly plus or minus one more residue) with
s = x - p * rint(x * fl(1/p)) in IEEE double precision.  This test evaluates that
rule for every modulus of the largest moduli set on all x in a window around 0,
around every multiple of p / 2 up to the accumulator bound's neighbourhood, and on
random and extreme INT32 values, and compares the result with the exact symmetric
residue (byte-wise for p = 256, where a tie gives +128 for -128, the same byte, and
where INT32 wrap-around is allowed).
"""
import numpy as np
import pytest

from oracle import core

BOUND = (1 << 17) * 127 * 127 + 127  # largest |x| for odd p


def _inputs(p, rng):
    lim = (1 << 31) - 1 if p == 256 else BOUND
    parts = [np.arange(-200000, 200001, dtype=np.int64),
             rng.integers(-lim, lim + 1, 3_000_000, dtype=np.int64),
             np.array([-lim, lim, -lim + 1, lim - 1, -(1 << 31) if p == 256 else -lim], dtype=np.int64)]
    # neighbourhoods of half-integers of x / p far from 0 (where the rounding of x * (1/p) matters)
    m = rng.integers(-(lim // p), lim // p, 20000, dtype=np.int64)
    for d in (-1, 0, 1):
        parts.append(np.clip(m * p + p // 2 + d, -lim, lim))
        parts.append(np.clip(m * p - p // 2 + d, -lim, lim))
    return np.concatenate(parts)


@pytest.mark.parametrize("p", core.constants(24)["p"])
def test_fp64_rule_matches_exact_residue(p):
    rng = np.random.default_rng(p)
    x = _inputs(p, rng)
    xd = x.astype(np.float64)
    q = np.rint(xd * (1.0 / p))  # double product, round half to even
    s = (xd - q * p).astype(np.int64)  # q p and the difference are exact
    r = np.mod(x, p)
    half = (p + 1) // 2
    want = np.where(r >= half, r - p, r)
    if p == 256:
        assert np.array_equal(s & 0xFF, want & 0xFF)
    else:
        assert np.array_equal(s, want)
        assert np.abs(s).max() <= (p - 1) // 2
