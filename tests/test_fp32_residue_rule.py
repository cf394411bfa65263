"""The FP32 residue rule of the split kernel, checked exhaustively on the host.

The split computes symmetric residues of integers x with |x| <= 9 * 2047 * 128
(sums of signed 11-bit chunks times symmetric residues of 2^(11 j)) in FP32 as
s = x - p * rint(x * fl(1/p)).  This test evaluates that rule in IEEE single
precision for every such x and every modulus of the largest moduli set, and
compares the result with the exact symmetric residue in [-(p-1)/2, p/2)
(byte-wise for p = 256, where a tie gives +128 for -128, the same byte).
"""
import numpy as np
import pytest

from oracle import core

X_MAX = 9 * 2047 * 128


@pytest.mark.parametrize("p", core.constants(24)["p"])
def test_fp32_rule_matches_exact_residue(p):
    x = np.arange(-X_MAX, X_MAX + 1, dtype=np.int64)
    xf = x.astype(np.float32)
    assert np.array_equal(xf.astype(np.int64), x)  # exact in FP32
    ip = np.float32(1) / np.float32(p)
    q = np.rint(xf * ip)  # float32 product, round half to even
    s = (xf - q * np.float32(p)).astype(np.int64)  # q p and the difference are exact
    r = np.mod(x, p)
    half = (p + 1) // 2
    want = np.where(r >= half, r - p, r)
    if p == 256:
        assert np.array_equal(s & 0xFF, want & 0xFF)
    else:
        assert np.array_equal(s, want)
