"""The residue split's arithmetic, checked on the host.

The split writes the truncated integer a' (signed like its input, |a'| < 2^(32 W - 1))
as the W-word integer u = a' + 2^(32 W - 1), takes x' = sum_j u_j w_j + 128 - (2^(32 W - 1)
mod p) over the bytes u_j of u with w_j = 2^(8 j) mod p (unsigned 4-byte dot products,
the offsets as the accumulator's start), so that x = x' - 128 is congruent to a', and
forms the byte s + 128 of the symmetric residue s of x in FP32 as
x' - p floor(fl(x' fl(1/p) + (0.5 - 128 fl(1/p)))) (one fma inside the floor).

1. That rule is evaluated for every integer with |x| <= 16 * 255 * 255 + 255 (the largest
   byte sum) and every modulus of the largest moduli set: the fma is replayed exactly
   (the product and sum are exact in double, then rounded once to single), and the
   result must be an integer in [0, 255] equal to s + 128 for the exact symmetric
   residue s in [-(p-1)/2, (p-1)/2] (for p = 256: in [-128, 127]).
2. The words come from FP64 steps (a' = trunc(x 2^mu), then q_{i+1} = floor(q_i 2^-32)
   and word_i = q_i - 2^32 q_{i+1} from the bottom, the top word's sign bit flipped);
   they are replayed here in IEEE double for values at the edges of every word count
   and compared with the exact biased integer, and the byte sum is compared with a'
   modulo every p, with the weights and offsets derived from Python integers.
"""
import math

import numpy as np
import pytest

from oracle import core

X_MAX = 16 * 255 * 255 + 255
MODULI = [int(p) for p in core.constants(24)["p"]]


@pytest.mark.parametrize("p", MODULI)
def test_fp32_byte_rule_matches_exact_residue(p):
    x = np.arange(-X_MAX, X_MAX + 1, dtype=np.int64)
    xs = (x + 128).astype(np.float32)
    assert np.array_equal(xs.astype(np.int64), x + 128)  # exact in FP32
    ip = np.float32(1) / np.float32(p)
    rb = np.float32(0.5) - np.float32(128) * ip
    assert float(rb) == 0.5 - 128 * float(ip)  # the offset is exact
    y = np.float32(xs.astype(np.float64) * float(ip) + float(rb))  # fma: one rounding
    q = np.floor(y).astype(np.float64)
    s = xs.astype(np.float64) - q * p  # q p and the difference are exact
    assert np.all(s == np.round(s)) and s.min() >= 0 and s.max() <= 255
    r = np.mod(x, p)
    half = (p + 1) // 2 if p % 2 else p // 2
    want = np.where(r >= half, r - p, r)
    assert np.array_equal(s.astype(np.int64) - 128, want)


def test_fp32_byte_rule_catches_plain_rounding():
    """Rounding half to even instead of the floor rule gives +128 at p = 256 ties,
    which is no byte of [0, 255] once shifted."""
    x = np.array([128, 384, -128], dtype=np.float64)
    q = np.rint(x / 256.0)
    assert (x - 256 * q + 128).max() == 256


def _words_fp64(x, mu, W):
    """The device steps in IEEE double: biased words of trunc(x 2^mu)."""
    q = math.trunc(math.ldexp(x, mu))  # exact integer-valued double, kept as a float
    q = float(q)
    out = []
    for _ in range(W - 1):
        hi = math.floor(q * 2.0 ** -32)
        w = q - hi * 2.0 ** 32  # exact: an integer in [0, 2^32)
        assert 0 <= w < 2 ** 32 and w == int(w)
        out.append(int(w))
        q = float(hi)
    assert -2 ** 31 <= q < 2 ** 31
    out.append((int(q) & 0xFFFFFFFF) ^ 0x80000000)
    return out


def _edge_values(W):
    top = 32 * W - 1  # |a'| < 2^top
    vals = [0.0, -0.0, 1.0, -1.0, 0.75, -0.75, 2.0 ** 31, -2.0 ** 31, 2.0 ** 32 - 1, -(2.0 ** 32 - 1)]
    for e in range(0, top):
        for m in (1.0, 1.0 + 2.0 ** -52, 2.0 - 2.0 ** -52, 1.5):
            v = math.ldexp(m, e)
            if v < 2.0 ** top:
                vals += [v, -v]
    rng = np.random.default_rng(8)
    for _ in range(400):
        v = math.ldexp(float(rng.uniform(1.0, 2.0)), int(rng.integers(0, top)))
        if v < 2.0 ** top:
            vals += [v, -v]
    return vals


@pytest.mark.parametrize("W", [1, 2, 3, 4])
def test_biased_words_and_byte_sums(W):
    weights = {p: [pow(2, 8 * j, p) for j in range(4 * W)] for p in MODULI}
    offset = {p: pow(2, 32 * W - 1, p) for p in MODULI}
    for v in _edge_values(W):
        for mu in (0, 3, -2):
            x = math.ldexp(v, -mu)  # so that x 2^mu = v
            a = math.trunc(math.ldexp(x, mu))
            if abs(a) >= 2 ** (32 * W - 1):
                continue
            words = _words_fp64(x, mu, W)
            u = a + 2 ** (32 * W - 1)
            assert words == [(u >> (32 * i)) & 0xFFFFFFFF for i in range(W)], (v, mu, W)
            by = [(words[j // 4] >> (8 * (j % 4))) & 0xFF for j in range(4 * W)]
            for p in MODULI:
                s = sum(b * w for b, w in zip(by, weights[p])) + 128 - offset[p]
                assert abs(s - 128) <= X_MAX
                assert (s - 128 - a) % p == 0


def test_planted_mistakes_fail():
    """A wrong bias, a signed top word or weights of 2^(11 j) break the congruence."""
    W, p = 2, 251
    a = -123456789
    u = a + 2 ** 63
    by = [(u >> (8 * j)) & 0xFF for j in range(8)]
    good = sum(b * pow(2, 8 * j, p) for j, b in enumerate(by)) - pow(2, 63, p)
    assert (good - a) % p == 0
    no_bias = sum(b * pow(2, 8 * j, p) for j, b in enumerate(by))
    assert (no_bias - a) % p != 0
    wrong_w = sum(b * pow(2, 11 * j, p) for j, b in enumerate(by)) - pow(2, 63, p)
    assert (wrong_w - a) % p != 0
    unbiased = a & (2 ** 64 - 1)
    by2 = [(unbiased >> (8 * j)) & 0xFF for j in range(8)]
    assert (sum(b * pow(2, 8 * j, p) for j, b in enumerate(by2)) - pow(2, 63, p) - a) % p != 0
