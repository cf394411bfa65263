"""Pins of the CPU network reference (oracle/mlp.py).

Gradients are pinned to central finite differences; the loss to closed forms
(uniform logits give log C; a confident correct prediction gives ~0); Adam to
its first-step closed form (every coordinate moves by lr sign(g)).
"""
import math

import numpy as np
import pytest

from oracle import mlp

F, H, C = 5, 7, 4


def _params(seed, f=F, h=H, c=C):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.5, mlp.n_params(f, h, c))
    n = mlp.n_params(f, h, c)
    p[n - 2 * f:n - f] = rng.normal(0, 1, f)          # mu
    p[n - f:] = rng.uniform(0.5, 2.0, f)              # sd
    return p


def test_param_layout_roundtrip():
    p = _params(0)
    parts = mlp.unpack(p, F, H, C)
    assert [x.size for x in parts] == mlp.sizes(F, H, C)
    assert np.array_equal(np.concatenate([x.ravel() for x in parts]), p)


def test_uniform_logits_give_log_c():
    p = _params(1)
    n = mlp.n_params(F, H, C)
    # zero the last layer: z = 0 for every row
    o = sum(mlp.sizes(F, H, C)[:4])
    p[o:o + C * H + C] = 0.0
    X = np.random.default_rng(2).normal(size=(9, F))
    y = np.arange(9) % C
    assert mlp.loss(p, X, y, F, H, C) == pytest.approx(math.log(C), rel=1e-12)
    del n


def test_confident_prediction_has_near_zero_loss():
    p = _params(3)
    o = sum(mlp.sizes(F, H, C)[:4])
    p[o:o + C * H] = 0.0
    p[o + C * H:o + C * H + C] = [60.0, 0.0, 0.0, 0.0]   # b3 favours class 0
    X = np.random.default_rng(4).normal(size=(6, F))
    assert mlp.loss(p, X, np.zeros(6, int), F, H, C) < 1e-20
    assert np.all(mlp.predict(p, X, F, H, C) == 0)


def test_gradient_matches_finite_differences():
    p = _params(5)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(11, F))
    y = rng.integers(0, C, 11)
    g = mlp.grad(p, X, y, F, H, C)
    n_train = mlp.n_params(F, H, C) - 2 * F
    eps = 1e-6
    for i in rng.choice(n_train, 60, replace=False):
        q1, q2 = p.copy(), p.copy()
        q1[i] += eps
        q2[i] -= eps
        fd = (mlp.loss(q1, X, y, F, H, C) - mlp.loss(q2, X, y, F, H, C)) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), i
    assert np.all(g[n_train:] == 0)


def test_adam_first_step_moves_by_lr_sign():
    rng = np.random.default_rng(7)
    p = rng.normal(size=30)
    g = rng.normal(size=30)
    p1, m, v = mlp.adam(p, g, np.zeros(30), np.zeros(30), 1, lr=1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step = lr g / (|g| + eps)
    assert np.allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_respects_trainable_prefix():
    p = np.arange(10.0)
    g = np.ones(10)
    p1, _, _ = mlp.adam(p, g, np.zeros(10), np.zeros(10), 1, lr=0.5, n_train=6)
    assert np.all(p1[6:] == p[6:]) and np.all(p1[:6] < p[:6])


# ------------------------------------------------------------ predictor features

def test_features_closed_forms():
    from oracle import features as ft

    k = 8
    # A: one row of equal magnitudes (l2 = 0.5 log2(2k), l1 = log2(2k)); one row with a
    # single nonzero (l2 = l1 = 0 after normalisation by its own power of two)
    A = np.zeros((2, k), complex)
    A[0] = 3.0 * (1 + 1j)
    A[1, 3] = 5.0
    B = np.zeros((k, 1), complex)
    B[:, 0] = 0.75
    f = ft.features(A, B)
    assert f[:3].tolist() == [1.0, 0.0, 3.0]
    l2_eq = 0.5 * math.log2(2 * k * (3.0 / 2.0) ** 2)   # |x| / 2^e = 1.5
    l1_eq = math.log2(2 * k * 1.5)
    l2_one = 0.5 * math.log2((5.0 / 4.0) ** 2)
    assert f[3] == pytest.approx(min(l2_eq, l2_one)) and f[4] == pytest.approx(max(l2_eq, l2_one))
    assert f[7] == pytest.approx(min(l1_eq, math.log2(1.25)))
    # B column: k equal reals (imaginary parts zero) -> l2 = 0.5 log2(k * 1.5^2)
    assert f[11] == pytest.approx(0.5 * math.log2(k * 1.5 ** 2)) and f[14] == 0.0
    zeros = (2 * k - 1) + k          # A row 1: 15 zero reals; B: k zero imaginary parts
    assert f[19] == pytest.approx(zeros / (2.0 * (2 + 1) * k))


def test_features_invariant_under_power_of_two_row_scaling():
    """Scaling rows of op(A) / columns of op(B) by powers of two leaves the features unchanged
    (the exponent rules of Section III-B make the emulation invariant in the same way)."""
    import workloads
    from oracle import features as ft

    A = workloads.complex_matrix(12, 40, 2.0, 81)
    B = workloads.complex_matrix(40, 9, 2.0, 82)
    rng = np.random.default_rng(83)
    As = workloads.skewed(A, row_exp=rng.integers(-30, 30, 12))
    Bs = workloads.skewed(B, col_exp=rng.integers(-30, 30, 9))
    assert np.allclose(ft.features(A, B), ft.features(As, Bs), rtol=0, atol=1e-12)


def test_features_ceil_resolution_and_subnormal_rows():
    """The statistics are the scaling pass's integers: every nonzero magnitude adds at least
    1 to the sums at 2^-20 of the row maximum (here 1 and 2^-40: sigma = 2^40 + 1,
    tau = 2^20 + 1), and a row whose maximum is subnormal is normalised exactly."""
    from oracle import features as ft

    A = np.zeros((2, 1), complex)
    A[0, 0] = complex(1.0, 2.0 ** -40)
    A[1, 0] = complex(3 * 2.0 ** -1074, 2.0 ** -1074)  # max 3 * 2^-1074, e = -1073
    B = np.ones((1, 1), complex)
    f = ft.features(A, B)
    l2 = [0.5 * math.log2(2 ** 40 + 1) - 20, 0.5 * math.log2(1.5 ** 2 + 0.5 ** 2)]
    l1 = [math.log2(2 ** 20 + 1) - 20, math.log2(2.0)]
    assert f[3] == pytest.approx(min(l2), abs=1e-15) and f[4] == pytest.approx(max(l2), abs=1e-15)
    assert f[7] == pytest.approx(min(l1), abs=1e-15) and f[8] == pytest.approx(max(l1), abs=1e-15)
    assert np.isfinite(f).all()
