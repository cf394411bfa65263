"""Training data, training and evaluation of the moduli-count predictor.

Instances follow the paper's generator (Section IV-A: entries (u - 0.5)
exp(phi g), u uniform, g standard normal) with uneven shapes, phi up to 8 and
power-of-two skews along k (skews of whole rows or columns do not change the
required N, since the exponent rules of Section III-B absorb them).

Labels are certified: the label of an instance is the smallest N in [6, 24] with

    max_ij (|C_N - C_24|_ij + b_ij) / (|A||B|)_ij <= target,

where C_24 is the 24-moduli result and b_ij bounds its own error against the
exact product: the reconstruction is exact, so C_24 differs from AB only by the
truncation of the scaled inputs (each real part of a 2^mu_i and b 2^nu_j is cut by
less than 1) and the final rounding,

    |C_24 - AB|_ij <= sqrt(2) (2^-mu_i ||b_j||_1 + 2^-nu_j ||a_i||_1) + 2^-53 |C_24|_ij

(complex moduli in the norms).  The left side is therefore an upper bound of the
true error of C_N, and an instance whose bound at 24 moduli already misses the
target gets the extra class.  |A||B| comes from the emulation at 16 moduli on the
moduli of the entries (a product of nonnegative matrices, relative error far below
the margin 2^-30 taken off it).  Everything runs through the C-ABI (statistics,
emulation, exponents, training, prediction); torch only adds and compares.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import Handle, MLP_CLASSES, MLP_FEATURES, MLP_MIN_N

MAX_N = 24


def draw_instance(rng, lo=64, hi=512, klo=64, khi=4096, phi_max=8.0, skew_max=40, square=True,
                  device="cuda"):
    """One instance (A, B) as column-major device tensors (op = N) plus its parameters."""
    import torch

    m = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    n = m if square else int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    k = int(round(math.exp(rng.uniform(math.log(klo), math.log(khi)))))
    phi = float(rng.uniform(0.0, phi_max))
    sigma = int(rng.integers(0, skew_max + 1))
    seed = int(rng.integers(0, 2 ** 62))
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)

    def mat(rows, cols):
        x = torch.rand((2, cols, rows), dtype=torch.float64, device=device, generator=gen) - 0.5
        g = torch.randn((2, cols, rows), dtype=torch.float64, device=device, generator=gen)
        x = x * torch.exp(phi * g)
        return torch.complex(x[0], x[1])  # (cols, rows): column-major rows x cols

    A = mat(m, k)
    B = mat(k, n)
    if sigma > 0:  # power-of-two skew along k (columns of A, rows of B), exact scaling
        ea = torch.from_numpy(rng.integers(0, sigma + 1, k).astype(np.float64)).to(device)
        eb = torch.from_numpy(rng.integers(0, sigma + 1, k).astype(np.float64)).to(device)
        A = A * torch.exp2(-ea)[:, None]
        B = B * torch.exp2(-eb)[None, :]
    return dict(m=m, n=n, k=k, phi=phi, sigma=sigma, A=A.contiguous(), B=B.contiguous())


def _emulate(h, inst, N, C):
    h.set_config(N, "fast", "karatsuba")
    m, n, k = inst["m"], inst["n"], inst["k"]
    h.zgemm("N", "N", m, n, k, 1.0, inst["A"], m, inst["B"], k, 0.0, C, m)


class Reference:
    """The 24-moduli result of an instance with the bound of its own error, and |A||B|."""

    def __init__(self, h, inst):
        import torch

        m, n, k = inst["m"], inst["n"], inst["k"]
        self.inst = inst
        h.set_config(MAX_N, "fast", "karatsuba")
        self.C = torch.empty((n, m), dtype=torch.complex128, device="cuda")
        mu = torch.empty(m, dtype=torch.int16, device="cuda")
        nu = torch.empty(n, dtype=torch.int16, device="cuda")
        h.inspect(False, "N", "N", m, n, k, inst["A"], m, inst["B"], k, mu=mu, nu=nu, C=self.C,
                  ldc=m)
        absA, absB = inst["A"].abs(), inst["B"].abs()   # (k, m) and (n, k) views
        na = absA.sum(dim=0)                             # ||a_i||_1, rows of A
        nb = absB.sum(dim=1)                             # ||b_j||_1, columns of B
        zero = -32768                                    # rows without scaling contribute 0
        sa = torch.where(mu == zero, torch.zeros_like(na),
                         torch.exp2(-mu.to(torch.float64)))
        sb = torch.where(nu == zero, torch.zeros_like(nb),
                         torch.exp2(-nu.to(torch.float64)))
        # C is held as (n, m): entry (i, j) at [j, i]
        self.bound = (math.sqrt(2.0) * (sb[:, None] * na[None, :] + nb[:, None] * sa[None, :])
                      + 2.0 ** -53 * self.C.abs())
        cA = torch.complex(absA, torch.zeros_like(absA))
        cB = torch.complex(absB, torch.zeros_like(absB))
        absAB = torch.empty((n, m), dtype=torch.complex128, device="cuda")
        h.set_config(16, "fast", "karatsuba")
        h.zgemm("N", "N", m, n, k, 1.0, cA, m, cB, k, 0.0, absAB, m)
        self.den = (absAB.real * (1.0 - 2.0 ** -30)).clamp_min(torch.finfo(torch.float64).tiny)

    def error(self, C):
        """Certified bound of max_ij |C - AB|_ij / (|A||B|)_ij."""
        return float((((C - self.C).abs() + self.bound) / self.den).max())


def error_profile(h, inst, Ns, ref=None):
    """Certified relative errors (against |A||B|) of the N-moduli results, N in Ns."""
    import torch

    ref = ref or Reference(h, inst)
    C = torch.empty_like(ref.C)
    out = {}
    for N in Ns:
        _emulate(h, inst, N, C)
        out[N] = ref.error(C)
    return out


def label(h, inst, target):
    """Smallest N in [6, 24] whose certified error meets the target, by bisection
    (the error falls with N); MAX_N + 1 if even the bound at 24 misses it."""
    lo, hi = MLP_MIN_N, MAX_N
    cache = {}
    ref = Reference(h, inst)

    def ok(N):
        if N not in cache:
            cache.update(error_profile(h, inst, [N], ref))
        return cache[N] <= target

    if not ok(hi):
        return MAX_N + 1
    while lo < hi:
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid + 1
    return lo


def features(h, inst):
    import torch

    out = torch.empty(MLP_FEATURES, dtype=torch.float32, device="cuda")
    m, n, k = inst["m"], inst["n"], inst["k"]
    h.features("N", "N", m, n, k, inst["A"], m, inst["B"], k, out)
    return out


def generate(h, count, seed, target=1e-15, log=None, **kw):
    """Features (count x F, float32, device) and labels (count, int32 classes, device)."""
    import torch

    rng = np.random.default_rng(seed)
    X = torch.empty((count, MLP_FEATURES), dtype=torch.float32, device="cuda")
    y = torch.empty(count, dtype=torch.int32, device="cuda")
    meta = []
    t0 = time.perf_counter()
    for i in range(count):
        inst = draw_instance(rng, **kw)
        X[i] = features(h, inst)
        N = label(h, inst, target)
        y[i] = N - MLP_MIN_N
        meta.append((inst["m"], inst["k"], inst["phi"], inst["sigma"], N))
        if log and (i + 1) % max(1, count // 10) == 0:
            log(f"[autoN] {i + 1}/{count} instances labelled ({time.perf_counter() - t0:.1f} s)")
    return X, y, meta


def fixed_rule(labels_N, quantile=0.999):
    """The conservative fixed count: smallest N meeting the target on the given share
    of the training instances (at most 24)."""
    Ns = np.sort(np.asarray(labels_N))
    idx = min(len(Ns) - 1, int(math.ceil(quantile * len(Ns))) - 1)
    return int(min(MAX_N, Ns[idx]))


def evaluate(h, insts, target, margin=0, check=None):
    """Run every instance with the learned N (Freivalds check at the target, escalation
    by 2): returns per instance the predicted N, the N used, the escalations, the
    certified error bound of the result and the call's status.  check(inst, C), when
    given, sees each result (C column-major as an (n, m) tensor) and its return value is
    kept under "check"."""
    import torch

    res = []
    h.set_auto_moduli(fallback=MAX_N, margin=margin)
    for inst in insts:
        m, n, k = inst["m"], inst["n"], inst["k"]
        N_hat = h.predict_moduli("N", "N", m, n, k, inst["A"], m, inst["B"], k)
        C = torch.empty((n, m), dtype=torch.complex128, device="cuda")
        h.set_config(0, "fast", "karatsuba")
        h.set_verify(True, rel=target, escalate=True)
        try:
            h.zgemm("N", "N", m, n, k, 1.0, inst["A"], m, inst["B"], k, 0.0, C, m)
            status = 0
        except Exception as e:  # verification failure at 24 moduli
            status = getattr(e, "status", -1)
        info = h.last_info()
        h.set_verify(False)
        r = dict(N_hat=N_hat, N_used=info["num_moduli"], esc=info["escalations"],
                 err=Reference(h, inst).error(C), status=status)
        if check is not None:
            r["check"] = check(inst, C)
        res.append(r)
    h.set_config(14, "fast", "karatsuba")
    return res
