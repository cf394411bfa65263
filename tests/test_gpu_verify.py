"""GPU Freivalds check and moduli escalation (through the C-ABI) against the
CPU oracle: outputs bit-exact with the oracle's emulation at the N the
library ends on, verdicts equal to the CPU check's on the same output."""
import numpy as np
import pytest

import workloads
from gpu_helpers import from_device, stored, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import torch

    import paper_2512_08321_amd as ozc

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = ozc.Handle(0)
    yield h
    torch.cuda.synchronize()
    h.close()


@pytest.fixture(scope="module")
def orc():
    from oracle import core

    return core


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nan_a = np.isnan(a.real) | np.isnan(a.imag)
    nan_b = np.isnan(b.real) | np.isnan(b.imag)
    return np.array_equal(nan_a, nan_b) and np.array_equal(a[~nan_a], b[~nan_b])


def _call(h, A, B, C, alpha, beta, N, ta="N", tb="N", mode="fast", fault=0, escalate=True):
    """Returns (output, info, status) of one verified call."""
    import torch

    import paper_2512_08321_amd as ozc

    m, k = A.shape
    n = B.shape[1]
    print(f"verify m,n,k={m},{n},{k} N={N} {mode} {ta}{tb} fault={fault} "
          f"single={A.dtype == np.complex64}", flush=True)
    h.set_config(N, mode, "karatsuba")
    h.set_verify(True, 0.0, escalate)
    h.debug_inject(fault)
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_device(As)
    dB, ldb = to_device(Bs)
    dC, ldc = to_device(np.asfortranarray(C.astype(A.dtype)), m + 3)
    fn = h.zgemm if A.dtype == np.complex128 else h.cgemm
    status = 0
    try:
        fn(ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc)
    except ozc.OzcError as e:
        status = e.status
    finally:
        h.debug_inject(0)
        h.set_verify(False)
    torch.cuda.synchronize()
    return from_device(dC, m, n, ldc), h.last_info(), status


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "C"), ("C", "N")])
def test_clean_call_passes_without_escalation(handle, orc, single, ta, tb):
    from oracle import freivalds as fv

    dt = np.complex64 if single else np.complex128
    N = 8 if single else 14
    A = workloads.complex_matrix(150, 70, 0.5, 61, dtype=dt)
    B = workloads.complex_matrix(70, 90, 0.5, 62, dtype=dt)
    C = workloads.complex_matrix(150, 90, 0.5, 63, dtype=dt)
    for alpha, beta in [(1.0, 0.0), (0.5 - 2j, 1.5 + 0.25j)]:
        got, info, st = _call(handle, A, B, C, alpha, beta, N, ta, tb)
        ref = orc.emulate(A, B, N, alpha=alpha, beta=beta, C=C, single=single)["out"]
        assert st == 0 and _same(got, ref)
        assert info["verified"] == 1 and info["escalations"] == 0 and info["verify_failed_rows"] == 0
        al = complex(np.complex64(alpha)) if single else alpha
        be = complex(np.complex64(beta)) if single else beta
        ratio, failed = fv.check(A, B, ref, al, be, C, single=single)
        assert failed == 0 and info["verify_ratio"] < 1.0


@pytest.mark.parametrize("single", [False, True])
def test_flipped_residue_rejected_then_escalated(handle, orc, single):
    """A corrupted E' (first attempt only) fails the check; the rerun at N + 2
    reproduces the oracle's N + 2 output bit for bit."""
    from oracle import freivalds as fv

    dt = np.complex64 if single else np.complex128
    N = 6 if single else 12
    A = workloads.complex_matrix(64, 40, 0.5, 71, dtype=dt)
    B = workloads.complex_matrix(40, 48, 0.5, 72, dtype=dt)
    C = workloads.complex_matrix(64, 48, 0.5, 73, dtype=dt)
    alpha, beta = 1.25 + 0.5j, -0.5 + 1j
    al = complex(np.complex64(alpha)) if single else alpha
    be = complex(np.complex64(beta)) if single else beta
    # without escalation: the faulty output is returned and flagged
    got, info, st = _call(handle, A, B, C, alpha, beta, N, fault=1, escalate=False)
    bad = orc.emulate(A, B, N, alpha=alpha, beta=beta, C=C, single=single, fault=1)["out"]
    assert _same(got, bad)
    ratio, failed = fv.check(A, B, bad, al, be, C, single=single)
    assert failed == 1 and ratio[0] > 1.0
    assert st == 7 and info["verify_failed_rows"] == 1 and info["escalations"] == 0
    assert info["verify_ratio"] == pytest.approx(ratio.max(), rel=1e-6)
    # with escalation: one rerun with N + 2 moduli from the saved C_in
    got, info, st = _call(handle, A, B, C, alpha, beta, N, fault=1)
    ref = orc.emulate(A, B, N + 2, alpha=alpha, beta=beta, C=C, single=single)["out"]
    assert st == 0 and info["escalations"] == 1 and info["verify_failed_rows"] == 0
    assert _same(got, ref)


def test_too_few_moduli_escalate_until_accepted(handle, orc):
    """N = 6 for ZGEMM is far too coarse for the FP64 tolerance; the library
    steps N by 2 until the CPU check on the oracle's output also passes."""
    from oracle import freivalds as fv

    A = workloads.complex_matrix(96, 64, 0.5, 81)
    B = workloads.complex_matrix(64, 80, 0.5, 82)
    C = np.zeros((96, 80), np.complex128)
    verdicts = {}
    for N in range(6, 25, 2):
        out = orc.emulate(A, B, N)["out"]
        ratio, failed = fv.check(A, B, out)
        verdicts[N] = (failed, ratio.max())
    expect = next(N for N in range(6, 25, 2) if verdicts[N][0] == 0)
    # the CPU verdicts must not sit at the threshold for the comparison to be meaningful
    assert all(abs(np.log2(max(r, 1e-300))) > 0.5 for _, r in verdicts.values() if r > 0)
    got, info, st = _call(handle, A, B, C, 1.0, 0.0, 6)
    assert st == 0 and info["escalations"] == (expect - 6) // 2
    assert _same(got, orc.emulate(A, B, expect)["out"])


def test_exponent_fault_persists_and_fails(handle):
    """Row 0's scaling pushed 12 bits past the uniqueness bound on every attempt:
    escalation cannot help, the call reports a verification failure."""
    A = workloads.complex_matrix(64, 48, 0.5, 91)
    B = workloads.complex_matrix(48, 32, 0.5, 92)
    C = np.zeros((64, 32), np.complex128)
    got, info, st = _call(handle, A, B, C, 1.0, 0.0, 20, fault=2)
    assert st == 7 and info["escalations"] == 2 and info["verify_failed_rows"] >= 1


def test_verify_is_deterministic_and_off_by_default(handle, orc):
    A = workloads.complex_matrix(33, 65, 1.0, 95)
    B = workloads.complex_matrix(65, 17, 1.0, 96)
    C = np.zeros((33, 17), np.complex128)
    g1, i1, _ = _call(handle, A, B, C, 1.0, 0.0, 14)
    g2, i2, _ = _call(handle, A, B, C, 1.0, 0.0, 14)
    assert _same(g1, g2) and i1["verify_ratio"] == i2["verify_ratio"]
    # a plain call after set_verify(False) reports no verification
    import torch

    handle.set_config(14, "fast", "karatsuba")
    dA, lda = to_device(A)
    dB, ldb = to_device(B)
    dC, ldc = to_device(C)
    handle.zgemm("N", "N", 33, 17, 65, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc)
    torch.cuda.synchronize()
    assert handle.last_info()["verified"] == 0
