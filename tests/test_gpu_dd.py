"""ozc_zgemm_dd (the product as a double-double pair) against the oracle, through the
C-ABI: the high parts equal ozc_zgemm's result and the oracle's RNE(C') scaled, the low
parts the oracle's rounded residual C' - RNE(C') scaled, bit for bit; with 24 moduli the
pair is far more accurate than double precision against the oracle's double-double
product."""
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


def _dd_call(h, A, B, N, mode="fast", algo="karatsuba", ta="N", tb="N"):
    import torch

    m, k = A.shape
    n = B.shape[1]
    h.set_config(N, mode, algo)
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_device(As, As.shape[0] + 1)
    dB, ldb = to_device(Bs)
    hi, ldc = to_device(np.zeros((m, n), complex), m + 3)
    lo, _ = to_device(np.zeros((m, n), complex), m + 3)
    h.zgemm_dd(ta, tb, m, n, k, dA, lda, dB, ldb, hi, lo, ldc)
    torch.cuda.synchronize()
    return from_device(hi, m, n, ldc), from_device(lo, m, n, ldc)


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint64)


@pytest.mark.parametrize("N,mode,algo", [(8, "fast", "karatsuba"), (16, "accurate", "4m"),
                                         (24, "fast", "karatsuba")])
def test_dd_parts_bit_exact(handle, N, mode, algo):
    from oracle import core

    A = workloads.complex_matrix(300, 150, 2.0, 1201)
    B = workloads.complex_matrix(150, 200, 2.0, 1202)
    print(f"zgemm_dd 300x200x150 N={N} {mode} {algo}", flush=True)
    hi, lo = _dd_call(handle, A, B, N, mode, algo, ta="C", tb="T")
    ref = core.emulate(A, B, N, mode, algo, want_lo=True)
    assert np.array_equal(_bits(hi), _bits(ref["out"]))
    assert np.array_equal(_bits(lo), _bits(ref["lo"]))
    # the high parts are ozc_zgemm's result
    import torch

    m, n, k = 300, 200, 150
    dA, lda = to_device(stored(A, "C"))
    dB, ldb = to_device(stored(B, "T"))
    dC, ldc = to_device(np.zeros((m, n), complex))
    handle.zgemm("C", "T", m, n, k, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(from_device(dC, m, n, ldc)), _bits(hi))


def test_dd_large_tiles_and_accuracy(handle):
    """256-tiles (m, n >= 1024), 24 moduli: bit-exact with the oracle on sampled rows, and
    the pair's error against the double-double product far below double precision."""
    from oracle import core

    m, n, k = 1100, 1030, 256
    A = workloads.complex_matrix(m, k, 0.5, 1211)
    B = workloads.complex_matrix(k, n, 0.5, 1212)
    hi, lo = _dd_call(handle, A, B, 24)
    rows = np.array([0, 1, 255, 256, 700, m - 1])
    cols = np.array([0, 3, 255, 256, 999, n - 1])
    ref = core.emulate(A[rows], B[:, cols], 24, want_lo=True)
    assert np.array_equal(_bits(hi[np.ix_(rows, cols)]), _bits(ref["out"]))
    assert np.array_equal(_bits(lo[np.ix_(rows, cols)]), _bits(ref["lo"]))
    dh, dl = core.dd_gemm(A[rows], B[:, cols])
    ab = core.abs_product(A[rows], B[:, cols])
    d = ((hi[np.ix_(rows, cols)] - dh) + (lo[np.ix_(rows, cols)] - dl))
    err_dd = float(np.max(np.abs(d) / ab))
    err_hi = core.err_nc(hi[np.ix_(rows, cols)], dh, dl, ab)
    print(f"N = 24: error of hi + lo {err_dd:.2e}, of hi alone {err_hi:.2e}", flush=True)
    assert err_dd < 1e-24 < err_hi


def test_dd_edge_cases(handle):
    import torch

    import paper_2512_08321_amd as ozc
    from oracle import core

    # integer inputs: the product is exact, the low parts zero
    A = workloads.integer_matrix(20, 30, 12, 1221)
    B = workloads.integer_matrix(30, 10, 12, 1222)
    hi, lo = _dd_call(handle, A, B, 12)
    assert np.array_equal(hi, A @ B) and not lo.any()
    # non-finite input: NaN rows and columns in both parts, as the oracle's
    A = workloads.complex_matrix(17, 9, 1.0, 1223)
    B = workloads.complex_matrix(9, 11, 1.0, 1224)
    A[4, 2] = np.inf
    hi, lo = _dd_call(handle, A, B, 12)
    ref = core.emulate(A, B, 12, want_lo=True)
    assert np.isnan(hi[4]).all() and np.isnan(lo[4]).all()
    ok = ~np.isnan(ref["out"])
    assert np.array_equal(hi[ok], ref["out"][ok]) and np.array_equal(lo[ok], ref["lo"][ok])
    # k == 0: zeros in both parts; k above the INT32 limit: refused before any work
    hi, lo = _dd_call(handle, A[:, :0], B[:0], 12)
    assert not hi.any() and not lo.any()
    kbig = ozc.MAX_K + 1
    dA = torch.zeros(4 * kbig, dtype=torch.complex128, device="cuda")
    dB = torch.zeros(kbig * 4, dtype=torch.complex128, device="cuda")
    dC = torch.full((16,), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    dL = torch.full((16,), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    with pytest.raises(ozc.OzcError) as e:
        handle.zgemm_dd("N", "N", 4, 4, kbig, dA, 4, dB, kbig, dC, dL, 4)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert bool(torch.all(dC == 7.0)) and bool(torch.all(dL == 7.0))
