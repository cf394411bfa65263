"""GPU parity at the sizes of the benchmark configurations, through the C-ABI.

Fast-mode exponents depend on one row of op(A) (column of op(B)) only, so the
oracle's result on sampled rows and columns is the exact result at those
entries.  Accurate-mode exponents depend on the whole bound product
(Section III-B), so the oracle computes them on the full matrices and is
handed them for the sampled entries.  The bar is bit-exact (both sides
reconstruct exactly and round once).
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import EXP_NONFINITE, EXP_ZERO, oracle_exp

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


def _dev(mat):
    """Column-major numpy matrix -> contiguous torch buffer (cols, rows)."""
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.asarray(mat).T)).cuda()


def _sample(n, count, seed, tile=256):
    """Sorted distinct indices: random ones plus both ends and tile edges."""
    rng = np.random.default_rng(seed)
    fixed = {0, n - 1, min(tile - 1, n - 1), min(tile, n - 1), n // 2}
    pick = set(rng.choice(n, size=min(count, n), replace=False).tolist()) | fixed
    return np.array(sorted(pick), dtype=np.int64)


def _gather(dC, rows, cols):
    """Entries (rows x cols) of the column-major result held as a (n, m) buffer."""
    import torch

    r = torch.from_numpy(rows).cuda()
    c = torch.from_numpy(cols).cuda()
    return dC.index_select(0, c).index_select(1, r).cpu().numpy().T


def _bits_equal(a, b):
    """Same dtype and bit-identical entries."""
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))


@pytest.fixture(scope="module")
def cgemm4096():
    m = n = k = 4096
    A = workloads.complex_matrix(m, k, 0.5, workloads.seed_for(2, 0, "A"), np.complex64)
    B = workloads.complex_matrix(k, n, 0.5, workloads.seed_for(2, 0, "B"), np.complex64)
    return A, B


@pytest.mark.parametrize("N", [6, 12])
@pytest.mark.parametrize("algo", ["karatsuba", "4m"])
def test_cgemm_4096(handle, cgemm4096, N, algo):
    """CGEMM 4096^3 (complex64 in and out), phi = 0.5: sampled entries bit-exact."""
    import torch

    from oracle import core

    A, B = cgemm4096
    m, k = A.shape
    n = B.shape[1]
    print(f"CGEMM {m}x{n}x{k} N={N} {algo}", flush=True)
    handle.set_config(N, "fast", algo)
    dA, dB = _dev(A), _dev(B)
    dC = torch.zeros((n, m), dtype=torch.complex64, device="cuda")
    handle.cgemm("N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m)
    torch.cuda.synchronize()
    rows, cols = _sample(m, 40, 1 + N), _sample(n, 40, 2 + N)
    got = _gather(dC, rows, cols)
    ref = core.emulate(A[rows, :], B[:, cols], N, algo=algo, single=True)["out"]
    assert got.dtype == np.complex64 and ref.dtype == np.complex64
    assert _bits_equal(got, ref)


def test_cgemm_4096_wide_range(handle):
    """CGEMM 4096^3 at phi = 4 (entries spread over e^+-16), 9 moduli: sampled entries."""
    import torch

    from oracle import core

    m = n = k = 4096
    A = workloads.complex_matrix(m, k, 4.0, workloads.seed_for(2, 1, "A"), np.complex64)
    B = workloads.complex_matrix(k, n, 4.0, workloads.seed_for(2, 1, "B"), np.complex64)
    print("CGEMM 4096^3 phi=4 N=9", flush=True)
    handle.set_config(9, "fast", "karatsuba")
    dC = torch.zeros((n, m), dtype=torch.complex64, device="cuda")
    handle.cgemm("N", "N", m, n, k, 1.0, _dev(A), m, _dev(B), k, 0.0, dC, m)
    torch.cuda.synchronize()
    rows, cols = _sample(m, 32, 5), _sample(n, 32, 6)
    ref = core.emulate(A[rows, :], B[:, cols], 9, single=True)["out"]
    assert _bits_equal(_gather(dC, rows, cols), ref)


def _accurate_case(handle, m, n, k, N, algo, phi, seed, ta="N", tb="N"):
    """Accurate mode: full exponents against the oracle's (all m + n of them), then
    sampled outputs computed by the oracle with those exponents."""
    import torch

    from oracle import core

    print(f"accurate ZGEMM {m}x{n}x{k} N={N} {algo} {ta}{tb}", flush=True)
    A = workloads.complex_matrix(m, k, phi, seed)
    B = workloads.complex_matrix(k, n, phi, seed + 1)
    As = A if ta == "N" else np.asfortranarray(A.T)
    Bs = B if tb == "N" else np.asfortranarray(B.T)
    handle.set_config(N, "accurate", algo)
    dC = torch.zeros((n, m), dtype=torch.complex128, device="cuda")
    mu = torch.zeros(m, dtype=torch.int16, device="cuda")
    nu = torch.zeros(n, dtype=torch.int16, device="cuda")
    handle.inspect(False, ta, tb, m, n, k, _dev(As), As.shape[0], _dev(Bs), Bs.shape[0],
                   mu=mu, nu=nu, C=dC, ldc=m)
    torch.cuda.synchronize()
    Are, Aim = core.rows_of_A(A)
    Bre, Bim = core.rows_of_B(B)
    omu, onu, fa, fb, _, _ = core.accurate_exponents(Are, Aim, Bre, Bim, N)
    assert np.array_equal(mu.cpu().numpy(), oracle_exp(omu, fa))
    assert np.array_equal(nu.cpu().numpy(), oracle_exp(onu, fb))
    rows, cols = _sample(m, 40, seed + 2), _sample(n, 40, seed + 3)
    ref = core.emulate(A[rows, :], B[:, cols], N, mode="accurate", algo=algo,
                       exponents=(omu[rows], fa[rows], onu[cols], fb[cols]))["out"]
    assert _bits_equal(_gather(dC, rows, cols), ref)
    handle.set_config(14, "fast", "karatsuba")


def test_accurate_zgemm_4096(handle):
    """ZGEMM 4096^3, accurate mode, 16 moduli, phi = 2 (the oracle's bound product is
    the full 4096^3 integer product of the 7-bit magnitudes)."""
    _accurate_case(handle, 4096, 4096, 4096, 16, "karatsuba", 2.0, workloads.seed_for(3, 0, "A"))


def test_accurate_long_k(handle):
    """Accurate mode on the long-k product schedule (256-tiles, k >= 16384), expanded
    products, transposed operands."""
    _accurate_case(handle, 1024, 1280, 16384, 20, "4m", 0.5, 3101, ta="T", tb="T")


@pytest.fixture(scope="module")
def long_k():
    m = n = 1024
    k = 65536
    A = workloads.complex_matrix(m, k, 2.0, 3201)
    B = workloads.complex_matrix(k, n, 2.0, 3202)
    return A, B, _dev(A), _dev(B)


@pytest.mark.parametrize("algo", ["karatsuba", "4m"])
def test_fast_long_k_65536(handle, long_k, algo):
    """Fast mode at 1024 x 1024 x 65536, 20 moduli (the shape class of the rectangular
    4096 x 4096 x 65536 configuration): sampled entries bit-exact."""
    import torch

    from oracle import core

    A, B, dA, dB = long_k
    m, k = A.shape
    n = B.shape[1]
    print(f"ZGEMM {m}x{n}x{k} N=20 {algo}", flush=True)
    handle.set_config(20, "fast", algo)
    dC = torch.zeros((n, m), dtype=torch.complex128, device="cuda")
    handle.zgemm("N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m)
    torch.cuda.synchronize()
    rows, cols = _sample(m, 24, 3203), _sample(n, 24, 3204)
    ref = core.emulate(A[rows, :], B[:, cols], 20, algo=algo)["out"]
    assert _bits_equal(_gather(dC, rows, cols), ref)
    handle.set_config(14, "fast", "karatsuba")
