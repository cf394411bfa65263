"""GPU path (through the C-ABI) against the CPU oracle, element by element.

Bar: exponents, residues, INT32 products and E' bit-exact; outputs bit-exact
(the reconstruction is exact on both sides, and alpha/beta follow the same
fused multiply-add order).  NaN outputs compare as NaN.
"""
import os

import numpy as np
import pytest

import workloads
from gpu_helpers import from_device, oracle_exp, stored, to_device

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
    a = np.asarray(a)
    b = np.asarray(b)
    nan_a = np.isnan(a.real) | np.isnan(a.imag)
    nan_b = np.isnan(b.real) | np.isnan(b.imag)
    return np.array_equal(nan_a, nan_b) and np.array_equal(a[~nan_a], b[~nan_b])


def _run_inspect(h, orc, A, B, N, mode, algo, ta="N", tb="N", single=False, lda_pad=0, ldb_pad=0):
    import torch

    print(f"inspect m,n,k={A.shape[0]},{B.shape[1]},{A.shape[1]} N={N} {mode} {algo} {ta}{tb} "
          f"single={single}", flush=True)
    m, k = A.shape
    n = B.shape[1]
    h.set_config(N, mode, algo)
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_device(As, As.shape[0] + lda_pad)
    dB, ldb = to_device(Bs, Bs.shape[0] + ldb_pad)
    planes = 3 if algo == "karatsuba" else 2
    nprod = 3 if algo == "karatsuba" else 4
    dev = "cuda"
    mu = torch.zeros(m, dtype=torch.int16, device=dev)
    nu = torch.zeros(n, dtype=torch.int16, device=dev)
    rA = torch.zeros((N, planes, m, k), dtype=torch.int8, device=dev)
    rB = torch.zeros((N, planes, n, k), dtype=torch.int8, device=dev)
    pr = torch.zeros((N, nprod, n, m), dtype=torch.int32, device=dev)
    ep = torch.zeros((N, 2, n, m), dtype=torch.int8, device=dev)
    dC, ldc = to_device(np.zeros((m, n), dtype=A.dtype))
    h.inspect(single, ta, tb, m, n, k, dA, lda, dB, ldb, mu, nu, rA, rB, pr, ep, dC, ldc)
    torch.cuda.synchronize()
    ref = orc.emulate(A, B, N, mode, algo, single=single, want_raw=True)
    return dict(mu=mu.cpu().numpy(), nu=nu.cpu().numpy(), rA=rA.cpu().numpy(), rB=rB.cpu().numpy(),
                pr=pr.cpu().numpy(), ep=ep.cpu().numpy(), out=from_device(dC, m, n, ldc)), ref


def _check_inspect(g, ref, algo):
    planes = 3 if algo == "karatsuba" else 2
    assert np.array_equal(g["mu"], oracle_exp(ref["mu"], ref["fa"])), "mu"
    assert np.array_equal(g["nu"], oracle_exp(ref["nu"], ref["fb"])), "nu"
    assert np.array_equal(g["rA"], ref["resA"][:, :planes]), "residues of A"
    assert np.array_equal(g["rB"], ref["resB"][:, :planes]), "residues of B"
    assert np.array_equal(g["pr"].transpose(0, 1, 3, 2), ref["raw"].astype(np.int32)), "INT32 products"
    assert np.array_equal(g["ep"].transpose(0, 1, 3, 2), ref["Ep"]), "E'"
    assert _same(g["out"], ref["out"]), "output"


# several tiles in every dimension plus ragged tails
@pytest.mark.parametrize("mode", ["fast", "accurate"])
@pytest.mark.parametrize("algo", ["karatsuba", "4m"])
def test_intermediates_bit_exact(handle, orc, mode, algo):
    A = workloads.complex_matrix(300, 150, 1.0, 11)
    B = workloads.complex_matrix(150, 200, 1.0, 12)
    g, ref = _run_inspect(handle, orc, A, B, 14, mode, algo)
    _check_inspect(g, ref, algo)


@pytest.mark.parametrize("mode,algo", [("fast", "karatsuba"), ("accurate", "4m")])
def test_large_tile_path_bit_exact(handle, orc, mode, algo):
    """m, n >= 1024 selects the 256 x 256 product tile; ragged edges in every dimension."""
    A = workloads.complex_matrix(1100, 96, 2.0, 91)
    B = workloads.complex_matrix(96, 1030, 2.0, 92)
    g, ref = _run_inspect(handle, orc, A, B, 13, mode, algo)
    _check_inspect(g, ref, algo)


@pytest.mark.parametrize("ta,tb", [("N", "T"), ("T", "N"), ("C", "C"), ("T", "C"), ("C", "N")])
def test_transpose_ops(handle, orc, ta, tb):
    A = workloads.complex_matrix(131, 77, 2.0, 21)
    B = workloads.complex_matrix(77, 140, 2.0, 22)
    g, ref = _run_inspect(handle, orc, A, B, 13, "fast", "karatsuba", ta, tb, lda_pad=3, ldb_pad=5)
    _check_inspect(g, ref, "karatsuba")


@pytest.mark.parametrize("N", [2, 3, 6, 9, 12, 16, 20, 24])
def test_moduli_counts(handle, orc, N):
    A = workloads.complex_matrix(129, 64, 4.0, 30 + N)
    B = workloads.complex_matrix(64, 130, 4.0, 60 + N)
    for mode in ("fast", "accurate"):
        g, ref = _run_inspect(handle, orc, A, B, N, mode, "karatsuba")
        _check_inspect(g, ref, "karatsuba")


@pytest.mark.parametrize("N", [6, 8, 12])
def test_cgemm_intermediates(handle, orc, N):
    A = workloads.complex_matrix(200, 96, 0.5, 41, dtype=np.complex64)
    B = workloads.complex_matrix(96, 160, 0.5, 42, dtype=np.complex64)
    for algo in ("karatsuba", "4m"):
        g, ref = _run_inspect(handle, orc, A, B, N, "fast", algo, single=True)
        _check_inspect(g, ref, algo)
        assert g["out"].dtype == np.complex64


def _gemm_call(h, A, B, C, alpha, beta, N, mode="fast", algo="karatsuba", ta="N", tb="N"):
    import torch

    m, k = A.shape
    n = B.shape[1]
    h.set_config(N, mode, algo)
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_device(As)
    dB, ldb = to_device(Bs)
    dC, ldc = to_device(np.asfortranarray(C.astype(A.dtype)), m + 2)
    fn = h.zgemm if A.dtype == np.complex128 else h.cgemm
    fn(ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc)
    torch.cuda.synchronize()
    return from_device(dC, m, n, ldc)


@pytest.mark.parametrize("single", [False, True])
def test_alpha_beta(handle, orc, single):
    dt = np.complex64 if single else np.complex128
    A = workloads.complex_matrix(70, 33, 1.0, 51, dtype=dt)
    B = workloads.complex_matrix(33, 90, 1.0, 52, dtype=dt)
    C = workloads.complex_matrix(70, 90, 1.0, 53, dtype=dt)
    for alpha, beta in [(0.5 - 2j, 1.5 + 0.25j), (-1.0, 0.75j), (2.0, 0.0), (1.0, 1.0)]:
        got = _gemm_call(handle, A, B, C, alpha, beta, 11)
        ref = orc.emulate(A, B, 11, alpha=alpha, beta=beta, C=C, single=single)["out"]
        assert _same(got, ref), (alpha, beta)


def test_edge_cases(handle, orc):
    import torch

    # 1x1x1, zero rows/columns, integer-valued inputs
    for (m, n, k) in [(1, 1, 1), (1, 7, 3), (5, 1, 200), (128, 128, 64), (129, 127, 65)]:
        A = workloads.complex_matrix(m, k, 1.0, m + k)
        B = workloads.complex_matrix(k, n, 1.0, n + k)
        if m > 2:
            A[1, :] = 0
        if n > 2:
            B[:, 2] = 0
        got = _gemm_call(handle, A, B, np.zeros((m, n)), 1.0, 0.0, 14)
        assert _same(got, orc.emulate(A, B, 14)["out"]), (m, n, k)
    A = workloads.integer_matrix(64, 512, 12, 1)
    B = workloads.integer_matrix(512, 48, 12, 2)
    got = _gemm_call(handle, A, B, np.zeros((64, 48)), 1.0, 0.0, 14, "accurate")
    assert np.array_equal(got, A @ B)
    # k == 0 and alpha == 0: C := beta C
    C = workloads.complex_matrix(9, 11, 1.0, 5)
    A = workloads.complex_matrix(9, 4, 1.0, 6)
    B = workloads.complex_matrix(4, 11, 1.0, 7)
    got = _gemm_call(handle, A, B, C, 0.0, 0.5 - 1j, 14)
    ref = orc.emulate(A, B, 14, alpha=0.0, beta=0.5 - 1j, C=C)["out"]
    assert _same(got, ref)
    got = _gemm_call(handle, A[:, :0], B[:0, :], C, 2.0, -1.0, 14)
    ref = orc.emulate(A[:, :0], B[:0, :], 14, alpha=2.0, beta=-1.0, C=C)["out"]
    assert _same(got, ref)
    # m == 0: nothing happens
    handle.zgemm("N", "N", 0, 5, 5, 1.0, 0, 1, 0, 5, 0.0, 0, 1)
    torch.cuda.synchronize()


def _extreme_operands():
    """Rows and columns scaled across the whole double range (subnormal rows, rows near
    2^900), a spread of 2^-80..1 inside every row, signed zeros and lone subnormals in
    normal rows; every product stays finite."""
    m, k, n = 70, 80, 66
    A = workloads.complex_matrix(m, k, 2.0, 901)
    B = workloads.complex_matrix(k, n, 2.0, 902)
    rng = np.random.default_rng(903)
    inner_a = rng.integers(-80, 1, size=(m, k))
    inner_b = rng.integers(-80, 1, size=(k, n))
    A = np.ldexp(A.real, inner_a) + 1j * np.ldexp(A.imag, inner_a)
    B = np.ldexp(B.real, inner_b) + 1j * np.ldexp(B.imag, inner_b)
    row_exp = np.array([-1060, -1030, -520, 0, 480, 900] * 12)[:m]
    col_exp = np.array([-900, -400, 0, 60, -1000, 30] * 11)[:n]
    A = workloads.skewed(np.asfortranarray(A), row_exp=row_exp)
    B = workloads.skewed(np.asfortranarray(B), col_exp=col_exp)
    A[3, :5] = -0.0
    A[4, 7] = complex(-0.0, 0.0)
    A[5, 9] = complex(5e-324, -5e-324)
    B[11, 3] = complex(0.0, -0.0)
    B[12, 4] = complex(-2.5e-320, 1e-310)
    return np.asfortranarray(A), np.asfortranarray(B)


@pytest.mark.parametrize("N,mode", [(6, "fast"), (14, "fast"), (14, "accurate"), (20, "fast"),
                                    (24, "accurate")])
def test_extreme_magnitudes_bit_exact(handle, orc, N, mode):
    """Every word count of the residue split (1 to 4) on inputs across the double range."""
    A, B = _extreme_operands()
    assert np.isfinite(A).all() and np.isfinite(B).all()
    g, ref = _run_inspect(handle, orc, A, B, N, mode, "karatsuba")
    _check_inspect(g, ref, "karatsuba")


def _random_case(i):
    rng = np.random.default_rng(7000 + i)
    dims = []
    for _ in range(3):
        if rng.random() < 0.25:  # near a tile or slab edge
            d = int(rng.choice([64, 128, 256])) + int(rng.integers(-1, 2))
        else:
            d = int(round(np.exp(rng.uniform(0.0, np.log(400)))))
        dims.append(max(1, d))
    m, n, k = dims
    single = bool(rng.random() < 0.3)
    N = int(rng.integers(2, 17 if single else 25))
    mode = str(rng.choice(["fast", "accurate"]))
    algo = str(rng.choice(["karatsuba", "4m"]))
    ta, tb = (str(rng.choice(["N", "T", "C"])) for _ in range(2))
    phi = float(rng.uniform(0.0, 6.0))
    pads = tuple(int(x) for x in rng.integers(0, 4, size=2))
    return m, n, k, single, N, mode, algo, ta, tb, phi, pads


@pytest.mark.parametrize("i", range(int(os.environ.get("OZC_RANDOM_CASES", "200"))))
def test_randomized_configurations(handle, orc, i):
    """Seeded random shapes (1..400, tile edges +-1), moduli counts, modes, product forms,
    op() forms, value spreads, precisions and leading-dimension padding (200 cases; the
    environment variable OZC_RANDOM_CASES runs more)."""
    m, n, k, single, N, mode, algo, ta, tb, phi, (pa, pb) = _random_case(i)
    dt = np.complex64 if single else np.complex128
    A = workloads.complex_matrix(m, k, phi, 8000 + 2 * i, dtype=dt)
    B = workloads.complex_matrix(k, n, phi, 8001 + 2 * i, dtype=dt)
    g, ref = _run_inspect(handle, orc, A, B, N, mode, algo, ta, tb, single=single, lda_pad=pa,
                          ldb_pad=pb)
    _check_inspect(g, ref, algo)


@pytest.mark.parametrize("algo", ["karatsuba", "4m"])
def test_row_padding_left_from_an_earlier_call(handle, orc, algo):
    """The split leaves the padding rows of the residue planes as an earlier call left
    them (they meet only output rows and columns past the product): a ragged product
    right after a larger one with other data and moduli count in the same workspace keeps
    every intermediate and the output bit-exact."""
    A = workloads.complex_matrix(600, 300, 4.0, 901)
    B = workloads.complex_matrix(300, 500, 4.0, 902)
    _gemm_call(handle, A, B, np.zeros((600, 500)), 1.0, 0.0, 20, "fast", algo)
    A = workloads.complex_matrix(131, 190, 0.5, 903)
    B = workloads.complex_matrix(190, 77, 0.5, 904)
    g, ref = _run_inspect(handle, orc, A, B, 14, "fast", algo)
    _check_inspect(g, ref, algo)


def test_nonfinite_inputs(handle, orc):
    A = workloads.complex_matrix(40, 20, 1.0, 71)
    B = workloads.complex_matrix(20, 30, 1.0, 72)
    A[3, 5] = complex(np.inf, 0)
    B[7, 9] = complex(0, np.nan)
    got = _gemm_call(handle, A, B, np.zeros((40, 30)), 1.0, 0.0, 12)
    info = handle.last_info()
    assert info["nonfinite"] == 1
    ref = orc.emulate(A, B, 12)["out"]
    assert _same(got, ref)
    assert np.isnan(got[3, :].real).all() and np.isnan(got[:, 9].real).all()


def test_argument_errors(handle):
    """Rejected before any work.  The operands are real device buffers of the declared
    shapes, so that a regression in the checks would compute on valid memory and fail
    an assertion instead of touching unowned addresses."""
    import torch

    import paper_2512_08321_amd as ozc

    kbig = ozc.MAX_K + 1
    A = torch.zeros(4 * kbig, dtype=torch.complex128, device="cuda")  # 4 x kbig, lda 4
    B = torch.zeros(kbig * 4, dtype=torch.complex128, device="cuda")  # kbig x 4, ldb kbig
    C = torch.zeros(16, dtype=torch.complex128, device="cuda")        # 4 x 4, ldc 4
    with pytest.raises(ozc.OzcError) as e:
        handle.zgemm("N", "N", 4, 4, 4, 1.0, A, 3, B, 4, 0.0, C, 4)  # lda < m
    assert e.value.status == 1
    with pytest.raises(ozc.OzcError) as e:  # k above the INT32 limit: inspect does not chunk
        handle.inspect(False, "N", "N", 4, 4, kbig, A, 4, B, kbig, C=C, ldc=4)
    assert e.value.status == 2
    with pytest.raises(ozc.OzcError) as e:
        handle.gemm_vbatched([dict(transa="N", transb="N", m=4, n=4, k=kbig, alpha=1.0,
                                   beta=0.0, A=A, lda=4, B=B, ldb=kbig, C=C, ldc=4)])
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert not bool(torch.any(C != 0))
    with pytest.raises(ozc.OzcError):
        handle.set_config(25)
    handle.set_config(14)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "T")])
def test_k_above_int32_limit_is_chunked(handle, orc, ta, tb):
    """k > 2^17: near-equal k chunks, each emulated on its own, accumulated with beta = 1;
    bit-exact with the oracle doing the same chunking."""
    import paper_2512_08321_amd as ozc

    k = ozc.MAX_K + 1000
    m, n = 6, 5
    print(f"k-chunk {ta}{tb} k={k}", flush=True)
    A = workloads.complex_matrix(m, k, 0.5, 141)
    B = workloads.complex_matrix(k, n, 0.5, 142)
    C = workloads.complex_matrix(m, n, 1.0, 143)
    alpha, beta = 0.75 - 0.5j, 0.5 + 1j
    got = _gemm_call(handle, A, B, C, alpha, beta, 14, ta=ta, tb=tb)
    half = k // 2
    ref = orc.emulate(A[:, :half], B[:half], 14, alpha=alpha, beta=beta, C=C)["out"]
    ref = orc.emulate(A[:, half:], B[half:], 14, alpha=alpha, beta=1.0, C=ref)["out"]
    assert _same(got, ref)


def test_k_chunks_keep_nonfinite_status(handle, orc):
    """An inf in the first k-chunk (k = 2^17 + 1000: two chunks) still reports the
    non-finite status after the last chunk, and the NaN rows and columns equal the
    oracle's chunked result."""
    import paper_2512_08321_amd as ozc

    k = ozc.MAX_K + 1000
    m, n = 6, 5
    print(f"k-chunk nonfinite k={k}", flush=True)
    A = workloads.complex_matrix(m, k, 0.5, 151)
    B = workloads.complex_matrix(k, n, 0.5, 152)
    A[2, 10] = complex(np.inf, 0.0)   # first chunk, row 2
    B[20, 3] = complex(0.0, np.nan)   # first chunk, column 3
    got = _gemm_call(handle, A, B, np.zeros((m, n)), 1.0, 0.0, 14)
    info = handle.last_info()
    assert info["nonfinite"] == 1
    half = k // 2
    ref = orc.emulate(A[:, :half], B[:half], 14)["out"]
    ref = orc.emulate(A[:, half:], B[half:], 14, alpha=1.0, beta=1.0, C=ref)["out"]
    assert _same(got, ref)
    assert np.isnan(got[2, :].real).all() and np.isnan(got[:, 3].real).all()
    # a clean call afterwards clears the flag
    got = _gemm_call(handle, A[:, 100:], B[100:], np.zeros((m, n)), 1.0, 0.0, 14)
    assert handle.last_info()["nonfinite"] == 0


@pytest.mark.parametrize("algo", ["karatsuba", "4m"])
def test_accumulators_near_int32_limit(handle, orc, algo):
    """k = 2^17 (the largest unchunked k) with constant operands: every term of a
    residue product has the same sign, so the INT32 accumulators reach 0.87 * 2^31
    (Karatsuba; 0.67 * 2^31 expanded) for an odd modulus, and the epilogue adds a carried
    residue to an unreduced accumulator; bit-exact with the oracle."""
    import paper_2512_08321_amd as ozc

    k = ozc.MAX_K
    a, b = 0.9833534339803927 + 0.44735250930159265j, 0.6176876180693398 - 0.6942699537086543j
    A = np.full((3, k), a)
    B = np.full((k, 2), b)
    print(f"int32-limit {algo} k={k}", flush=True)
    ref = orc.emulate(A, B, 14, algo=algo)
    ra, rb = np.asarray(ref["resA"]), np.asarray(ref["resB"])
    pairs = [(0, 0), (1, 1), (2, 2)] if algo == "karatsuba" else [(0, 0), (1, 1), (0, 1), (1, 0)]
    biggest = max(abs(int(ra[l, pa].flat[0]) * int(rb[l, pb].flat[0])) * k
                  for l in range(1, 14) for pa, pb in pairs)
    assert biggest >= (0.85 if algo == "karatsuba" else 0.65) * 2.0 ** 31
    got = _gemm_call(handle, A, B, np.zeros((3, 2)), 1.0, 0.0, 14, "fast", algo)
    assert _same(got, ref["out"])


def test_config0_workload_bit_exact(handle, orc):
    """256^3 complex128, 14 moduli, 4-GEMM products, alpha = 1, beta = 0, phi = 0.5."""
    A = workloads.complex_matrix(256, 256, 0.5, workloads.seed_for(0, 0, "A"))
    B = workloads.complex_matrix(256, 256, 0.5, workloads.seed_for(0, 0, "B"))
    got = _gemm_call(handle, A, B, np.zeros((256, 256)), 1.0, 0.0, 14, "fast", "4m")
    ref = orc.emulate(A, B, 14, "fast", "4m")["out"]
    assert _same(got, ref)
    hi, lo = orc.dd_gemm(A, B)
    err = orc.err_nc(got, hi, lo, orc.abs_product(A, B))
    assert err <= 4 * 256 * 2.0 ** -53


def test_deterministic_and_row_major_api(handle):
    import torch

    import paper_2512_08321_amd as ozc

    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    A = torch.randn(300, 257, dtype=torch.complex128, device="cuda", generator=g)
    B = torch.randn(257, 190, dtype=torch.complex128, device="cuda", generator=g)
    c1 = ozc.gemm(A, B, num_moduli=14, handle=handle)
    c2 = ozc.gemm(A, B, num_moduli=14, handle=handle)
    assert torch.equal(c1, c2)
    ref = (A.cpu() @ B.cpu())
    rel = ((c1.cpu() - ref).abs() / (A.cpu().abs() @ B.cpu().abs())).max().item()
    assert rel < 4 * 257 * 2.0 ** -53


@pytest.mark.parametrize("algo", ["karatsuba", "4m"])
def test_large_tiles_both_schedules_sampled(handle, orc, algo):
    """256 x 256 product tiles with k below and at the long-k bound (16384): the two
    product schedules.  Fast-mode exponents depend only on their own row or column, so
    sampled rows and columns of the full GPU result are checked bit for bit against the
    oracle run on those rows and columns alone (full k)."""
    rng = np.random.default_rng(151)
    for k in (8192, 16384):
        m, n = 1030, 1100
        print(f"large tiles {algo} k={k}", flush=True)
        A = workloads.complex_matrix(m, k, 1.0, 152 + k)
        B = workloads.complex_matrix(k, n, 1.0, 153 + k)
        got = _gemm_call(handle, A, B, np.zeros((m, n)), 1.0, 0.0, 14, "fast", algo)
        rows = np.unique(np.r_[0, m - 1, rng.choice(m, 10, replace=False)])
        cols = np.unique(np.r_[0, n - 1, rng.choice(n, 10, replace=False)])
        ref = orc.emulate(A[rows], B[:, cols], 14, "fast", algo)["out"]
        assert _same(got[np.ix_(rows, cols)], ref)
