"""Real products (ozc_dgemm / ozc_sgemm, Algorithm 1 for real A and B) against the
oracle's real path, through the C-ABI: exponents, residues, INT32 products, E' and
outputs bit-exact; argument semantics as for complex products."""
import numpy as np
import pytest

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


def real_matrix(rows, cols, phi, seed, dtype=np.float64):
    """Column-major real matrix with entries (u - 0.5) exp(phi g) (the real parts of the
    complex generator's distribution)."""
    import workloads

    z = workloads.complex_matrix(rows, cols, phi, seed)
    return np.asfortranarray(z.real.astype(dtype))


def to_dev(mat, ld=None):
    """Column-major real matrix -> device buffer with leading dimension ld (NaN padding)."""
    import torch

    rows, cols = mat.shape
    ld = max(1, rows) if ld is None else ld
    host = np.full((max(cols, 1), ld), np.nan, dtype=mat.dtype)
    host[:cols, :rows] = mat.T
    return torch.from_numpy(host).cuda(), ld


def from_dev(buf, rows, cols, ld):
    return np.asfortranarray(buf.cpu().numpy()[:cols, :rows].T)


def stored(op_mat, op):
    return op_mat if op == "N" else np.asfortranarray(op_mat.T)


def _exp(mu, flags):
    out = np.array(mu, dtype=np.int64)
    out[flags == 0] = -32768
    out[flags == 2] = 32767
    return out.astype(np.int16)


def _inspect(h, orc, A, B, N, mode, ta="N", tb="N", pad=(0, 0)):
    import torch

    single = A.dtype == np.float32
    m, k = A.shape
    n = B.shape[1]
    print(f"real inspect {m}x{n}x{k} N={N} {mode} {ta}{tb} single={single}", flush=True)
    h.set_config(N, mode, "karatsuba")
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_dev(As, As.shape[0] + pad[0])
    dB, ldb = to_dev(Bs, Bs.shape[0] + pad[1])
    mu = torch.zeros(m, dtype=torch.int16, device="cuda")
    nu = torch.zeros(n, dtype=torch.int16, device="cuda")
    rA = torch.zeros((N, 1, m, k), dtype=torch.int8, device="cuda")
    rB = torch.zeros((N, 1, n, k), dtype=torch.int8, device="cuda")
    pr = torch.zeros((N, 1, n, m), dtype=torch.int32, device="cuda")
    ep = torch.zeros((N, 1, n, m), dtype=torch.int8, device="cuda")
    dC, ldc = to_dev(np.zeros((m, n), dtype=A.dtype), m + 1)
    h.inspect(3 if single else 2, ta, tb, m, n, k, dA, lda, dB, ldb, mu, nu, rA, rB, pr, ep, dC, ldc)
    torch.cuda.synchronize()
    ref = orc.emulate_real(A, B, N, mode, single=single, want_raw=True)
    assert np.array_equal(mu.cpu().numpy(), _exp(ref["mu"], ref["fa"])), "mu"
    assert np.array_equal(nu.cpu().numpy(), _exp(ref["nu"], ref["fb"])), "nu"
    assert np.array_equal(rA.cpu().numpy()[:, 0], ref["resA"]), "residues of A"
    assert np.array_equal(rB.cpu().numpy()[:, 0], ref["resB"]), "residues of B"
    assert np.array_equal(pr.cpu().numpy()[:, 0].transpose(0, 2, 1), ref["raw"].astype(np.int32)), "products"
    assert np.array_equal(ep.cpu().numpy()[:, 0].transpose(0, 2, 1), ref["Ep"]), "E'"
    got = from_dev(dC, m, n, ldc)
    assert got.dtype == ref["out"].dtype
    assert np.array_equal(got, ref["out"]), "output"


@pytest.mark.parametrize("mode", ["fast", "accurate"])
def test_real_intermediates(handle, orc, mode):
    _inspect(handle, orc, real_matrix(300, 150, 1.0, 11), real_matrix(150, 200, 1.0, 12), 14, mode)


@pytest.mark.parametrize("mode", ["fast", "accurate"])
def test_real_large_tiles(handle, orc, mode):
    """m, n >= 1024: 256 x 256 product tiles, ragged edges."""
    _inspect(handle, orc, real_matrix(1100, 96, 2.0, 13), real_matrix(96, 1030, 2.0, 14), 15, mode)


@pytest.mark.parametrize("ta,tb", [("T", "N"), ("N", "T"), ("T", "T"), ("C", "C")])
def test_real_ops_and_padding(handle, orc, ta, tb):
    _inspect(handle, orc, real_matrix(131, 77, 2.0, 15), real_matrix(77, 140, 2.0, 16), 13, "fast",
             ta, tb, pad=(3, 5))


@pytest.mark.parametrize("N", [2, 5, 9, 16, 20, 24])
def test_real_moduli_counts(handle, orc, N):
    for mode in ("fast", "accurate"):
        _inspect(handle, orc, real_matrix(129, 64, 4.0, 20 + N), real_matrix(64, 130, 4.0, 50 + N),
                 N, mode)


def test_sgemm_intermediates(handle, orc):
    _inspect(handle, orc, real_matrix(200, 96, 0.5, 31, np.float32),
             real_matrix(96, 160, 0.5, 32, np.float32), 8, "fast")


def _call(h, A, B, C, alpha, beta, N, ta="N", tb="N", mode="fast"):
    import torch

    m, k = A.shape
    n = B.shape[1]
    h.set_config(N, mode, "karatsuba")
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_dev(As)
    dB, ldb = to_dev(Bs)
    dC, ldc = to_dev(np.asfortranarray(C.astype(A.dtype)), m + 2)
    fn = h.sgemm if A.dtype == np.float32 else h.dgemm
    fn(ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc)
    torch.cuda.synchronize()
    return from_dev(dC, m, n, ldc)


def _same(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_real_alpha_beta(handle, orc, dtype):
    A = real_matrix(70, 33, 1.0, 41, dtype)
    B = real_matrix(33, 90, 1.0, 42, dtype)
    C = real_matrix(70, 90, 1.0, 43, dtype)
    for alpha, beta in [(0.5, 1.5), (-1.0, -0.25), (2.0, 0.0), (1.0, 1.0)]:
        got = _call(handle, A, B, C, alpha, beta, 11)
        ref = orc.emulate_real(A, B, 11, alpha=alpha, beta=beta, C=C,
                               single=dtype == np.float32)["out"]
        assert np.array_equal(got, ref), (alpha, beta)


def test_real_edge_cases(handle, orc):
    A = real_matrix(37, 19, 1.0, 51)
    B = real_matrix(19, 23, 1.0, 52)
    C = real_matrix(37, 23, 1.0, 53)
    A[5, :] = 0.0
    B[:, 7] = 0.0
    got = _call(handle, A, B, C, 1.0, 0.0, 12)
    ref = orc.emulate_real(A, B, 12)["out"]
    assert np.array_equal(got, ref) and not got[5].any() and not got[:, 7].any()
    # alpha = 0: C := beta C without reading A, B; k = 0 likewise
    got = _call(handle, A, B, C, 0.0, 2.0, 12)
    assert np.array_equal(got, 2.0 * C)
    got = _call(handle, A[:, :0], B[:0, :], C, 1.0, -1.0, 12)
    assert np.array_equal(got, -C)
    # 1 x 1 x 1 and integer inputs (exact)
    Ai = np.asfortranarray(np.array([[3.0, -7.0, 11.0]]))
    Bi = np.asfortranarray(np.array([[2.0], [5.0], [-1.0]]))
    assert _call(handle, Ai, Bi, np.zeros((1, 1)), 1.0, 0.0, 6)[0, 0] == 3 * 2 - 35 - 11
    got = _call(handle, A[:1, :1], B[:1, :1], C[:1, :1], 1.0, 0.0, 14)
    assert np.array_equal(got, orc.emulate_real(A[:1, :1], B[:1, :1], 14)["out"])


def test_real_nonfinite(handle, orc):
    A = real_matrix(40, 20, 1.0, 61)
    B = real_matrix(20, 30, 1.0, 62)
    A[3, 5] = np.inf
    B[7, 9] = np.nan
    got = _call(handle, A, B, np.zeros((40, 30)), 1.0, 0.0, 12)
    assert handle.last_info()["nonfinite"] == 1
    assert _same(got, orc.emulate_real(A, B, 12)["out"])
    assert np.isnan(got[3, :]).all() and np.isnan(got[:, 9]).all()


def test_real_k_chunks(handle, orc):
    """k > 2^17: near-equal chunks, each emulated with its own exponents, beta = 1 after
    the first; the oracle does the same chunking."""
    import paper_2512_08321_amd as ozc

    k = ozc.MAX_K + 777
    A = real_matrix(6, k, 0.5, 71)
    B = real_matrix(k, 5, 0.5, 72)
    C = real_matrix(6, 5, 1.0, 73)
    got = _call(handle, A, B, C, 0.75, 0.5, 14, ta="T", tb="N")
    half = k // 2
    ref = orc.emulate_real(A[:, :half], B[:half], 14, alpha=0.75, beta=0.5, C=C)["out"]
    ref = orc.emulate_real(A[:, half:], B[half:], 14, alpha=0.75, beta=1.0, C=ref)["out"]
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("mode,N", [("fast", 14), ("accurate", 16)])
def test_dgemm_4096_sampled(handle, orc, mode, N):
    """DGEMM 4096^3 (phi = 0.5): exponents of every row and column and sampled outputs
    bit-exact (accurate mode: the oracle's bound product over the full matrices)."""
    import torch

    m = n = k = 4096
    A = real_matrix(m, k, 0.5, 81)
    B = real_matrix(k, n, 0.5, 82)
    print(f"DGEMM 4096^3 {mode} N={N}", flush=True)
    handle.set_config(N, mode, "karatsuba")
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    dC = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    mu = torch.zeros(m, dtype=torch.int16, device="cuda")
    nu = torch.zeros(n, dtype=torch.int16, device="cuda")
    handle.inspect(2, "N", "N", m, n, k, dA, m, dB, k, mu=mu, nu=nu, C=dC, ldc=m)
    torch.cuda.synchronize()
    Are = np.ascontiguousarray(A)
    Bre = np.ascontiguousarray(B.T)
    if mode == "fast":
        omu, fa, _, _ = orc.fast_exponents(Are, np.zeros_like(Are), N)
        onu, fb, _, _ = orc.fast_exponents(Bre, np.zeros_like(Bre), N)
    else:
        omu, onu, fa, fb, _, _ = orc.accurate_exponents(Are, np.zeros_like(Are), Bre,
                                                        np.zeros_like(Bre), N)
    assert np.array_equal(mu.cpu().numpy(), _exp(omu, fa))
    assert np.array_equal(nu.cpu().numpy(), _exp(onu, fb))
    rng = np.random.default_rng(83)
    rows = np.unique(np.concatenate([rng.choice(m, 40, replace=False), [0, 255, 256, m - 1]]))
    cols = np.unique(np.concatenate([rng.choice(n, 40, replace=False), [0, 255, 256, n - 1]]))
    ref = orc.emulate_real(A[rows, :], B[:, cols], N, mode,
                           exponents=(omu[rows], fa[rows], onu[cols], fb[cols]))["out"]
    r = torch.from_numpy(rows).cuda()
    c = torch.from_numpy(cols).cuda()
    got = dC.index_select(0, c).index_select(1, r).cpu().numpy().T
    assert np.array_equal(got, ref)
