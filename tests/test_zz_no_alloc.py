"""ozc_zgemm_noalloc (the entry point for callers that cannot allocate device
memory) against ozc_zgemm, through the C-ABI: bit-identical outputs on two calls
in a row, the second smaller than the first, so the second runs on the fixed
workspace the first left behind; shapes beyond the fixed workspace, the
Freivalds check and the learned moduli count are refused before any work."""
import numpy as np
import pytest

import workloads
from gpu_helpers import from_device, to_device

pytestmark = pytest.mark.gpu


def _call(h, fn, A, B, C, alpha, beta, ta="N", tb="N"):
    import torch

    m, k = A.shape
    n = B.shape[1]
    As = A if ta == "N" else np.asfortranarray(A.T if ta == "T" else A.conj().T)
    Bs = B if tb == "N" else np.asfortranarray(B.T if tb == "T" else B.conj().T)
    dA, lda = to_device(As, As.shape[0] + 3)
    dB, ldb = to_device(Bs)
    dC, ldc = to_device(np.asfortranarray(C), m + 1)
    fn(ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc)
    torch.cuda.synchronize()
    return from_device(dC, m, n, ldc)


def _same(a, b):
    """Bit-identical (NaN payloads and signed zeros included)."""
    return np.array_equal(np.ascontiguousarray(a).view(np.uint64),
                          np.ascontiguousarray(b).view(np.uint64))


@pytest.mark.parametrize("N,mode,algo", [(14, "fast", "karatsuba"), (9, "accurate", "4m")])
def test_noalloc_matches_zgemm_two_calls(N, mode, algo):
    import torch

    import paper_2512_08321_amd as ozc

    assert torch.cuda.is_available()
    h = ozc.Handle(0, num_moduli=N, mode=mode, algo=algo)
    try:
        # first a large call (several 128-tiles, ragged), then a smaller one with other
        # operations, alpha and beta: the second sees the first's leftovers in the array
        cases = [((600, 530, 700), "N", "N", 1.0, 0.0, 11),
                 ((97, 130, 75), "C", "T", 0.5 - 2j, 1.25 + 0.5j, 21)]
        for (m, n, k), ta, tb, alpha, beta, seed in cases:
            print(f"noalloc {m}x{n}x{k} {ta}{tb} N={N} {mode} {algo}", flush=True)
            A = workloads.complex_matrix(m, k, 1.0, seed)
            B = workloads.complex_matrix(k, n, 1.0, seed + 1)
            C = workloads.complex_matrix(m, n, 1.0, seed + 2)
            need = h.workspace_size(ta, tb, m, n, k)
            assert 0 < need <= ozc.NOALLOC_WORKSPACE
            want = _call(h, h.zgemm, A, B, C, alpha, beta, ta, tb)
            got = _call(h, h.zgemm_noalloc, A, B, C, alpha, beta, ta, tb)
            assert _same(got, want)
            assert np.isfinite(got.real).all() and np.isfinite(got.imag).all()
    finally:
        torch.cuda.synchronize()
        h.close()


def test_noalloc_refusals():
    import torch

    import paper_2512_08321_amd as ozc

    h = ozc.Handle(0, num_moduli=14)
    try:
        m = n = k = 1024   # 256-tiles: about 101 MiB of workspace at 14 moduli
        assert h.workspace_size("N", "N", m, n, k) > ozc.NOALLOC_WORKSPACE
        A = torch.zeros(m * k, dtype=torch.complex128, device="cuda")
        B = torch.zeros(k * n, dtype=torch.complex128, device="cuda")
        C = torch.full((m * n,), 3.0 + 0j, dtype=torch.complex128, device="cuda")
        with pytest.raises(ozc.OzcError) as e:
            h.zgemm_noalloc("N", "N", m, n, k, 1.0, A, m, B, k, 0.0, C, m)
        assert e.value.status == 2
        small = 64
        h.set_verify(True)
        with pytest.raises(ozc.OzcError) as e:
            h.zgemm_noalloc("N", "N", small, small, small, 1.0, A, small, B, small, 0.0, C, small)
        assert e.value.status == 2
        h.set_verify(False)
        h.set_config(0)
        with pytest.raises(ozc.OzcError) as e:
            h.zgemm_noalloc("N", "N", small, small, small, 1.0, A, small, B, small, 0.0, C, small)
        assert e.value.status == 2
        with pytest.raises(ozc.OzcError) as e:   # argument checks as ozc_zgemm
            h.zgemm_noalloc("N", "N", small, small, small, 1.0, A, small - 1, B, small, 0.0, C,
                            small)
        assert e.value.status == 1
        torch.cuda.synchronize()
        assert bool(torch.all(C == 3.0))   # nothing ran
    finally:
        torch.cuda.synchronize()
        h.close()
