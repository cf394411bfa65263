"""hipBLAS redirection (Section III-D: the emulation serves an unmodified program's
vendor BLAS GEMM calls through LD_PRELOAD).

An ordinary hipBLAS program (paper_2512_08321_amd/_build/blas_client, linked to the
image's libhipblas) runs one GEMM on inputs written here; with libozc_blas.so preloaded,
its result must equal the oracle's emulation bit for bit, for the typed calls
(hipblasZgemm, Cgemm, Dgemm, Sgemm), for hipblasGemmEx, and with scalars on the device.
Without the preload the same program runs the vendor routine (no redirection trace).
A GemmEx call with a compute type the emulation does not serve goes to the vendor."""
import os
import subprocess

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2512_08321_amd")
SHIM = os.path.join(PKG, "libozc_blas.so")
CLIENT = os.path.join(PKG, "_build", "blas_client")

DT = {"z": np.complex128, "c": np.complex64, "d": np.float64, "s": np.float32}


def _write(path, mat, ld):
    rows, cols = mat.shape
    host = np.zeros((cols, ld), dtype=mat.dtype)
    host[:, :rows] = mat.T
    host.tofile(path)


def _run(tmp, kind, api, ptr, A, B, C, alpha, beta, ta, tb, preload=True):
    """Run the client on op(A) = A, op(B) = B (stored per ta, tb) and return (C, stderr)."""
    m, k = A.shape
    n = B.shape[1]
    As = A if ta == "N" else (A.T if ta == "T" else A.conj().T)
    Bs = B if tb == "N" else (B.T if tb == "T" else B.conj().T)
    lda, ldb, ldc = As.shape[0] + 2, Bs.shape[0] + 1, m + 3
    fa, fb, fc, fo = (str(tmp / x) for x in ("A.bin", "B.bin", "C.bin", "out.bin"))
    _write(fa, np.asarray(As), lda)
    _write(fb, np.asarray(Bs), ldb)
    _write(fc, C, ldc)
    a, b = complex(alpha), complex(beta)
    env = dict(os.environ)
    env["OZC_BLAS_TRACE"] = "1"
    env["OZC_BLAS_DOUBLE_MODULI"] = "14"
    env["OZC_BLAS_SINGLE_MODULI"] = "8"
    if preload:
        env["LD_PRELOAD"] = SHIM + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    args = [CLIENT, kind, api, ptr, str(m), str(n), str(k), ta, tb, repr(a.real), repr(a.imag),
            repr(b.real), repr(b.imag), str(lda), str(ldb), str(ldc), fa, fb, fc, fo]
    print("client:", kind, api, ptr, m, n, k, ta, tb, "preload" if preload else "vendor", flush=True)
    r = subprocess.run(args, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(fo, dtype=C.dtype).reshape(n, ldc)[:, :m].T
    return out, r.stderr


def _oracle(kind, A, B, C, alpha, beta):
    from oracle import core

    if kind in "zc":
        return core.emulate(A, B, 14 if kind == "z" else 8, alpha=alpha, beta=beta, C=C,
                            single=kind == "c")["out"]
    return core.emulate_real(A, B, 14 if kind == "d" else 8, alpha=alpha, beta=beta, C=C,
                             single=kind == "s")["out"]


def _inputs(kind, m, n, k, seed):
    A = workloads.complex_matrix(m, k, 1.0, seed)
    B = workloads.complex_matrix(k, n, 1.0, seed + 1)
    C = workloads.complex_matrix(m, n, 1.0, seed + 2)
    if kind in "ds":
        A, B, C = A.real, B.real, C.real
    dt = DT[kind]
    return (np.asfortranarray(A.astype(dt)), np.asfortranarray(B.astype(dt)),
            np.asfortranarray(C.astype(dt)))


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint8)


@pytest.mark.parametrize("kind", ["z", "c", "d", "s"])
@pytest.mark.parametrize("api", ["typed", "ex"])
def test_redirected_gemm_equals_oracle(tmp_path, kind, api):
    assert os.path.exists(SHIM) and os.path.exists(CLIENT), "build() first"
    A, B, C = _inputs(kind, 70, 45, 130, 900 + ord(kind))
    cplx = kind in "zc"
    alpha = 0.75 - 0.25j if cplx else -1.25
    beta = 0.5 + 1.0j if cplx else 0.5
    ta, tb = ("C", "T") if cplx else ("T", "N")
    got, err = _run(tmp_path, kind, api, "host", A, B, C, alpha, beta, ta, tb)
    assert f"ozc-blas: {kind}gemm 70 x 45 x 130" in err
    ref = _oracle(kind, A, B, C, alpha, beta)
    assert got.dtype == ref.dtype and np.array_equal(_bits(got), _bits(ref))


def test_device_pointer_mode(tmp_path):
    A, B, C = _inputs("z", 33, 29, 57, 950)
    got, err = _run(tmp_path, "z", "typed", "device", A, B, C, 1.5 + 0.5j, -0.25j, "N", "N")
    assert "ozc-blas: zgemm" in err
    assert np.array_equal(_bits(got), _bits(_oracle("z", A, B, C, 1.5 + 0.5j, -0.25j)))


def test_without_preload_the_vendor_runs(tmp_path):
    A, B, C = _inputs("d", 40, 30, 50, 960)
    got, err = _run(tmp_path, "d", "typed", "host", A, B, C, 1.0, 0.0, "N", "N", preload=False)
    assert "ozc-blas" not in err
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.max(np.abs(got - exact)) <= 1e-12 * np.max(np.abs(A) @ np.abs(B))


def test_unserved_types_go_to_the_vendor(tmp_path):
    """hipblasGemmEx on half-precision A, B with float C: not a type the emulation serves,
    so the call reaches the vendor routine (no trace; result at half-precision accuracy)."""
    A, B, C = _inputs("s", 40, 30, 50, 970)
    got, err = _run(tmp_path, "s", "ex16", "host", A, B, C, 1.0, 0.0, "N", "N")
    assert "ozc-blas" not in err
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.max(np.abs(got - exact)) <= 1e-2 * np.max(np.abs(A) @ np.abs(B))
