"""The C-ABI library loads and exports every symbol include/ozc.h declares (no GPU needed)."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ozc.h")).read()
    return sorted(set(re.findall(r"\b(ozc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_all_declared_symbols():
    import paper_2512_08321_amd as ozc

    lib = ozc.lib()
    names = _declared()
    assert "ozc_zgemm" in names and "ozc_cgemm" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", ozc.library_path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ozc_\w+)", out))
    assert set(names) <= exported
    assert set(ozc.EXPORTS) == set(names)


def test_status_strings_and_no_device_errors():
    import ctypes

    import paper_2512_08321_amd as ozc

    lib = ozc.lib()
    assert lib.ozc_status_string(0) == b"success"
    assert lib.ozc_status_string(5) == b"non-finite input"
    # calls on a NULL handle report an error instead of crashing
    assert lib.ozc_set_config(None, 14, 0, 0) == 6
    assert lib.ozc_last_info(None, None) == 6
    h = ctypes.c_void_p()
    assert lib.ozc_create(None, 0) == 1


def test_header_constants_match_binding():
    import paper_2512_08321_amd as ozc

    text = open(os.path.join(ROOT, "include", "ozc.h")).read()
    m = re.search(r"#define OZC_NOALLOC_WORKSPACE \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == ozc.NOALLOC_WORKSPACE
    assert re.search(r"#define OZC_MAX_K (\d+)", text).group(1) == str(ozc.MAX_K)


def test_blas_shim_exports_the_redirected_calls():
    """libozc_blas.so defines the hipBLAS GEMM entry points it serves (Section III-D list)."""
    from paper_2512_08321_amd import build

    out = subprocess.run(["nm", "-D", "--defined-only", build.SHIM], capture_output=True,
                         text=True, check=True).stdout
    defined = set(re.findall(r"\bT (hipblas\w+)", out))
    want = {"hipblasSgemm", "hipblasDgemm", "hipblasCgemm", "hipblasZgemm", "hipblasGemmEx",
            "hipblasSgemm_64", "hipblasDgemm_64", "hipblasCgemm_64", "hipblasZgemm_64",
            "hipblasGemmEx_64"}
    assert want <= defined
    assert os.access(build.CLIENT, os.X_OK)
