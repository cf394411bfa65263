"""Build the HIP library libozc.so for gfx950 with hipcc (in-tree).

Every source under csrc/ is compiled to an object in _build/ and linked into
paper_2512_08321_amd/libozc.so.  Flags: -O3, gfx950 only, packed FP32
instructions disabled in device code.  Then the hipBLAS redirection library
libozc_blas.so (shim/hipblas_shim.cpp, linked to libozc.so) and its test client
_build/blas_client (an ordinary hipBLAS program).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libozc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["tables.cpp", "api.cpp", "batched.cpp", "autoN.cpp", "prep.hip", "gemm.hip", "crt.hip",
           "verify.hip", "mlp.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"-I{os.path.join(ROOT, 'include')}"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, "-c", "-x", "hip", *COMMON, os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if verbose and out.strip():
        print(out, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_shim(verbose)
    return LIB


SHIM = os.path.join(HERE, "libozc_blas.so")
CLIENT = os.path.join(BUILD, "blas_client")
ROCM_LIB = "/opt/rocm/lib"


def build_shim(verbose: bool = False) -> str:
    """libozc_blas.so (hipBLAS GEMM entry points served by libozc.so) and the client."""
    src = os.path.join(HERE, "shim", "hipblas_shim.cpp")
    cmd = [HIPCC, "-x", "hip", *COMMON, "-shared", src, "-o", SHIM + ".tmp", f"-L{HERE}", "-lozc",
           "-Wl,-rpath,$ORIGIN", f"-L{ROCM_LIB}", "-lhipblas", f"-Wl,-rpath,{ROCM_LIB}", "-ldl"]
    client = [HIPCC, "-x", "hip", "-O2", "-std=c++17", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              os.path.join(HERE, "shim", "blas_client.cpp"), "-o", CLIENT + ".tmp",
              f"-L{ROCM_LIB}", "-lhipblas", f"-Wl,-rpath,{ROCM_LIB}"]
    for c, out in ((cmd, SHIM), (client, CLIENT)):
        if verbose:
            print(" ".join(c), flush=True)
        r = subprocess.run(c, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {os.path.basename(out)}:\n{msg}")
        os.replace(out + ".tmp", out)
    return SHIM


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
